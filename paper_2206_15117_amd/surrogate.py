"""Learned A x W kernel generator.

A network (pg_mlp: SiLU hidden layers, linear head, bfloat16 matrix-core products) maps
(w, frequency, parallactic angle, Mueller cell) to one oversampled gridding-kernel cell,
[os][os][S][S] complex.  Its teacher is pg_make_kernels, which also stays the fallback and the
judge of error: training pairs are the FFT generator's own cells, exported from its tables.

Features of one cell: [w / w_max, (nu - nu_mid) / nu_half, sin pa, cos pa, one-hot(q npol + c)].
Targets are divided by a per-cell scale (the RMS of that Mueller cell over a reference draw) so
every output of the network is of order one; pg_kernels_import multiplies the scale back in.

Training (fit): the teacher's kernels span a low-dimensional space (a few dozen directions per
Mueller cell), so the head is trained in two stages.  A rank-r orthonormal basis B of the
(scaled) kernels is taken from a first block of teacher calls (randomised SVD: a Gaussian range
finder with power iterations, every large product in the library's float32 GEMM, orthonormalised
by shifted Cholesky QR whose r x r Gram factors are the only host arithmetic); the network is
trained with its output layer in basis coordinates (targets K B^T, r outputs), which is cheap
enough for many epochs over every teacher kernel; the output layer is then folded with the basis,
W_head = W_r B, b_head = b_r B, giving the network of the stated shape that emits kernels
directly, and optionally fine-tuned on kernel-space targets.  Every training step runs in the
library's forward/backward/Adam kernels.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import polgrid as pg

N_CELLS = 16


EXTENDED = True


def n_features() -> int:
    return (8 if EXTENDED else 4) + N_CELLS


def features(w, nu, pa, cell, w_max: float, nu_lo: float, nu_hi: float) -> np.ndarray:
    """float32 [B][n_features()] rows for per-row (w, nu, pa, Mueller cell index):
    w / w_max, (nu - nu_mid) / nu_half, sin pa, cos pa, then (extended set) sin 2pa, cos 2pa (the
    feed rotation enters the Mueller matrix through the double angle), nu_lo / nu (beam widths scale
    with 1/nu) and (w / w_max)^2, then the one-hot Mueller cell."""
    w, nu, pa, cell = (np.atleast_1d(np.asarray(a, dtype=np.float64)) for a in (w, nu, pa, cell))
    b = max(len(w), len(nu), len(pa), len(cell))
    w, nu, pa = (np.broadcast_to(a, (b,)) for a in (w, nu, pa))
    nf = n_features() - N_CELLS
    x = np.zeros((b, nf + N_CELLS), dtype=np.float32)
    mid, half = 0.5 * (nu_lo + nu_hi), 0.5 * (nu_hi - nu_lo)
    x[:, 0] = w / w_max
    x[:, 1] = (nu - mid) / half
    x[:, 2] = np.sin(pa)
    x[:, 3] = np.cos(pa)
    if EXTENDED:
        x[:, 4] = np.sin(2 * pa)
        x[:, 5] = np.cos(2 * pa)
        x[:, 6] = nu_lo / nu
        x[:, 7] = (w / w_max) ** 2
    x[np.arange(b), nf + np.broadcast_to(cell, (b,)).astype(np.int64)] = 1.0
    return x


class Teacher:
    """Training pairs from the FFT generator: one pg_make_kernels call per (nu, pa) draw with
    `planes` sorted w draws gives planes x 16 cells."""

    def __init__(self, setup, jones_fn, planes: int = 16, eps_null: float = 0.2, seed: int = 1):
        self.setup = setup
        self.jones_fn = jones_fn            # (beam, mk, fov) -> complex128 [2][2][mk][mk]
        self.planes = planes
        self.eps_null = eps_null
        self.rng = np.random.default_rng(seed)
        g = setup.geom
        self.cell_len = g.os * g.os * int(g.support[0]) ** 2 * 2   # floats per cell
        self.seconds = 0.0
        self.calls = 0

    def call(self, out):
        """Fill out [planes * 16][cell_len] (device float32) and return the matching features."""
        import torch

        t0 = time.perf_counter()
        s = self.setup
        w, nu, pa = s.draw(self.planes, self.rng)
        w = np.sort(w)
        nu, pa = float(nu[0]), float(pa[0])
        g = s.plane_geometry(w)
        jones = self.jones_fn(s.beam(nu, pa), g.mk, g.fov)
        k = pg.make_kernels(g, 4, pg.KIND_GRID, jones=jones, eps_null=self.eps_null)
        k.export_planes(0, self.planes, out=out)
        torch.cuda.synchronize()
        del k
        self.seconds += time.perf_counter() - t0
        self.calls += 1
        rows = np.repeat(np.arange(self.planes), N_CELLS)
        cells = np.tile(np.arange(N_CELLS), self.planes)
        return features(w[rows], nu, pa, cells, s.w_max, s.nu_lo, s.nu_hi)


def cell_scale(teacher, calls: int = 4):
    """Per-Mueller-cell RMS of the teacher's cells over a few draws (float32 [16])."""
    import torch

    buf = torch.empty((teacher.planes * N_CELLS, teacher.cell_len), dtype=torch.float32, device="cuda")
    acc = torch.zeros(N_CELLS, dtype=torch.float64, device="cuda")
    for _ in range(calls):
        teacher.call(buf)
        acc += buf.double().pow(2).mean(dim=1).view(teacher.planes, N_CELLS).mean(dim=0)
    return (acc / calls).sqrt().float().cpu().numpy()


def train(net, teacher, scale, steps: int, batch: int = 256, pool_calls: int = 32, refresh_every: int = 8,
          lr: float = 1e-3, lr_final: float = 2e-5, log=None, seed: int = 7):
    """Adam on random batches from a pool of teacher calls; one pool slot is regenerated every
    `refresh_every` steps, so steps / refresh_every + pool_calls calls pass through.  The learning
    rate decays on a cosine from lr to lr_final.  Returns (losses, kernels seen)."""
    import torch

    per = teacher.planes * N_CELLS
    pool = torch.empty((pool_calls * per, teacher.cell_len), dtype=torch.float32, device="cuda")
    xs = torch.empty((pool_calls * per, n_features()), dtype=torch.float32, device="cuda")
    inv = torch.from_numpy(1.0 / scale).cuda()

    inv_rows = inv.float().repeat(teacher.planes).contiguous()

    def fill(slot):
        rows = slice(slot * per, (slot + 1) * per)
        x = teacher.call(pool[rows])
        pg.scale_rows(pool[rows], inv_rows)
        xs[rows] = torch.from_numpy(x).cuda()

    for slot in range(pool_calls):
        fill(slot)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    losses = []
    seen = pool_calls * per
    for it in range(steps):
        if it and it % refresh_every == 0:
            fill((it // refresh_every) % pool_calls)
            seen += per
        idx = torch.randint(0, pool_calls * per, (batch,), device="cuda", generator=gen)
        x, t = xs.index_select(0, idx), pool.index_select(0, idx)
        rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * it / max(1, steps - 1)))
        loss = net.train_step(x, t, rate)
        if log is not None and (it % 500 == 0 or it == steps - 1):
            lv = float(loss.item())
            losses.append((it, lv))
            log(f"step {it} loss {lv:.4e} lr {rate:.2e}")
    return losses, seen


def surrogate_kernels(net, setup, w_planes, nu: float, pa: float, scale, chunk_planes: int = 16,
                      storage: int = pg.STORE_F32):
    """A grid kernel set on the given w planes, every cell emitted by the network."""
    import torch

    g = setup.plane_geometry(w_planes)
    k = pg.kernels_alloc(g, 4, pg.KIND_GRID, storage=storage)
    p_total = len(w_planes)
    cl = g.os * g.os * int(g.support[0]) ** 2 * 2
    out = torch.empty((chunk_planes * N_CELLS, cl), dtype=torch.float32, device="cuda")
    for p0 in range(0, p_total, chunk_planes):
        np_ = min(chunk_planes, p_total - p0)
        rows = np.repeat(np.arange(p0, p0 + np_), N_CELLS)
        cells = np.tile(np.arange(N_CELLS), np_)
        x = torch.from_numpy(features(np.asarray(w_planes)[rows], nu, pa, cells, setup.w_max, setup.nu_lo,
                                      setup.nu_hi)).cuda()
        y = net.forward(x, out=out[:np_ * N_CELLS])
        k.import_planes(p0, np_, y, cell_scale=scale)
    return k


def _orthonormalise(y, passes: int = 3):
    """Orthonormal columns spanning the columns of y (device float32 [n][q]): shifted Cholesky QR
    (a first pass with a small diagonal shift of the Gram matrix, then passes that restore
    orthogonality to rounding).  The teacher's kernels have fewer significant directions than q, so
    the float32 Gram matrix can be singular to rounding; a pass whose factorisation fails is
    repeated with a larger shift (the directions it then damps are rounding noise).  Gram products
    and the re-basing y R^-1 run in pg_gemm_f32; only the q x q Cholesky factor and its inverse are
    formed on the host, in float64."""
    import torch

    q = y.shape[1]
    for it in range(passes):
        gram = pg.gemm_f32(y, y, transa=True).double().cpu().numpy()
        gram = 0.5 * (gram + gram.T)
        mean_diag = np.trace(gram) / q
        shift = 1e-6 * mean_diag if it == 0 else 0.0
        for _ in range(8):
            try:
                r = np.linalg.cholesky(gram + shift * np.eye(q)).T   # gram + shift = r^T r
                break
            except np.linalg.LinAlgError:
                shift = max(100.0 * shift, 1e-7 * mean_diag)
        else:
            raise np.linalg.LinAlgError("Gram matrix not positive definite even with a shift")
        rinv = torch.from_numpy(np.linalg.inv(r).astype(np.float32)).cuda()
        y = pg.gemm_f32(y, rinv)
    return y


def row_basis(k, rank: int, oversample: int = 16, power_iters: int = 4, seed: int = 1):
    """Orthonormal rows [rank][d] spanning the dominant row space of k [n][d] (device float32): a
    randomised SVD (Halko, Martinsson and Tropp's range finder with power iterations) on k^T, every
    large product in pg_gemm_f32.  The Gaussian test matrix is drawn by torch's generator and passed
    in; the q x q eigenproblem of the projected matrix is solved on the host in float64."""
    import torch

    n, d = k.shape
    q = min(rank + oversample, n)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    omega = torch.randn((n, q), dtype=torch.float32, device="cuda", generator=gen)
    y = _orthonormalise(pg.gemm_f32(k, omega, transa=True))          # [d][q]: range of k^T
    for _ in range(power_iters):
        z = _orthonormalise(pg.gemm_f32(k, y))                        # [n][q]
        y = _orthonormalise(pg.gemm_f32(k, z, transa=True))           # [d][q]
    b = pg.gemm_f32(k, y)                                             # k y = u s w^T
    gram = pg.gemm_f32(b, b, transa=True).double().cpu().numpy()      # w s^2 w^T
    evals, w = np.linalg.eigh(0.5 * (gram + gram.T))
    w_top = np.ascontiguousarray(w[:, np.argsort(evals)[::-1][:rank]].T.astype(np.float32))
    return pg.gemm_f32(torch.from_numpy(w_top).cuda(), y, transb=True)  # [rank][d] = (y w)^T


def _residual(k, c, basis) -> float:
    """Mean relative squared residual |k - c basis|^2 / |k|^2 of rows projected onto the basis."""
    r = pg.gemm_f32(c, basis, out=k.clone(), alpha=-1.0, beta=1.0)
    return float((r.pow(2).sum(1) / k.pow(2).sum(1)).mean())


def teacher_data(teacher, scale, calls: int, basis_calls: int = 64, rank: int = 256, seed: int = 1, log=None):
    """Teacher kernels of `calls` calls reduced to basis coordinates.

    Returns (features [N][F], coefficients [N][rank], basis [rank][cell_len], info), device tensors."""
    import torch

    t_start = time.perf_counter()
    per = teacher.planes * N_CELLS
    d = teacher.cell_len
    inv = torch.from_numpy((1.0 / scale).astype(np.float32)).cuda().repeat(teacher.planes).contiguous()
    nb = min(basis_calls, calls)
    k0 = torch.empty((nb * per, d), dtype=torch.float32, device="cuda")
    feats = []
    for c in range(nb):
        rows = slice(c * per, (c + 1) * per)
        feats.append(teacher.call(k0[rows]))
        pg.scale_rows(k0[rows], inv)
    basis = row_basis(k0, rank, seed=seed)                   # [rank][d], orthonormal rows
    coef = [pg.gemm_f32(k0, basis, transb=True)]
    resid0 = _residual(k0[:512], coef[0][:512], basis)
    del k0
    torch.cuda.empty_cache()
    buf = torch.empty((per, d), dtype=torch.float32, device="cuda")
    resid = []
    for c in range(nb, calls):
        feats.append(teacher.call(buf))
        if log is not None and (c + 1) % 256 == 0:
            log(f"teacher call {c + 1}/{calls}")
        pg.scale_rows(buf, inv)
        cc = pg.gemm_f32(buf, basis, transb=True)
        coef.append(cc)
        if c < nb + 8:
            resid.append(_residual(buf, cc, basis))
    del buf
    x_all = torch.from_numpy(np.concatenate(feats)).cuda()
    c_all = torch.cat(coef)
    info = dict(kernels=int(x_all.shape[0]), rank=rank, basis_residual=resid0,
                basis_residual_heldout=float(np.mean(resid)) if resid else None,
                teacher_s=time.perf_counter() - t_start)
    if log:
        log(f"basis: rank {rank}, in-sample residual {resid0:.2e}, held-out residual "
            f"{info['basis_residual_heldout']}; {info['kernels']} kernels in {info['teacher_s']:.1f} s")
    return x_all, c_all, basis, info


def train_coefficients(x_all, c_all, steps: int = 20000, batch: int = 1024, lr: float = 2e-3,
                       lr_final: float = 1e-5, seed: int = 1, log=None):
    """The network with its output layer in basis coordinates, trained by Adam on random batches."""
    import torch

    n, rank = c_all.shape
    net_r = pg.MLP(x_all.shape[1], 256, 3, rank, batch, seed=seed)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    losses = []
    for it in range(steps):
        idx = torch.randint(0, n, (batch,), device="cuda", generator=gen)
        rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * it / max(1, steps - 1)))
        loss = net_r.train_step(x_all.index_select(0, idx), c_all.index_select(0, idx), rate)
        if it % 2000 == 0 or it == steps - 1:
            losses.append((it, float(loss.item())))
            if log is not None:
                log(f"coef step {it} loss {losses[-1][1]:.3e} lr {rate:.2e}")
    return net_r, losses


def fold(net_r, basis, max_batch: int = 256, seed: int = 1):
    """The kernel-emitting network: hidden layers of net_r, output layer W_r B, b_r B."""
    import torch

    d = basis.shape[1]
    net = pg.MLP(net_r.dims[0], 256, 3, d, max_batch, seed=seed)
    for layer in range(3):
        net.load(layer, net_r.copy(pg.MLP_W, layer), net_r.copy(pg.MLP_B, layer))
    w_r, b_r = net_r.copy(pg.MLP_W, 3), net_r.copy(pg.MLP_B, 3)
    net.load(3, pg.gemm_f32(w_r.contiguous(), basis), pg.gemm_f32(b_r.view(1, -1).contiguous(), basis)[0])
    torch.cuda.synchronize()
    return net


def fit(teacher, scale, calls: int, basis_calls: int = 64, rank: int = 256, steps: int = 20000,
        batch: int = 1024, lr: float = 2e-3, lr_final: float = 1e-5, tune_steps: int = 0, tune_lr: float = 1e-5,
        max_batch: int = 256, seed: int = 1, log=None):
    """Train a kernel network on `calls` teacher calls (planes x 16 kernels each).

    Returns (network emitting scaled kernels [B][cell_len], info dict)."""
    x_all, c_all, basis, info = teacher_data(teacher, scale, calls, basis_calls, rank, seed, log)
    t0 = time.perf_counter()
    net_r, losses = train_coefficients(x_all, c_all, steps, batch, lr, lr_final, seed, log)
    net = fold(net_r, basis, max_batch, seed)
    info["train_s"] = time.perf_counter() - t0
    if tune_steps:
        tl, _ = train(net, teacher, scale, tune_steps, batch=max_batch, pool_calls=16, refresh_every=8,
                      lr=tune_lr, lr_final=tune_lr * 0.1, log=log)
        losses += [(steps + i, v) for i, v in tl]
    info.update(losses=losses, steps=steps, batch=batch)
    return net, info


def heldout_error(net, teacher, scale, calls: int = 4):
    """Root-mean per-cell relative error |y - t| / |t| of the network on fresh teacher draws (float [16])."""
    import torch

    per = teacher.planes * N_CELLS
    buf = torch.empty((per, teacher.cell_len), dtype=torch.float32, device="cuda")
    sc = torch.from_numpy(scale).cuda().repeat(teacher.planes)[:, None]
    acc = torch.zeros(N_CELLS, dtype=torch.float64, device="cuda")
    out = torch.empty_like(buf)
    for _ in range(calls):
        x = torch.from_numpy(teacher.call(buf)).cuda()
        for r0 in range(0, per, net.max_batch):
            r1 = min(per, r0 + net.max_batch)
            net.forward(x[r0:r1], out=out[r0:r1])
        y = out * sc
        e = ((y - buf).double().pow(2).sum(1) / buf.double().pow(2).sum(1)).view(teacher.planes, N_CELLS).mean(0)
        acc += e
    return (acc / calls).sqrt().cpu().numpy()
