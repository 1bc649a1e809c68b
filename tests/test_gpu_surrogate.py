"""GPU tests of the learned-kernel path: cell export/import, empty kernel sets, the teacher's
training pairs, and what the trained network gains over nearest-plane kernels.

Expected values come from the FP64 oracle (kernel tables, direct Fourier transforms); the
network is trained here, on the GPU, by the library's own forward/backward/Adam kernels.
"""
import time

import numpy as np
import pytest

import synth
from oracle import imaging, kernels, mueller

torch = pytest.importorskip("torch")
pg = pytest.importorskip("paper_2206_15117_amd.polgrid")
sg = pytest.importorskip("paper_2206_15117_amd.surrogate")

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.fixture(scope="module")
def small():
    pg.use_torch_allocator(True)
    w = synth.scaled_config2(4000, n=256, nplanes=8, mk=64, support=[16, 12, 10, 8, 8, 10, 12, 16])
    jones = synth.jones_on_lattice(w.beam, w.geom.mk, w.geom.fov)
    phi = mueller.phi_grid(jones, w.eps_null)
    tabs = kernels.make_tables(w.geom, phi, planes=[3, 4])
    k = pg.make_kernels(w.geom, 4, pg.KIND_GRID, jones=jones, eps_null=w.eps_null)
    return w, jones, tabs, k


def test_export_is_the_oracle_table(small):
    w, _, tabs, k = small
    got = k.export_planes(3, 2).cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    want = np.stack([tabs[3], tabs[4]])
    assert got.shape == want.shape == (2, 4, 4, 8, 8, 8, 8)
    assert rel(got, want) < 1e-6


def test_export_rejects_mixed_supports_and_bad_ranges(small):
    _, _, _, k = small
    for p0, n in [(2, 2), (7, 2), (-1, 1)]:
        with pytest.raises(pg.PolgridError):
            k.export_planes(p0, n, out=torch.empty(1 << 22, device="cuda"))


@pytest.mark.parametrize("storage", [pg.STORE_F32, pg.STORE_F16])
def test_import_into_empty_set_reproduces_tables_and_grid(small, storage):
    w, jones, _, _ = small
    g = w.geom
    k = pg.make_kernels(g, 4, pg.KIND_GRID, jones=jones, eps_null=w.eps_null, storage=storage)
    e = pg.kernels_alloc(g, 4, pg.KIND_GRID, storage=storage)
    assert torch.count_nonzero(e.table()).item() == 0
    assert np.array_equal(e.aa_pixels, k.aa_pixels)
    assert np.array_equal(e.plane_offset, k.plane_offset)
    p = 0
    while p < g.nplanes:
        q = p
        while q + 1 < g.nplanes and g.support[q + 1] == g.support[p]:
            q += 1
        e.import_planes(p, q - p + 1, k.export_planes(p, q - p + 1))
        p = q + 1
    assert torch.equal(e.table(), k.table())
    uvw = torch.from_numpy(w.uvw).cuda()
    vis = torch.from_numpy(synth.random_vis(w.nvis, 4, np.random.default_rng(2))).cuda()
    pk = pg.plan(k, uvw, max_chunk=64)
    ge = pg.grid(pk, e, vis)
    gk = pg.grid(pk, k, vis)
    assert rel(ge.cpu().numpy(), gk.cpu().numpy()) < 1e-6


def test_import_applies_cell_scale(small):
    w, _, tabs, k = small
    e = pg.kernels_alloc(w.geom, 4, pg.KIND_GRID)
    src = k.export_planes(3, 2).contiguous()
    scale = np.arange(1, 17, dtype=np.float32) / 4.0
    e.import_planes(3, 2, src, cell_scale=scale)
    got = e.export_planes(3, 2).cpu().numpy()
    want = src.cpu().numpy() * scale.reshape(1, 4, 4, 1, 1, 1, 1, 1)
    assert np.array_equal(got, want.astype(np.float32))
    assert torch.count_nonzero(e.export_planes(0, 1)).item() == 0


def test_teacher_pairs_are_make_kernels_cells():
    """A teacher call returns the FFT generator's cells for its (w, nu, pa) draw, row = plane * 16 + cell."""
    s = synth.config4()
    small_geom = synth.Geometry(n=64, cell=0.1 / 64, os=4, w_planes=s.geom.w_planes[:2],
                                support=np.full(2, 8, np.int32), tile=np.full(2, 8, np.int32), aa_support=7,
                                mk=32)
    s.geom = small_geom
    t = sg.Teacher(s, synth.jones_on_lattice, planes=3, seed=4)
    buf = torch.empty((48, t.cell_len), dtype=torch.float32, device="cuda")
    x = t.call(buf)
    w, nu, pa = s.draw(3, np.random.default_rng(4))
    w = np.sort(w)
    assert np.allclose(x[::16, 0] * s.w_max, w)
    g = s.plane_geometry(w)
    phi = mueller.phi_grid(synth.jones_on_lattice(s.beam(nu[0], pa[0]), g.mk, g.fov), 0.2)
    tabs = kernels.make_tables(g, phi)
    want = np.stack(tabs).reshape(48, -1)
    got = buf.cpu().numpy().reshape(48, -1, 2)
    assert rel(got[..., 0] + 1j * got[..., 1], want) < 1e-6


# ------------------------------------------------------------------ trained network (c4 geometry)

@pytest.fixture(scope="module")
def trained():
    """A kernel network trained on 300 teacher calls x 4 w planes x 16 cells (19,200 kernels)."""
    pg.use_torch_allocator(True)
    s = synth.config4()
    teacher = sg.Teacher(s, synth.jones_on_lattice, planes=16, seed=1)
    scale = sg.cell_scale(teacher, 2)
    teacher = sg.Teacher(s, synth.jones_on_lattice, planes=4, seed=1)
    t0 = time.perf_counter()
    x, c, basis, info = sg.teacher_data(teacher, scale, calls=300, basis_calls=64, rank=256)
    net_r, losses = sg.train_coefficients(x, c, steps=8000, batch=2048, lr=5e-3)
    net = sg.fold(net_r, basis)
    print(f"teacher {info['teacher_s']:.1f} s, total {time.perf_counter() - t0:.1f} s, "
          f"basis residual {info['basis_residual']:.2e} / held-out {info['basis_residual_heldout']:.2e}, "
          f"final loss {losses[-1][1]:.3e}")
    return s, scale, net, net_r, basis, info


def test_basis_spans_unseen_kernels(trained):
    """The rank-256 basis from the first calls reproduces later calls' kernels (relative residual)."""
    _, _, _, _, _, info = trained
    assert info["basis_residual"] < 1e-6
    assert info["basis_residual_heldout"] < 1e-4


def test_folded_network_emits_basis_expansion(trained):
    """Folding the output layer with the basis changes the map only by bfloat16 rounding."""
    s, scale, net, net_r, basis, _ = trained
    x = torch.from_numpy(sg.features(np.linspace(-150, 150, 64), 1.1e9, 0.7, np.arange(64) % 16, s.w_max,
                                     s.nu_lo, s.nu_hi)).cuda()
    y = net.forward(x)
    want = net_r.forward(x) @ basis
    assert float((y - want).norm() / want.norm()) < 1e-2


def test_network_generalises_to_unseen_draws(trained):
    """Per-cell relative kernel error on fresh (w, nu, pa) draws."""
    s, scale, net, _, _, _ = trained
    err = sg.heldout_error(net, sg.Teacher(s, synth.jones_on_lattice, planes=16, seed=999), scale, calls=2)
    print("held-out relative error per Mueller cell:", np.array2string(err, precision=3))
    assert np.all(np.isfinite(err))
    assert err.mean() < 0.25
    assert max(err[0], err[3]) < 0.1        # the I rows' dominant cells (I <- XX, I <- YY)


def test_surrogate_gain_over_channel_averaged_beam(trained):
    """What the network gains: per-channel A x W kernels at the cost of one network evaluation,
    where the FFT generator's cost per kernel set leads to beams averaged over channels.  Four
    channels (700-1600 MHz) of the config-1 sky and uv coverage, predicted through each channel's
    beam; truth is the direct Fourier image with each channel's exact gridding screens.  The
    surrogate's per-channel kernels must beat one kernel set from the channel-averaged Jones field."""
    s, scale, net, _, _, _ = trained
    g = s.geom
    chans = [700e6, 1000e6, 1300e6, 1600e6]
    pa = s.pa_eval
    rng = np.random.default_rng(6)
    nper = 500
    uvws = [s.uvw[np.sort(rng.choice(len(s.uvw), nper, replace=False))] for _ in chans]
    vis = [imaging.dft_predict(u, s.src_l, s.src_m, s.src_iquv, beam=s.beam(nu, pa)).astype(np.complex64)
           for u, nu in zip(uvws, chans)]
    jl = [synth.jones_on_lattice(s.beam(nu, pa), g.mk, g.fov) for nu in chans]
    truth = sum(imaging.dft_image(g, u, v, float(nper * len(chans)), phi_pixels=mueller.phi_grid(j, 0.2))
                for u, v, j in zip(uvws, vis, jl))

    def image_with(kset):
        grid = torch.zeros((4, g.n, g.n), dtype=torch.complex64, device="cuda")
        tot = 0
        for k, u, v in zip(kset, uvws, vis):
            p = pg.plan(k, torch.from_numpy(u).cuda(), max_chunk=256)
            pg.grid(p, k, torch.from_numpy(v).cuda(), out=grid, accumulate=True, fftshift=True)
            tot += p.n_kept
        assert tot == nper * len(chans)
        out = torch.empty((4, g.n, g.n), dtype=torch.float32, device="cuda")
        return pg.taper(kset[0], torch.fft.fft2(grid), out, pg.TAPER_IMAGE, float(tot)).cpu().numpy()

    im_avg = image_with([pg.make_kernels(g, 4, pg.KIND_GRID, jones=sum(jl) / len(jl), eps_null=0.2)] * len(chans))
    im_fft = image_with([pg.make_kernels(g, 4, pg.KIND_GRID, jones=j, eps_null=0.2) for j in jl])
    im_mlp = image_with([sg.surrogate_kernels(net, s, g.w_planes, nu, pa, scale) for nu in chans])
    n = g.n
    inner = np.zeros((n, n), bool)
    inner[n // 4:3 * n // 4, n // 4:3 * n // 4] = True
    peak = np.abs(truth[0][inner]).max()

    def err(im):
        return float(np.sqrt(np.mean((im[0][inner] - truth[0][inner]) ** 2)) / peak)

    e_avg, e_fft, e_mlp = err(im_avg), err(im_fft), err(im_mlp)
    resid = float(np.sqrt(np.mean((im_mlp[:, inner] - im_fft[:, inner]) ** 2)) / peak)
    print(f"Stokes I rms error / peak: averaged beam {e_avg:.3e}, FFT per channel {e_fft:.3e}, "
          f"network per channel {e_mlp:.3e}; network vs FFT kernels, all Stokes {resid:.3e}")
    assert e_fft < 5e-3
    assert e_mlp < 0.5 * e_avg
