"""Parity at full size, in the launch configuration the benchmark times (the autotuned tiles, chunk
length, waves per workgroup and XCD grouping, centring folded into grid/degrid):
  c2  full-pol 2048^2 x 4, 32 planes, supports 16-48, os 8, 2.3M rows;
  c5  major cycle 8192^2 x 4, 128 planes, supports 16-48, os 8, 20M rows (288 channels).

The oracle cannot grid millions of rows in seconds, so: the plan is compared bit-exactly in full;
grid and degrid are compared on a seeded sample of rows drawn from every populated plane (c2: all
31, so every (support, tile) launch shape the benchmark runs) or from the most populated plane of
every support class (c5: 17 planes), with every other visibility set to zero for grid; the
adjoint identity is checked over all rows.
"""
import numpy as np
import pytest

import synth
from oracle import geometry, gridding, kernels, mueller
from oracle import plan as oplan
from oracle_pool import tables_in_parallel

torch = pytest.importorskip("torch")
pg = pytest.importorskip("paper_2206_15117_amd.polgrid")

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module", params=["c2", "c5"])
def full(request):
    from paper_2206_15117_amd import autotune

    w = synth.config2() if request.param == "c2" else synth.config5()
    launch = autotune.apply(w.geom, 4, pg.STORE_F32)
    g = launch.geom
    w.geom = g
    jones = synth.jones_on_lattice(w.beam, g.mk, g.fov)
    kg = pg.make_kernels(g, 4, pg.KIND_GRID, jones=jones, eps_null=w.eps_null)
    kd = pg.make_kernels(g, 4, pg.KIND_DEGRID, jones=jones)
    uvw = torch.from_numpy(w.uvw).cuda()
    p = autotune.plan(kg, uvw, launch)
    loc = geometry.locate(g, w.uvw)
    counts = np.bincount(loc["plane"], minlength=g.nplanes)
    if request.param == "c2":
        planes = [int(q) for q in np.flatnonzero(counts > 0)]
        per = 40
    else:
        planes = sorted(int(max(np.flatnonzero(g.support == s), key=lambda q: counts[q]))
                        for s in np.unique(g.support) if counts[g.support == s].sum() > 0)
        per = 60
    rng = np.random.default_rng(2022)
    sample = np.concatenate([rng.choice(np.flatnonzero(loc["plane"] == q), min(per, int(counts[q])), replace=False)
                             for q in planes])
    tg = tables_in_parallel(g, mueller.phi_grid(jones, w.eps_null), planes, request.param + " grid")
    td = tables_in_parallel(g, mueller.phi_degrid(jones), planes, request.param + " degrid")
    n = g.n
    sign = ((-1.0) ** (np.arange(n)[:, None] + np.arange(n)[None, :]))[None]
    return dict(w=w, kg=kg, kd=kd, uvw=uvw, p=p, sample=np.sort(sample), tg=tg, td=td, sign=sign,
                chunk=launch.max_chunk, planes=planes)


def test_full_plan_bit_exact(full):
    w, p = full["w"], full["p"]
    want = oplan.plan(w.geom, w.uvw, full["chunk"])
    perm, fine, items = (t.cpu().numpy() for t in p.arrays())
    assert (p.n_kept, p.n_dropped, p.n_items) == (want["n_kept"], want["n_dropped"], want["items"].shape[0])
    assert np.array_equal(perm, want["perm"])
    kept = want["perm"][:want["n_kept"]]
    assert np.array_equal(fine[:, 0], want["loc"]["fine_x"][kept])
    assert np.array_equal(fine[:, 1], want["loc"]["fine_y"][kept])
    it = want["items"]
    t = w.geom.tile[it[:, 0]]
    assert np.array_equal(items[:, :5], np.stack([it[:, 0], it[:, 1] * t, it[:, 2] * t, it[:, 3], it[:, 4]], 1))


def test_full_sample_covers_every_launch_shape(full):
    """The sampled planes cover every (support, tile) pair of the launch (c2) or every support (c5)."""
    g, planes = full["w"].geom, full["planes"]
    counts = np.bincount(geometry.locate(g, full["w"].uvw)["plane"], minlength=g.nplanes)
    used = {(int(g.support[q]), int(g.tile[q])) for q in np.flatnonzero(counts > 0)}
    got = {(int(g.support[q]), int(g.tile[q])) for q in planes}
    if len(planes) >= np.count_nonzero(counts):
        assert got == used
    else:
        assert {s for s, _ in got} == {s for s, _ in used}


def test_full_grid_sampled_rows(full):
    w, s = full["w"], full["sample"]
    rng = np.random.default_rng(7)
    vis = np.zeros((w.nvis, 4), np.complex64)
    vis[s] = synth.random_vis(len(s), 4, rng)
    got = pg.grid(full["p"], full["kg"], torch.from_numpy(vis).cuda(), fftshift=True).cpu().numpy()
    want = gridding.grid(w.geom, full["tg"], w.uvw[s], vis[s]) * full["sign"]
    for q in range(4):
        assert rel(got[q], want[q]) < TOL, q


def test_full_degrid_sampled_rows(full):
    w, s = full["w"], full["sample"]
    n = w.geom.n
    gen = torch.Generator(device="cuda").manual_seed(11)
    gr = torch.randn((4, n, n), dtype=torch.complex64, device="cuda", generator=gen)
    got = pg.degrid(full["p"], full["kd"], gr, fftshift=True).cpu().numpy()[s]
    want = gridding.degrid(w.geom, full["td"], w.uvw[s], gr.cpu().numpy().astype(np.complex128) * full["sign"])
    for c in range(4):
        assert rel(got[:, c], want[:, c]) < TOL, c


def test_full_adjoint_identity(full):
    w, p, kg = full["w"], full["p"], full["kg"]
    n = w.geom.n
    gen = torch.Generator(device="cuda").manual_seed(12)
    x = torch.randn((4, n, n), dtype=torch.complex64, device="cuda", generator=gen)
    v = torch.randn((w.nvis, 4), dtype=torch.complex64, device="cuda", generator=gen)
    dx = pg.degrid(p, kg, x).to(torch.complex128)
    gv = pg.grid(p, kg, v).to(torch.complex128)
    lhs = torch.vdot(dx.flatten(), v.to(torch.complex128).flatten()).item()
    rhs = torch.vdot(x.to(torch.complex128).flatten(), gv.flatten()).item()
    scale = dx.norm().item() * v.to(torch.complex128).norm().item()
    assert abs(lhs - rhs) <= TOL * scale


def test_full_shared_taps_match_row_bands_on_all_rows(full):
    """Every row carrying data, at full size: the tuned kernel (shared taps, exact fixed-point
    sub-grids, items up to the tuned chunk length) against the row-band float kernel, which the
    sampled tests above tie to the oracle."""
    w = full["w"]
    vis = torch.from_numpy(synth.random_vis(w.nvis, 4, np.random.default_rng(21))).cuda()
    a = pg.grid(full["p"], full["kg"], vis, variant=pg.VARIANT_SHARED)
    b = pg.grid(full["p"], full["kg"], vis, variant=pg.VARIANT_BANDED)
    torch.cuda.synchronize()
    for q in range(4):
        d = float((a[q] - b[q]).abs().norm() / b[q].abs().norm())
        assert d < 1e-6, (q, d)
