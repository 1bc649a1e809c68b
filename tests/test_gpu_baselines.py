"""GPU tests of per-baseline Mueller kernels (Sec. 3.2: non-identical antennas make the Mueller
matrix J_a (x) conj(J_b) unique to the baseline): one kernel set per ordered antenna-type pair, rows
split by their baseline's pair, every pair gridded onto ONE grid by one batched launch (and degridded
from one model grid), against the float64 oracle with per-pair tables."""
import numpy as np
import pytest

import synth
from oracle import gridding, kernels, mueller

torch = pytest.importorskip("torch")
pg = pytest.importorskip("paper_2206_15117_amd.polgrid")

pytestmark = pytest.mark.gpu

K = 3


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def case():
    pg.use_torch_allocator(True)
    rng = np.random.default_rng(71)
    w = synth.scaled_config2(3780, n=128, nplanes=4, mk=64, support=[12, 8, 8, 12])
    g = w.geom
    types = synth.antenna_types(0.5 * g.fov, K, rng, pointing_sigma=0.03 * g.fov, level=0.04)
    jl = [synth.jones_on_lattice(t, g.mk, g.fov) for t in types]
    pair = synth.baseline_type_pairs(w.nvis, 36, K)
    vis = synth.random_vis(w.nvis, 4, rng)
    groups = []
    for p in range(K * K):
        rows = np.flatnonzero(pair == p)
        groups.append((p // K, p % K, rows))
    return g, jl, w.uvw, vis, groups


def test_make_kernels_with_equal_second_antenna_is_the_identical_antenna_set(case):
    g, jl, *_ = case
    a = pg.make_kernels(g, 4, pg.KIND_GRID, jones=jl[0], eps_null=0.2)
    b = pg.make_kernels(g, 4, pg.KIND_GRID, jones=jl[0], jones_b=jl[0], eps_null=0.2)
    ta, tb = a.table(), b.table()
    torch.cuda.synchronize()
    assert torch.equal(ta, tb)


def test_per_pair_grid_onto_one_grid_matches_oracle(case):
    g, jl, uvw, vis, groups = case
    grid = torch.empty((4, g.n, g.n), dtype=torch.complex64, device="cuda")
    fields, keep = [], []
    want = 0
    for ta, tb, rows in groups:
        k = pg.make_kernels(g, 4, pg.KIND_GRID, jones=jl[ta], jones_b=jl[tb], eps_null=0.2)
        p = pg.plan(k, torch.from_numpy(np.ascontiguousarray(uvw[rows])).cuda(), max_chunk=128)
        v = torch.from_numpy(np.ascontiguousarray(vis[rows])).cuda()
        fields.append((p, k, v, grid))
        keep.append((k, p, v))
        tabs = kernels.make_tables(g, mueller.phi_grid(jl[ta], 0.2, jones_b=jl[tb]))
        want = want + gridding.grid(g, tabs, uvw[rows], vis[rows])
    b = pg.batch(fields)
    b.grid()
    torch.cuda.synchronize()
    got = grid.cpu().numpy()
    for q in range(4):
        assert rel(got[q], want[q]) < 1e-5, q


def test_per_pair_degrid_from_one_grid_matches_oracle(case):
    g, jl, uvw, vis, groups = case
    rng = np.random.default_rng(72)
    gm = (rng.standard_normal((4, g.n, g.n)) + 1j * rng.standard_normal((4, g.n, g.n))).astype(np.complex64)
    gmt = torch.from_numpy(gm).cuda()
    fields, outs, wants = [], [], []
    for ta, tb, rows in groups:
        k = pg.make_kernels(g, 4, pg.KIND_DEGRID, jones=jl[ta], jones_b=jl[tb])
        p = pg.plan(k, torch.from_numpy(np.ascontiguousarray(uvw[rows])).cuda(), max_chunk=128)
        o = torch.empty((rows.size, 4), dtype=torch.complex64, device="cuda")
        fields.append((p, k, o, gmt))
        outs.append(o)
        tabs = kernels.make_tables(g, mueller.phi_degrid(jl[ta], jones_b=jl[tb]))
        wants.append(gridding.degrid(g, tabs, uvw[rows], gm.astype(np.complex128)))
    b = pg.batch(fields)
    b.degrid()
    torch.cuda.synchronize()
    for o, want in zip(outs, wants):
        assert rel(o.cpu().numpy(), want) < 1e-5
