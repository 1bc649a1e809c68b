"""Invariants of the oracle grid/degrid pair: adjointness, Hermitian symmetry, linearity, shifts."""
import numpy as np
import pytest

import synth
from oracle import gridding, kernels


def _crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def _geom(n=48, os_=4, planes=(-40.0, 0.0, 40.0), support=(9, 7, 9), mk=32):
    planes = np.asarray(planes, dtype=np.float64)
    return synth.Geometry(n=n, cell=0.3 / n, os=os_, w_planes=planes,
                          support=np.asarray(support, np.int32),
                          tile=np.full(planes.size, 8, np.int32), mk=mk)


def _uvw(rng, g, nv, spread=0.35):
    lim = spread * g.n / g.fov
    return np.stack([rng.uniform(-lim, lim, nv), rng.uniform(-lim, lim, nv), rng.uniform(-60, 60, nv)], 1)


@pytest.mark.parametrize("npol", [1, 4])
def test_adjoint_identity(npol):
    """P2: <degrid(x), v> = <x, grid(v)> to 1e-12 for random tables, grids and visibilities."""
    rng = np.random.default_rng(11 + npol)
    g = _geom()
    phi = _crandn(rng, npol, npol, g.mk, g.mk)
    tabs = kernels.make_tables(g, phi)
    uvw = _uvw(rng, g, 400, spread=0.55)  # some fall off the edge
    v = _crandn(rng, 400, npol)
    x = _crandn(rng, npol, g.n, g.n)
    lhs = np.vdot(gridding.degrid(g, tabs, uvw, x), v)
    rhs = np.vdot(x, gridding.grid(g, tabs, uvw, v))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(v)
    assert abs(lhs) > 1e-3 * np.linalg.norm(x) * np.linalg.norm(v) / 100


def test_hermitian_symmetry():
    """P3: gridding V and its conjugate partner at -uvw with real screens gives G(n-X, n-Y) = conj G."""
    rng = np.random.default_rng(12)
    g = _geom()
    phi = rng.standard_normal((4, 4, g.mk, g.mk)).astype(complex)
    tabs = kernels.make_tables(g, phi)
    uvw = _uvw(rng, g, 200)
    v = _crandn(rng, 200, 4)
    allu = np.concatenate([uvw, -uvw])
    allv = np.concatenate([v, np.conj(v)])
    gr = gridding.grid(g, tabs, allu, allv)
    n = g.n
    inner = gr[:, 1:, 1:]
    mirror = gr[:, ::-1, ::-1][:, :n - 1, :n - 1]  # G(n-Y, n-X) for X, Y in 1..n-1
    assert np.max(np.abs(inner - np.conj(mirror))) < 1e-12 * np.max(np.abs(gr))
    assert np.max(np.abs(gr[:, 0, :])) == 0 and np.max(np.abs(gr[:, :, 0])) == 0


def test_linearity_and_integer_shift():
    """P12: grid is linear in V, and moving every uv by whole cells moves the grid by whole pixels."""
    rng = np.random.default_rng(13)
    g = _geom(planes=(0.0,), support=(7,))
    tabs = kernels.make_tables(g, _crandn(rng, 4, 4, g.mk, g.mk))
    uvw = _uvw(rng, g, 150, spread=0.3)
    uvw[:, 2] = 0.0
    a, b = _crandn(rng, 150, 4), _crandn(rng, 150, 4)
    ga, gb = gridding.grid(g, tabs, uvw, a), gridding.grid(g, tabs, uvw, b)
    gab = gridding.grid(g, tabs, uvw, 2.0 * a - 1j * b)
    assert np.max(np.abs(gab - (2.0 * ga - 1j * gb))) < 1e-12 * np.max(np.abs(gab))
    shifted = uvw.copy()
    shifted[:, 0] += 3 / g.fov
    shifted[:, 1] -= 2 / g.fov
    gs = gridding.grid(g, tabs, shifted, a)
    ref = np.zeros_like(ga)
    ref[:, :g.n - 2, 3:] = ga[:, 2:, :g.n - 3]
    assert np.max(np.abs(gs - ref)) < 1e-12 * np.max(np.abs(ga))
    dv = gridding.degrid(g, tabs, uvw, ga)
    dvs = gridding.degrid(g, tabs, shifted, ref)
    assert np.max(np.abs(dv - dvs)) < 1e-12 * np.max(np.abs(dv))


def test_dropped_visibilities_contribute_nothing():
    rng = np.random.default_rng(14)
    g = _geom(planes=(0.0,), support=(7,))
    tabs = kernels.make_tables(g, np.ones((1, 1, g.mk, g.mk), complex))
    far = np.array([[0.49 * g.n / g.fov, 0.0, 0.0], [0.0, -0.5 * g.n / g.fov, 0.0]])
    out = gridding.grid(g, tabs, far, np.ones((2, 1)))
    assert np.max(np.abs(out)) == 0
    assert np.max(np.abs(gridding.degrid(g, tabs, far, _crandn(rng, 1, g.n, g.n)))) == 0
