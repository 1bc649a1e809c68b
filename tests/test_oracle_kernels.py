"""Pins of the kernel tables: direct evaluation of the DFT definition and the unit-visibility case."""
import numpy as np
import pytest

import synth
from oracle import geometry, gridding, kernels, mueller


def _geom(support=7, os_=4, n=32, mk=32, planes=(0.0,)):
    planes = np.asarray(planes, dtype=np.float64)
    return synth.Geometry(n=n, cell=0.3 / n, os=os_, w_planes=planes,
                          support=np.full(planes.size, support, np.int32),
                          tile=np.full(planes.size, 8, np.int32), mk=mk)


def _direct_tap(f2d, d_x, d_y, os_):
    """T(d) as the plain double sum of the definition, no matrix products."""
    mk = f2d.shape[0]
    acc = 0j
    for b in range(mk):
        for a in range(mk):
            acc += f2d[b, a] * np.exp(2j * np.pi * (d_x * (a - mk // 2) + d_y * (b - mk // 2)) / (os_ * mk))
    return acc / (mk * mk)


def test_table_entries_equal_direct_dft():
    g = _geom(support=5, os_=4, n=16, mk=16, planes=(40.0,))
    rng = np.random.default_rng(7)
    phi = (rng.standard_normal((1, 1, 16, 16)) + 1j * rng.standard_normal((1, 1, 16, 16)))
    t = kernels.make_tables(g, phi)[0][0, 0]
    f = kernels.image_function(g, 0, phi)[0, 0]
    s, os_ = 5, 4
    for _ in range(12):
        py, px, ty, tx = rng.integers(0, os_), rng.integers(0, os_), rng.integers(0, s), rng.integers(0, s)
        dy = py - s * os_ // 2 + 1 + ty * os_
        dx = px - s * os_ // 2 + 1 + tx * os_
        want = 0j if max(abs(dx), abs(dy)) >= s * os_ / 2 else _direct_tap(f, dx, dy, os_)
        assert abs(t[py, px, ty, tx] - want) < 1e-13


def test_w_screen_is_conjugate_of_predict_phase():
    """Image-domain function of plane w carries exp(-2 pi i w (n-1)) on top of AA."""
    g = _geom(planes=(-120.0, 120.0), n=16, mk=16)
    phi = np.ones((1, 1, 16, 16), complex)
    f0 = kernels.image_function(g, 0, phi)[0, 0]
    f1 = kernels.image_function(g, 1, phi)[0, 0]
    x = kernels.lattice(16, g.fov)
    mm, ll = np.meshgrid(x, x, indexing="ij")
    nm1 = np.sqrt(1 - ll ** 2 - mm ** 2) - 1
    aa = kernels.aa_lattice(16, 7)
    assert np.allclose(f1, np.outer(aa, aa) * np.exp(-2j * np.pi * 120.0 * nm1), atol=1e-14)
    assert np.allclose(f0, np.conj(f1), atol=1e-14)


@pytest.mark.parametrize("npol", [1, 4])
def test_unit_visibility_reproduces_kernel(npol):
    """P1: gridding V_c = delta_{c,c0} puts T_{q,c0}(X os - fine) on the brute-force footprint, 0 elsewhere."""
    g = _geom(support=7, os_=4, n=32, mk=32, planes=(-30.0, 30.0))
    rng = np.random.default_rng(8)
    phi = rng.standard_normal((npol, npol, 32, 32)) + 1j * rng.standard_normal((npol, npol, 32, 32))
    tabs = kernels.make_tables(g, phi)
    f = [kernels.image_function(g, p, phi) for p in range(2)]
    for trial in range(4):
        uvw = np.array([[rng.uniform(-10, 10) / g.fov, rng.uniform(-10, 10) / g.fov, rng.uniform(-60, 60)]])
        c0 = trial % npol
        vis = np.zeros((1, npol), complex)
        vis[0, c0] = 1.0
        got = gridding.grid(g, tabs, uvw, vis)
        fx, fy = geometry.fine_position(uvw, g.n, g.cell, g.os)
        p = int(np.argmin(np.abs(uvw[0, 2] - g.w_planes)))
        expect = np.zeros_like(got)
        half = 7 * 4 / 2
        for Y in range(g.n):
            for X in range(g.n):
                dx, dy = X * 4 - fx[0], Y * 4 - fy[0]
                if abs(dx) < half and abs(dy) < half:
                    for q in range(npol):
                        expect[q, Y, X] = _direct_tap(f[p][q, c0], dx, dy, 4)
        assert np.max(np.abs(got - expect)) < 1e-13
        assert np.count_nonzero(np.abs(got[0]) > 0) in (36, 42, 49)


def test_aa_only_kernel_sums_to_one_over_a_period():
    """Summed over one full period of integer offsets, the AA-only kernel gives AA(0)^2 = 1."""
    mk = 16
    g = _geom(support=mk + 1, os_=2, n=mk, mk=mk)
    t = kernels.make_tables(g, np.ones((1, 1, mk, mk), complex))[0][0, 0]
    # phase 0 has offsets d = 2 t - 16 (integer uv cells -8 .. 8); cells -8 .. 7 make one period
    assert abs(t[0, 0][:mk, :mk].sum() - 1.0) < 1e-12
    # any other lattice point l_a of the image is recovered the same way
    a = 5
    ph = np.exp(-2j * np.pi * np.arange(-8, 8) * (a - mk // 2) / mk)
    aa = kernels.aa_lattice(mk, 7)
    assert abs(ph @ t[0, 0][:mk, :mk] @ ph - aa[a] * aa[a]) < 1e-12


def test_grid_and_degrid_kernels_follow_mueller_screens():
    """Grid/degrid screens reduce to S and S^-1 conj-transposed for an identity beam."""
    s = mueller.stokes_matrix()
    g = mueller.phi_grid(np.broadcast_to(np.eye(2)[:, :, None, None], (2, 2, 2, 2)), eps=0.0)
    assert np.allclose(g[:, :, 0, 0], s, atol=1e-14)
    d = mueller.phi_degrid(np.broadcast_to(np.eye(2)[:, :, None, None], (2, 2, 2, 2)))
    assert np.allclose(d[:, :, 1, 1], np.linalg.inv(s).conj().T, atol=1e-14)
