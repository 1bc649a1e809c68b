"""Brute-force pins of the imaging chain: grid -> FFT -> taper against direct Fourier transforms.

Tolerances were fixed from the FP64 oracle's own runs before any GPU work: they bound the
kernel truncation and aliasing error of the method on these tiny grids, with visibilities on
the oversampled lattice so that no position snapping error enters.
"""
import numpy as np
import pytest

import synth
from oracle import gridding, imaging, kernels, mueller


def _lattice_uvw(rng, g, nv, reach, w=None):
    c = g.n // 2 * g.os
    fx = rng.integers(c - reach, c + reach, nv)
    fy = rng.integers(c - reach, c + reach, nv)
    ww = np.zeros(nv) if w is None else w
    return np.stack([(fx / g.os - g.n / 2) / g.fov, (fy / g.os - g.n / 2) / g.fov, ww], 1)


def _pixel_sources(rng, g, k):
    n = g.n
    ii = rng.integers(n // 4, 3 * n // 4, k)
    jj = rng.integers(n // 4, 3 * n // 4, k)
    return ii, jj, (jj - n // 2) * g.cell, (ii - n // 2) * g.cell


def test_p4_dirty_image_matches_dft():
    rng = np.random.default_rng(21)
    n = 64
    g = synth.Geometry(n=n, cell=0.1 / n, os=4, w_planes=np.zeros(1), support=np.array([7]),
                       tile=np.array([16]), mk=n)
    uvw = _lattice_uvw(rng, g, 3000, 60)
    _, _, sl, sm = _pixel_sources(rng, g, 5)
    v = imaging.dft_predict(uvw, sl, sm, rng.uniform(0.1, 1, (5, 1)))
    tabs = kernels.make_tables(g, mueller.phi_identity(1, n, n))
    img = imaging.image_from_grid(g, gridding.grid(g, tabs, uvw, v), uvw.shape[0])[0]
    truth = imaging.dft_image(g, uvw, v, uvw.shape[0])[0]
    inner = slice(n // 4, 3 * n // 4)
    assert np.max(np.abs(img - truth)[inner, inner]) < 2e-4 * np.max(np.abs(truth))


def test_p5_w_projection_matches_dft_with_w_term():
    rng = np.random.default_rng(22)
    n, fov = 64, 0.4
    planes = np.array([-150.0, 0.0, 150.0])
    g = synth.Geometry(n=n, cell=fov / n, os=4, w_planes=planes, support=np.array([31, 7, 31]),
                       tile=np.array([16, 16, 16]), mk=n)
    uvw = _lattice_uvw(rng, g, 1500, 40, w=planes[rng.integers(0, 3, 1500)])
    _, _, sl, sm = _pixel_sources(rng, g, 5)
    v = imaging.dft_predict(uvw, sl, sm, rng.uniform(0.1, 1, (5, 1)))
    tabs = kernels.make_tables(g, mueller.phi_identity(1, n, n))
    img = imaging.image_from_grid(g, gridding.grid(g, tabs, uvw, v), uvw.shape[0])[0]
    truth = imaging.dft_image(g, uvw, v, uvw.shape[0])[0]
    inner = slice(n // 4, 3 * n // 4)
    err = np.max(np.abs(img - truth)[inner, inner]) / np.max(np.abs(truth))
    assert err < 5e-4
    # the same data without w-projection is far off: the pin is sensitive to the w screen
    g0 = synth.Geometry(n=n, cell=fov / n, os=4, w_planes=np.zeros(1), support=np.array([7]),
                        tile=np.array([16]), mk=n)
    t0 = kernels.make_tables(g0, mueller.phi_identity(1, n, n))
    img0 = imaging.image_from_grid(g0, gridding.grid(g0, t0, uvw, v), uvw.shape[0])[0]
    assert np.max(np.abs(img0 - truth)[inner, inner]) / np.max(np.abs(truth)) > 0.1


def test_p6_a_projection_predict_matches_dft():
    """Degrid of the model through Mueller kernels equals Eq. 2 evaluated directly."""
    rng = np.random.default_rng(23)
    n, fov = 64, 0.1
    g = synth.Geometry(n=n, cell=fov / n, os=4, w_planes=np.zeros(1), support=np.array([11]),
                       tile=np.array([16]), mk=n)
    beam = synth.seeded_leakage_beam(0.06, rng, level=0.05)
    tabs = kernels.make_tables(g, mueller.phi_degrid(synth.jones_on_lattice(beam, n, fov)))
    uvw = _lattice_uvw(rng, g, 300, 60)
    ii, jj, sl, sm = _pixel_sources(rng, g, 4)
    iquv = np.zeros((4, 4))
    iquv[:, 0] = rng.uniform(0.1, 1, 4)
    iquv[:, 1:] = rng.uniform(-0.1, 0.1, (4, 3))
    model = np.zeros((4, n, n))
    for s in range(4):
        model[:, ii[s], jj[s]] += iquv[s]
    vg = gridding.degrid(g, tabs, uvw, imaging.grid_from_model(g, model))
    vt = imaging.dft_predict(uvw, sl, sm, iquv, beam)
    assert np.max(np.abs(vg - vt)) < 1e-4 * np.max(np.abs(vt))
    # without the beam the prediction is wrong by the beam attenuation
    flat = kernels.make_tables(g, mueller.phi_identity(4, n, n, kind="degrid"))
    vf = gridding.degrid(g, flat, uvw, imaging.grid_from_model(g, model))
    assert np.max(np.abs(vf - vt)) > 1e-2 * np.max(np.abs(vt))


def test_p9_eq6_flux_recovery_closed_form():
    """Gridding with the Eq. 6 inverse recovers I B^2 / (B^2 + beta) for a Stokes-I source."""
    rng = np.random.default_rng(24)
    n, fov = 64, 0.1
    g = synth.Geometry(n=n, cell=fov / n, os=4, w_planes=np.zeros(1), support=np.array([11]),
                       tile=np.array([16]), mk=n)
    theta = 0.08
    beam = synth.GaussianLeakageBeam(theta=theta, level=0.0)
    eps = 0.2
    tabs = kernels.make_tables(g, mueller.phi_grid(synth.jones_on_lattice(beam, n, fov), eps))
    i0, j0 = 40, 22
    sl, sm = (j0 - n // 2) * g.cell, (i0 - n // 2) * g.cell
    uvw = _lattice_uvw(rng, g, 2000, 80)
    v = imaging.dft_predict(uvw, [sl], [sm], np.array([[1.0, 0, 0, 0]]), beam)
    img = imaging.image_from_grid(g, gridding.grid(g, tabs, uvw, v), uvw.shape[0])
    b = np.exp(-4 * np.log(2) * (sl ** 2 + sm ** 2) / theta ** 2)  # power beam at the source
    beta = (eps / 2) ** 2  # max |B| = 1 at the centre lattice point
    want = b * b / (b * b + beta)
    assert img[0, i0, j0] == pytest.approx(want, rel=1e-3)
    assert abs(img[1, i0, j0]) < 1e-3 and abs(img[2, i0, j0]) < 1e-3 and abs(img[3, i0, j0]) < 1e-3
    assert want < 0.99  # the source sits off the beam centre


def test_p11_unit_visibility_at_origin_gives_flat_image():
    n = 64
    g = synth.Geometry(n=n, cell=0.1 / n, os=4, w_planes=np.zeros(1), support=np.array([7]),
                       tile=np.array([16]), mk=n)
    tabs = kernels.make_tables(g, mueller.phi_identity(1, n, n))
    img = imaging.image_from_grid(g, gridding.grid(g, tabs, np.zeros((1, 3)), np.ones((1, 1))), 1.0)[0]
    inner = slice(n // 4, 3 * n // 4)
    assert np.max(np.abs(img[inner, inner] - 1.0)) < 2e-4


def test_predict_transform_is_adjoint_of_image_transform():
    """grid_from_model and the untapered image transform are an adjoint pair up to the real part."""
    rng = np.random.default_rng(25)
    n = 16
    g = synth.Geometry(n=n, cell=0.1 / n, os=4, w_planes=np.zeros(1), support=np.array([7]), mk=n)
    gr = (rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n)))
    model = rng.standard_normal((1, n, n))
    img = imaging.image_from_grid(g, gr, 1.0)  # Re(F gr) / (AA AA)
    rhs = np.vdot(imaging.grid_from_model(g, model), gr).real  # <F^H (model / AA AA), gr>
    assert np.sum(img * model) == pytest.approx(rhs, rel=1e-10)


# dft_image with per-pixel screens Phi_qc(l, m): the image is Re sum_c Phi_qc(l, m) A_c(l, m) / weight_sum,
# A_c the direct transform of correlation c.  The pins below catch a transposed Mueller index (q, c),
# screens applied at transposed pixels (y, x), a conjugated screen and a dropped imaginary part.

def _small_geom(n=16):
    return synth.Geometry(n=n, cell=0.05 / n, os=4, w_planes=np.zeros(1), support=np.array([7]), mk=n)


def test_dft_image_single_visibility_constant_screen_is_a_cosine_image():
    """One visibility V_c at (u, v, w) with a constant complex 4x4 screen A:
    I_q(l, m) = sum_c |A_qc V_c| cos(arg(A_qc V_c) - 2 pi (u l + v m + w (n - 1)))."""
    g = _small_geom()
    rng = np.random.default_rng(31)
    a = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    vis = (rng.standard_normal(4) + 1j * rng.standard_normal(4))[None]
    u, v, w = 37.0, -12.5, 80.0
    phi = np.broadcast_to(a[:, :, None, None], (4, 4, g.n, g.n))
    img = imaging.dft_image(g, np.array([[u, v, w]]), vis, 2.0, phi_pixels=phi)
    x = (np.arange(g.n) - g.n // 2) * g.cell
    mm, ll = np.meshgrid(x, x, indexing="ij")
    nm1 = -(ll ** 2 + mm ** 2) / (1 + np.sqrt(1 - ll ** 2 - mm ** 2))
    theta = 2 * np.pi * (u * ll + v * mm + w * nm1)
    for q in range(4):
        want = sum(abs(a[q, c] * vis[0, c]) * np.cos(np.angle(a[q, c] * vis[0, c]) - theta) for c in range(4)) / 2.0
        np.testing.assert_allclose(img[q], want, rtol=0, atol=1e-12)


def test_dft_image_screen_combines_correlation_images_linearly():
    """Re(A acc) = Re(A) Re(acc) - Im(A) Im(acc), with Re(acc) and -Im(acc) the identity-screen images of
    V and of i V: the screened image follows from two unscreened ones for any non-symmetric A."""
    g = _small_geom()
    rng = np.random.default_rng(32)
    uvw = np.stack([rng.uniform(-60, 60, 9), rng.uniform(-60, 60, 9), rng.uniform(-100, 100, 9)], 1)
    vis = rng.standard_normal((9, 4)) + 1j * rng.standard_normal((9, 4))
    a = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    phi = np.broadcast_to(a[:, :, None, None], (4, 4, g.n, g.n))
    got = imaging.dft_image(g, uvw, vis, 3.0, phi_pixels=phi)
    re_acc = imaging.dft_image(g, uvw, vis, 3.0)          # Re(acc_c) / 3
    m_im_acc = imaging.dft_image(g, uvw, 1j * vis, 3.0)  # Re(i acc_c) / 3 = -Im(acc_c) / 3
    want = np.einsum("qc,cyx->qyx", a.real, re_acc) + np.einsum("qc,cyx->qyx", a.imag, m_im_acc)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_dft_image_screen_is_applied_at_its_own_pixel():
    """With one visibility at the origin every A_c(l, m) equals V_c, so the image is Re(Phi_qc(i, j) V_c):
    a screen that varies along columns only (or rows only) must come out unchanged in layout."""
    g = _small_geom()
    rng = np.random.default_rng(33)
    vis = np.array([[1.0 + 0.5j, -0.25j, 2.0, 0.75 - 1j]])
    col = np.arange(g.n, dtype=np.float64)
    phi = np.zeros((4, 4, g.n, g.n), dtype=np.complex128)
    phi[0, 2] = col[None, :]                 # varies with j (l)
    phi[3, 1] = 1j * col[:, None]            # varies with i (m)
    phi[1, 0] = rng.standard_normal((g.n, g.n))
    img = imaging.dft_image(g, np.zeros((1, 3)), vis, 1.0, phi_pixels=phi)
    np.testing.assert_allclose(img[0], np.broadcast_to(col[None, :] * 2.0, (g.n, g.n)), atol=1e-12)
    np.testing.assert_allclose(img[3], np.broadcast_to((1j * col[:, None] * (-0.25j)).real, (g.n, g.n)), atol=1e-12)
    np.testing.assert_allclose(img[1], phi[1, 0].real * 1.0, atol=1e-12)
    np.testing.assert_allclose(img[2], 0.0, atol=1e-12)
