"""Pins of the UV-domain mosaic oracle (Sec. 2.2, Eq. 1): gamma's closed forms, and the whole
chain (per-field beam kernels -> common grid -> FFT -> taper -> gamma) against direct Fourier
transforms and against the flux of point sources times the normalised primary-beam pattern."""
import numpy as np
import pytest

import synth
from oracle import imaging, mueller, uvmosaic


def gauss(n, cell, l0, m0, fwhm):
    return synth.power_on_pixels(synth.OffsetBeam(synth.GaussianLeakageBeam(fwhm, level=0.0), l0, m0), n, cell)


def test_gamma_one_field_is_inverse_beam_times_peak():
    """One field: gamma = [B / max B] / B^2 = 1 / (B max B) wherever B^2 clears the floor."""
    b = gauss(48, 0.002, 0.01, -0.005, 0.05)
    g = uvmosaic.gamma(b[None], floor=1e-3)
    ok = b ** 2 >= 1e-3 * (b ** 2).max()
    assert ok.sum() > 100 and (~ok).sum() > 10
    np.testing.assert_allclose(g[ok], 1.0 / (b[ok] * b.max()), rtol=1e-12)
    assert np.all(g[~ok] == 0)


def test_gamma_identical_fields_and_pattern_normalisation():
    """N coincident fields: gamma = 1 / (N B max B); for any set, gamma sum B^2 is the pattern
    sqrt(S / max S), which is 1 at the sensitivity peak and below 1 elsewhere."""
    b = gauss(40, 0.003, 0.0, 0.0, 0.06)
    g3 = uvmosaic.gamma(np.stack([b, b, b]), floor=0.0)
    np.testing.assert_allclose(g3, 1.0 / (3.0 * b * b.max()), rtol=1e-12)
    bs = np.stack([gauss(40, 0.003, dl, dm, 0.05) for dl, dm in [(-0.02, 0), (0.02, 0), (0, 0.03)]])
    s = (bs ** 2).sum(0)
    pat = uvmosaic.gamma(bs, floor=0.0) * s
    assert abs(pat.max() - 1.0) < 1e-12 and pat.flat[np.argmax(s)] == pytest.approx(1.0, abs=1e-12)
    np.testing.assert_allclose(pat, np.sqrt(s / s.max()), rtol=1e-12)


def _mosaic_case(seed=31, leakage=0.0):
    rng = np.random.default_rng(seed)
    n, fov = 64, 0.12
    g = synth.Geometry(n=n, cell=fov / n, os=4, w_planes=np.zeros(1), support=np.array([13]),
                       tile=np.array([16]), mk=n)
    base = synth.seeded_leakage_beam(0.05, rng, level=leakage)
    pointings = [(-0.02, -0.01), (0.02, -0.01), (0.0, 0.02)]
    beams = [synth.OffsetBeam(base, l0, m0) for l0, m0 in pointings]
    # two unpolarised point sources on pixel centres, inside the mosaic
    ii = np.array([n // 2 - 5, n // 2 + 7])
    jj = np.array([n // 2 + 6, n // 2 - 4])
    sl, sm = (jj - n // 2) * g.cell, (ii - n // 2) * g.cell
    iquv = np.array([[0.8, 0, 0, 0], [0.5, 0, 0, 0]], dtype=np.float64)
    fields = []
    for k, b in enumerate(beams):
        c = n // 2 * g.os
        nv = 900 + 150 * k
        fx, fy = rng.integers(c - 90, c + 90, nv), rng.integers(c - 90, c + 90, nv)
        uvw = np.stack([(fx / g.os - n / 2) / g.fov, (fy / g.os - n / 2) / g.fov, np.zeros(nv)], 1)
        vis = imaging.dft_predict(uvw, sl, sm, iquv, beam=b) / nv  # each field normalised on its own
        fields.append((uvw, vis, synth.jones_on_lattice(b, n, fov)))
    pix = np.stack([synth.power_on_pixels(b, n, g.cell) for b in beams])
    return g, fields, pix, (ii, jj, iquv)


def test_uv_mosaic_matches_direct_transforms():
    """The gridded mosaic equals, pixel by pixel, gamma / 2 times the sum over fields of the direct
    Fourier transform of each field's visibilities through the same screens (S^-1 M_i^S)^H."""
    g, fields, pix, _ = _mosaic_case(leakage=0.02)
    got = uvmosaic.mosaic_image(g, fields, pix)
    direct = 0
    for uvw, vis, jones in fields:
        direct = direct + imaging.dft_image(g, uvw, vis, 1.0, phi_pixels=mueller.phi_degrid(jones))
    want = 0.5 * direct * uvmosaic.gamma(pix)[None]
    n = g.n
    inner = slice(n // 4, 3 * n // 4)
    err = np.max(np.abs(got - want)[:, inner, inner]) / np.max(np.abs(want[0]))
    assert err < 1e-5, err  # 7e-7 in the float64 run


def test_uv_mosaic_recovers_flux_times_beam_pattern():
    """At each source pixel the Stokes-I mosaic is the source flux times sqrt(S / max S) (the
    primary-beam pattern of Eq. 1), within the dirty-image sidelobes of the other source; Q, U, V
    stay near zero.  Kernels from the gridding screens (M'^S)^-1 S instead, or a missing 1/2, miss."""
    g, fields, pix, (ii, jj, iquv) = _mosaic_case()
    img = uvmosaic.mosaic_image(g, fields, pix)
    s = (pix ** 2).sum(0)
    pat = np.sqrt(s / s.max())
    for k in range(2):
        want = iquv[k, 0] * pat[ii[k], jj[k]]
        assert img[0, ii[k], jj[k]] == pytest.approx(want, rel=0.01)  # 0.1-0.3 % in the float64 run
        assert np.all(np.abs(img[1:, ii[k], jj[k]]) < 0.01 * want)
    wrong = [(u, v, j) for u, v, j in fields]
    from oracle import gridding, kernels
    gg = 0
    for uvw, vis, jones in wrong:
        gg = gg + gridding.grid(g, kernels.make_tables(g, mueller.phi_grid(jones, 0.2)), uvw, vis)
    bad = 0.5 * imaging.image_from_grid(g, gg, 1.0) * uvmosaic.gamma(pix)[None]
    assert abs(bad[0, ii[0], jj[0]] - iquv[0, 0] * pat[ii[0], jj[0]]) > 0.2 * iquv[0, 0] * pat[ii[0], jj[0]]
