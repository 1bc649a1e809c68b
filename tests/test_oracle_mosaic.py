"""Pins of the image-domain mosaicing reference (no GPU).

- Direction cosines against an independent construction: the unit vector of (ra, dec) projected
  on the east and north unit vectors at the phase centre, plus textbook values.
- Bilinear interpolation reproduces a function linear in the source pixel coordinates exactly,
  and a reprojection onto the same frame is an exact copy.
- A point placed on a source pixel reappears, after reprojection to a frame with another phase
  centre and a finer cell, with its centroid at the destination pixel computed from the sky
  position directly.
- Mosaic weighting: one field gives the field image where covered; fields that see the same
  constant sky give that constant on their union; low total weight gives 0.
- Phase rotation: point-source visibilities predicted about one centre and rotated to another
  equal the direct Fourier transform about the other centre; rotating onto the same centre
  changes nothing; a round trip returns the input.
"""
import math

import numpy as np

from oracle import imaging, mosaic

DEG = math.pi / 180.0


def unit(ra, dec):
    return np.stack([np.cos(dec) * np.cos(ra), np.cos(dec) * np.sin(ra), np.sin(dec)], axis=-1)


def test_direction_cosines_against_vector_basis():
    rng = np.random.default_rng(1)
    ra0, dec0 = 1.1, -0.7
    east = np.array([-math.sin(ra0), math.cos(ra0), 0.0])
    north = np.array([-math.sin(dec0) * math.cos(ra0), -math.sin(dec0) * math.sin(ra0), math.cos(dec0)])
    centre = unit(ra0, dec0)
    ra = ra0 + rng.uniform(-0.5, 0.5, 200)
    dec = np.clip(dec0 + rng.uniform(-0.5, 0.5, 200), -1.5, 1.5)
    s = unit(ra, dec)
    l, m, n = mosaic.radec_to_lm(ra, dec, ra0, dec0)
    np.testing.assert_allclose(l, s @ east, atol=1e-14)
    np.testing.assert_allclose(m, s @ north, atol=1e-14)
    np.testing.assert_allclose(n, s @ centre, atol=1e-14)
    ra2, dec2 = mosaic.lm_to_radec(l, m, ra0, dec0)
    np.testing.assert_allclose(np.angle(np.exp(1j * (ra2 - ra))), 0.0, atol=1e-12)
    np.testing.assert_allclose(dec2, dec, atol=1e-12)


def test_direction_cosine_textbook_values():
    assert np.allclose(mosaic.radec_to_lm(0.3, 0.2, 0.3, 0.2), (0.0, 0.0, 1.0))
    assert np.allclose(mosaic.radec_to_lm(0.3 + math.pi / 2, 0.0, 0.3, 0.0), (1.0, 0.0, 0.0))
    th = 0.1
    assert np.allclose(mosaic.radec_to_lm(0.3, 0.2 + th, 0.3, 0.2), (0.0, math.sin(th), math.cos(th)))


def test_bilinear_is_exact_on_linear_functions_and_identity_copies():
    rng = np.random.default_rng(2)
    n = 64
    src_frame = (n, 0.4 * DEG / n, 0.50, -0.60)
    dst_frame = (48, 0.5 * DEG / 48, 0.50 + 0.07 * DEG, -0.60 + 0.05 * DEG)
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    img = 0.3 * xx - 1.7 * yy + 2.0
    v, w = mosaic.reproject(img, src_frame, dst_frame)
    x, y, front = mosaic.source_pixels(dst_frame, src_frame)
    e = mosaic.EDGE
    cov = (x >= -e) & (y >= -e) & (x <= n - 1 + e) & (y <= n - 1 + e) & front
    assert 0.3 < cov.mean() < 1.0
    np.testing.assert_allclose(v[cov], (0.3 * x - 1.7 * y + 2.0)[cov], atol=1e-12)
    assert np.all(v[~cov] == 0) and np.array_equal(w, cov.astype(float))
    # the destination centre pixel looks at the destination phase centre
    l, m, _ = mosaic.radec_to_lm(dst_frame[2], dst_frame[3], src_frame[2], src_frame[3])
    assert abs(x[24, 24] - (l / src_frame[1] + n // 2)) < 1e-9 and abs(y[24, 24] - (m / src_frame[1] + n // 2)) < 1e-9
    r = rng.standard_normal((2, n, n))
    same, ws = mosaic.reproject(r, src_frame, src_frame)
    np.testing.assert_allclose(same, r, atol=1e-12)
    assert np.all(ws == 1.0)


def test_point_source_lands_at_its_sky_position():
    n = 128
    src_frame = (n, 0.01 * DEG, 2.0, 0.4)
    dst_frame = (256, 0.0025 * DEG, 2.0 + 0.15 * DEG, 0.4 - 0.1 * DEG)
    img = np.zeros((n, n))
    i, j = 60, 70
    img[i, j] = 1.0
    ra, dec = mosaic.lm_to_radec((j - n // 2) * src_frame[1], (i - n // 2) * src_frame[1], src_frame[2], src_frame[3])
    l, m, _ = mosaic.radec_to_lm(ra, dec, dst_frame[2], dst_frame[3])
    want_x, want_y = l / dst_frame[1] + 128, m / dst_frame[1] + 128
    v, _ = mosaic.reproject(img, src_frame, dst_frame)
    yy, xx = np.mgrid[0:256, 0:256]
    tot = v.sum()
    assert abs(tot / 16.0 - 1.0) < 0.02  # the tent covers 4 x 4 destination cells per source cell
    assert abs((v * xx).sum() / tot - want_x) < 0.05 and abs((v * yy).sum() / tot - want_y) < 0.05


def test_mosaic_weighting():
    n = 64
    f1 = (n, 0.02 * DEG, 1.0, 0.3)
    f2 = (n, 0.02 * DEG, 1.0 + 0.5 * DEG, 0.3)
    dst = (96, 0.02 * DEG, 1.0 + 0.25 * DEG, 0.3)
    rng = np.random.default_rng(3)
    a = rng.standard_normal((4, n, n))
    wa = rng.uniform(0.5, 1.0, (n, n))
    one, den = mosaic.mosaic([a], [f1], [wa], dst, 1e-6)
    v, w = mosaic.reproject(a, f1, dst, wa)
    cov = w > 0
    np.testing.assert_allclose(one[:, cov], v[:, cov], atol=1e-12)
    assert np.all(one[:, ~cov] == 0)
    const = np.full((1, n, n), 2.5)
    both, den = mosaic.mosaic([const, const], [f1, f2], [wa, wa[::-1]], dst, 1e-6)
    covered = den >= 1e-6
    assert covered.mean() > 0.5
    np.testing.assert_allclose(both[:, covered], 2.5, atol=1e-12)
    none, _ = mosaic.mosaic([const], [f1], [wa], dst, 10.0)
    assert np.all(none == 0)


def test_phase_rotation_matches_the_direct_transform_about_the_new_centre():
    rng = np.random.default_rng(7)
    a = (1.2, -0.6)
    b = (1.2 + 0.8 * DEG / math.cos(-0.6), -0.6 + 0.5 * DEG)
    ra = a[0] + rng.uniform(-1, 1, 6) * DEG
    dec = a[1] + rng.uniform(-1, 1, 6) * DEG
    flux = rng.uniform(0.2, 1.0, (6, 1))
    uvw = rng.uniform(-3000, 3000, (500, 3))
    la, ma, _ = mosaic.radec_to_lm(ra, dec, *a)
    va = imaging.dft_predict(uvw, la, ma, flux)
    uvw_b, vb = mosaic.phase_rotate(uvw, va, a, b)
    lb, mb, _ = mosaic.radec_to_lm(ra, dec, *b)
    want = imaging.dft_predict(uvw_b, lb, mb, flux)
    np.testing.assert_allclose(vb, want, rtol=0, atol=1e-9 * np.abs(want).max())
    np.testing.assert_allclose(np.linalg.norm(uvw_b, axis=1), np.linalg.norm(uvw, axis=1), rtol=1e-13)
    same_uvw, same = mosaic.phase_rotate(uvw, va, a, a)
    np.testing.assert_allclose(same_uvw, uvw, atol=1e-9)
    np.testing.assert_allclose(same, va, atol=1e-12)
    back_uvw, back = mosaic.phase_rotate(uvw_b, vb, b, a)
    np.testing.assert_allclose(back_uvw, uvw, atol=1e-8)
    np.testing.assert_allclose(back, va, atol=1e-9)

