"""Pins of the Hogbom reference against closed forms (no GPU).

A dirty image that is exactly F x psf centred on a pixel is the textbook case: every iteration
takes the same pixel, the residual there falls as F (1 - g)^k and the components sum to
F (1 - (1 - g)^k); the number of iterations before a threshold t is the least k with
F (1 - g)^k < t.
"""
import math

import numpy as np

from oracle import clean


def gaussian_psf(n, sigma=2.0):
    y, x = np.mgrid[0:n, 0:n]
    return np.exp(-((x - n // 2) ** 2 + (y - n // 2) ** 2) / (2 * sigma ** 2)).astype(np.float32)


def shifted(psf, py, px):
    n = psf.shape[0]
    out = np.zeros_like(psf)
    for y in range(n):
        for x in range(n):
            sy, sx = y - py + n // 2, x - px + n // 2
            if 0 <= sy < n and 0 <= sx < n:
                out[y, x] = psf[sy, sx]
    return out


def test_single_source_geometric_series():
    n, f, g = 32, 2.0, 0.25
    psf = gaussian_psf(n)
    img = (np.float32(f) * shifted(psf, 13, 17))[None]
    r, comps = clean.hogbom(img, psf, gain=g, max_iter=10)
    assert len(comps) == 10 and all(c[0] == 13 * n + 17 for c in comps)
    assert math.isclose(float(r[0, 13, 17]), f * (1 - g) ** 10, rel_tol=1e-5)
    assert math.isclose(sum(float(c[1][0]) for c in comps), f * (1 - (1 - g) ** 10), rel_tol=1e-5)
    # the whole image is the same multiple of the shifted psf
    np.testing.assert_allclose(r[0], f * (1 - g) ** 10 * shifted(psf, 13, 17), atol=1e-6)


def test_threshold_gives_the_closed_form_iteration_count():
    n, f, g, t = 32, 1.0, 0.1, 0.05
    psf = gaussian_psf(n)
    img = shifted(psf, 10, 10)[None] * np.float32(f)
    _, comps = clean.hogbom(img, psf, gain=g, threshold=t, max_iter=1000)
    assert len(comps) == math.ceil(math.log(t / f) / math.log(1 - g))


def test_mask_keeps_sources_outside_it():
    n = 32
    psf = gaussian_psf(n, 1.0)
    img = (3.0 * shifted(psf, 5, 5) + 1.0 * shifted(psf, 25, 25))[None].astype(np.float32)
    mask = np.zeros((n, n), np.uint8)
    mask[16:, 16:] = 1
    r, comps = clean.hogbom(img, psf, mask=mask, gain=0.5, max_iter=20)
    assert all(divmod(c[0], n)[0] >= 16 and divmod(c[0], n)[1] >= 16 for c in comps)
    assert math.isclose(float(r[0, 5, 5]), 3.0, rel_tol=1e-6)
    assert clean.hogbom(img, psf, mask=np.zeros((n, n), np.uint8))[1] == []


def test_ties_take_the_first_pixel_and_all_planes_follow():
    n = 16
    psf = np.zeros((n, n), np.float32)
    psf[n // 2, n // 2] = 1.0
    img = np.zeros((2, n, n), np.float32)
    img[0, 3, 4] = img[0, 9, 2] = -2.0   # |I| ties; the first in row-major order wins
    img[1, 3, 4] = 0.5
    r, comps = clean.hogbom(img, psf, gain=1.0, max_iter=1)
    assert comps[0][0] == 3 * n + 4
    np.testing.assert_array_equal(comps[0][1], np.array([-2.0, 0.5], np.float32))
    assert r[0, 3, 4] == 0.0 and r[1, 3, 4] == 0.0 and r[0, 9, 2] == -2.0


def test_patch_limits_the_subtraction():
    n = 32
    psf = np.ones((n, n), np.float32)
    img = np.ones((1, n, n), np.float32)
    img[0, 16, 16] = 2.0
    r, _ = clean.hogbom(img, psf, gain=0.5, max_iter=1, psf_patch=2)
    changed = r[0] != img[0]
    assert changed.sum() == 25 and changed[14:19, 14:19].all()


def test_beam_mask_fraction():
    p = np.array([[1.0, 0.5], [0.2, 0.1]])
    np.testing.assert_array_equal(clean.beam_mask(p, 0.2), [[1, 1], [1, 0]])
