"""Image-domain mosaicing (test infrastructure only).

Sec. 2.2, image-domain mosaics: every mosaic component (field) is imaged with the phase centre at
its own pointing centre; image-plane reprojection then builds the mosaic at one common phase
centre; before the degridding stage of clean the model image is reprojected back to the phase
centre of each field, and each field gets its own FFT and degridding.

Phase rotation (listed with reprojection among the GPU-suited steps, Sec. 4) brings
visibilities stored about one phase centre to another, so that a field can be imaged about its
own pointing centre.

The paper gives no formulas for these steps; these are the readings used here:
- An image is an orthographic (SIN) projection about its phase centre (a0, d0).  Pixel (row i,
  column j) of an n x n image with cell size `cell` holds the direction cosines
  l = (j - n/2) cell, m = (i - n/2) cell (the gridder's image convention), with
      l = cos d sin(a - a0),   m = sin d cos d0 - cos d sin d0 cos(a - a0),
  the components of the unit direction vector along the east and north axes at the centre.
  Only the hemisphere in front of the centre (n = sqrt(1 - l^2 - m^2) > 0) is covered.
- Reprojection samples the source image at the source-frame pixel position of every
  destination pixel by bilinear interpolation.  A destination pixel is covered when that
  position lies within the source pixel centres, -1e-6 <= x, y <= n_src - 1 + 1e-6 (the margin
  keeps border pixels of an identical frame covered despite rounding; positions are then clamped
  to [0, n_src - 1]) and the direction is in front of both centres; uncovered pixels get value 0
  and weight 0.
- The mosaic is the weighted mean  I = sum_f w_f I_f / sum_f w_f,  with w_f a weight image per
  field (for example the squared power beam inside the beam mask) reprojected like the image;
  mosaic pixels whose total weight is below `min_weight` are 0.
- Phase rotation from centre A to centre B: the baseline b = u e_A + v n_A + w c_A (wavelengths,
  on A's east/north/centre axes) gets coordinates (b.e_B, b.n_B, b.c_B) about B, and with the
  predict convention V = sum I exp(+2 pi i (u l + v m + w (n - 1))) every correlation is
  multiplied by exp(2 pi i (w_A - w_B)).
Everything is float64.
"""
import numpy as np


def radec_to_lm(ra, dec, ra0, dec0):
    """Direction cosines (l, m, n) of (ra, dec) about the centre (ra0, dec0)."""
    ra, dec = np.asarray(ra, dtype=np.float64), np.asarray(dec, dtype=np.float64)
    da = ra - ra0
    l = np.cos(dec) * np.sin(da)
    m = np.sin(dec) * np.cos(dec0) - np.cos(dec) * np.sin(dec0) * np.cos(da)
    n = np.sin(dec) * np.sin(dec0) + np.cos(dec) * np.cos(dec0) * np.cos(da)
    return l, m, n


def lm_to_radec(l, m, ra0, dec0):
    """Inverse of radec_to_lm on the front hemisphere (l^2 + m^2 <= 1)."""
    l, m = np.asarray(l, dtype=np.float64), np.asarray(m, dtype=np.float64)
    n = np.sqrt(np.maximum(0.0, 1.0 - l * l - m * m))
    dec = np.arcsin(np.clip(m * np.cos(dec0) + n * np.sin(dec0), -1.0, 1.0))
    ra = ra0 + np.arctan2(l, n * np.cos(dec0) - m * np.sin(dec0))
    return ra, dec


def source_pixels(dst_frame, src_frame):
    """Source-frame pixel coordinates (x, y) of every destination pixel, shape [n_dst, n_dst] each,
    and a mask of destination pixels whose direction is on both front hemispheres.
    A frame is (n, cell, ra, dec)."""
    nd, cd, rad, decd = dst_frame
    ns, cs, ras, decs = src_frame
    c = (np.arange(nd) - nd // 2) * cd
    l0, m0 = np.meshgrid(c, c)  # column index -> l, row index -> m
    front = l0 * l0 + m0 * m0 < 1.0
    ra, dec = lm_to_radec(l0, m0, rad, decd)
    l, m, n = radec_to_lm(ra, dec, ras, decs)
    return l / cs + ns // 2, m / cs + ns // 2, front & (n > 0)


EDGE = 1e-6  # pixels


def bilinear(img, x, y):
    """Bilinear samples of img[..., row, col] at (x = column, y = row), and the covered mask
    -EDGE <= x, y <= n - 1 + EDGE (positions clamped to [0, n - 1]); uncovered samples are 0."""
    img = np.asarray(img, dtype=np.float64)
    n = img.shape[-1]
    inside = (x >= -EDGE) & (y >= -EDGE) & (x <= n - 1 + EDGE) & (y <= n - 1 + EDGE)
    xc = np.where(inside, np.clip(x, 0.0, n - 1.0), 0.0)
    yc = np.where(inside, np.clip(y, 0.0, n - 1.0), 0.0)
    x0 = np.minimum(np.floor(xc).astype(np.int64), n - 2)
    y0 = np.minimum(np.floor(yc).astype(np.int64), n - 2)
    fx, fy = xc - x0, yc - y0
    v = ((1 - fy) * ((1 - fx) * img[..., y0, x0] + fx * img[..., y0, x0 + 1])
         + fy * ((1 - fx) * img[..., y0 + 1, x0] + fx * img[..., y0 + 1, x0 + 1]))
    return np.where(inside, v, 0.0), inside


def reproject(src, src_frame, dst_frame, src_weight=None):
    """(dst [..., n_dst, n_dst], weight [n_dst, n_dst]): src resampled onto the destination frame;
    weight = the bilinear sample of src_weight (1 where covered if None), 0 where uncovered."""
    x, y, front = source_pixels(dst_frame, src_frame)
    v, inside = bilinear(src, x, y)
    cov = inside & front
    v = np.where(cov, v, 0.0)
    if src_weight is None:
        w = cov.astype(np.float64)
    else:
        w = np.where(cov, bilinear(src_weight, x, y)[0], 0.0)
    return v, w


def mosaic(images, frames, weights, dst_frame, min_weight):
    """Weighted mean of the reprojected field images: sum_f w_f I_f / sum_f w_f where the total
    weight is at least min_weight, else 0."""
    num, den = 0.0, 0.0
    for img, fr, wt in zip(images, frames, weights):
        v, w = reproject(img, fr, dst_frame, wt)
        num = num + w * v
        den = den + w
    return np.where(den >= min_weight, num / np.where(den > 0, den, 1.0), 0.0), den


def axes(ra0, dec0):
    """East, north and centre unit vectors of the frame about (ra0, dec0), rows of a 3 x 3 array."""
    sa, ca, sd, cd = np.sin(ra0), np.cos(ra0), np.sin(dec0), np.cos(dec0)
    return np.array([[-sa, ca, 0.0], [-sd * ca, -sd * sa, cd], [cd * ca, cd * sa, sd]])


def phase_rotate(uvw, vis, centre_from, centre_to):
    """(uvw about centre_to, vis about centre_to) from uvw float64 [nvis][3] and vis [nvis][npol]
    about centre_from; centres are (ra, dec) in radians."""
    uvw = np.asarray(uvw, dtype=np.float64)
    b = uvw @ axes(*centre_from)           # baseline vectors, equatorial Cartesian
    out = b @ axes(*centre_to).T
    ph = np.exp(2j * np.pi * (uvw[:, 2] - out[:, 2]))
    return out, np.asarray(vis, dtype=np.complex128) * ph[:, None]

