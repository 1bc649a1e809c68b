"""UV-domain mosaicing (Sec. 2.2, Eq. 1) in float64 (test infrastructure only).

Each mosaic component (field) is gridded onto one common uv grid about the mosaic phase centre,
weighted by its primary beam through the gridding kernel, and the weighting is removed from the
image afterwards by gamma(l, m) of Eq. 1: the primary-beam pattern sqrt(sum_i B_i^2), normalised to
a maximum of one over the image, times the weighting correction 1 / sum_i B_i^2.

Readings taken here (the paper gives Eq. 1 and no more):

  * The kernel of field i is the adjoint of its prediction: the degridding screens
    Phi = (S^-1 M_i^S)^H of field i's Jones field (the beam centred on the field's pointing, on the
    common lattice).  For the Stokes matrix of Eq. 4, (S^-1)^H S^-1 = 2 I, so an unpolarised sky
    enters the common image as 2 sum_i B_i^2 I; the factor 1/2 is applied with gamma.
  * Each field's visibilities are divided by that field's own weight sum before gridding, so every
    field's dirty image is normalised on its own, which the weighting correction assumes.
  * B_i is the power beam at the image pixels; the maximum in gamma is over the image pixels.
  * Where sum_i B_i^2 is below `floor` times its maximum the mosaic holds no data: gamma is 0
    there (Eq. 1 would divide by a vanishing sum).
"""
import numpy as np

from . import gridding, imaging, kernels, mueller


def gamma(beams, floor: float = 1e-3) -> np.ndarray:
    """Eq. 1 on the pixel grid: beams [N][n][n] (B_i), result [n][n]."""
    s = np.sum(np.asarray(beams, dtype=np.float64) ** 2, axis=0)
    smax = s.max()
    out = np.zeros_like(s)
    ok = s >= floor * smax
    pbp = np.sqrt(s[ok]) / np.sqrt(smax)
    out[ok] = pbp * (1.0 / s[ok])
    return out


def common_grid(geom, fields) -> np.ndarray:
    """Sum over fields of the grid of each field's (already weight-normalised) visibilities,
    each through its own degridding-screen kernels.  fields: (uvw, vis, jones) triples."""
    g = None
    for uvw, vis, jones in fields:
        tables = kernels.make_tables(geom, mueller.phi_degrid(jones))
        gi = gridding.grid(geom, tables, uvw, vis)
        g = gi if g is None else g + gi
    return g


def mosaic_image(geom, fields, beams, floor: float = 1e-3) -> np.ndarray:
    """The corrected UV-domain mosaic [4][n][n]: image of the common grid (weight sum 1) times
    gamma / 2 (see the readings)."""
    img = imaging.image_from_grid(geom, common_grid(geom, fields), 1.0)
    return 0.5 * img * gamma(beams, floor)[None]
