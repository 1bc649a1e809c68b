"""Image-domain and UV-domain mosaics on the device (Sec. 2.2).

Each field (pointing) is imaged with the phase centre at its own pointing centre (grid -> FFT ->
taper in the library's kernels); image-plane reprojection (pg_reproject) accumulates every field
image, weighted by its weight image, onto a common mosaic frame, and pg_weight_normalise turns the
sums into the weighted mean.  In the other direction the mosaic model is reprojected onto each
field's frame and predicted through that field's degridding kernels.

UV-domain mosaics (uv_image) grid every field onto one common grid about the mosaic phase centre
through that field's own primary-beam kernels (its degridding-kind kernel set, whose Jones field is
the beam centred on the field's pointing), image the common grid once, and remove the beam
weighting with gamma of Eq. 1 (pg_mosaic_gamma).

A frame is an n x n orthographic projection about (ra, dec) with `cell` radians per pixel; the
pixel convention is the imager's (column j at l = (j - n/2) cell, row i at m = (i - n/2) cell).
"""
from __future__ import annotations

from collections import namedtuple
from dataclasses import dataclass

from . import polgrid as pg

SkyFrame = namedtuple("SkyFrame", "n cell ra dec")


@dataclass
class Field:
    frame: SkyFrame        # the field's image frame (phase centre = pointing centre)
    plan: object           # pg.Plan of the field's visibilities
    kernels_grid: object   # pg.Kernels (grid direction)
    kernels_degrid: object  # pg.Kernels (degrid direction), same geometry as the plan
    weight: object         # float32 [n][n] device: the field's mosaic weight image
    weight_sum: float      # natural-weighting normalisation of the field image


def image(fields, vis_list, mosaic_frame, min_weight: float, out=None, weight_out=None, grid_buf=None,
          field_buf=None, deterministic: bool = False):
    """Mosaic of the fields' dirty images: sum_f w_f I_f / sum_f w_f on mosaic_frame (0 where the
    total weight is below min_weight).  Returns (mosaic float32 [npol][n][n], weight [n][n]).
    deterministic: field images gridded in the reproducible mode."""
    import torch

    npol = fields[0].kernels_grid.npol
    n = mosaic_frame.n
    dev = vis_list[0].device
    if out is None:
        out = torch.empty((npol, n, n), dtype=torch.float32, device=dev)
    if weight_out is None:
        weight_out = torch.empty((n, n), dtype=torch.float32, device=dev)
    out.zero_()
    weight_out.zero_()
    for f, vis in zip(fields, vis_list):
        img = pg.image(f.plan, f.kernels_grid, vis, f.weight_sum, grid_buf=grid_buf, out=field_buf,
                       deterministic=deterministic)
        pg.reproject(img, f.frame, out, mosaic_frame, src_weight=f.weight, dst_weight=weight_out, accumulate=True)
    pg.weight_normalise(out, weight_out, min_weight)
    return out, weight_out


def predict(fields, model, mosaic_frame, outs=None, field_buf=None, subtract: bool = False):
    """Model visibilities of every field: the mosaic model reprojected onto the field's frame,
    then taper -> inverse FFT -> degrid with the field's kernels (with subtract: outs[f] -= ...)."""
    import torch

    res = []
    for i, f in enumerate(fields):
        npol = model.shape[0]
        if field_buf is None or tuple(field_buf.shape) != (npol, f.frame.n, f.frame.n):
            field_buf = torch.empty((npol, f.frame.n, f.frame.n), dtype=torch.float32, device=model.device)
        pg.reproject(model, mosaic_frame, field_buf, f.frame)
        res.append(pg.predict(f.plan, f.kernels_degrid, field_buf, out=None if outs is None else outs[i],
                              subtract=subtract))
    return res


def uv_image(fields, beams, floor: float = 1e-3, out=None, grid_buf=None, weight_out=None):
    """UV-domain mosaic (Sec. 2.2, Eq. 1).  fields: (plan, kernels, vis) triples on one common
    geometry, where kernels are the field's PG_KIND_DEGRID set (its beam as the gridding kernel) and
    vis are already divided by the field's own weight sum; beams float32 [nfields][n][n] are the
    fields' power beams at the image pixels.  Returns (mosaic float32 [npol][n][n], S = sum B^2)."""
    import torch

    k0 = fields[0][1]
    npol, n = k0.npol, k0.n
    if grid_buf is None:
        grid_buf = torch.empty((npol, n, n), dtype=torch.complex64, device=beams.device)
    for i, (p, k, vis) in enumerate(fields):
        pg.grid(p, k, vis, out=grid_buf, accumulate=i > 0, fftshift=True)
    if out is None:
        out = torch.empty((npol, n, n), dtype=torch.float32, device=beams.device)
    img = pg.taper(k0, torch.fft.fft2(grid_buf), out, pg.TAPER_IMAGE, 1.0)
    weight = pg.mosaic_gamma(beams, img, floor=floor, scale=0.5, weight_sum=weight_out)
    return img, weight
