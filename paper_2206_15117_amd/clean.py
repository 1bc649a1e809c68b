"""Cotton-Schwab clean on the device (Sec. 2.1): major cycles image the residual visibilities with
the A x W gridding kernels (grid -> FFT -> taper); minor cycles (Hogbom, pg_hogbom) take point
components out of the residual image inside the beam mask; the model image is then predicted
through the degridding kernels and subtracted from the visibilities (taper x -1 -> inverse FFT
-> accumulating degrid), and the next major cycle starts from the new residual.

Every arithmetic step of the cycles (imaging, peak search, PSF normalisation, minor cycles,
prediction) runs in the library's kernels; torch provides buffers, the FFT and the AND of the
two component masks when they are set up.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import polgrid as pg


@dataclass
class CleanResult:
    model: object                    # float32 [npol][n][n] component image
    residual: object                 # float32 [npol][n][n] final residual image
    components: int = 0              # components found over all minor cycles
    peaks: list = field(default_factory=list)  # |I| peak of the residual at the start of each major cycle


def psf(plan, kernels, weight_sum: float):
    """The point-spread function: Stokes-I image of unit Stokes-I visibilities (XX = YY = 1) on the
    same plan and kernels, float32 [n][n], divided by its value at the phase centre (n/2, n/2) so
    the peak is one (the largest |value| can sit at the image edge, where the taper correction
    amplifies rounding noise)."""
    import torch

    npol = kernels.npol
    unit = torch.zeros((plan.nvis, npol), dtype=torch.complex64, device="cuda")
    unit[:, 0] = 1.0
    if npol == 4:
        unit[:, 3] = 1.0
    img = pg.image(plan, kernels, unit, weight_sum)[0].contiguous()
    n = img.shape[-1]
    return pg.normalise_at(img, (n // 2) * n + n // 2)


def taper_mask(kernels, aa_min: float = 0.1):
    """uint8 [n][n]: 1 where AA(l) AA(m) >= aa_min.  Towards the image edge the taper correction
    divides by an anti-aliasing function that falls to zero, so noise there is amplified without
    bound; clean is kept to the region where the correction is well conditioned."""
    import numpy as np
    import torch

    aa = np.outer(kernels.aa_pixels, kernels.aa_pixels)
    return torch.from_numpy((aa >= aa_min).astype(np.uint8)).cuda()


def cotton_schwab(plan, kernels_grid, kernels_degrid, vis, mask=None, gain: float = 0.1, threshold: float = 0.0,
                  cycles: int = 5, minor_iter: int = 500, cycle_factor: float = 0.2, psf_patch: int = 0,
                  beam=None, aa_min: float = 0.1):
    """Clean `vis` (complex64 [nvis][npol], device).  Components are taken only where `mask` (e.g.
    the beam mask of Sec. 3.3; uint8 [n][n]) and the taper mask (taper_mask(aa_min)) are both set.
    A minor cycle stops at max(threshold, cycle_factor x the residual peak at its start) or after
    minor_iter components; clean stops after `cycles` major cycles, or when the residual peak is
    below threshold."""
    import torch

    n, npol = kernels_grid.n, kernels_grid.npol
    wsum = float(plan.n_kept)
    beam = psf(plan, kernels_grid, wsum) if beam is None else beam
    tm = taper_mask(kernels_grid, aa_min)
    mask = tm if mask is None else (tm * mask).contiguous()
    model = torch.zeros((npol, n, n), dtype=torch.float32, device="cuda")
    resid_vis = vis.clone()
    grid_buf = torch.empty((npol, n, n), dtype=torch.complex64, device="cuda")
    out = CleanResult(model=model, residual=None)
    for _ in range(cycles):
        img = pg.image(plan, kernels_grid, resid_vis, wsum, grid_buf=grid_buf)
        peak, _ = pg.masked_peak(img[0], mask)
        out.peaks.append(peak)
        if peak < threshold:
            out.residual = img
            return out
        pos, _ = pg.hogbom(img, beam, mask, gain=gain, threshold=max(threshold, cycle_factor * peak),
                           max_iter=minor_iter, psf_patch=psf_patch, model=model)
        out.components += int(pos.numel())
        if pos.numel() == 0:
            break
        resid_vis.copy_(vis)
        pg.predict(plan, kernels_degrid, model, out=resid_vis, subtract=True)
    out.residual = pg.image(plan, kernels_grid, resid_vis, wsum, grid_buf=grid_buf)
    return out
