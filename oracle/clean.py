"""Hogbom minor cycle of Cotton-Schwab clean (test infrastructure only).

The imager cleans with the Cotton-Schwab algorithm (Sec. 2.1): major cycles image the residual
visibilities; minor cycles (Hogbom) find and subtract point components in the image with the
point-spread function; the model is then predicted back and subtracted from the visibilities.
The image is masked where the beam is weak (Sec. 3.3: below a fraction eps of its peak).

The minor cycle decides integers (which pixel is the peak, when to stop) from floating point, so
this reference takes those decisions in the same precision as the device, float32, with every
product and difference rounded on its own: it is the algorithm written out, one component at a
time, in float32.
"""
import numpy as np


def hogbom(residual, psf, mask=None, gain=0.1, threshold=0.0, max_iter=1000, psf_patch=0):
    """Returns (cleaned residual float32 [npol][n][n], [(flat pixel index, float32 values [npol])]).

    Each iteration: the peak is the masked pixel of largest |I| (plane 0), the first one in
    row-major order on ties; stop if it is below threshold; the component is gain x residual at
    the peak in every plane; subtract component x psf shifted so its centre (n/2, n/2) lands on
    the peak, where it overlaps the image and lies within psf_patch pixels of the peak
    (psf_patch <= 0: no limit)."""
    r = np.array(residual, dtype=np.float32, copy=True)
    psf = np.asarray(psf, dtype=np.float32)
    n = r.shape[-1]
    patch = n if (psf_patch <= 0 or psf_patch > n) else psf_patch
    keep = None if mask is None else (np.asarray(mask).ravel() != 0)
    g = np.float32(gain)
    comps = []
    for _ in range(max_iter):
        a = np.abs(r[0]).ravel()
        if keep is not None:
            if not keep.any():
                break
            a = np.where(keep, a, np.float32(-1.0))
        idx = int(np.argmax(a))
        if not (a[idx] >= np.float32(threshold)):
            break
        py, px = divmod(idx, n)
        v = (g * r[:, py, px]).astype(np.float32)
        comps.append((idx, v.copy()))
        y0, y1 = max(0, py - n // 2, py - patch), min(n, py + n // 2, py + patch + 1)
        x0, x1 = max(0, px - n // 2, px - patch), min(n, px + n // 2, px + patch + 1)
        if y1 <= y0 or x1 <= x0:
            continue
        shifted = psf[y0 - py + n // 2:y1 - py + n // 2, x0 - px + n // 2:x1 - px + n // 2]
        prod = (v[:, None, None] * shifted[None]).astype(np.float32)
        r[:, y0:y1, x0:x1] = (r[:, y0:y1, x0:x1] - prod).astype(np.float32)
    return r, comps


def beam_mask(power, eps):
    """uint8 mask: 1 where the power beam is at least eps times its peak (Sec. 3.3)."""
    power = np.asarray(power, dtype=np.float64)
    return (power >= eps * power.max()).astype(np.uint8)
