"""Grid geometry: image coordinates, uv snapping, footprints and w-planes.

The paper does not state its gridding geometry (Sec. 2.1 only says w-projection
with a configurable number of w-planes); the readings taken here are:

  * image pixel (i, j) sits at l = (j - n/2) * cell, m = (i - n/2) * cell;
  * the uv cell is 1/fov, so visibility k lands at x = u n cell + n/2;
  * positions are snapped in float64 onto the 1/os fine grid with round-half-up;
  * the footprint is the open interval |X os - fine| < S os / 2 per axis, which
    holds S points, or S-1 when the interval ends fall on grid points;
  * the plane is the nearest w-plane centre, ties going to the lower plane;
  * a visibility is dropped when its S x S box (X0 .. X0+S-1) leaves [0, n).
"""
import numpy as np


def pixel_coords(n: int, cell: float) -> np.ndarray:
    """l (or m) of every image column (row): (j - n/2) * cell."""
    return (np.arange(n) - n // 2) * cell


def n_minus_one(l, m):
    """n - 1 = sqrt(1 - l^2 - m^2) - 1, written without cancellation."""
    r2 = l * l + m * m
    return -r2 / (1.0 + np.sqrt(1.0 - r2))


def fine_position(uvw: np.ndarray, n: int, cell: float, os: int):
    """Fine-grid integer positions (round-half-up of x*os) of every visibility, float64 math."""
    x = uvw[:, 0] * (n * cell) + n / 2
    y = uvw[:, 1] * (n * cell) + n / 2
    return np.floor(x * os + 0.5).astype(np.int64), np.floor(y * os + 0.5).astype(np.int64)


def anchor_phase(fine, support, os):
    """First footprint point X0 and the table phase of one axis.

    X0 is the smallest integer with X0*os > fine - S*os/2.  Tap t of the S x S box
    sits at offset d = X0*os + t*os - fine = phase - S*os/2 + 1 + t*os, so the
    phase lies in [0, os).
    """
    fine = np.asarray(fine, dtype=np.int64)
    support = np.asarray(support, dtype=np.int64)
    half = support * os // 2
    lo = fine - half + 1
    x0 = -((-lo) // os)  # ceil(lo / os)
    phase = x0 * os - fine + half - 1
    return x0, phase


def nearest_plane(w, w_planes):
    """argmin_p |w - w_p|; numpy's argmin keeps the first (lowest) index on ties."""
    w = np.asarray(w, dtype=np.float64)
    return np.argmin(np.abs(w[:, None] - np.asarray(w_planes)[None, :]), axis=1).astype(np.int64)


def keep_mask(x0, y0, support, n):
    support = np.asarray(support)
    return (x0 >= 0) & (y0 >= 0) & (x0 + support <= n) & (y0 + support <= n)


def locate(geom, uvw):
    """Everything the gridder needs per visibility: fine positions, plane, anchors, phases, keep."""
    fx, fy = fine_position(uvw, geom.n, geom.cell, geom.os)
    plane = nearest_plane(uvw[:, 2], geom.w_planes)
    s = geom.support[plane].astype(np.int64)
    x0, px = anchor_phase(fx, s, geom.os)
    y0, py = anchor_phase(fy, s, geom.os)
    keep = keep_mask(x0, y0, s, geom.n)
    return dict(fine_x=fx, fine_y=fy, plane=plane, support=s, x0=x0, y0=y0,
                phase_x=px, phase_y=py, keep=keep)
