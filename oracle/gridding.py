"""Gridding and degridding with 4x4 Mueller A x W kernels.

grid (Sec. 3.2, gridding stage; Sec. 4 lists gridding as the GPU step):
    G_q(X, Y) = sum_k sum_c T_{p_k,q,c}(X os - fine_x,k, Y os - fine_y,k) V_{k,c}
degrid (Sec. 3.2, degridding stage of Cotton-Schwab clean):
    V_{k,c} = sum_q sum_{X,Y} conj(T_{p_k,q,c}(...)) G_q(X, Y)

The pair is an exact adjoint for any table.  Visibilities are pre-weighted by
the caller (natural weighting, every weight 1).  Grids are [Q][n][n]
(row = Y = v, column = X = u); visibilities are [nvis][C].
"""
import numpy as np

from .geometry import locate


def grid(geom, tables, uvw, vis) -> np.ndarray:
    vis = np.asarray(vis).astype(np.complex128)
    loc = locate(geom, uvw)
    q = next(t for t in tables if t is not None).shape[0]
    g = np.zeros((q, geom.n, geom.n), dtype=np.complex128)
    for k in np.nonzero(loc["keep"])[0]:
        p, s = loc["plane"][k], loc["support"][k]
        y0, x0 = loc["y0"][k], loc["x0"][k]
        taps = tables[p][:, :, loc["phase_y"][k], loc["phase_x"][k]]  # [Q][C][S][S]
        g[:, y0:y0 + s, x0:x0 + s] += np.einsum("qcyx,c->qyx", taps, vis[k])
    return g


def degrid(geom, tables, uvw, g) -> np.ndarray:
    loc = locate(geom, uvw)
    c = next(t for t in tables if t is not None).shape[1]
    out = np.zeros((uvw.shape[0], c), dtype=np.complex128)
    for k in np.nonzero(loc["keep"])[0]:
        p, s = loc["plane"][k], loc["support"][k]
        y0, x0 = loc["y0"][k], loc["x0"][k]
        taps = tables[p][:, :, loc["phase_y"][k], loc["phase_x"][k]]
        out[k] = np.einsum("qcyx,qyx->c", np.conj(taps), g[:, y0:y0 + s, x0:x0 + s])
    return out
