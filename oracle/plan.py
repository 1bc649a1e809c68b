"""Visibility binning for the gridder (the paper says nothing about ordering).

Each kept visibility gets the key
    ((plane * NT + tile_y) * NT + tile_x) * os^2 + phase_y * os + phase_x
with tile = anchor // T_p (per-plane tile side) and NT = ceil(n / min_p T_p);
dropped visibilities sort last.  The permutation is the stable argsort of the
key, and work items are the runs of equal (plane, tile_y, tile_x) cut into
chunks of at most `max_chunk` visibilities.
"""
import numpy as np

from .geometry import locate


def plan(geom, uvw, max_chunk: int):
    loc = locate(geom, uvw)
    os = geom.os
    tile = geom.tile.astype(np.int64)
    nt = -(-geom.n // int(tile.min()))
    p = loc["plane"]
    t = tile[p]
    ty, tx = loc["y0"] // t, loc["x0"] // t
    key = (((p * nt + ty) * nt + tx) * os + loc["phase_y"]) * os + loc["phase_x"]
    big = np.int64(np.iinfo(np.int64).max)
    key = np.where(loc["keep"], key, big)
    perm = np.argsort(key, kind="stable")
    nkeep = int(loc["keep"].sum())
    bins = key[perm[:nkeep]] // (os * os)
    items = []
    starts = np.concatenate([[0], np.flatnonzero(np.diff(bins)) + 1]) if nkeep else np.zeros(0, np.int64)
    ends = np.concatenate([starts[1:], [nkeep]]) if nkeep else np.zeros(0, np.int64)
    for start, end in zip(starts, ends):
        pl, rest = divmod(int(bins[start]), nt * nt)
        iy, ix = divmod(rest, nt)
        for s0 in range(int(start), int(end), max_chunk):
            items.append((pl, iy, ix, s0, min(int(end), s0 + max_chunk)))
    return dict(loc=loc, key=key, perm=perm, n_kept=nkeep, n_dropped=uvw.shape[0] - nkeep,
                items=np.asarray(items, dtype=np.int64).reshape(-1, 5), nt=nt)
