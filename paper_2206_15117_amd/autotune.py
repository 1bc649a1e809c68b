"""Autotuner for the gridder's launch shape.

Searches, per geometry class (npol, storage, os, per-plane supports):
  * workgroups per CU (1-4): sets each plane's tile T to the largest sub-grid that fits
    1/k of the LDS, so every item of a launch has the same LDS footprint;
  * waves per workgroup for grid and degrid (4, 6, 8, 16);
  * output planes per gridder workgroup (all, 2 or 1 of the four correlations), and output
    correlations per degridder workgroup (all or 2, float32 tables);
  * the grid variant (row bands, shared taps with fixed-point LDS accumulation, or LDS float
    atomics) and the chunk length of work items;
  * how many consecutive work items share one XCD (and its L2), for the best shape found.
Each candidate is timed with HIP events on a representative workload; the best choice is
cached in tuning.json beside this file and read back by `tuned_config`.
"""
from __future__ import annotations

import json
import os
import time
from collections import namedtuple

import numpy as np

Launch = namedtuple("Launch", "geom max_chunk variant grid_waves degrid_waves xcd_group batch_grid_waves "
                               "batch_degrid_waves grid_planes degrid_corrs batch_grid")
# the batched gridder's own shape where it differs from the single-plan one: geometry (tiles),
# chunk length, variant and output planes per workgroup; the batched degrid keeps the entry's
BatchGrid = namedtuple("BatchGrid", "geom max_chunk variant planes")

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")
LDS_CU = 163840            # LDS per CU
LDS_SCRATCH = 1280         # per-workgroup gridder scratch (row loads and band bounds), rounded up


def lds_pitch(width: int, support: int) -> int:
    return width + (support - width) % 32


def tiles_for(support, npol: int, wgs_per_cu: int, min_tile: int = 1):
    """Largest tile per plane whose (T+S-1) x pitch x npol x 8 B sub-grid, plus the gridder
    scratch, lets wgs_per_cu workgroups share one CU's LDS.  All npol planes count: the degridder
    holds every plane, and grid and degrid share one plan (a gridder with fewer output planes per
    workgroup then fits more workgroups per CU)."""
    budget = LDS_CU // wgs_per_cu - LDS_SCRATCH
    out = []
    for s in np.asarray(support):
        s = int(s)
        t = min_tile
        while t < 512:
            w = t + 1 + s - 1
            if w * lds_pitch(w, s) * npol * 8 > budget:
                break
            t += 1
        w = t + s - 1
        if w * lds_pitch(w, s) * npol * 8 > budget:
            return None
        out.append(t)
    return np.asarray(out, dtype=np.int32)


def key_of(npol, storage, os_, support) -> str:
    return f"np{npol}-st{storage}-os{os_}-S" + ",".join(str(int(s)) for s in support)


def tuned_config(npol, storage, os_, support):
    """Cached best launch shape for this geometry class; else the entry of the same npol and storage
    (its launch shape, with tiles recomputed for these supports); else None."""
    if not os.path.exists(CACHE):
        return None
    with open(CACHE) as fh:
        data = json.load(fh)
    hit = data.get(key_of(npol, storage, os_, support))
    if hit is not None:
        return hit
    prefix = f"np{npol}-st{storage}-"
    for k, v in sorted(data.items()):
        if k.startswith(prefix):
            out = json.loads(json.dumps(v))
            for d in ("grid", "degrid"):
                t = tiles_for(support, npol, out[d]["wgs_per_cu"])
                if t is None:
                    return None
                out[d]["tiles"] = t.tolist()
            return out
    return None


def apply(geom, npol, storage) -> Launch:
    """Launch(geometry with tuned tiles, max_chunk, grid variant, grid waves, degrid waves, XCD group)
    for this geometry, using the grid direction's tiles for both directions when they differ."""
    import copy

    cfg = tuned_config(npol, storage, geom.os, geom.support)
    g = copy.copy(geom)
    if cfg is None:
        return Launch(g, 1024, 0, 16, 16, 1, 16, 16, 0, 0, None)
    g.tile = np.asarray(cfg["grid"]["tiles"], dtype=np.int32)
    same = cfg["grid"]["wgs_per_cu"] == cfg["degrid"]["wgs_per_cu"]
    gw, dw = int(cfg["grid"]["waves"]), int(cfg["degrid"]["waves"]) if same else 16
    batch = cfg.get("batch", {})
    bgrid = None
    if "grid_wgs_per_cu" in batch:
        tiles = tiles_for(geom.support, npol, int(batch["grid_wgs_per_cu"]))
        if tiles is not None:
            gb = copy.copy(geom)
            gb.tile = tiles
            bgrid = BatchGrid(gb, int(batch["grid_max_chunk"]), int(batch["grid_variant"]), int(batch["grid_planes"]))
    return Launch(g, int(cfg["grid"]["max_chunk"]), int(cfg["grid"].get("variant", 2)), gw, dw,
                  int(cfg.get("xcd_group", 1)), int(batch.get("grid_waves", gw)), int(batch.get("degrid_waves", dw)),
                  int(cfg["grid"].get("planes", 0)), int(cfg["degrid"].get("corrs", 0)), bgrid)


def batch_grid_geom(launch: Launch):
    """Geometry (tiles) for the gridding kernels of a batched launch."""
    return launch.batch_grid.geom if launch.batch_grid is not None else launch.geom


def batch_plans(kernels_grid, kernels_degrid, uvw, launch: Launch):
    """(grid plan, degrid plan) for one field of a batched launch, with the batched kernels'
    waves per workgroup and, where the tuned entry gives one, the batched gridder's own chunk
    length, variant and output planes (kernels_grid built on `batch_grid_geom(launch)`); a batch
    takes its launch shape from its first field's plan."""
    from . import polgrid as pg

    bgr = launch.batch_grid
    pg_ = pg.plan(kernels_grid, uvw, max_chunk=bgr.max_chunk if bgr is not None else launch.max_chunk)
    pd_ = pg.plan(kernels_degrid, uvw, max_chunk=launch.max_chunk)
    pg_.set_launch(bgr.variant if bgr is not None else launch.variant, launch.batch_grid_waves, launch.degrid_waves,
                   launch.xcd_group, bgr.planes if bgr is not None else launch.grid_planes, launch.degrid_corrs)
    pd_.set_launch(0, launch.grid_waves, launch.batch_degrid_waves, launch.xcd_group, launch.grid_planes,
                   launch.degrid_corrs)
    return pg_, pd_


def plan(kernels, uvw, launch: Launch):
    """A plan binned for `kernels` with the tuned chunk length and launch shape."""
    from . import polgrid as pg

    return pg.plan(kernels, uvw, max_chunk=launch.max_chunk).set_launch(launch.variant, launch.grid_waves,
                                                                        launch.degrid_waves, launch.xcd_group,
                                                                        launch.grid_planes, launch.degrid_corrs)


def _time(fn, reps):
    import torch

    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(geom, npol, jones, uvw, vis, eps_null=0.2, storage=0, reps=3, wgs=(1, 2, 3, 4),
         waves=(4, 6, 8, 16), chunks=(256, 1024), planes=(0, 2, 1), verbose=True):
    """Time every candidate; returns (best dict, list of all results)."""
    import copy

    import torch

    from . import polgrid as pg

    grid = torch.empty((npol, geom.n, geom.n), dtype=torch.complex64, device="cuda")
    out = torch.empty_like(vis)
    results = []
    for k in wgs:
        tiles = tiles_for(geom.support, npol, k)
        if tiles is None:
            continue
        g = copy.copy(geom)
        g.tile = tiles
        kg = pg.make_kernels(g, npol, pg.KIND_GRID, jones=jones, eps_null=eps_null, storage=storage)
        kd = pg.make_kernels(g, npol, pg.KIND_DEGRID, jones=jones, storage=storage)
        for chunk in chunks:
            p = pg.plan(kg, uvw, max_chunk=chunk)
            for nw in waves:
                cands = [(v, q) for v in (2, 3) for q in planes if q == 0 or npol % q == 0] + [(1, 0)]
                for variant, gp in cands:
                    if variant == 1 and nw != 16:
                        continue
                    p.set_launch(variant, nw, nw, 1, gp)
                    tg = _time(lambda: pg.grid(p, kg, vis, out=grid, fftshift=True), reps)
                    td = _time(lambda: pg.degrid(p, kd, grid, out=out, fftshift=True), reps)
                    corrs = 0
                    if storage == 0 and npol == 4 and gp == planes[0]:
                        p.set_launch(variant, nw, nw, 1, gp, 2)
                        td2 = _time(lambda: pg.degrid(p, kd, grid, out=out, fftshift=True), reps)
                        if td2 < td:
                            td, corrs = td2, 2
                    r = dict(wgs_per_cu=k, max_chunk=chunk, waves=nw, variant=variant, planes=gp, corrs=corrs,
                             grid_ms=tg, degrid_ms=td, tiles=tiles.tolist())
                    results.append(r)
                    if verbose:
                        print(json.dumps(r), flush=True)
    bg = min(results, key=lambda r: r["grid_ms"])
    bd = min(results, key=lambda r: r["degrid_ms"])
    best = dict(grid=dict(wgs_per_cu=bg["wgs_per_cu"], max_chunk=bg["max_chunk"], waves=bg["waves"],
                          variant=bg["variant"], planes=bg["planes"], ms=bg["grid_ms"], tiles=bg["tiles"]),
                degrid=dict(wgs_per_cu=bd["wgs_per_cu"], max_chunk=bd["max_chunk"], waves=bd["waves"],
                            corrs=bd["corrs"], ms=bd["degrid_ms"], tiles=bd["tiles"]))
    # XCD grouping for the best grid shape: sum of grid and degrid time
    g = copy.copy(geom)
    g.tile = np.asarray(bg["tiles"], dtype=np.int32)
    kg = pg.make_kernels(g, npol, pg.KIND_GRID, jones=jones, eps_null=eps_null, storage=storage)
    kd = pg.make_kernels(g, npol, pg.KIND_DEGRID, jones=jones, storage=storage)
    p = pg.plan(kg, uvw, max_chunk=bg["max_chunk"])
    best_x = (float("inf"), 1)
    for xg in (1, 2, 4, 8, 16, 32):
        p.set_launch(bg["variant"], bg["waves"], bd["waves"], xg, bg["planes"], bd["corrs"])
        t = (_time(lambda: pg.grid(p, kg, vis, out=grid, fftshift=True), reps)
             + _time(lambda: pg.degrid(p, kd, grid, out=out, fftshift=True), reps))
        results.append(dict(xcd_group=xg, grid_plus_degrid_ms=t))
        if verbose:
            print(json.dumps(results[-1]), flush=True)
        best_x = min(best_x, (t, xg))
    best["xcd_group"] = best_x[1]
    return best, results


def save(npol, storage, os_, support, best, results=None, note=""):
    data = {}
    if os.path.exists(CACHE):
        with open(CACHE) as fh:
            data = json.load(fh)
    entry = dict(best)
    entry["note"] = note
    entry["when"] = time.strftime("%Y-%m-%d")
    data[key_of(npol, storage, os_, support)] = entry
    with open(CACHE, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


def main():
    import argparse
    import sys

    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c2", choices=["c2"])
    ap.add_argument("--storage", type=int, default=0)
    ap.add_argument("--quick", action="store_true", help="fewer candidates")
    ap.add_argument("--wgs", default="1,2,3,4", help="workgroups per CU to try")
    ap.add_argument("--waves", default="4,6,8,16", help="waves per workgroup to try")
    ap.add_argument("--chunks", default="256,1024", help="work item lengths to try")
    ap.add_argument("--planes", default="0,2,1", help="output planes per gridder workgroup to try (0 = all)")
    ap.add_argument("--save", action="store_true")
    args = ap.parse_args()
    from . import polgrid as pg

    torch.cuda.set_device(0)
    pg.use_torch_allocator(True)
    w = synth.config2()
    g = w.geom
    jones = synth.jones_on_lattice(w.beam, g.mk, g.fov)
    uvw = torch.from_numpy(w.uvw).cuda()
    vis = torch.from_numpy(synth.random_vis(w.nvis, 4, np.random.default_rng(3))).cuda()
    ints = lambda t: tuple(int(v) for v in t.split(","))
    kw = dict(wgs=(1, 2, 4), waves=(4, 16), chunks=(256,)) if args.quick else dict(
        wgs=ints(args.wgs), waves=ints(args.waves), chunks=ints(args.chunks), planes=ints(args.planes))
    best, results = tune(g, 4, jones, uvw, vis, w.eps_null, storage=args.storage, **kw)
    print("BEST", json.dumps(best), flush=True)
    if args.save:
        save(4, args.storage, g.os, g.support, best, results, note=f"{w.name}, {w.nvis} rows")
        print("CACHE", json.dumps({key_of(4, args.storage, g.os, g.support): best}), flush=True)


if __name__ == "__main__":
    main()
