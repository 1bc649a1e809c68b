"""Save and restore kernel tables, kernel-surrogate networks and their training state.

Files are safetensors (tensors plus a string metadata map; nothing in them is executed on load):

  kernel set   tensor "table", the device table entry for entry as [entries][2] (re, im) float32
               (float32 storage) or float16 (float16 storage); metadata: format, geometry (n, cell,
               os, w_planes, support, tile, aa_support, mk), npol, kind, storage.  Restored with
               pg_kernels_alloc of the same spec and pg_kernels_load_table, so grids made with the
               restored set are bit-identical to grids made with the original.
  network      tensors "w.<l>", "b.<l>" per layer and, with training state, "mw.<l>", "vw.<l>",
               "mb.<l>", "vb.<l>" (Adam moments); metadata: format, shape (n_in, width, hidden,
               n_out, max_batch), the Adam step and optional caller fields (the surrogate stores
               its per-cell output scale there).  Restored through pg_mlp_set and
               pg_mlp_set_step, so training resumes where it stopped.
"""
from __future__ import annotations

import json
from dataclasses import dataclass

import numpy as np

from . import polgrid as pg

KERNELS_FORMAT = "polgrid-kernels-1"
NETWORK_FORMAT = "polgrid-mlp-1"


@dataclass
class SavedGeometry:
    """The geometry a kernel set was built for, as stored in a kernel-set file."""

    n: int
    cell: float
    os: int
    w_planes: np.ndarray
    support: np.ndarray
    tile: np.ndarray
    aa_support: int
    mk: int

    @property
    def fov(self) -> float:
        return self.n * self.cell

    @property
    def nplanes(self) -> int:
        return int(len(self.w_planes))


def _geometry_meta(g) -> str:
    return json.dumps(dict(n=int(g.n), cell=float(g.cell), os=int(g.os), w_planes=[float(v) for v in g.w_planes],
                           support=[int(v) for v in g.support], tile=[int(v) for v in g.tile],
                           aa_support=int(g.aa_support), mk=int(g.mk)))


def _geometry_from(meta: str) -> SavedGeometry:
    d = json.loads(meta)
    return SavedGeometry(int(d["n"]), float(d["cell"]), int(d["os"]), np.asarray(d["w_planes"], dtype=np.float64),
                         np.asarray(d["support"], dtype=np.int32), np.asarray(d["tile"], dtype=np.int32),
                         int(d["aa_support"]), int(d["mk"]))


def _check_format(meta: dict, want: str, path: str) -> None:
    got = (meta or {}).get("format")
    if got != want:
        raise ValueError(f"{path}: format {got!r}, expected {want!r}")


def save_kernels(k: pg.Kernels, path: str) -> None:
    """Write kernel set `k` (its geometry, spec fields and whole table) to `path`."""
    import torch
    from safetensors.torch import save_file

    table = k.table()
    if table.dtype == torch.complex64:
        table = torch.view_as_real(table)
    torch.cuda.synchronize()
    meta = dict(format=KERNELS_FORMAT, geometry=_geometry_meta(k.geom), npol=str(k.npol), kind=str(k.kind),
                storage=str(k.storage))
    save_file({"table": table.contiguous().cpu()}, path, metadata=meta)


def load_kernels(path: str, stream=None) -> pg.Kernels:
    """The kernel set saved in `path`, on the current device."""
    import torch
    from safetensors import safe_open

    with safe_open(path, framework="pt") as f:
        meta = f.metadata()
        _check_format(meta, KERNELS_FORMAT, path)
        table = f.get_tensor("table")
    geom = _geometry_from(meta["geometry"])
    k = pg.kernels_alloc(geom, int(meta["npol"]), int(meta["kind"]), int(meta["storage"]), stream=stream)
    src = table.cuda()
    if k.storage == pg.STORE_F32:
        if src.dtype != torch.float32:
            raise ValueError(f"{path}: float32 storage needs a float32 table")
        src = torch.view_as_complex(src.contiguous())
    k.load_table(src.contiguous(), stream=stream)
    torch.cuda.synchronize()
    return k


def save_network(net: pg.MLP, path: str, training_state: bool = True, extra: dict | None = None) -> None:
    """Write the weights of `net` (and, with training_state, its Adam moments and step) to `path`.
    `extra`: caller fields stored as JSON in the metadata (numpy arrays become lists)."""
    import torch
    from safetensors.torch import save_file

    tensors = {}
    layers = len(net.dims) - 1
    for layer in range(layers):
        tensors[f"w.{layer}"] = net.copy(pg.MLP_W, layer)
        tensors[f"b.{layer}"] = net.copy(pg.MLP_B, layer)
        if training_state:
            for name, what in (("mw", pg.MLP_MW), ("vw", pg.MLP_VW), ("mb", pg.MLP_MB), ("vb", pg.MLP_VB)):
                tensors[f"{name}.{layer}"] = net.copy(what, layer)
    torch.cuda.synchronize()
    tensors = {key: v.cpu() for key, v in tensors.items()}
    meta = dict(format=NETWORK_FORMAT, n_in=str(net.n_in), width=str(net.width), hidden=str(net.hidden),
                n_out=str(net.n_out), max_batch=str(net.max_batch), step=str(net.step),
                training_state=str(int(training_state)))
    if extra:
        meta["extra"] = json.dumps({key: (v.tolist() if isinstance(v, np.ndarray) else v) for key, v in extra.items()})
    save_file(tensors, path, metadata=meta)


def load_network(path: str, max_batch: int | None = None):
    """(network, extra) restored from `path`.  The network has the saved shape, weights and, when
    they were saved, Adam moments and step; max_batch defaults to the saved one."""
    import torch
    from safetensors import safe_open

    with safe_open(path, framework="pt") as f:
        meta = f.metadata()
        _check_format(meta, NETWORK_FORMAT, path)
        tensors = {key: f.get_tensor(key) for key in f.keys()}
    net = pg.MLP(int(meta["n_in"]), int(meta["width"]), int(meta["hidden"]), int(meta["n_out"]),
                 int(max_batch or meta["max_batch"]))
    layers = len(net.dims) - 1
    names = [("w", pg.MLP_W), ("b", pg.MLP_B)]
    if meta.get("training_state") == "1":
        names += [("mw", pg.MLP_MW), ("vw", pg.MLP_VW), ("mb", pg.MLP_MB), ("vb", pg.MLP_VB)]
    keep = []
    for layer in range(layers):
        for name, what in names:
            src = tensors[f"{name}.{layer}"].to(torch.float32).contiguous().cuda()
            keep.append(src)
            net.set(what, layer, src)
    net.step = int(meta["step"]) if meta.get("training_state") == "1" else 0
    torch.cuda.synchronize()
    extra = json.loads(meta["extra"]) if "extra" in meta else {}
    return net, extra
