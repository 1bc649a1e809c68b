"""ctypes binding of libpolgrid.so (the C ABI in include/polgrid.h).

Argument marshalling only: device buffers are torch tensors on the current HIP
device, streams are torch's current stream, and every step of the path runs in
the library's HIP kernels.  torch.fft (rocFFT) moves between grid and image.
There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpolgrid.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
KIND_GRID, KIND_DEGRID = 0, 1
STORE_F32, STORE_F16 = 0, 1
STOKES_IAU, STOKES_PAPER = 0, 1
ACCUMULATE, FFTSHIFT, VARIANT_ATOMIC, VARIANT_BANDED, DETERMINISTIC, VARIANT_SHARED = 1, 2, 4, 8, 16, 32
TAPER_IMAGE, TAPER_PREDICT = 0, 1


class PgGeometry(ctypes.Structure):
    _fields_ = [("n", c_int32), ("cell", c_double), ("os", c_int32), ("nplanes", c_int32),
                ("w_planes", POINTER(c_double)), ("support", POINTER(c_int32)), ("tile", POINTER(c_int32)),
                ("aa_support", c_int32), ("mk", c_int32)]


class PgKernelSpec(ctypes.Structure):
    _fields_ = [("g", PgGeometry), ("npol", c_int32), ("kind", c_int32), ("jones", POINTER(c_double)),
                ("eps_null", c_double), ("stokes_convention", c_int32), ("storage", c_int32),
                ("jones_b", POINTER(c_double))]


class PgKernelsDesc(ctypes.Structure):
    _fields_ = [("npol", c_int32), ("kind", c_int32), ("storage", c_int32), ("os", c_int32), ("n", c_int32),
                ("nplanes", c_int32), ("table", c_void_p), ("plane_offset", POINTER(c_int64)),
                ("aa_pixels", POINTER(c_double))]


class PgPlanDesc(ctypes.Structure):
    _fields_ = [("nvis", c_int64), ("n_kept", c_int64), ("n_dropped", c_int64), ("n_items", c_int64),
                ("perm", c_void_p), ("fine", c_void_p), ("items", c_void_p)]


class PgField(ctypes.Structure):
    _fields_ = [("plan", c_void_p), ("kernels", c_void_p), ("vis", c_void_p), ("grid", c_void_p)]


class PgSkyFrame(ctypes.Structure):
    _fields_ = [("n", c_int32), ("cell", c_double), ("ra", c_double), ("dec", c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p)

EXPORTS = {
    "pg_version": (c_int, []),
    "pg_last_error": (ctypes.c_char_p, []),
    "pg_set_allocator": (None, [ALLOC_FN, FREE_FN, c_void_p]),
    "pg_make_kernels": (c_int, [POINTER(PgKernelSpec), c_void_p, POINTER(c_void_p)]),
    "pg_kernels_info": (c_int, [c_void_p, POINTER(PgKernelsDesc)]),
    "pg_kernels_copy_table": (c_int, [c_void_p, c_void_p, c_void_p]),
    "pg_kernels_load_table": (c_int, [c_void_p, c_void_p, c_void_p]),
    "pg_kernels_destroy": (None, [c_void_p]),
    "pg_plan_create": (c_int, [c_void_p, c_void_p, c_int64, c_int32, c_void_p, POINTER(c_void_p), POINTER(c_int64)]),
    "pg_plan_info": (c_int, [c_void_p, POINTER(PgPlanDesc)]),
    "pg_plan_copy": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pg_plan_destroy": (None, [c_void_p]),
    "pg_plan_set_launch": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32]),
    "pg_grid": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "pg_degrid": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "pg_taper": (c_int, [c_void_p, c_void_p, c_void_p, c_int32, c_double, c_void_p]),
    "pg_batch_create": (c_int, [POINTER(PgField), c_int32, c_void_p, POINTER(c_void_p)]),
    "pg_batch_grid": (c_int, [c_void_p, c_int32, c_void_p]),
    "pg_batch_degrid": (c_int, [c_void_p, c_int32, c_void_p]),
    "pg_batch_work_items": (c_int64, [c_void_p]),
    "pg_batch_destroy": (None, [c_void_p]),
    "pg_reproject": (c_int, [c_void_p, c_void_p, POINTER(PgSkyFrame), c_void_p, c_void_p, POINTER(PgSkyFrame), c_int32,
                             c_int32, c_void_p]),
    "pg_weight_normalise": (c_int, [c_void_p, c_void_p, c_int32, c_int32, ctypes.c_float, c_void_p]),
    "pg_phase_rotate": (c_int, [c_void_p, c_void_p, c_int64, c_int32, c_double, c_double, c_double, c_double,
                                c_void_p, c_void_p, c_void_p]),
    "pg_kernels_write_cell": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "pg_kernels_alloc": (c_int, [POINTER(PgKernelSpec), c_void_p, POINTER(c_void_p)]),
    "pg_hogbom": (c_int, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, ctypes.c_float, ctypes.c_float, c_int32,
                          c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pg_hogbom_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, ctypes.c_float, ctypes.c_float,
                                  c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pg_masked_peak": (c_int, [c_void_p, c_void_p, c_int64, POINTER(ctypes.c_float), POINTER(c_int64), c_void_p]),
    "pg_normalise_at": (c_int, [c_void_p, c_int64, c_int64, c_void_p]),
    "pg_mosaic_gamma": (c_int, [c_void_p, c_int32, c_int32, c_double, c_double, c_void_p, c_void_p, c_int32,
                                c_void_p]),
    "pg_gemm_f32": (c_int, [c_int32, c_int32, c_int64, c_int64, c_int64, ctypes.c_float, c_void_p, c_int64,
                            c_void_p, c_int64, ctypes.c_float, c_void_p, c_int64, c_void_p]),
    "pg_scale_rows": (c_int, [c_void_p, c_int64, c_int64, c_void_p, c_void_p]),
    "pg_kernels_export": (c_int, [c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "pg_kernels_import": (c_int, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "pg_mlp_create": (c_int, [c_int32, c_int32, c_int32, c_int64, c_int32, ctypes.c_uint64, c_void_p,
                              POINTER(c_void_p)]),
    "pg_mlp_forward": (c_int, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "pg_mlp_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_int32, ctypes.c_float, c_int32, c_void_p,
                                  c_void_p]),
    "pg_mlp_copy": (c_int, [c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "pg_mlp_load": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "pg_mlp_set": (c_int, [c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "pg_mlp_get_step": (c_int, [c_void_p, POINTER(c_int64)]),
    "pg_mlp_set_step": (c_int, [c_void_p, c_int64]),
    "pg_mlp_destroy": (None, [c_void_p]),
}

_lib = None


class PolgridError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"polgrid error {code}: {msg}")
        self.code = code


def lib():
    """The loaded library; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_2206_15117_amd.build)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(rc: int):
    if rc != OK:
        raise PolgridError(rc, lib().pg_last_error().decode())


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _ptr(t):
    return c_void_p(0 if t is None else t.data_ptr())


# The callback pair handed to the library.  Every device buffer keeps the function pointers it was
# allocated with and frees through them, so the pair is created once and never released.
_torch_hooks = None


def use_torch_allocator(enable: bool = True):
    """Route the library's device allocations through torch's caching allocator (idempotent);
    enable=False returns new allocations to hipMalloc (buffers already made still free through torch)."""
    global _torch_hooks
    import torch

    if not enable:
        lib().pg_set_allocator(ALLOC_FN(), FREE_FN(), None)
        return
    if _torch_hooks is None:
        def _alloc(size, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(size), stream=int(stream or 0))
            except Exception:
                return None

        def _free(ptr, stream, ctx):
            torch.cuda.caching_allocator_delete(int(ptr))

        _torch_hooks = (ALLOC_FN(_alloc), FREE_FN(_free))
    lib().pg_set_allocator(_torch_hooks[0], _torch_hooks[1], None)


def _geometry_struct(geom):
    w = np.ascontiguousarray(geom.w_planes, dtype=np.float64)
    s = np.ascontiguousarray(geom.support, dtype=np.int32)
    t = np.ascontiguousarray(geom.tile, dtype=np.int32)
    g = PgGeometry(int(geom.n), float(geom.cell), int(geom.os), int(w.shape[0]),
                   w.ctypes.data_as(POINTER(c_double)), s.ctypes.data_as(POINTER(c_int32)),
                   t.ctypes.data_as(POINTER(c_int32)), int(geom.aa_support), int(geom.mk))
    return g, (w, s, t)


(MLP_W, MLP_W_BF16, MLP_B, MLP_GW, MLP_GB, MLP_ACT, MLP_PRE, MLP_GY, MLP_GY_BF16, MLP_GZ, MLP_GZ_BF16, MLP_MW,
 MLP_VW, MLP_MB, MLP_VB) = range(15)


class Kernels:
    """A kernel table set (pg_kernels)."""

    def __init__(self, handle, geom):
        self._h = handle
        self.geom = geom
        d = PgKernelsDesc()
        _check(lib().pg_kernels_info(self._h, ctypes.byref(d)))
        self.npol, self.kind, self.storage = d.npol, d.kind, d.storage
        self.os, self.n, self.nplanes = d.os, d.n, d.nplanes
        self.plane_offset = np.array([d.plane_offset[i] for i in range(d.nplanes + 1)], dtype=np.int64)
        self.aa_pixels = np.array([d.aa_pixels[i] for i in range(d.n)])

    @property
    def handle(self):
        return self._h

    def table(self):
        """Device copy of the whole table: complex64 (F32) or float16 pairs [entries, 2] (F16)."""
        import torch

        n = int(self.plane_offset[-1])
        if self.storage == STORE_F16:
            out = torch.empty((n, 2), dtype=torch.float16, device="cuda")
        else:
            out = torch.empty(n, dtype=torch.complex64, device="cuda")
        _check(lib().pg_kernels_copy_table(self._h, _ptr(out), _stream()))
        return out

    def load_table(self, src, stream=None):
        """Overwrite the whole table from a device tensor laid out as table() returns it."""
        n = int(self.plane_offset[-1])
        want = (n, 2) if self.storage == STORE_F16 else (n,)
        dt = "torch.float16" if self.storage == STORE_F16 else "torch.complex64"
        if tuple(src.shape) != want or str(src.dtype) != dt or not src.is_contiguous():
            raise ValueError(f"src must be a contiguous {dt} tensor of shape {want}")
        _check(lib().pg_kernels_load_table(self._h, _ptr(src), _stream(stream)))

    def write_cell(self, plane: int, q: int, c: int, src, stream=None):
        """Overwrite cell (q, c) of `plane` from device float [os][os][S][S][2]."""
        _check(lib().pg_kernels_write_cell(self._h, int(plane), int(q), int(c), _ptr(src), _stream(stream)))

    def export_planes(self, plane0: int, nplanes: int, out=None, stream=None):
        """Cells of planes plane0.. (one support S) as float32 [nplanes][npol][npol][os][os][S][S][2]."""
        import torch

        s = int(self.geom.support[plane0])
        shape = (nplanes, self.npol, self.npol, self.os, self.os, s, s, 2)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device="cuda")
        elif out.numel() < int(np.prod(shape)) or not out.is_contiguous() or out.dtype != torch.float32:
            raise ValueError("out must be a contiguous float32 tensor of at least the export size")
        _check(lib().pg_kernels_export(self._h, int(plane0), int(nplanes), _ptr(out), _stream(stream)))
        return out.view(-1)[:int(np.prod(shape))].view(shape)

    def import_planes(self, plane0: int, nplanes: int, src, cell_scale=None, stream=None):
        """Overwrite every cell of planes plane0.. with cell_scale[q npol + c] * src (layout of export_planes)."""
        s = int(self.geom.support[plane0])
        need = nplanes * self.npol ** 2 * self.os ** 2 * s * s * 2
        if src.numel() < need or not src.is_contiguous() or str(src.dtype) != "torch.float32":
            raise ValueError("src must be a contiguous float32 tensor of at least the import size")
        sp = None
        if cell_scale is not None:
            sc = np.ascontiguousarray(cell_scale, dtype=np.float32)
            if sc.size != self.npol ** 2:
                raise ValueError("cell_scale needs npol^2 values")
            sp = sc.ctypes.data_as(c_void_p)
        _check(lib().pg_kernels_import(self._h, int(plane0), int(nplanes), _ptr(src), sp, _stream(stream)))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pg_kernels_destroy(self._h)
            self._h = None


def make_kernels(geom, npol: int, kind: int = KIND_GRID, jones=None, eps_null: float = 0.2,
                 storage: int = STORE_F32, convention: int = STOKES_IAU, stream=None, jones_b=None) -> Kernels:
    """Kernel set (pg_make_kernels).  jones: the antennas' Jones field [2][2][mk][mk]; jones_b: the
    second antenna's of a baseline between two antenna types (Mueller J_a (x) conj(J_b))."""
    g, keep = _geometry_struct(geom)
    ptrs = []
    for j in (jones, jones_b):
        if j is None:
            ptrs.append(None)
            continue
        jarr = np.ascontiguousarray(j, dtype=np.complex128)
        if jarr.shape != (2, 2, geom.mk, geom.mk):
            raise ValueError(f"Jones fields must be complex128 [2][2][mk][mk], got {jarr.shape}")
        keep = keep + (jarr,)
        ptrs.append(jarr.ctypes.data_as(POINTER(c_double)))
    spec = PgKernelSpec(g, int(npol), int(kind), ptrs[0], float(eps_null), int(convention), int(storage), ptrs[1])
    h = c_void_p()
    _check(lib().pg_make_kernels(ctypes.byref(spec), _stream(stream), ctypes.byref(h)))
    return Kernels(h, geom)


def kernels_alloc(geom, npol: int, kind: int = KIND_GRID, storage: int = STORE_F32, stream=None) -> Kernels:
    """A kernel set of this geometry whose table is zero, to be filled with Kernels.import_planes."""
    g, keep = _geometry_struct(geom)
    spec = PgKernelSpec(g, int(npol), int(kind), None, 0.0, STOKES_IAU, int(storage), None)
    h = c_void_p()
    _check(lib().pg_kernels_alloc(ctypes.byref(spec), _stream(stream), ctypes.byref(h)))
    return Kernels(h, geom)


class Plan:
    """Binned visibilities (pg_plan)."""

    def __init__(self, handle):
        self._h = handle
        d = PgPlanDesc()
        _check(lib().pg_plan_info(self._h, ctypes.byref(d)))
        self.nvis, self.n_kept, self.n_dropped, self.n_items = d.nvis, d.n_kept, d.n_dropped, d.n_items

    @property
    def handle(self):
        return self._h

    def arrays(self):
        """(perm [nvis], fine [n_kept, 2], items [n_items, 8]) as int32 device tensors."""
        import torch

        perm = torch.empty(max(self.nvis, 1), dtype=torch.int32, device="cuda")
        fine = torch.empty((max(self.n_kept, 1), 2), dtype=torch.int32, device="cuda")
        items = torch.empty((max(self.n_items, 1), 8), dtype=torch.int32, device="cuda")
        _check(lib().pg_plan_copy(self._h, _ptr(perm), _ptr(fine), _ptr(items), _stream()))
        return perm[:self.nvis], fine[:self.n_kept], items[:self.n_items]

    def set_launch(self, grid_variant: int = 0, grid_waves: int = 16, degrid_waves: int = 16, xcd_group: int = 1,
                   grid_planes: int = 0, degrid_corrs: int = 0):
        """Launch tuning (grid variant 0 auto / 1 atomic / 2 banded / 3 shared taps, waves per workgroup, consecutive
        work items per XCD, output planes per banded-gridder workgroup: 0 = all, 1, 2 or 4, output
        correlations per degrid workgroup: 0 = all, 2 or 4)."""
        _check(lib().pg_plan_set_launch(self._h, int(grid_variant), int(grid_waves), int(degrid_waves),
                                        int(xcd_group), int(grid_planes), int(degrid_corrs)))
        return self

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pg_plan_destroy(self._h)
            self._h = None


def plan(kernels: Kernels, uvw, max_chunk: int = 1024, stream=None) -> Plan:
    import torch

    if uvw.dtype != torch.float64 or uvw.dim() != 2 or uvw.shape[1] != 3 or not uvw.is_contiguous():
        raise ValueError("uvw must be a contiguous float64 [nvis, 3] device tensor")
    h = c_void_p()
    nd = c_int64()
    _check(lib().pg_plan_create(kernels.handle, _ptr(uvw), uvw.shape[0], int(max_chunk), _stream(stream),
                                ctypes.byref(h), ctypes.byref(nd)))
    return Plan(h)


def _grid_shape(k: Kernels):
    return (k.npol, k.n, k.n)


def grid(p: Plan, k: Kernels, vis, out=None, accumulate: bool = False, fftshift: bool = False, stream=None,
         variant: int = 0, deterministic: bool = False):
    """Grid `vis` [nvis, npol] onto `out` [npol, n, n].  deterministic=True gives bit-for-bit
    reproducible grids (fixed-point accumulation; allocates npol n^2 16 bytes of scratch per call)."""
    import torch

    if vis.dtype != torch.complex64 or not vis.is_contiguous() or tuple(vis.shape) != (p.nvis, k.npol):
        raise ValueError(f"vis must be contiguous complex64 [{p.nvis}, {k.npol}]")
    if out is None:
        out = torch.empty(_grid_shape(k), dtype=torch.complex64, device=vis.device)
    elif out.dtype != torch.complex64 or tuple(out.shape) != _grid_shape(k) or not out.is_contiguous():
        raise ValueError("out must be contiguous complex64 [npol, n, n]")
    flags = (ACCUMULATE if accumulate else 0) | (FFTSHIFT if fftshift else 0) | int(variant) | \
        (DETERMINISTIC if deterministic else 0)
    _check(lib().pg_grid(p.handle, k.handle, _ptr(vis), _ptr(out), flags, _stream(stream)))
    return out


def degrid(p: Plan, k: Kernels, g, out=None, fftshift: bool = False, accumulate: bool = False, stream=None):
    import torch

    if g.dtype != torch.complex64 or tuple(g.shape) != _grid_shape(k) or not g.is_contiguous():
        raise ValueError("grid must be contiguous complex64 [npol, n, n]")
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs out")
        out = torch.empty((p.nvis, k.npol), dtype=torch.complex64, device=g.device)
    elif out.dtype != torch.complex64 or tuple(out.shape) != (p.nvis, k.npol) or not out.is_contiguous():
        raise ValueError("out must be contiguous complex64 [nvis, npol]")
    flags = (FFTSHIFT if fftshift else 0) | (ACCUMULATE if accumulate else 0)
    _check(lib().pg_degrid(p.handle, k.handle, _ptr(g), _ptr(out), flags, _stream(stream)))
    return out


def taper(k: Kernels, inp, out, direction: int, weight_sum: float = 1.0, stream=None):
    """Taper correction between grid and image (pg_taper).  TAPER_IMAGE: inp complex64 [npol, n, n]
    (the transformed grid) -> out float32 [npol, n, n]; TAPER_PREDICT: inp float32 [npol, n, n] (the
    model) -> out complex64 [npol, n, n].  Both contiguous, on one device."""
    import torch

    if direction == TAPER_IMAGE:
        want_in, want_out = torch.complex64, torch.float32
    elif direction == TAPER_PREDICT:
        want_in, want_out = torch.float32, torch.complex64
    else:
        raise ValueError("direction must be TAPER_IMAGE or TAPER_PREDICT")
    shape = _grid_shape(k)
    for t, dt, what in ((inp, want_in, "input"), (out, want_out, "output")):
        if not isinstance(t, torch.Tensor) or t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"taper {what} must be a contiguous {dt} tensor of shape {list(shape)}")
    if inp.device != out.device:
        raise ValueError("taper input and output must be on the same device")
    _check(lib().pg_taper(k.handle, _ptr(inp), _ptr(out), int(direction), float(weight_sum), _stream(stream)))
    return out


def image(p: Plan, k: Kernels, vis, weight_sum: float, grid_buf=None, out=None, deterministic: bool = False):
    """Dirty image: grid (centring folded in) -> FFT (rocFFT via torch) -> taper correction.
    deterministic: grid in the reproducible mode (the same image bits on every call)."""
    import torch

    g = grid(p, k, vis, out=grid_buf, fftshift=True, deterministic=deterministic)
    f = torch.fft.fft2(g)
    if out is None:
        out = torch.empty(_grid_shape(k), dtype=torch.float32, device=vis.device)
    return taper(k, f, out, TAPER_IMAGE, weight_sum)


def predict(p: Plan, k: Kernels, model, out=None, buf=None, subtract: bool = False):
    """Model visibilities: taper correction -> unnormalised inverse FFT -> degrid.  With subtract,
    out -= the model visibilities (dropped rows untouched)."""
    import torch

    if buf is None:
        buf = torch.empty(_grid_shape(k), dtype=torch.complex64, device=model.device)
    taper(k, model, buf, TAPER_PREDICT, -1.0 if subtract else 1.0)
    g = torch.fft.ifft2(buf, norm="forward")
    return degrid(p, k, g, out=out, fftshift=True, accumulate=subtract)


def _frame(f) -> PgSkyFrame:
    """A sky frame (n, cell, ra, dec) (tuple, namedtuple or object with those attributes)."""
    if hasattr(f, "cell"):
        return PgSkyFrame(int(f.n), float(f.cell), float(f.ra), float(f.dec))
    n, cell, ra, dec = f
    return PgSkyFrame(int(n), float(cell), float(ra), float(dec))


def _image_check(t, npol: int, n: int, what: str):
    import torch

    if t.dtype != torch.float32 or tuple(t.shape[-2:]) != (n, n) or not t.is_contiguous() or t.numel() != npol * n * n:
        raise ValueError(f"{what} must be a contiguous float32 [{npol}][{n}][{n}] device tensor")


def reproject(src, src_frame, dst, dst_frame, src_weight=None, dst_weight=None, accumulate: bool = False,
              stream=None):
    """Image-plane reprojection of src (float32 [npol][n][n], frame src_frame) onto dst (frame
    dst_frame): without accumulate dst = the bilinear samples (dst_weight = the sampled weight);
    with accumulate dst += weight x sample and dst_weight += weight."""
    sf, df = _frame(src_frame), _frame(dst_frame)
    npol = src.shape[0] if src.dim() == 3 else 1
    _image_check(src, npol, sf.n, "src")
    _image_check(dst, npol, df.n, "dst")
    if src_weight is not None:
        _image_check(src_weight, 1, sf.n, "src_weight")
    if dst_weight is not None:
        _image_check(dst_weight, 1, df.n, "dst_weight")
    _check(lib().pg_reproject(_ptr(src), _ptr(src_weight) if src_weight is not None else None, ctypes.byref(sf),
                              _ptr(dst), _ptr(dst_weight) if dst_weight is not None else None, ctypes.byref(df),
                              npol, ACCUMULATE if accumulate else 0, _stream(stream)))
    return dst


def phase_rotate(uvw, vis, centre_from, centre_to, uvw_out=None, vis_out=None, stream=None):
    """Visibilities (complex64 [nvis][npol]) and uvw (float64 [nvis][3]) about centre_from moved to
    centre_to ((ra, dec) radians).  Returns (uvw_out, vis_out); pass the inputs as outputs to
    rotate in place."""
    import torch

    if uvw.dtype != torch.float64 or uvw.dim() != 2 or uvw.shape[1] != 3 or not uvw.is_contiguous():
        raise ValueError("uvw must be a contiguous float64 [nvis, 3] device tensor")
    if vis.dtype != torch.complex64 or vis.dim() != 2 or vis.shape[0] != uvw.shape[0] or not vis.is_contiguous():
        raise ValueError("vis must be a contiguous complex64 [nvis, npol] device tensor")
    if uvw_out is None:
        uvw_out = torch.empty_like(uvw)
    if vis_out is None:
        vis_out = torch.empty_like(vis)
    _check(lib().pg_phase_rotate(_ptr(uvw), _ptr(vis), uvw.shape[0], vis.shape[1], float(centre_from[0]),
                                 float(centre_from[1]), float(centre_to[0]), float(centre_to[1]), _ptr(uvw_out),
                                 _ptr(vis_out), _stream(stream)))
    return uvw_out, vis_out


def weight_normalise(img, weight, min_weight: float, stream=None):
    """img /= weight where weight >= min_weight, else 0 (in place)."""
    n = img.shape[-1]
    npol = img.shape[0] if img.dim() == 3 else 1
    _image_check(img, npol, n, "img")
    _image_check(weight, 1, n, "weight")
    _check(lib().pg_weight_normalise(_ptr(img), _ptr(weight), n, npol, float(min_weight), _stream(stream)))
    return img


HOGBOM_STATIC_MAX_ITER = 65536


def hogbom(residual, psf, mask=None, gain: float = 0.1, threshold: float = 0.0, max_iter: int = 1000,
           psf_patch: int = 0, model=None, stream=None, noalloc: bool = False):
    """Hogbom minor cycle on the device (pg_hogbom, or pg_hogbom_noalloc with noalloc=True, whose
    scratch is the library's fixed device array): residual float32 [npol, n, n] is cleaned in
    place; returns (component pixel indices int32 [m], component values float32 [m, npol])."""
    import torch

    npol, n = residual.shape[0], residual.shape[-1]
    if residual.dtype != torch.float32 or not residual.is_contiguous() or residual.shape[1] != n:
        raise ValueError("residual must be contiguous float32 [npol, n, n]")
    if psf.dtype != torch.float32 or tuple(psf.shape) != (n, n) or not psf.is_contiguous():
        raise ValueError("psf must be contiguous float32 [n, n]")
    if mask is not None and (mask.dtype != torch.uint8 or tuple(mask.shape) != (n, n) or not mask.is_contiguous()):
        raise ValueError("mask must be contiguous uint8 [n, n]")
    if model is not None and (model.dtype != torch.float32 or tuple(model.shape) != tuple(residual.shape)
                              or not model.is_contiguous()):
        raise ValueError("model must be contiguous float32 like residual")
    pos = torch.empty(max(max_iter, 1), dtype=torch.int32, device=residual.device)
    val = torch.empty((max(max_iter, 1), npol), dtype=torch.float32, device=residual.device)
    cnt = torch.zeros(1, dtype=torch.int32, device=residual.device)
    fn = lib().pg_hogbom_noalloc if noalloc else lib().pg_hogbom
    _check(fn(_ptr(residual), _ptr(psf), _ptr(mask), int(n), int(npol), ctypes.c_float(gain),
              ctypes.c_float(threshold), int(psf_patch), int(max_iter), _ptr(pos), _ptr(val), _ptr(model), _ptr(cnt),
              _stream(stream)))
    m = int(cnt.item())
    return pos[:m], val[:m]


def masked_peak(img, mask=None, stream=None):
    """(largest |img| over the mask, its flat index) by pg_masked_peak; img float32, mask uint8 of
    the same number of elements (None: all).  (0.0, -1) when no pixel is masked in."""
    import torch

    if img.dtype != torch.float32 or not img.is_contiguous():
        raise ValueError("img must be contiguous float32")
    if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != img.numel() or not mask.is_contiguous()):
        raise ValueError("mask must be contiguous uint8 with img's number of elements")
    peak, index = ctypes.c_float(), c_int64()
    _check(lib().pg_masked_peak(_ptr(img), _ptr(mask), img.numel(), ctypes.byref(peak), ctypes.byref(index),
                                _stream(stream)))
    return float(peak.value), int(index.value)


def normalise_at(img, ref_index: int, stream=None):
    """img /= img.flatten()[ref_index] in place (pg_normalise_at); img contiguous float32."""
    import torch

    if img.dtype != torch.float32 or not img.is_contiguous():
        raise ValueError("img must be contiguous float32")
    _check(lib().pg_normalise_at(_ptr(img), img.numel(), int(ref_index), _stream(stream)))
    return img


def mosaic_gamma(beams, img, floor: float = 1e-3, scale: float = 0.5, weight_sum=None, stream=None):
    """UV-domain mosaic correction (pg_mosaic_gamma, Eq. 1): img float32 [npol, n, n] is multiplied in
    place by scale x gamma from the fields' power beams float32 [nfields, n, n]; returns S = sum B^2."""
    import torch

    if beams.dtype != torch.float32 or beams.dim() != 3 or not beams.is_contiguous() or beams.shape[1] != beams.shape[2]:
        raise ValueError("beams must be contiguous float32 [nfields, n, n]")
    n = beams.shape[-1]
    if img.dtype != torch.float32 or img.dim() != 3 or tuple(img.shape[1:]) != (n, n) or not img.is_contiguous():
        raise ValueError("img must be contiguous float32 [npol, n, n] on the beams' grid")
    if weight_sum is None:
        weight_sum = torch.empty((n, n), dtype=torch.float32, device=beams.device)
    elif weight_sum.dtype != torch.float32 or tuple(weight_sum.shape) != (n, n) or not weight_sum.is_contiguous():
        raise ValueError("weight_sum must be contiguous float32 [n, n]")
    _check(lib().pg_mosaic_gamma(_ptr(beams), int(beams.shape[0]), int(n), float(floor), float(scale),
                                 _ptr(weight_sum), _ptr(img), int(img.shape[0]), _stream(stream)))
    return weight_sum


class Batch:
    """Many fields gridded or degridded by one launch each way (pg_batch)."""

    def __init__(self, fields, stream=None):
        self._keep = list(fields)
        arr = (PgField * len(fields))()
        for i, (p, k, vis, g) in enumerate(fields):
            arr[i] = PgField(p.handle, k.handle, vis.data_ptr() if vis is not None else None, g.data_ptr())
        h = c_void_p()
        _check(lib().pg_batch_create(arr, len(fields), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.work_items = int(lib().pg_batch_work_items(self._h))

    def grid(self, fftshift: bool = False, accumulate: bool = False, stream=None):
        flags = (FFTSHIFT if fftshift else 0) | (ACCUMULATE if accumulate else 0)
        _check(lib().pg_batch_grid(self._h, flags, _stream(stream)))

    def degrid(self, fftshift: bool = False, stream=None):
        _check(lib().pg_batch_degrid(self._h, FFTSHIFT if fftshift else 0, _stream(stream)))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pg_batch_destroy(self._h)
            self._h = None


def batch(fields, stream=None) -> Batch:
    """fields: list of (Plan, Kernels, vis tensor, grid tensor) sharing npol and table storage."""
    return Batch(fields, stream)


def gemm_f32(a, b, out=None, transa: bool = False, transb: bool = False, alpha: float = 1.0, beta: float = 0.0,
             stream=None):
    """out = alpha op(a) op(b) + beta out (pg_gemm_f32) for contiguous float32 2-D device tensors,
    op(x) = x or x^T; out is allocated (and beta ignored) when None."""
    import torch

    for t, nm in ((a, "a"), (b, "b")):
        if t.dtype != torch.float32 or t.dim() != 2 or not t.is_contiguous():
            raise ValueError(f"{nm} must be a contiguous float32 matrix")
    m, k = (a.shape[1], a.shape[0]) if transa else (a.shape[0], a.shape[1])
    kb, n = (b.shape[1], b.shape[0]) if transb else (b.shape[0], b.shape[1])
    if k != kb:
        raise ValueError(f"inner dimensions differ: {k} vs {kb}")
    if out is None:
        out = torch.empty((m, n), dtype=torch.float32, device=a.device)
        beta = 0.0
    elif out.dtype != torch.float32 or tuple(out.shape) != (m, n) or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous float32 [{m}, {n}] tensor")
    _check(lib().pg_gemm_f32(int(bool(transa)), int(bool(transb)), m, n, k, ctypes.c_float(alpha), _ptr(a),
                             a.shape[1], _ptr(b), b.shape[1], ctypes.c_float(beta), _ptr(out), n, _stream(stream)))
    return out


def scale_rows(x, scale, stream=None):
    """x[r, :] *= scale[r] in place (pg_scale_rows) for contiguous float32 x [rows, cols], scale [rows]."""
    import torch

    if x.dtype != torch.float32 or x.dim() != 2 or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 matrix")
    if scale.dtype != torch.float32 or tuple(scale.shape) != (x.shape[0],) or not scale.is_contiguous():
        raise ValueError("scale must be contiguous float32 [rows]")
    _check(lib().pg_scale_rows(_ptr(x), x.shape[0], x.shape[1], _ptr(scale), _stream(stream)))
    return x


class MLP:
    """Kernel surrogate network (pg_mlp): BF16 matrix-core products, FP32 masters, Adam."""

    def __init__(self, n_in: int, width: int, hidden: int, n_out: int, max_batch: int, seed: int = 1, stream=None):
        h = c_void_p()
        _check(lib().pg_mlp_create(int(n_in), int(width), int(hidden), int(n_out), int(max_batch),
                                   ctypes.c_uint64(int(seed)), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.dims = [n_in] + [width] * hidden + [n_out]
        self.n_in, self.width, self.hidden, self.n_out = int(n_in), int(width), int(hidden), int(n_out)
        self.max_batch = max_batch

    def forward(self, x, out=None, stream=None):
        import torch

        if x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 2 or x.shape[1] != self.dims[0]:
            raise ValueError(f"x must be contiguous float32 [batch, {self.dims[0]}]")
        if out is None:
            out = torch.empty((x.shape[0], self.dims[-1]), dtype=torch.float32, device=x.device)
        elif (out.dtype != torch.float32 or not out.is_contiguous()
              or tuple(out.shape) != (x.shape[0], self.dims[-1])):
            raise ValueError(f"out must be contiguous float32 [{x.shape[0]}, {self.dims[-1]}]")
        _check(lib().pg_mlp_forward(self._h, _ptr(x), int(x.shape[0]), _ptr(out), _stream(stream)))
        return out

    def train_step(self, x, target, lr: float, update: bool = True, stream=None):
        import torch

        loss = torch.zeros(1, dtype=torch.float32, device=x.device)
        _check(lib().pg_mlp_train_step(self._h, _ptr(x), _ptr(target), int(x.shape[0]), ctypes.c_float(lr),
                                       1 if update else 0, _ptr(loss), _stream(stream)))
        return loss

    def copy(self, what: int, layer: int, batch: int = 0):
        """A parameter, gradient or activation of `layer` as a device tensor."""
        import torch

        din, dout = self.dims[layer], self.dims[layer + 1]
        shapes = {MLP_W: ((din, dout), torch.float32), MLP_W_BF16: ((din, dout), torch.bfloat16),
                  MLP_B: ((dout,), torch.float32), MLP_GW: ((din, dout), torch.float32),
                  MLP_GB: ((dout,), torch.float32), MLP_ACT: ((batch, din), torch.bfloat16),
                  MLP_PRE: ((batch, dout), torch.float32), MLP_GY: ((batch, self.dims[-1]), torch.float32),
                  MLP_GY_BF16: ((batch, self.dims[-1]), torch.bfloat16), MLP_GZ: ((batch, self.dims[1]), torch.float32),
                  MLP_GZ_BF16: ((batch, self.dims[1]), torch.bfloat16), MLP_MW: ((din, dout), torch.float32),
                  MLP_VW: ((din, dout), torch.float32), MLP_MB: ((dout,), torch.float32),
                  MLP_VB: ((dout,), torch.float32)}
        shape, dt = shapes[what]
        out = torch.empty(shape, dtype=dt, device="cuda")
        _check(lib().pg_mlp_copy(self._h, int(what), int(layer), _ptr(out), _stream()))
        return out

    def load(self, layer: int, w, b):
        _check(lib().pg_mlp_load(self._h, int(layer), _ptr(w.contiguous()), _ptr(b.contiguous()), _stream()))

    def set(self, what: int, layer: int, src):
        """Restore weights, bias or an Adam moment of `layer` (pg_mlp_set) from a float32 device tensor."""
        import torch

        din, dout = self.dims[layer], self.dims[layer + 1]
        shape = (din, dout) if what in (MLP_W, MLP_MW, MLP_VW) else (dout,)
        if tuple(src.shape) != shape or src.dtype != torch.float32 or not src.is_contiguous():
            raise ValueError(f"src must be a contiguous float32 tensor of shape {shape}")
        _check(lib().pg_mlp_set(self._h, int(what), int(layer), _ptr(src), _stream()))

    @property
    def step(self) -> int:
        """Adam updates taken so far."""
        v = c_int64()
        _check(lib().pg_mlp_get_step(self._h, ctypes.byref(v)))
        return int(v.value)

    @step.setter
    def step(self, value: int):
        _check(lib().pg_mlp_set_step(self._h, int(value)))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pg_mlp_destroy(self._h)
            self._h = None
