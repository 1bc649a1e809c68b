"""The C ABI: the library loads, exports every declared symbol, and validates arguments on the
host before anything reaches the GPU (these calls never touch HIP, so they run without one)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2206_15117_amd import polgrid as pg

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "polgrid.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = pg.lib()
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(pg.EXPORTS) == names


def test_version():
    v = pg.lib().pg_version()
    assert v >> 16 == 1


def _geom(n=64, os_=4, support=(7,), tile=(16,), planes=(0.0,), mk=64, cell=None):
    class G:
        pass

    g = G()
    g.n, g.os, g.mk, g.aa_support = n, os_, mk, 7
    g.cell = cell if cell is not None else 0.1 / n
    g.w_planes = np.asarray(planes, np.float64)
    g.support = np.asarray(support, np.int32)
    g.tile = np.asarray(tile, np.int32)
    return g


def _spec(g, npol=1, kind=0, storage=0, conv=0, eps=0.2):
    gs, keep = pg._geometry_struct(g)
    return pg.PgKernelSpec(gs, npol, kind, None, eps, conv, storage), keep


@pytest.mark.parametrize("mutate,code,needle", [
    (dict(n=63), pg.EINVAL, "n must be even"),
    (dict(os_=3), pg.EINVAL, "os must be even"),
    (dict(cell=-1.0), pg.EINVAL, "cell"),
    (dict(cell=1.0), pg.EINVAL, "field of view"),
    (dict(planes=(1.0, 0.0), support=(7, 7), tile=(16, 16)), pg.EINVAL, "ascending"),
    (dict(support=(65,)), pg.EINVAL, "support"),
    (dict(tile=(0,)), pg.EINVAL, "tile"),
    (dict(mk=7), pg.EINVAL, "mk"),
    (dict(support=(48,), tile=(64,)), pg.EUNSUPPORTED, "LDS"),
])
def test_make_kernels_rejects_bad_geometry(mutate, code, needle):
    g = _geom(**mutate)
    npol = 4 if code == pg.EUNSUPPORTED else 1
    spec, keep = _spec(g, npol=npol)
    h = ctypes.c_void_p()
    rc = pg.lib().pg_make_kernels(ctypes.byref(spec), None, ctypes.byref(h))
    assert rc == code
    assert needle in pg.lib().pg_last_error().decode()
    assert not h.value


@pytest.mark.parametrize("field,value,needle", [
    ("npol", 2, "npol"), ("kind", 5, "kind"), ("storage", 3, "storage"),
    ("stokes_convention", 9, "stokes_convention"), ("eps_null", -1.0, "eps_null"),
])
def test_make_kernels_rejects_bad_spec(field, value, needle):
    spec, keep = _spec(_geom())
    setattr(spec, field, value)
    h = ctypes.c_void_p()
    assert pg.lib().pg_make_kernels(ctypes.byref(spec), None, ctypes.byref(h)) == pg.EINVAL
    assert needle in pg.lib().pg_last_error().decode()


def test_stokes_i_with_jones_is_unsupported():
    spec, keep = _spec(_geom())
    j = np.zeros(2 * 2 * 64 * 64 * 2)
    spec.jones = j.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    assert pg.lib().pg_make_kernels(ctypes.byref(spec), None, ctypes.byref(h)) == pg.EUNSUPPORTED


def test_null_handles_are_rejected():
    lib = pg.lib()
    h = ctypes.c_void_p()
    nd = ctypes.c_int64()
    assert lib.pg_make_kernels(None, None, ctypes.byref(h)) == pg.EINVAL
    assert lib.pg_plan_create(None, None, 0, 16, None, ctypes.byref(h), ctypes.byref(nd)) == pg.EINVAL
    assert lib.pg_grid(None, None, None, None, 0, None) == pg.EINVAL
    assert lib.pg_degrid(None, None, None, None, 0, None) == pg.EINVAL
    assert lib.pg_taper(None, None, None, 0, 1.0, None) == pg.EINVAL
    assert lib.pg_kernels_info(None, None) == pg.EINVAL
    assert lib.pg_plan_info(None, None) == pg.EINVAL
    assert lib.pg_plan_copy(None, None, None, None, None) == pg.EINVAL
    assert lib.pg_kernels_copy_table(None, None, None) == pg.EINVAL
    assert lib.pg_plan_set_launch(None, 0, 16, 16, 1, 0, 0) == pg.EINVAL
    assert lib.pg_kernels_alloc(None, None, ctypes.byref(h)) == pg.EINVAL
    assert lib.pg_kernels_export(None, 0, 1, None, None) == pg.EINVAL
    f = pg.PgSkyFrame(64, 1e-4, 0.0, 0.0)
    assert lib.pg_reproject(None, None, f, None, None, f, 4, 0, None) == pg.EINVAL
    assert lib.pg_reproject(1024, None, None, 2048, None, f, 4, 0, None) == pg.EINVAL
    assert lib.pg_weight_normalise(None, None, 64, 4, 1.0, None) == pg.EINVAL
    assert lib.pg_phase_rotate(None, None, 10, 4, 0.0, 0.0, 0.1, 0.1, None, None, None) == pg.EINVAL
    assert lib.pg_phase_rotate(None, None, 0, 4, 0.0, 0.0, 0.1, 2.0, None, None, None) == pg.EINVAL
    assert lib.pg_kernels_import(None, 0, 1, None, None, None) == pg.EINVAL
    lib.pg_kernels_destroy(None)
    lib.pg_plan_destroy(None)
    assert "non-NULL" in lib.pg_last_error().decode()


def test_last_error_is_cleared_by_a_successful_call():
    lib = pg.lib()
    assert lib.pg_grid(None, None, None, None, 0, None) == pg.EINVAL
    assert lib.pg_last_error().decode()
    # an empty phase rotation validates its arguments and succeeds without touching a device
    rc = lib.pg_phase_rotate(None, None, 0, 4, 0.0, 0.0, 0.1, 0.1, None, None, None)
    assert rc == pg.OK
    assert lib.pg_last_error().decode() == ""
    # and the next failure sets a fresh message
    d = pg.PgPlanDesc()
    assert lib.pg_plan_info(None, ctypes.byref(d)) == pg.EINVAL
    assert "non-NULL" in lib.pg_last_error().decode()


def test_binding_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(pg, "_lib", None)
    monkeypatch.setattr(pg, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        pg.lib()


def test_torch_allocator_hooks_are_created_once():
    """Objects free through the hooks they were allocated with, so re-enabling the torch allocator
    must hand the library the same callback objects (a fresh pair would free the old ones)."""
    pytest.importorskip("torch")
    pg.use_torch_allocator(True)
    first = pg._torch_hooks
    pg.use_torch_allocator(False)
    pg.use_torch_allocator(True)
    assert pg._torch_hooks is first and first is not None
    pg.use_torch_allocator(False)


def test_header_is_plain_c_and_links(tmp_path):
    """include/polgrid.h compiles as C99, and a C program links against the library and gets
    argument errors back through the ABI without touching a GPU."""
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    inc = os.path.join(root, "include")
    libdir = os.path.join(root, "paper_2206_15117_amd")
    src = tmp_path / "abi.c"
    src.write_text(
        "#include <stdio.h>\n#include \"polgrid.h\"\n"
        "int main(void) {\n"
        "  pg_sky_frame f = {64, 1e-4, 0.0, 0.0};\n"
        "  if (pg_reproject(NULL, NULL, &f, NULL, NULL, &f, 4, 0, NULL) != PG_EINVAL) return 1;\n"
        "  if (pg_weight_normalise(NULL, NULL, 64, 4, 1.0f, NULL) != PG_EINVAL) return 2;\n"
        "  if (pg_grid(NULL, NULL, NULL, NULL, 0, NULL) != PG_EINVAL) return 3;\n"
        "  printf(\"%s\\n\", pg_last_error());\n"
        "  return 0;\n}\n")
    exe = tmp_path / "abi"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", inc, str(src), "-o", str(exe), "-L", libdir,
                    "-lpolgrid", "-Wl,-rpath," + libdir], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "non-NULL" in r.stdout
