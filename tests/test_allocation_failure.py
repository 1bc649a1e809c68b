"""Allocation-failure handling through the C ABI, on the host: with an allocator hook that returns
NULL, every entry point that allocates reports PG_ENOMEM with a message, creates no object, and the
library works again once the default allocator is back.  (Each call below fails at its first device
allocation, before any launch, so no GPU is needed; tests/test_gpu_parity.py covers failures after
some allocations have succeeded.)"""
import ctypes

import numpy as np
import pytest

import synth
from paper_2206_15117_amd import polgrid as pg


@pytest.fixture
def failing_allocator():
    calls = {"alloc": 0}

    def _alloc(size, stream, ctx):
        calls["alloc"] += 1
        return None

    def _free(ptr, stream, ctx):
        raise AssertionError("nothing was allocated, so nothing may be freed")

    hooks = (pg.ALLOC_FN(_alloc), pg.FREE_FN(_free))
    pg._keep_forever = getattr(pg, "_keep_forever", []) + [hooks]
    pg.lib().pg_set_allocator(hooks[0], hooks[1], None)
    yield calls
    pg.lib().pg_set_allocator(pg.ALLOC_FN(), pg.FREE_FN(), None)


def _last_error():
    return pg.lib().pg_last_error().decode()


def test_make_kernels_reports_enomem(failing_allocator):
    w = synth.config1(nvis=10)
    g, keep = pg._geometry_struct(w.geom)
    spec = pg.PgKernelSpec(g, 1, pg.KIND_GRID, None, 0.2, pg.STOKES_IAU, pg.STORE_F32, None)
    h = ctypes.c_void_p()
    assert pg.lib().pg_make_kernels(ctypes.byref(spec), None, ctypes.byref(h)) == pg.ENOMEM
    assert not h.value and "allocation" in _last_error()
    assert failing_allocator["alloc"] >= 1


def test_network_create_reports_enomem(failing_allocator):
    h = ctypes.c_void_p()
    rc = pg.lib().pg_mlp_create(8, 16, 2, 32, 4, ctypes.c_uint64(1), None, ctypes.byref(h))
    assert rc == pg.ENOMEM and not h.value and "allocation" in _last_error()


def test_hogbom_and_mosaic_gamma_report_enomem(failing_allocator):
    fake = ctypes.c_void_p(256)  # never dereferenced: the scratch allocation fails first
    rc = pg.lib().pg_hogbom(fake, fake, None, 64, 1, ctypes.c_float(0.1), ctypes.c_float(0.0), 0, 10, fake, fake,
                            None, fake, None)
    assert rc == pg.ENOMEM and "allocation" in _last_error()
    rc = pg.lib().pg_mosaic_gamma(fake, 2, 64, 1e-3, 0.5, fake, fake, 1, None)
    assert rc == pg.ENOMEM and "allocation" in _last_error()


def test_library_recovers_after_the_failure():
    """With the default hooks back, a validation error is again EINVAL (not a stale ENOMEM)."""
    assert pg.lib().pg_grid(None, None, None, None, 0, None) == pg.EINVAL
    assert "non-NULL" in _last_error()
