"""Host-side logic without a GPU: launch-shape cache, tile sizing, workload generators, network
features, the XCD work-item map and the benchmark's refusal of several GPUs."""
import json
import math
import subprocess
import sys

import numpy as np
import pytest

import synth
from paper_2206_15117_amd import autotune, surrogate


def test_tiles_fill_the_lds_budget_exactly():
    """The tile is the largest T whose (T + S - 1) x pitch x npol x 8 B sub-grid fits 1/k of the
    LDS less the gridder scratch; one more row would not fit."""
    for k in (1, 2, 3):
        budget = autotune.LDS_CU // k - autotune.LDS_SCRATCH
        for s in (7, 16, 24, 33, 48):
            t = autotune.tiles_for([s], 4, k)
            if t is None:
                w = s
                assert w * autotune.lds_pitch(w, s) * 32 > budget
                continue
            w = int(t[0]) + s - 1
            assert w * autotune.lds_pitch(w, s) * 32 <= budget
            assert (w + 1) * autotune.lds_pitch(w + 1, s) * 32 > budget


def test_lds_pitch_is_congruent_to_support():
    for s in range(1, 65):
        for w in range(s, 200):
            p = autotune.lds_pitch(w, s)
            assert p >= w and (p - s) % 32 == 0 and p - w < 32


def test_tuned_config_exact_and_prefix_fallback():
    w = synth.config2(nvis=1000)
    exact = autotune.tuned_config(4, 0, 8, w.geom.support)
    assert exact is not None and exact["grid"]["waves"] in (4, 6, 8, 16)
    other = np.array([16, 20, 24, 48], dtype=np.int32)
    fb = autotune.tuned_config(4, 0, 8, other)
    assert fb is not None
    want = autotune.tiles_for(other, 4, fb["grid"]["wgs_per_cu"])
    assert fb["grid"]["tiles"] == want.tolist()
    assert autotune.tuned_config(2, 0, 8, other) is None


def test_apply_without_cache_entry_gives_defaults():
    g = synth.config1().geom
    launch = autotune.apply(g, 1, 0)
    assert launch.max_chunk == 1024 and launch.grid_waves == 16 and launch.xcd_group == 1
    assert np.array_equal(launch.geom.tile, g.tile)


def test_batched_gridder_shape_only_where_the_entry_names_one():
    """The float16 entry gives the batched gridder its own tiles and shape (one-workgroup-per-CU
    tiles, shared taps, one plane, 1024-row items) while its degrid keeps the entry's tiles; the
    float32 entry names none, so its batches use the single-plan shape."""
    w = synth.config3()[0]
    l16 = autotune.apply(w.geom, 4, 1)
    bg = l16.batch_grid
    assert bg is not None and (bg.variant, bg.planes, bg.max_chunk) == (3, 1, 1024)
    assert np.array_equal(bg.geom.tile, autotune.tiles_for(w.geom.support, 4, 1))
    assert autotune.batch_grid_geom(l16) is bg.geom
    assert not np.array_equal(bg.geom.tile, l16.geom.tile)  # the degrid's tiles differ
    l32 = autotune.apply(synth.config2().geom, 4, 0)
    assert l32.batch_grid is None and autotune.batch_grid_geom(l32) is l32.geom


def test_tuning_cache_is_well_formed():
    data = json.load(open(autotune.CACHE))
    for key, v in data.items():
        assert key.startswith("np")
        for d in ("grid", "degrid"):
            assert v[d]["waves"] in (4, 6, 8, 16) and v[d]["max_chunk"] >= 1
            assert len(v[d]["tiles"]) == len(key.split("-S")[1].split(","))
        assert 1 <= v.get("xcd_group", 1) <= 4096


def _xcd_item(b, group):
    x, j = b & 7, b >> 3
    return ((j // group) * 8 + x) * group + (j % group)


@pytest.mark.parametrize("group", [1, 2, 3, 4, 64])
def test_xcd_item_map_is_a_bijection_keeping_groups_on_one_xcd(group):
    """The launch pads to 8 x group blocks; block b runs on XCD b mod 8 and takes one item, every
    item of [0, padded) exactly once, `group` consecutive items per XCD."""
    n_items = 1000
    span = 8 * group
    padded = n_items if group == 1 else -(-n_items // span) * span
    items = [_xcd_item(b, group) for b in range(padded)]
    assert sorted(items) == list(range(padded))
    for b in range(padded):
        assert (items[b] // group) % 8 == b % 8


def test_config5_shape_and_geometry():
    w = synth.config5(nvis=200_000, nchan=4, ndump=10, nsrc=10)
    assert w.uvw.shape == (200_000, 3) and w.geom.n == 8192 and w.geom.nplanes == 128
    assert abs(w.geom.fov - 8192 * 1.76 / 3600 * math.pi / 180) < 1e-12
    assert w.geom.support.min() >= 16 and w.geom.support.max() <= 48
    assert np.all(np.abs(w.uvw[:, 2]) <= w.geom.w_planes[-1])


def test_config4_rotated_beam():
    """At pa = 0 the rotated beam is the base beam; the feed rotation is orthogonal, so the
    beam power |J|_F^2 is unchanged by pa at a rotated sky position."""
    s = synth.config4()
    l, m = np.array([0.01, -0.02]), np.array([0.005, 0.0])
    b0 = s.beam(1e9, 0.0)
    base = synth.GaussianLeakageBeam(theta=1.4 * math.pi / 180, dxy=s.leakage.dxy, dyx=s.leakage.dyx,
                                     level=s.leakage.level)
    assert np.allclose(b0.jones(l, m), base.jones(l, m))
    pa = 0.7
    c, sn = math.cos(pa), math.sin(pa)
    lr, mr = c * l - sn * m, sn * l + c * m          # a position that rotates onto (l, m)
    jr = s.beam(1e9, pa).jones(lr, mr)
    assert np.allclose(np.sum(np.abs(jr) ** 2, axis=(-2, -1)), np.sum(np.abs(base.jones(l, m)) ** 2, axis=(-2, -1)))


def test_network_features_layout():
    x = surrogate.features(np.array([-200.0, 100.0]), 1250e6, np.array([0.0, math.pi / 2]), np.array([0, 15]),
                           200.0, 700e6, 1800e6)
    assert x.shape == (2, surrogate.n_features()) == (2, 24) and x.dtype == np.float32
    np.testing.assert_allclose(x[:, 0], [-1.0, 0.5])
    np.testing.assert_allclose(x[:, 1], [0.0, 0.0], atol=1e-7)
    np.testing.assert_allclose(x[:, 2:4], [[0.0, 1.0], [1.0, 0.0]], atol=1e-7)
    np.testing.assert_allclose(x[:, 4:6], [[0.0, 1.0], [0.0, -1.0]], atol=1e-7)
    np.testing.assert_allclose(x[:, 6], [0.56, 0.56], rtol=1e-6)
    np.testing.assert_allclose(x[:, 7], [1.0, 0.25])
    assert x[0, 8] == 1.0 and x[1, 23] == 1.0 and x[:, 8:].sum() == 2.0


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True,
                       cwd=autotune.os.path.dirname(autotune.HERE), timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stdout
