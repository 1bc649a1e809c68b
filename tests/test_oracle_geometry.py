"""Pins of the oracle's geometry and binning against brute force on small inputs."""
import numpy as np
import pytest

import synth
from oracle import geometry, plan as oplan


def test_round_half_up_snapping():
    # x*os exactly k + 0.5 rounds up; just below rounds down (float64 snapping).
    n, cell, os = 64, 0.01, 4
    fov = n * cell
    xs = np.array([10.125, 10.124, 33.0, 31.875])  # grid-pixel positions
    uvw = np.zeros((4, 3))
    uvw[:, 0] = (xs - n / 2) / fov
    uvw[:, 1] = (xs - n / 2) / fov
    fx, fy = geometry.fine_position(uvw, n, cell, os)
    assert list(fx) == [41, 40, 132, 128]
    assert list(fx) == list(fy)


@pytest.mark.parametrize("os_", [2, 4, 8])
@pytest.mark.parametrize("support", [7, 8, 16, 31, 48])
def test_footprint_brute_force(os_, support):
    """X0..X0+S-1 minus the one zero slot is exactly {X : |X os - fine| < S os / 2}."""
    if (support * os_) % 2:
        pytest.skip("S*os must be even")
    rng = np.random.default_rng(support * 10 + os_)
    fine = rng.integers(-50, 500, 400)
    x0, ph = geometry.anchor_phase(fine, np.full(fine.shape, support), os_)
    half = support * os_ / 2
    for f, a, p in zip(fine, x0, ph):
        brute = [X for X in range(-200, 400) if abs(X * os_ - f) < half]
        box = [a + t for t in range(support)
               if abs(p - support * os_ // 2 + 1 + t * os_) < half]
        assert brute == box
        assert 0 <= p < os_
        assert len(brute) in (support, support - 1)
        assert (len(brute) == support - 1) == (p == os_ - 1)


def test_nearest_plane_brute_force_and_ties():
    planes = np.array([-30.0, -10.0, 10.0, 30.0])
    w = np.array([-100.0, -20.0, 0.0, 20.0, 29.0, 100.0, -10.0])
    got = geometry.nearest_plane(w, planes)
    # -20 ties between planes 0 and 1 -> lower; 0 ties 1/2 -> 1; 20 ties 2/3 -> 2
    assert list(got) == [0, 0, 1, 2, 3, 3, 1]
    rng = np.random.default_rng(3)
    w = rng.uniform(-50, 50, 500)
    got = geometry.nearest_plane(w, planes)
    for wi, gi in zip(w, got):
        d = [abs(wi - pp) for pp in planes]
        assert gi == min(range(4), key=lambda i: (d[i], i))


def test_keep_mask_matches_box_in_grid():
    n = 32
    rng = np.random.default_rng(4)
    x0 = rng.integers(-10, 40, 300)
    y0 = rng.integers(-10, 40, 300)
    s = rng.integers(4, 12, 300)
    keep = geometry.keep_mask(x0, y0, s, n)
    for a, b, ss, k in zip(x0, y0, s, keep):
        inside = all(0 <= a + t < n and 0 <= b + t < n for t in range(ss))
        assert inside == k


def _tiny_geom():
    planes = synth.linear_w_planes(4, 60.0)
    return synth.Geometry(n=64, cell=0.4 / 64, os=4, w_planes=planes,
                          support=np.array([9, 7, 7, 9], np.int32),
                          tile=np.array([8, 12, 12, 8], np.int32), mk=64)


def test_plan_brute_force():
    g = _tiny_geom()
    rng = np.random.default_rng(5)
    nv = 3000
    uvw = np.stack([rng.uniform(-90, 90, nv), rng.uniform(-90, 90, nv), rng.uniform(-80, 80, nv)], 1)
    pl = oplan.plan(g, uvw, max_chunk=7)
    loc = pl["loc"]
    # brute force: sort tuples (plane, ty, tx, phy, phx, index) of kept visibilities
    rows = []
    for k in range(nv):
        if not loc["keep"][k]:
            continue
        p = loc["plane"][k]
        t = g.tile[p]
        rows.append((p, loc["y0"][k] // t, loc["x0"][k] // t, loc["phase_y"][k], loc["phase_x"][k], k))
    rows.sort()
    assert pl["n_kept"] == len(rows)
    assert pl["n_dropped"] == nv - len(rows) and pl["n_dropped"] > 0
    assert list(pl["perm"][:len(rows)]) == [r[5] for r in rows]
    assert sorted(pl["perm"]) == list(range(nv))
    # items: consecutive chunks of runs of equal (plane, ty, tx), at most 7 long, covering all
    expect = []
    i = 0
    while i < len(rows):
        j = i
        while j < len(rows) and rows[j][:3] == rows[i][:3]:
            j += 1
        for s0 in range(i, j, 7):
            expect.append((rows[i][0], rows[i][1], rows[i][2], s0, min(j, s0 + 7)))
        i = j
    assert [tuple(int(v) for v in it) for it in pl["items"]] == expect
