"""Pins of the per-baseline Mueller kernels (Sec. 3.2: the Mueller matrix of a baseline is the
Kronecker product of its two antennas' Jones matrices; non-identical antennas make it unique to the
baseline): the coherency transform with two different Jones matrices, baseline reversal, and the
degrid prediction through per-baseline-class kernels against Eq. 2 evaluated directly."""
import numpy as np

import synth
from oracle import gridding, imaging, kernels, mueller


def _crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def test_baseline_mueller_is_the_two_antenna_coherency_transform():
    """vec(J_a B J_b^H) = M_ab vec(B) for random, different J_a, J_b (a transposed or unconjugated
    factor, or swapped antennas, fails)."""
    rng = np.random.default_rng(61)
    for _ in range(10):
        ja, jb, b = _crandn(rng, 2, 2), _crandn(rng, 2, 2), _crandn(rng, 2, 2)
        m = mueller.mueller_from_jones(ja, jb)
        assert np.allclose((ja @ b @ jb.conj().T).reshape(4), m @ b.reshape(4), atol=1e-13)
        assert not np.allclose(mueller.mueller_from_jones(jb, ja) @ b.reshape(4), m @ b.reshape(4))
    j = _crandn(rng, 2, 2)
    assert np.array_equal(mueller.mueller_from_jones(j, j), mueller.mueller_from_jones(j))


def test_reversed_baseline_gives_the_conjugate_transposed_visibility():
    """For a Hermitian coherency B, the (b, a) baseline measures (J_a B J_b^H)^H: M_ba vec(B) equals
    the reordered conjugate of M_ab vec(B)."""
    rng = np.random.default_rng(62)
    for _ in range(10):
        ja, jb = _crandn(rng, 2, 2), _crandn(rng, 2, 2)
        h = _crandn(rng, 2, 2)
        b = h + h.conj().T
        vab = (mueller.mueller_from_jones(ja, jb) @ b.reshape(4)).reshape(2, 2)
        vba = (mueller.mueller_from_jones(jb, ja) @ b.reshape(4)).reshape(2, 2)
        assert np.allclose(vba, vab.conj().T, atol=1e-13)


def antenna_classes(rng, fov, k=3):
    """k antenna types: the 1-degree-style Gaussian beam with its own pointing error and leakage."""
    out = []
    for _ in range(k):
        b = synth.seeded_leakage_beam(0.5 * fov, rng, level=0.05)
        out.append(synth.OffsetBeam(b, rng.uniform(-0.03, 0.03) * fov, rng.uniform(-0.03, 0.03) * fov))
    return out


def test_per_baseline_degrid_matches_direct_prediction():
    """Rows split by baseline class (a, b); each class predicted through the degridding kernels of
    M_ab equals Eq. 2 with J_a B J_b^H at every source, to the P6 tolerance; kernels of the averaged
    (mean-Jones) beam instead are far off."""
    rng = np.random.default_rng(63)
    n, fov = 64, 0.1
    g = synth.Geometry(n=n, cell=fov / n, os=4, w_planes=np.zeros(1), support=np.array([13]),
                       tile=np.array([16]), mk=n)
    ants = antenna_classes(rng, fov)
    ii = rng.integers(n // 4, 3 * n // 4, 4)
    jj = rng.integers(n // 4, 3 * n // 4, 4)
    sl, sm = (jj - n // 2) * g.cell, (ii - n // 2) * g.cell
    iquv = np.zeros((4, 4))
    iquv[:, 0] = rng.uniform(0.3, 1, 4)
    iquv[:, 1:] = rng.uniform(-0.1, 0.1, (4, 3))
    model = np.zeros((4, n, n))
    for k in range(4):
        model[:, ii[k], jj[k]] += iquv[k]
    gm = imaging.grid_from_model(g, model)
    c = n // 2 * g.os
    worst, worst_avg = 0.0, 0.0
    jl = [synth.jones_on_lattice(a, n, fov) for a in ants]
    mean_j = sum(jl) / len(jl)
    for a in range(3):
        for b in range(a, 3):
            fx, fy = rng.integers(c - 60, c + 60, 120), rng.integers(c - 60, c + 60, 120)
            uvw = np.stack([(fx / g.os - n / 2) / g.fov, (fy / g.os - n / 2) / g.fov, np.zeros(120)], 1)
            tabs = kernels.make_tables(g, mueller.phi_degrid(jl[a], jones_b=jl[b]))
            got = gridding.degrid(g, tabs, uvw, gm)
            want = imaging.dft_predict(uvw, sl, sm, iquv, beam=ants[a], beam_b=ants[b])
            worst = max(worst, np.max(np.abs(got - want)) / np.max(np.abs(want)))
            avg = gridding.degrid(g, kernels.make_tables(g, mueller.phi_degrid(mean_j)), uvw, gm)
            worst_avg = max(worst_avg, np.max(np.abs(avg - want)) / np.max(np.abs(want)))
    assert worst < 1e-5, worst  # 1.1e-6 in the float64 run
    assert worst_avg > 0.03  # 6-11 % in the float64 run
