"""Pins of the Mueller algebra (Eqs. 3-6) against closed forms and the paper's Fig. 1 numbers."""
import json
import os

import numpy as np
import pytest

from oracle import mueller

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def test_stokes_matrix_recovers_textbook_coherency():
    """Correlations XX = I+Q, XY = U+iV, YX = U-iV, YY = I-Q map back to (I, Q, U, V)."""
    rng = np.random.default_rng(1)
    s = mueller.stokes_matrix()
    for _ in range(10):
        i, q, u, v = rng.standard_normal(4)
        corr = np.array([i + q, u + 1j * v, u - 1j * v, i - q])
        assert np.allclose(s @ corr, [i, q, u, v], atol=1e-14)


def test_mueller_is_the_coherency_transform():
    """vec(J B J^H) = M vec(B) for random J and B (row-major vec, order XX XY YX YY)."""
    rng = np.random.default_rng(2)
    for _ in range(10):
        j = _crandn(rng, 2, 2)
        b = _crandn(rng, 2, 2)
        m = mueller.mueller_from_jones(j)
        assert np.allclose((j @ b @ j.conj().T).reshape(4), m @ b.reshape(4), atol=1e-13)


def test_scalar_beam_gives_scaled_identity():
    e = 0.37
    m = mueller.mueller_from_jones(e * np.eye(2))
    ms = mueller.stokes_mueller(m, mueller.stokes_matrix())
    assert np.allclose(ms, e * e * np.eye(4), atol=1e-15)


def test_stokes_mueller_real_only_under_readings():
    """M^S is real for any J with J (x) conj(J) and U = (XY+YX)/2; the literal readings break it."""
    rng = np.random.default_rng(3)
    j = _crandn(rng, 2, 2)
    s = mueller.stokes_matrix("iau")
    ms = mueller.stokes_mueller(mueller.mueller_from_jones(j), s)
    assert np.max(np.abs(ms.imag)) < 1e-14
    literal_u = mueller.stokes_mueller(mueller.mueller_from_jones(j), mueller.stokes_matrix("paper"))
    assert np.max(np.abs(literal_u.imag)) > 1e-3
    no_conj = np.kron(j, j)
    assert np.max(np.abs(mueller.stokes_mueller(no_conj, s).imag)) > 1e-3


def test_eq6_touches_only_the_diagonal_and_follows_the_formula():
    rng = np.random.default_rng(4)
    ms = rng.standard_normal((5, 6, 4, 4))
    eps = 0.2
    out = mueller.regularise_diagonal(ms, eps)
    off = ~np.eye(4, dtype=bool)
    assert np.array_equal(out[..., off], ms[..., off])
    for p in range(4):
        b = ms[..., p, p]
        beta = ((eps / 2) * np.abs(b).max()) ** 2
        expect = b / np.abs(b) * (np.abs(b) + beta / np.abs(b))  # Eq. 6 as printed
        assert np.allclose(out[..., p, p], expect, rtol=1e-14)


def test_eq6_at_an_exact_null_stays_finite():
    ms = np.zeros((3, 4, 4))
    ms[:, range(4), range(4)] = [[1.0] * 4, [0.0] * 4, [0.5] * 4]
    reg = mueller.regularise_diagonal(ms, 0.2)
    inv = 1.0 / reg[:, 0, 0]
    assert np.all(np.isfinite(inv)) and abs(inv[1]) < 1e-140
    assert np.all(np.isfinite(np.linalg.inv(reg)))


def test_fig1_divergences():
    """Paper Fig. 1 text: divergence of 1/B' from 1/B on a sinc^2 beam with eps = 2 per cent."""
    gold = json.load(open(os.path.join(GOLDEN, "fig1_eq6_divergence.json")))
    eps = gold["epsilon"]
    x = np.linspace(-3.0, 3.0, 600001)
    b = np.sinc(x) ** 2
    ms = np.zeros((x.size, 4, 4))
    ms[:, range(4), range(4)] = b[:, None]
    bp = mueller.regularise_diagonal(ms, eps)[:, 0, 0].real
    with np.errstate(divide="ignore", invalid="ignore"):
        div = np.abs(1 / bp - 1 / b) * np.abs(b)
    centre = div[x.size // 2]
    half = div[np.argmin(np.abs(b[x.size // 2:] - 0.5)) + x.size // 2]
    side_region = (x > 1.2) & (x < 1.7)
    side_idx = np.flatnonzero(side_region)[np.argmax(b[side_region])]
    side = div[side_idx]
    pr = gold["printed"]
    # one printed digit: agree to within rounding of that digit
    assert centre == pytest.approx(pr["centre"], rel=0.05)
    assert side == pytest.approx(pr["first_sidelobe"], rel=0.1)
    # half power disagrees with the printed 4e-3 by ten times (recorded reading)
    assert half == pytest.approx(pr["half_power"] / 10, rel=0.05)
    # no infinities in the inverse of the modified beam, even at the nulls
    assert np.all(np.isfinite(1 / bp))


def test_phi_identity_screens():
    g = mueller.phi_identity(4, 3, 3, kind="grid", eps=0.2)
    s = mueller.stokes_matrix()
    assert np.allclose(np.moveaxis(g, (0, 1), (-2, -1))[1, 2], s / 1.01, atol=1e-14)
    d = mueller.phi_identity(4, 3, 3, kind="degrid")
    assert np.allclose(np.moveaxis(d, (0, 1), (-2, -1))[0, 0], np.linalg.inv(s).conj().T, atol=1e-14)
