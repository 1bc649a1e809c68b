"""Pins of the prolate spheroidal anti-aliasing function (textbook special function)."""
import numpy as np
import pytest
from scipy.special import pro_ang1

from oracle import pswf


@pytest.mark.parametrize("support", [5, 7, 9])
def test_matches_scipy_pro_ang1_inside(support):
    c = np.pi * support / 2
    x = np.linspace(-0.995, 0.995, 81)
    ref = np.array([pro_ang1(0, 0, c, v)[0] for v in x]) / pro_ang1(0, 0, c, 0.0)[0]
    assert np.max(np.abs(pswf.psi0(c, x) - ref)) < 1e-12


@pytest.mark.parametrize("support", [7, 12])
def test_finite_fourier_eigenfunction(support):
    """int_-1^1 exp(i c x t) psi(t) dt = lambda psi(x) with one real lambda for every x."""
    c = np.pi * support / 2
    t, wq = np.polynomial.legendre.leggauss(200)
    psi_t = pswf.psi0(c, t)
    x = np.linspace(-1.0, 1.0, 23)
    lhs = np.exp(1j * c * np.outer(x, t)) @ (wq * psi_t)
    lam = lhs[11]  # x = 0, psi(0) = 1
    assert abs(lam.imag) < 1e-12 and lam.real > 0
    assert np.max(np.abs(lhs - lam * pswf.psi0(c, x))) < 1e-11 * abs(lam)


def test_normalised_even_and_finite_at_edges():
    x = np.linspace(-1, 1, 101)
    v = pswf.aa_function(7, x)
    assert pswf.aa_function(7, 0.0) == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(v, v[::-1], rtol=0, atol=1e-15)
    assert np.all(np.isfinite(v)) and np.all(v > 0)
    # pixels: x = 2 (j - n/2) / n reaches -1 at the first pixel
    px = pswf.aa_pixels(8, 7)
    assert px[0] == pytest.approx(pswf.aa_function(7, -1.0))
    assert px[4] == pytest.approx(1.0)
