"""Order-0 prolate spheroidal anti-aliasing function.

The paper multiplies every kernel in the image domain by "an anti-aliasing
function" (Sec. 3.2) without naming it; the reading taken is the order-0
prolate spheroidal wave function psi_c on [-1, 1] with c = pi * S_aa / 2,
normalised to psi(0) = 1, applied as AA(l, m) = psi(2 l / fov) psi(2 m / fov).

Evaluation: expansion in even normalised Legendre polynomials whose
coefficients are the eigenvector of the smallest eigenvalue of the symmetric
tridiagonal matrix of the prolate differential operator in that basis
(Bouwkamp's method; Xiao, Rokhlin and Yarvin 2001).  scipy's `pro_ang1`
returns NaN at |x| = 1, which the kernel lattice reaches, so it serves only
as an independent pin inside (-1, 1).
"""
import numpy as np
from numpy.polynomial import legendre
from scipy.linalg import eigh_tridiagonal


def legendre_coefficients(c: float, nterms: int = 0) -> np.ndarray:
    """Coefficients b_k of psi_0 in P_k (plain Legendre basis), degrees 0, 1, ..., 2K."""
    if nterms == 0:
        nterms = int(c) + 40
    k = 2.0 * np.arange(nterms)
    diag = k * (k + 1) + c * c * (2 * k * (k + 1) - 1) / ((2 * k + 3) * (2 * k - 1))
    kk = k[:-1]
    off = c * c * (kk + 2) * (kk + 1) / ((2 * kk + 3) * np.sqrt((2 * kk + 1) * (2 * kk + 5)))
    _, vec = eigh_tridiagonal(diag, off, select="i", select_range=(0, 0))
    beta = vec[:, 0]
    coef = np.zeros(2 * nterms - 1)
    coef[0::2] = beta * np.sqrt(k + 0.5)  # normalised -> plain Legendre basis
    return coef


def psi0(c: float, x) -> np.ndarray:
    """psi_0(c, x) normalised to psi_0(c, 0) = 1."""
    coef = legendre_coefficients(c)
    v = legendre.legval(np.asarray(x, dtype=np.float64), coef)
    return v / legendre.legval(0.0, coef)


def aa_function(aa_support: int, x) -> np.ndarray:
    """The anti-aliasing function at normalised coordinate x = 2 l / fov."""
    return psi0(np.pi * aa_support / 2.0, x)


def aa_pixels(n: int, aa_support: int) -> np.ndarray:
    """AA at the n image pixels of one axis, x = 2 (j - n/2) / n."""
    return aa_function(aa_support, 2.0 * (np.arange(n) - n // 2) / n)
