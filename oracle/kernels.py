"""Oversampled uv kernel tables (Sec. 3.2: the kernels are the Fourier transform of
the Mueller cells after multiplication, in the image domain, by the anti-aliasing
function and the w-correction term).

Readings (the paper gives no sampling, padding or normalisation):

  * the image-domain function of plane p, output Stokes q and input
    correlation c is f = AA(l) AA(m) exp(-2 pi i w_p (n - 1)) Phi_qc(l, m),
    sampled on an mk x mk lattice l_a = (a - mk/2) fov / mk;
  * the table is its zero-padded (x os) inverse DFT restricted to offsets
    |d| < S os / 2 on the 1/os fine grid:
        T(d_x, d_y) = mk^-2 sum_ab f(l_a, m_b)
                      exp(+2 pi i [d_x (a - mk/2) + d_y (b - mk/2)] / (os mk)),
    a separable transform computed as two dense matrix products;
  * storage is [phase_y][phase_x][tap_y][tap_x] with tap t of phase ph at offset
    d = ph - S os / 2 + 1 + t os; the one slot with d = S os / 2 holds zero.
"""
import numpy as np

from .geometry import n_minus_one
from .pswf import aa_function


def lattice(mk: int, fov: float) -> np.ndarray:
    return (np.arange(mk) - mk // 2) * (fov / mk)


def aa_lattice(mk: int, aa_support: int) -> np.ndarray:
    """AA at the lattice points of one axis: psi(2 l_a / fov) = psi(2 (a - mk/2) / mk)."""
    return aa_function(aa_support, 2.0 * (np.arange(mk) - mk // 2) / mk)


def image_function(geom, plane: int, phi: np.ndarray) -> np.ndarray:
    """f[q][c][b][a] = AA(l_a) AA(m_b) W*_p(l_a, m_b) Phi[q][c][b][a]."""
    mk = geom.mk
    x = lattice(mk, geom.fov)
    mm, ll = np.meshgrid(x, x, indexing="ij")
    aa = aa_lattice(mk, geom.aa_support)
    screen = np.outer(aa, aa) * np.exp(-2j * np.pi * geom.w_planes[plane] * n_minus_one(ll, mm))
    return screen[None, None] * phi


def dft_table(f2d: np.ndarray, support: int, os: int) -> np.ndarray:
    """[os][os][S][S] oversampled table of one image-domain function f2d[b][a]."""
    mk = f2d.shape[0]
    half = support * os // 2
    d = np.arange(-(half - 1), half)
    e = np.exp(2j * np.pi * np.outer(d, np.arange(mk) - mk // 2) / (os * mk)) / mk
    full = e @ f2d @ e.T  # [d_y][d_x]
    pad = np.zeros((support * os, support * os), dtype=np.complex128)
    pad[:-1, :-1] = full
    # index d + half - 1 = phase + t * os
    return pad.reshape(support, os, support, os).transpose(1, 3, 0, 2)


def make_tables(geom, phi: np.ndarray, planes=None) -> list:
    """One table per plane, each [Q][C][os][os][S_p][S_p] complex128 (None for planes not asked for)."""
    tables = []
    for p in range(geom.nplanes):
        if planes is not None and p not in planes:
            tables.append(None)
            continue
        f = image_function(geom, p, phi)
        q, c = f.shape[:2]
        s = int(geom.support[p])
        t = np.empty((q, c, geom.os, geom.os, s, s), dtype=np.complex128)
        for qq in range(q):
            for cc in range(c):
                t[qq, cc] = dft_table(f[qq, cc], s, geom.os)
        tables.append(t)
    return tables


def round_tables(tables, dtype) -> list:
    """Tables rounded to the storage precision (complex64, or float16 pairs) and back to complex128."""
    out = []
    for t in tables:
        if t is None:
            out.append(None)
        elif dtype == np.float16:
            out.append(t.real.astype(np.float16).astype(np.float64)
                       + 1j * t.imag.astype(np.float16).astype(np.float64))
        else:
            out.append(t.astype(dtype).astype(np.complex128))
    return out
