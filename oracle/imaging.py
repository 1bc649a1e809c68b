"""FFT + taper correction, the predict direction, and direct Fourier transforms.

The paper moves between grid and image with an FFT (Sec. 2.2, Sec. 4) and
applies the anti-aliasing function in the image domain (Sec. 3.2), so the
image is divided by it afterwards.  Sign convention: Eq. 2 predicts with
exp(+2 pi i s.b); the imaging transform uses the opposite sign, and the w
term is phase-centre referenced, w (n - 1) (readings of Eq. 2).  Images are
the real part divided by the weight sum (natural weighting).
"""
import numpy as np

from .geometry import n_minus_one, pixel_coords
from .mueller import mueller_from_jones, stokes_matrix, stokes_mueller
from .pswf import aa_pixels


def image_from_grid(geom, g: np.ndarray, weight_sum: float) -> np.ndarray:
    """I_q(i, j) = Re{sum_XY G_q(X,Y) exp(-2 pi i [(X-n/2)(j-n/2) + (Y-n/2)(i-n/2)]/n)}
    / (AA(l_j) AA(m_i)) / weight_sum."""
    f = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(g, axes=(-2, -1)), axes=(-2, -1)), axes=(-2, -1))
    aa = aa_pixels(geom.n, geom.aa_support)
    return f.real / np.outer(aa, aa)[None] / weight_sum


def grid_from_model(geom, model: np.ndarray) -> np.ndarray:
    """Predict direction: G_q(X, Y) = sum_ij [model_q(i,j) / AA AA] exp(+2 pi i [...] / n)."""
    aa = aa_pixels(geom.n, geom.aa_support)
    m = np.asarray(model, dtype=np.complex128) / np.outer(aa, aa)[None]
    n2 = geom.n * geom.n
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(m, axes=(-2, -1)), axes=(-2, -1)), axes=(-2, -1)) * n2


def dft_predict(uvw, src_l, src_m, src_stokes, beam=None, convention: str = "iau", beam_b=None) -> np.ndarray:
    """Direct evaluation of Eq. 2 for point sources.

    Stokes-I only (src_stokes [nsrc][1], no beam): V = sum_j I_j e^{+2 pi i (u l + v m + w (n-1))}.
    Full polarisation (src_stokes [nsrc][4] = I, Q, U, V): the correlations
    XX, XY, YX, YY are V = sum_j S^-1 M^S(l_j, m_j) I_j e^{...}, with M from the beam's
    Jones matrix at the source (identity when beam is None); with beam_b, every row is a
    baseline between an antenna of `beam` and one of `beam_b`: M = J_a (x) conj(J_b).
    """
    src_l = np.asarray(src_l, dtype=np.float64)
    src_m = np.asarray(src_m, dtype=np.float64)
    stokes = np.asarray(src_stokes, dtype=np.float64)
    phase = np.exp(2j * np.pi * (np.outer(uvw[:, 0], src_l) + np.outer(uvw[:, 1], src_m)
                                  + np.outer(uvw[:, 2], n_minus_one(src_l, src_m))))
    if stokes.shape[1] == 1:
        return phase @ stokes.astype(np.complex128)
    s = stokes_matrix(convention)
    if beam is None:
        m = np.broadcast_to(np.eye(4, dtype=np.complex128), (src_l.shape[0], 4, 4))
    else:
        m = mueller_from_jones(beam.jones(src_l, src_m), None if beam_b is None else beam_b.jones(src_l, src_m))
    corr = np.einsum("jcq,jq->jc", np.linalg.inv(s)[None] @ stokes_mueller(m, s), stokes)
    return phase @ corr


def dft_image(geom, uvw, vis, weight_sum, phi_pixels=None) -> np.ndarray:
    """Direct dirty image at every pixel: Re sum_k sum_c Phi_qc(l,m) V_kc e^{-2 pi i (u l + v m + w (n-1))}
    / weight_sum.  phi_pixels [Q][C][n][n] defaults to the identity (C = Q)."""
    x = pixel_coords(geom.n, geom.cell)
    mm, ll = np.meshgrid(x, x, indexing="ij")
    nm1 = n_minus_one(ll, mm)
    vis = np.asarray(vis, dtype=np.complex128)
    c = vis.shape[1]
    acc = np.zeros((c, geom.n, geom.n), dtype=np.complex128)
    for k in range(uvw.shape[0]):
        ph = np.exp(-2j * np.pi * (uvw[k, 0] * ll + uvw[k, 1] * mm + uvw[k, 2] * nm1))
        acc += vis[k][:, None, None] * ph[None]
    if phi_pixels is None:
        return acc.real / weight_sum
    return np.einsum("qcyx,cyx->qyx", phi_pixels, acc).real / weight_sum

