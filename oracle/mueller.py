"""Jones -> Mueller -> Stokes Mueller, null regularisation and the kernel screens Phi.

Readings of the paper (Sec. 3.2-3.3):

  * Mueller from Jones (Sec. 3.2, the Kronecker product under Eq. 2): the
    paper writes J_i (x) J_j; the conjugate J_i (x) conj(J_j) is taken, the
    textbook measurement equation, without which M^S is not real.  Antennas
    are identical unless a second Jones field is given (a baseline between two
    antenna types); M^S is then complex in general.
  * Correlation order XX, XY, YX, YY (Eq. 3).
  * Stokes substitution (Eq. 4): the paper prints U with a factor i; the
    reading is U = (XY + YX)/2 (IAU), under which M^S is real.  The
    paper-literal variant is kept as convention "paper".
  * Stokes Mueller (Eq. 5): M^S = S M S^-1.
  * Eq. 6 acts on a copy of the diagonal entries B_p = M^S_pp:
    B'_p = B_p (1 + beta_p / |B_p|^2), beta_p = ((eps/2) max|B_p|)^2, the max
    taken over the kernel lattice; at an exact null B_p is replaced by 1e-150 so
    that B'_p is large and finite and 1/B'_p goes to its limit, 0.
  * Gridding screens Phi = (M'^S)^-1 S map correlations to Stokes (Sec. 3.2,
    gridding paragraph); degridding screens Phi = (S^-1 M^S)^H are the ones
    whose conjugate maps the Stokes sky to observed correlations (Eq. 2).
"""
import numpy as np


def stokes_matrix(convention: str = "iau") -> np.ndarray:
    """S with rows I, Q, U, V and columns XX, XY, YX, YY (Eq. 4)."""
    u = 0.5 if convention == "iau" else 0.5j
    return np.array([[0.5, 0, 0, 0.5],
                     [0.5, 0, 0, -0.5],
                     [0, u, u, 0],
                     [0, -0.5j, 0.5j, 0]], dtype=np.complex128)


def mueller_from_jones(j: np.ndarray, j_b: np.ndarray = None) -> np.ndarray:
    """M = J (x) conj(J) per sample; j is [..., 2, 2], the result [..., 4, 4].  With j_b, the
    Mueller matrix of a baseline between two different antennas, J_a (x) conj(J_b) (Sec. 3.2)."""
    j = np.asarray(j, dtype=np.complex128)
    jc = np.conj(j if j_b is None else np.asarray(j_b, dtype=np.complex128))
    out = np.empty(j.shape[:-2] + (4, 4), dtype=np.complex128)
    for a in range(2):
        for b in range(2):
            for c in range(2):
                for d in range(2):
                    out[..., 2 * a + b, 2 * c + d] = j[..., a, c] * jc[..., b, d]
    return out


def stokes_mueller(m: np.ndarray, s: np.ndarray) -> np.ndarray:
    """M^S = S M S^-1 (Eq. 5)."""
    return s @ m @ np.linalg.inv(s)


def regularise_diagonal(ms: np.ndarray, eps: float) -> np.ndarray:
    """Eq. 6 on a copy of the diagonal of a [..., 4, 4] field; off-diagonal entries unchanged."""
    out = np.array(ms, dtype=np.complex128, copy=True)
    flat = ms.reshape(-1, 4, 4)
    for p in range(4):
        b = ms[..., p, p]
        beta = ((eps / 2.0) * np.abs(flat[:, p, p]).max()) ** 2
        b = np.where(np.abs(b) > 0, b, 1e-150)
        out[..., p, p] = b * (1.0 + beta / np.abs(b) ** 2)
    return out


def jones_field_to_pixels(jones: np.ndarray) -> np.ndarray:
    """[2][2][rows][cols] (make_kernels layout) -> [rows][cols][2][2]."""
    return np.moveaxis(np.asarray(jones, dtype=np.complex128), (0, 1), (2, 3))


def _ms_field(jones, jones_b, s):
    jb = None if jones_b is None else jones_field_to_pixels(jones_b)
    return stokes_mueller(mueller_from_jones(jones_field_to_pixels(jones), jb), s)


def phi_grid(jones, eps: float, convention: str = "iau", jones_b=None) -> np.ndarray:
    """Gridding screens Phi = (M'^S)^-1 S, shape [Q=4][C=4][rows][cols] (Sec. 3.2-3.3); with jones_b,
    those of the baseline between antennas with Jones fields jones and jones_b."""
    s = stokes_matrix(convention)
    ms = _ms_field(jones, jones_b, s)
    minv = np.linalg.inv(regularise_diagonal(ms, eps))
    phi = minv @ s
    return np.moveaxis(phi, (-2, -1), (0, 1))


def phi_degrid(jones, convention: str = "iau", jones_b=None) -> np.ndarray:
    """Degridding screens Phi = (S^-1 M^S)^H, shape [Q=4][C=4][rows][cols] (Sec. 3.2, Eq. 2); with
    jones_b, those of the baseline between antennas with Jones fields jones and jones_b."""
    s = stokes_matrix(convention)
    ms = _ms_field(jones, jones_b, s)
    a = np.linalg.inv(s) @ ms
    phi = np.conj(np.swapaxes(a, -1, -2))
    return np.moveaxis(phi, (-2, -1), (0, 1))


def phi_identity(npol: int, rows: int, cols: int, kind: str = "grid", eps: float = 0.2,
                 convention: str = "iau") -> np.ndarray:
    """Screens without an A-term.

    npol 1 (Stokes I only): Phi = 1.  npol 4: the screens of J = identity, i.e.
    the Stokes conversion with (grid) or without (degrid) the Eq. 6 scaling.
    """
    if npol == 1:
        return np.ones((1, 1, rows, cols), dtype=np.complex128)
    jones = np.zeros((2, 2, rows, cols), dtype=np.complex128)
    jones[0, 0] = 1.0
    jones[1, 1] = 1.0
    if kind == "grid":
        return phi_grid(jones, eps, convention)
    return phi_degrid(jones, convention)
