"""Oracle: orthogonalisation and subspace diagonalisation
(TEST INFRASTRUCTURE ONLY).

Sec. 6.  States are state-major arrays psi[k, p]; the grid inner product is
<f|g> = h^3 sum_p f(p) g(p).

  overlap        eq. (7): S_jk = <phi_j|phi_k>
  cholesky_upper S = U^T U with U upper triangular, positive diagonal
  orthonormalize eq. (8), read as phi_j = sum_k U_kj phibar_k (Psi = Psibar U,
                 so Psibar = Psi U^-1, classical Gram-Schmidt order)
  subspace       eq. (9): h_jk = <phi_j|H|phi_k>, symmetrised
  rayleigh_ritz  diagonalise h (ascending eigenvalues) and rotate, eq. (10):
                 phibar_k = sum_j xi_jk phi_j (applied to H psi as well); each
                 eigenvector's largest-magnitude component is made positive
                 (the sign is otherwise arbitrary)
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


class NotPositiveDefinite(Exception):
    def __init__(self, pivot: int):
        super().__init__(f"overlap not positive definite at pivot {pivot}")
        self.pivot = pivot


def dots(f: np.ndarray, g: np.ndarray, dv: float) -> np.ndarray:
    """Per-state <f_k|g_k>."""
    return dv * np.einsum("kp,kp->k", f, g)


def overlap(psi: np.ndarray, dv: float, other: np.ndarray = None) -> np.ndarray:
    """Eq. (7): S[j, k] = h^3 sum_p conj(psi_j(p)) other_k(p) (other = psi by
    default), for state-major [N, np] arrays, real or complex."""
    y = psi if other is None else other
    return dv * (np.conj(psi) @ y.T)


def cholesky_upper(S: np.ndarray) -> np.ndarray:
    """Plain right-looking Cholesky, S = U^T U, raising with the 1-based
    failing pivot (LAPACK potrf convention)."""
    n = S.shape[0]
    A = np.array(S, dtype=np.float64, copy=True)
    U = np.zeros_like(A)
    for j in range(n):
        d = A[j, j] - U[:j, j] @ U[:j, j]
        if not d > 0.0:
            raise NotPositiveDefinite(j + 1)
        U[j, j] = np.sqrt(d)
        U[j, j + 1:] = (A[j, j + 1:] - U[:j, j] @ U[:j, j + 1:]) / U[j, j]
    return U


def orthonormalize(psi: np.ndarray, dv: float):
    """Returns (Psibar, U, S)."""
    S = overlap(psi, dv)
    U = cholesky_upper(S)
    # Psibar^T = U^-T Psi^T  (state-major: solve U^T X = Psi)
    psibar = scipy.linalg.solve_triangular(U.T, psi, lower=True)
    return psibar, U, S


def subspace(psi: np.ndarray, hpsi: np.ndarray, dv: float) -> np.ndarray:
    hm = dv * (psi @ hpsi.T)
    return 0.5 * (hm + hm.T)


def rayleigh_ritz(psi: np.ndarray, hpsi: np.ndarray, dv: float):
    """Returns (eigenvalues ascending, xi, rotated psi, rotated H psi)."""
    hm = subspace(psi, hpsi, dv)
    lam, xi = np.linalg.eigh(hm)
    xi = xi * fix_signs(xi)
    return lam, xi, xi.T @ psi, xi.T @ hpsi


def fix_signs(V: np.ndarray) -> np.ndarray:
    """+1/-1 per column so that each column's largest-|.| entry is positive."""
    arg = np.argmax(np.abs(V), axis=0)
    return np.where(V[arg, np.arange(V.shape[1])] < 0, -1.0, 1.0)
