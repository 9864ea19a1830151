"""Pins of the oracle's orthogonalisation and subspace diagonalisation
(CPU only): LAPACK QR / eigh are the independent routes."""
import numpy as np
import pytest

import synthetic
from oracle import hamiltonian, linalg


def test_orthonormalize_equals_qr():
    rng = np.random.default_rng(0)
    dv = 0.2 ** 3
    psi = rng.uniform(-1, 1, size=(12, 3000))
    psibar, U, S = linalg.orthonormalize(psi, dv)
    Q, R = np.linalg.qr(np.sqrt(dv) * psi.T)
    sgn = np.sign(np.diag(R))
    Q, R = Q * sgn, (R.T * sgn).T
    assert np.allclose(U, R, rtol=0, atol=1e-12 * np.max(np.abs(R)))
    assert np.allclose(psibar, Q.T / np.sqrt(dv), atol=1e-11)
    assert np.allclose(dv * psibar @ psibar.T, np.eye(12), atol=1e-12)
    # classical Gram-Schmidt order: the first state is only normalised
    assert np.allclose(psibar[0], psi[0] / np.sqrt(dv * psi[0] @ psi[0]), atol=1e-13)


def test_cholesky_matches_lapack_and_reports_pivot():
    rng = np.random.default_rng(1)
    A = rng.normal(size=(20, 20))
    S = A @ A.T + 20 * np.eye(20)
    U = linalg.cholesky_upper(S)
    assert np.allclose(U, np.linalg.cholesky(S).T, atol=1e-12)
    psi = rng.uniform(-1, 1, size=(6, 500))
    psi[4] = psi[2]                        # duplicated state -> singular overlap
    S = linalg.overlap(psi, 1.0)
    S[4, 4] -= 1e-9 * S[2, 2]              # push the zero pivot clearly negative
    with pytest.raises(linalg.NotPositiveDefinite) as e:
        linalg.cholesky_upper(S)
    assert e.value.pivot == 5


def test_rayleigh_ritz_matches_eigh_and_diagonalises():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=1.6, h=0.25, nat=2, atom_radius=0.6, rc=1.0)
    g, atoms, H = hamiltonian.build_system(w)
    rng = np.random.default_rng(2)
    psi, _, _ = linalg.orthonormalize(rng.uniform(-1, 1, size=(6, g.np)), g.dv)
    hpsi = H.apply(psi)
    lam, xi, p2, h2 = linalg.rayleigh_ritz(psi, hpsi, g.dv)
    # independent route: h from (H psi) psi^T via the dense matrix
    Hd = H.dense()
    hm = g.dv * psi @ Hd @ psi.T
    assert np.allclose(np.linalg.eigvalsh(hm), lam, atol=1e-10)
    sub = g.dv * p2 @ h2.T
    assert np.allclose(sub, np.diag(lam), atol=1e-10)
    # the rotated set spans the same subspace
    P1 = psi.T @ psi
    P2 = p2.T @ p2
    assert np.allclose(P1, P2, atol=1e-10 / g.dv)


def test_overlap_of_complex_states_is_hermitian_and_splits():
    """S = h^3 Psi^H Psi for complex states: Hermitian, positive definite,
    with real part S(a) + S(b) and imaginary part S(a, b) - S(b, a)."""
    rng = np.random.default_rng(31)
    a, b = rng.uniform(-1, 1, size=(2, 6, 50))
    z = a + 1j * b
    S = linalg.overlap(z, 0.3)
    assert np.allclose(S, S.conj().T, rtol=0, atol=1e-14)
    assert np.min(np.linalg.eigvalsh(S)) > 0
    assert np.allclose(S.real, 0.3 * (a @ a.T + b @ b.T), rtol=0, atol=1e-13)
    assert np.allclose(S.imag, 0.3 * (a @ b.T - b @ a.T), rtol=0, atol=1e-13)
    assert np.allclose(linalg.overlap(a, 0.3, b), 0.3 * a @ b.T, rtol=0, atol=1e-13)
