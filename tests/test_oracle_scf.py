"""Pins of the oracle's SCF loop (Sec. 3): LDA exchange-correlation, the
density, the Broyden/Anderson mixer, and a converged SCF checked against the
dense eigenproblem of its own effective Hamiltonian."""
import numpy as np
import pytest

import synthetic
from oracle import hamiltonian, linalg, rmmdiis, scf


def test_lda_potential_is_the_derivative_of_the_energy_density():
    """v_xc = d(n eps_xc)/dn by central differences, on both branches of the
    correlation (rs from 0.05 to 40)."""
    rs = np.geomspace(0.05, 40.0, 60)
    n = 3.0 / (4.0 * np.pi * rs ** 3)
    v, e = scf.lda_xc(n)
    d = 1e-6 * n
    _, ep = scf.lda_xc(n + d)
    _, em = scf.lda_xc(n - d)
    fd = ((n + d) * ep - (n - d) * em) / (2 * d)
    assert np.max(np.abs(fd - v) / np.abs(v)) < 1e-7


def test_lda_textbook_values():
    """Exchange of the uniform gas: eps_x = -0.458165 / rs Ha; the two
    correlation branches meet at rs = 1 (to the parametrisation's 4 digits)
    near the Ceperley-Alder value -0.0596 Ha; zero density gives zero."""
    for rs in (0.5, 1.0, 3.0):
        n = 3.0 / (4.0 * np.pi * rs ** 3)
        v, e = scf.lda_xc(np.array([n]))
        ex = -0.75 * (3 * n / np.pi) ** (1 / 3)
        assert abs(ex + 0.458165293 / rs) < 1e-8
    n1 = 3.0 / (4.0 * np.pi)
    _, e_hi = scf.lda_xc(np.array([n1 * (1 - 1e-12)]))
    _, e_lo = scf.lda_xc(np.array([n1 * (1 + 1e-12)]))
    ex1 = -0.458165293
    assert abs((e_hi[0] - ex1) - (e_lo[0] - ex1)) < 1e-4
    assert abs((e_hi[0] - ex1) + 0.0596) < 5e-4
    assert scf.lda_xc(np.zeros(3))[0].tolist() == [0.0, 0.0, 0.0]


def test_density_counts_the_electrons():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=2.0, h=0.25, nat=1, atom_radius=0.3, nstates=6)
    g, atoms, H = hamiltonian.build_system(w)
    psi, _, _ = linalg.orthonormalize(synthetic.draw_states(synthetic.rng_after_atoms(w), 6, g.np), g.dv)
    n = scf.density(psi, 4)
    assert abs(g.dv * n.sum() - 8.0) < 1e-12
    assert np.all(n >= 0.0)


def test_mixer_solves_a_linear_fixed_point():
    """On a linear map n -> M n + c in 5 dimensions, Anderson mixing with a
    history of 5 reaches the fixed point (like GMRES) within a few
    iterations, where plain linear mixing is still far off."""
    rng = np.random.default_rng(3)
    Q = np.linalg.qr(rng.normal(size=(5, 5)))[0]
    M = Q @ np.diag([0.9, 0.7, -0.5, 0.3, 0.95]) @ Q.T
    c = rng.normal(size=5)
    fixed = np.linalg.solve(np.eye(5) - M, c)
    mix = scf.Mixer(1.0, 0.3, 5)
    n = np.zeros(5)
    for _ in range(8):
        n = mix(n, M @ n + c - n)
    assert np.max(np.abs(n - fixed)) < 1e-9 * np.max(np.abs(fixed))
    lin = np.zeros(5)
    for _ in range(8):
        lin = lin + 0.3 * (M @ lin + c - lin)
    assert np.max(np.abs(lin - fixed)) > 1e-2 * np.max(np.abs(fixed))


def test_scf_reaches_its_own_fixed_point():
    """A tiny sphere with two wells and 2 electrons (gap 0.67 Ha to the
    next level): after convergence the density is (to the tolerance) the
    ground-state density of the dense effective Hamiltonian built from it,
    and the solver's eigenvalues are that Hamiltonian's."""
    w = synthetic.make_workload("sphere_r12_h0.2", radius=2.4, h=0.3, nat=2, atom_radius=0.8, rc=1.0, nstates=6)
    g, atoms, H = hamiltonian.build_system(w)
    psi = synthetic.draw_states(synthetic.rng_after_atoms(w), 6, g.np)
    opts = scf.ScfOptions(nocc=1, eig_steps=3, mix=0.3, history=5, tol=1e-8)
    psi, hist = scf.scf(H, psi, opts, rmmdiis.Options(m=3, block=6, tol=1e-12), max_iter=80)
    assert hist[-1][0] < 1e-8
    n = scf.density(psi, 1)
    Heff = hamiltonian.Hamiltonian(g, scf.effective_potential(g, H.vloc, n), H.proj)
    ev, vec = np.linalg.eigh(Heff.dense())
    vec = vec / np.sqrt(g.dv)
    n_dense = scf.density(vec.T, 1)
    assert np.max(np.abs(n_dense - n)) < 1e-6 * np.max(n)
    assert np.max(np.abs(hist[-1][1][:4] - ev[:4])) < 1e-6
