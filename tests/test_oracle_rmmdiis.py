"""Pins of the oracle's RMM-DIIS step, filter preconditioner and converged
eigenvalues (CPU only)."""
import numpy as np
import pytest
import scipy.optimize

import synthetic
from oracle import grid, hamiltonian, linalg, rmmdiis, stencil


@pytest.mark.parametrize("alpha", [0.5, 0.6, None])
def test_filter_symbol_on_plane_waves(alpha):
    """K on plane waves of a periodic grid: the closed-form symbol
    a + (1 - a)/3 sum cos(k h), 1 at k = 0 and 2a - 1 at the Nyquist corner
    (zero for a = 1/2; None = the default centre weight, 0.52)."""
    n, h = 12, 0.25
    g = grid.build_grid("periodic", h, n=n)
    L = n * h
    a = rmmdiis.Options().alpha if alpha is None else alpha
    kw = {} if alpha is None else {"alpha": alpha}
    for nvec in [(0, 0, 0), (1, 2, 0), (6, 6, 6), (6, 0, 0), (3, 5, 1)]:
        k = 2 * np.pi * np.array(nvec) / L
        f = np.cos(g.xyz @ k)
        got = rmmdiis.filter_precond(g, f, **kw)
        sym = a + (1.0 - a) / 3 * np.sum(np.cos(k * h))
        assert np.max(np.abs(got - sym * f)) < 1e-13
    f = np.cos(g.xyz @ (np.pi / h * np.ones(3)))
    assert np.max(np.abs(rmmdiis.filter_precond(g, f, **kw) - (2 * a - 1) * f)) < 1e-13


@pytest.mark.parametrize("alpha", [0.5, 0.6])
def test_filter_zero_outside_domain(alpha):
    g = grid.build_grid("box", 0.3, n=4)
    f = np.ones(g.np)
    out = rmmdiis.filter_precond(g, f, alpha=alpha)
    corner = np.nonzero(np.all(g.inner == 0, axis=1))[0][0]
    centre = np.nonzero(np.all(g.inner == 1, axis=1))[0][0]
    assert out[corner] == pytest.approx(alpha + (1 - alpha) / 6 * 3)
    assert out[centre] == pytest.approx(1.0)


def test_periodic_even_box_converges_to_dense_spectrum():
    """Periodic 16^3 box (even edges, so the alternating vector is a grid
    mode) with wells and projectors: from random states the default filter
    reaches the lowest eigenvalues of the dense matrix.  With alpha = 1/2
    the same solve keeps a residual floor, because K then annihilates that
    mode and the random start's component along it can never be removed."""
    w = synthetic.make_workload("periodic96_h0.25", n=16, nat=1, nstates=12, block=4)
    g, atoms, H = hamiltonian.build_system(w)
    ev = np.linalg.eigvalsh(H.dense())[:8]
    psi0 = synthetic.draw_states(synthetic.rng_after_atoms(w), 12, g.np)
    floors = {}
    a0 = rmmdiis.Options().alpha
    for alpha in (a0, 0.6, 0.5):
        opts = rmmdiis.Options(m=3, block=4, tol=1e-12, alpha=alpha)
        psi, hist = rmmdiis.eigensolve(H, psi0, opts, max_steps=150, eref=ev if alpha > 0.5 else None,
                                       etol=1e-10)
        eig, res = hist[-1]
        floors[alpha] = res[:8].max()
        if alpha > 0.5:
            assert np.max(np.abs(eig[:8] - ev)) < 1e-10
    assert floors[0.5] > 1e-4 and floors[0.5] > 1e3 * max(floors[0.6], floors[a0])


def test_trial_lambda_minimises_rayleigh_quotient():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=1.6, h=0.25, nat=2, atom_radius=0.6, rc=1.0)
    g, _, H = hamiltonian.build_system(w)
    rng = np.random.default_rng(7)
    dv = g.dv
    for _ in range(4):
        p = rng.uniform(-1, 1, g.np)
        d = rng.uniform(-1, 1, g.np)
        hp, hd = H.apply(p), H.apply(d)
        lam = rmmdiis.trial_lambda(dv * p @ hp, dv * 0.5 * (p @ hd + d @ hp), dv * d @ hd,
                                   dv * p @ p, dv * p @ d, dv * d @ d)
        rq = lambda t: ((p + t * d) @ H.apply(p + t * d)) / ((p + t * d) @ (p + t * d))
        best = scipy.optimize.minimize_scalar(rq, bracket=(lam - 1, lam, lam + 1), tol=1e-12)
        assert rq(lam) <= best.fun + 1e-10 * abs(best.fun)


def test_trial_mix_minimises_rayleigh_quotient():
    """The filter/network coefficients (a, b) of the learned trial step are
    the minimiser of the Rayleigh quotient of psi + a d + b e: no point found
    by Nelder-Mead from around them is lower, and a network direction that
    is a multiple of the filter's is reported singular."""
    w = synthetic.make_workload("sphere_r12_h0.2", radius=1.6, h=0.25, nat=2, atom_radius=0.6, rc=1.0)
    g, _, H = hamiltonian.build_system(w)
    rng = np.random.default_rng(9)
    dv = g.dv
    for _ in range(3):
        v = [rng.uniform(-1, 1, g.np) for _ in range(3)]
        hv = [H.apply(x) for x in v]
        A = np.array([[0.5 * dv * (v[i] @ hv[j] + v[j] @ hv[i]) for j in range(3)] for i in range(3)])
        Bq = np.array([[dv * (v[i] @ v[j]) for j in range(3)] for i in range(3)])
        a, b = rmmdiis.trial_mix(A, Bq)
        def rq(t):
            x = v[0] + t[0] * v[1] + t[1] * v[2]
            return (x @ H.apply(x)) / (x @ x)
        best = scipy.optimize.minimize(rq, [a, b], method="Nelder-Mead",
                                       options=dict(xatol=1e-10, fatol=1e-14, maxiter=4000))
        assert rq([a, b]) <= best.fun + 1e-10 * abs(best.fun)
        A2 = A.copy(); B2 = Bq.copy()
        A2[2], A2[:, 2] = 2 * A[1], 2 * A[:, 1]
        A2[2, 2] = 4 * A[1, 1]
        B2[2], B2[:, 2] = 2 * Bq[1], 2 * Bq[:, 1]
        B2[2, 2] = 4 * Bq[1, 1]
        assert rmmdiis.trial_mix(A2, B2) is None


def test_step_with_zero_network_is_the_filter_step():
    """A network that outputs zero (all weights zero) makes every 3x3 trial
    problem singular, so the step with it is exactly the filter's step."""
    from oracle import cnn
    w = synthetic.make_workload("periodic96_h0.25", n=12, nat=1, nstates=8, block=4)
    g, atoms, H = hamiltonian.build_system(w)
    psi, _, _ = linalg.orthonormalize(synthetic.draw_states(synthetic.rng_after_atoms(w), 8, g.np), g.dv)
    opts = rmmdiis.Options(m=3, block=4, tol=1e-12)
    p = np.zeros(cnn.NP)
    a = rmmdiis.rmmdiis_step(H, psi, opts)
    b = rmmdiis.rmmdiis_step(H, psi, opts, net=p)
    assert np.array_equal(a["psi"], b["psi"])
    assert np.all(b["mix"][:, 1] == 0.0)


def test_step_with_exact_inverse_beats_filter():
    """A direction that the trial subspace can use well: with (T - sigma)^-1
    r (the target the network is trained on, closed form on a periodic box)
    standing in for the network, the step's Rayleigh quotients are never
    above the filter step's and the network coefficient is nonzero."""
    from oracle import cnn
    w = synthetic.make_workload("periodic96_h0.25", n=12, nat=1, nstates=8, block=4)
    g, atoms, H = hamiltonian.build_system(w)
    psi, _, _ = linalg.orthonormalize(synthetic.draw_states(synthetic.rng_after_atoms(w), 8, g.np), g.dv)
    opts = rmmdiis.Options(m=1, block=4, tol=1e-12)
    orig = cnn.precondition
    try:
        cnn.precondition = lambda params, gg, r, sig: cnn.shifted_inverse_periodic(gg, r, sig)
        withnet = rmmdiis.rmmdiis_step(H, psi, opts, net=np.zeros(cnn.NP))
    finally:
        cnn.precondition = orig
    plain = rmmdiis.rmmdiis_step(H, psi, opts)
    assert np.all(withnet["mix"][:, 1] != 0.0)
    # m = 1: the returned states are the trial iterates, orthonormalised; the
    # Rayleigh-Ritz values of the new subspace are lower with the network
    def rr(x):
        return linalg.rayleigh_ritz(x, H.apply(x), g.dv)[0]
    assert np.sum(rr(withnet["psi"])) < np.sum(rr(plain["psi"]))


def test_diis_coefficients_minimise_ratio():
    rng = np.random.default_rng(8)
    for n in (2, 3):
        X = rng.normal(size=(n, 50))
        Y = rng.normal(size=(n, 50))
        A, B = X @ X.T, Y @ Y.T
        c = rmmdiis.diis_coefficients(A, B)
        assert c[0] == 1.0
        f = lambda z: (np.r_[1.0, z] @ A @ np.r_[1.0, z]) / (np.r_[1.0, z] @ B @ np.r_[1.0, z])
        best = scipy.optimize.minimize(f, np.zeros(n - 1), method="Nelder-Mead",
                                       options=dict(xatol=1e-12, fatol=1e-14, maxiter=20000))
        assert f(c[1:]) <= best.fun + 1e-9 * best.fun
    # singular B falls back to keeping the latest iterate
    c = rmmdiis.diis_coefficients(np.eye(2), np.zeros((2, 2)))
    assert list(c) == [1.0, 0.0]


def test_converged_eigenvalues_harmonic_box():
    """Lowest four levels of the 32^3 harmonic box (exact discrete values from
    the separable 1-D problems) from random starts."""
    w = synthetic.make_workload("box32_harmonic", nstates=4)
    g, _, H = hamiltonian.build_system(w)
    psi = synthetic.draw_states(synthetic.rng_after_atoms(w), 4, g.np)
    psi, hist = rmmdiis.eigensolve(H, psi, rmmdiis.Options(block=4, tol=1e-9), 120)
    want = np.array([1.4999991750, 2.4999964915, 2.4999964915, 2.4999964915])
    assert np.max(np.abs(hist[-1][0] - want)) < 1e-9
    assert np.max(hist[-1][1]) < 1e-9


def test_converged_eigenvalues_dense_bruteforce():
    """Tiny sphere with wells and projectors: the eigensolver reaches the
    lowest eigenvalues of the assembled dense matrix."""
    w = synthetic.make_workload("sphere_r12_h0.2", radius=1.6, h=0.2, nat=2, atom_radius=0.6, rc=1.0)
    g, _, H = hamiltonian.build_system(w)
    ev = np.linalg.eigvalsh(H.dense())
    psi = synthetic.draw_states(synthetic.rng_after_atoms(w), 4, g.np)
    psi, hist = rmmdiis.eigensolve(H, psi, rmmdiis.Options(block=4, tol=1e-9), 300)
    assert np.max(np.abs(hist[-1][0] - ev[:4])) < 1e-10


def test_step_keeps_orthonormality_and_block_stop():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=2.0, nat=2, atom_radius=0.8)
    g, _, H = hamiltonian.build_system(w)
    psi = synthetic.draw_states(synthetic.rng_after_atoms(w), 8, g.np)
    psi, _, _ = linalg.orthonormalize(psi, g.dv)
    out = rmmdiis.rmmdiis_step(H, psi, rmmdiis.Options(block=4))
    assert np.allclose(g.dv * out["psi"] @ out["psi"].T, np.eye(8), atol=1e-12)
    assert np.all(np.diff(out["eig"]) >= 0)
    # with a huge tolerance every block is frozen: the step is RR + ortho only
    frozen = rmmdiis.rmmdiis_step(H, psi, rmmdiis.Options(block=4, tol=1e9))
    assert not frozen["active"].any()
    lam, xi, p2, _ = linalg.rayleigh_ritz(psi, H.apply(psi), g.dv)
    p2, _, _ = linalg.orthonormalize(p2, g.dv)
    assert np.allclose(frozen["psi"], p2, atol=1e-10)
