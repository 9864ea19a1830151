"""Pins of the oracle's Kleinman-Bylander non-local potential (CPU only)."""
import numpy as np
import pytest

import synthetic
from oracle import grid, hamiltonian, kb


def _single_atom(h=0.2, R=4.0, pos=(0.0, 0.0, 0.0), D=(2.0, 1.0, 1.0, 1.0)):
    g = grid.build_grid("sphere", h, radius=R)
    ps = kb.build_projectors(g, np.array([pos]), np.array([D]), rc=2.5, sigma=0.7)
    return g, ps


def test_projector_normalisation_and_symmetry():
    """Continuum-normalised s and p Gaussians: the grid Gram matrix is the
    identity up to cut-off and quadrature error; s-p and p-p' overlaps vanish
    by symmetry for an atom on a grid point."""
    g, ps = _single_atom()
    G = g.dv * ps.gamma[0].T @ ps.gamma[0]
    assert np.allclose(np.diag(G), 1.0, atol=1e-4)
    off = G - np.diag(np.diag(G))
    assert np.max(np.abs(off)) < 1e-14
    # all three p projectors have the same norm (cubic symmetry)
    assert np.ptp(np.diag(G)[1:]) < 1e-14


def test_projector_is_eigenvector_of_vnl():
    """For one atom with a diagonal Gram matrix, V_nl gamma_i = D_i G_ii gamma_i."""
    g, ps = _single_atom()
    G = g.dv * ps.gamma[0].T @ ps.gamma[0]
    for i in range(4):
        f = np.zeros(g.np)
        f[ps.idx[0]] = ps.gamma[0][:, i]
        out = kb.apply_nonlocal(ps, f)
        lam = ps.D[0, i] * G[i, i]
        assert np.max(np.abs(out - lam * f)) < 1e-13 * np.max(np.abs(f))


def test_sphere_membership_inclusive_and_count():
    g, ps = _single_atom(h=0.5)
    # points at distance exactly 2.5 = 5 h (integer offsets (5,0,0), (3,4,0), ...)
    d2 = (ps_idx_xyz := g.xyz[ps.idx[0]]) @ np.ones(3)  # noqa: F841 (shape check)
    r2 = (g.xyz[ps.idx[0]] ** 2).sum(1)
    assert np.max(r2) == pytest.approx(6.25)
    # count = integer points with i^2+j^2+k^2 <= 25
    cnt = sum(1 for i in range(-5, 6) for j in range(-5, 6) for k in range(-5, 6)
              if i * i + j * j + k * k <= 25)
    assert len(ps.idx[0]) == cnt


def test_hermitian_and_rank_with_overlaps():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=1.6, h=0.25, nat=3, atom_radius=0.6, rc=1.0)
    g, atoms, H = hamiltonian.build_system(w)
    ps = H.proj
    assert ps.colour.max() >= 1          # spheres overlap, so >= 2 colours
    rng = np.random.default_rng(3)
    a, b = rng.uniform(-1, 1, size=(2, g.np))
    va, vb = kb.apply_nonlocal(ps, a), kb.apply_nonlocal(ps, b)
    assert abs(a @ vb - va @ b) < 1e-13 * np.linalg.norm(a) * np.linalg.norm(vb)
    Vd = kb.apply_nonlocal(ps, np.eye(g.np))
    s = np.linalg.svd(Vd, compute_uv=False)
    assert np.sum(s > 1e-10 * s[0]) <= 4 * ps.nat


def test_coloured_scatter_equals_plain_sum():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=3.0, nat=6, atom_radius=1.5)
    g, atoms, H = hamiltonian.build_system(w)
    ps = H.proj
    rng = np.random.default_rng(4)
    psi = rng.uniform(-1, 1, size=(2, g.np))
    P = kb.project(ps, psi)
    want = np.zeros_like(psi)
    for a in range(ps.nat):                   # every atom, in index order
        for i in range(4):
            for k in range(2):
                want[k, ps.idx[a]] += ps.gamma[a][:, i] * ps.D[a, i] * P[k, a, i]
    got = kb.apply_projections(ps, P, g.np)
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))


def test_colouring_greedy_and_disjoint():
    rng = np.random.default_rng(5)
    pos = rng.uniform(-4, 4, size=(30, 3))
    rc = 1.5
    col = kb.colour_atoms(pos, rc)
    d = np.linalg.norm(pos[:, None] - pos[None], axis=2)
    conflict = d <= 2 * rc
    for a in range(30):
        for b in range(a):
            if conflict[a, b]:
                assert col[a] != col[b]
        for c in range(col[a]):            # smallest free colour
            assert any(conflict[a, b] and col[b] == c for b in range(a))


def test_periodic_minimum_image():
    g = grid.build_grid("periodic", 0.25, n=24)
    L = 24 * 0.25
    D = np.array([[1.0, 1.0, 1.0, 1.0]] * 2)
    pos = np.array([[3.0, 3.0, 3.0], [0.0, 0.0, 0.0]])      # centre and corner
    ps = kb.build_projectors(g, pos, D, rc=1.3, sigma=0.5)
    assert len(ps.idx[0]) == len(ps.idx[1])
    G0 = ps.gamma[0].T @ ps.gamma[0]
    G1 = ps.gamma[1].T @ ps.gamma[1]
    assert np.allclose(G0, G1, atol=1e-13)


# ---------------------------------------------------------------- l <= 3
def _sphere_rule(nt=8, nphi=16):
    """Product rule on the unit sphere, exact for polynomials of degree <= 15:
    Gauss-Legendre in cos(theta) times the trapezoid in phi."""
    x, w = np.polynomial.legendre.leggauss(nt)
    phi = 2.0 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1.0 - ct * ct)
    u = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    wt = (w[:, None] * np.full(nphi, 2.0 * np.pi / nphi)[None, :]).reshape(-1)
    return u, wt


def test_real_harmonics_orthonormal_on_sphere():
    """int Y_i Y_j dOmega = delta_ij for all 16 functions of l <= 3 (a wrong
    constant, a wrong polynomial or a repeated function fails this)."""
    u, wt = _sphere_rule()
    Y = kb.solid_harmonics(u, 3)                 # r = 1
    G = (Y * wt[:, None]).T @ Y
    assert np.max(np.abs(G - np.eye(16))) < 1e-14


def test_addition_theorem():
    """sum_m Y_lm(u)^2 = (2l + 1) / (4 pi) for every direction u and each l."""
    u = np.random.default_rng(11).normal(size=(50, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    Y = kb.solid_harmonics(u, 3)
    for l in range(4):
        s = np.sum(Y[:, l * l:(l + 1) ** 2] ** 2, axis=1)
        assert np.allclose(s, (2 * l + 1) / (4 * np.pi), rtol=0, atol=1e-15)


def test_solid_harmonics_are_harmonic():
    """r^l Y_lm has zero Laplacian; for polynomials of degree <= 3 the second
    central difference with unit step equals the second derivative exactly."""
    rng = np.random.default_rng(12)
    d = rng.uniform(-2, 2, size=(40, 3))
    lap = -6.0 * kb.solid_harmonics(d, 3)
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1.0
        lap += kb.solid_harmonics(d + e, 3) + kb.solid_harmonics(d - e, 3)
    assert np.max(np.abs(lap)) < 1e-12
    # degree and parity: scaling d by t scales the l block by t^l
    t = 1.7
    for l in range(4):
        sl = slice(l * l, (l + 1) ** 2)
        assert np.allclose(kb.solid_harmonics(t * d, 3)[:, sl], t ** l * kb.solid_harmonics(d, 3)[:, sl],
                           rtol=1e-13, atol=1e-13)


def test_radial_norm_by_quadrature():
    from scipy.integrate import quad
    for l in range(4):
        for sigma in (0.5, 0.9):
            N = kb.radial_norm(l, sigma)
            val, _ = quad(lambda r: N * N * r ** (2 * l + 2) * np.exp(-r * r / sigma ** 2), 0, np.inf,
                          epsabs=1e-14, epsrel=1e-13)
            assert val == pytest.approx(1.0, abs=1e-12)


def test_lmax3_projectors_orthonormal_on_fine_grid():
    """The 16 projectors of one atom are orthonormal in the continuum; on a
    grid with h << sigma the grid Gram matrix is the identity to quadrature
    precision (off the grid point too), and l <= 1 reproduces the s/p set."""
    g = grid.build_grid("sphere", 0.14, radius=4.6)
    pos = np.array([[0.031, -0.047, 0.022]])
    ps = kb.build_projectors(g, pos, np.ones((1, 16)), rc=4.5, sigma=0.7, lmax=3)
    G = g.dv * ps.gamma[0].T @ ps.gamma[0]
    assert np.max(np.abs(G - np.eye(16))) < 1e-10
    ps1 = kb.build_projectors(g, pos, np.ones((1, 4)), rc=4.5, sigma=0.7, lmax=1)
    assert np.allclose(ps1.gamma[0], ps.gamma[0][:, :4], rtol=1e-14, atol=1e-16)
    ns, npn = kb.projector_norms(0.7)
    d = g.xyz[ps.idx[0]] - pos[0]
    e = np.exp(-(d * d).sum(1) / (2 * 0.49))
    assert np.allclose(ps1.gamma[0], np.c_[ns * e, npn * d * e[:, None]], rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("lmax", [0, 2, 3])
def test_vnl_hermitian_rank_and_scatter_lmax(lmax):
    """V_nl with (lmax+1)^2 projectors per atom: symmetric, rank <= nproj * nat,
    and the coloured scatter equals the plain per-atom sum."""
    w = synthetic.make_workload("sphere_r12_h0.2", radius=1.6, h=0.25, nat=3, atom_radius=0.6, rc=1.0)
    g, atoms, _ = hamiltonian.build_system(w, with_projectors=False)
    npj = (lmax + 1) ** 2
    D = np.random.default_rng(20 + lmax).uniform(0.5, 2.0, size=(atoms.pos.shape[0], npj))
    ps = kb.build_projectors(g, atoms.pos, D, w.rc, w.sigma, lmax=lmax)
    assert ps.gamma[0].shape[1] == npj
    Vd = kb.apply_nonlocal(ps, np.eye(g.np))
    assert np.max(np.abs(Vd - Vd.T)) < 1e-13 * np.max(np.abs(Vd))
    s = np.linalg.svd(Vd, compute_uv=False)
    assert np.sum(s > 1e-10 * s[0]) <= npj * ps.nat
    # brute force: V = h^3 sum_A sum_i D_Ai g_Ai g_Ai^T on the full grid
    want = np.zeros((g.np, g.np))
    for a in range(ps.nat):
        for i in range(npj):
            f = np.zeros(g.np)
            f[ps.idx[a]] = ps.gamma[a][:, i]
            want += g.dv * D[a, i] * np.outer(f, f)
    assert np.max(np.abs(Vd - want)) < 1e-13 * np.max(np.abs(want))


def test_complex_states_split_into_real_and_imaginary_parts():
    """The projectors are real, so V_nl (a + i b) = V_nl a + i V_nl b and the
    projections of a complex state are P(a) + i P(b)."""
    w = synthetic.make_workload("sphere_r12_h0.2", radius=1.6, h=0.25, nat=3, atom_radius=0.6, rc=1.0)
    g, atoms, _ = hamiltonian.build_system(w, with_projectors=False)
    ps = kb.build_projectors(g, atoms.pos, np.ones((atoms.pos.shape[0], 9)), w.rc, w.sigma, lmax=2)
    rng = np.random.default_rng(21)
    a, b = rng.uniform(-1, 1, size=(2, 3, g.np))
    z = a + 1j * b
    assert np.allclose(kb.project(ps, z), kb.project(ps, a) + 1j * kb.project(ps, b), rtol=0, atol=1e-15)
    assert np.allclose(kb.apply_nonlocal(ps, z), kb.apply_nonlocal(ps, a) + 1j * kb.apply_nonlocal(ps, b),
                       rtol=0, atol=1e-14)
    # Hermitian on complex states: <x|V y> = conj(<y|V x>)
    x, y = z[0], z[1]
    lhs = np.vdot(x, kb.apply_nonlocal(ps, y))
    rhs = np.conj(np.vdot(y, kb.apply_nonlocal(ps, x)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
