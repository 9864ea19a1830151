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
