"""Pins of the oracle's kinetic stencil and local potential (CPU only)."""
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import synthetic
from oracle import grid, hamiltonian, stencil

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_weights_match_textbook_table():
    rows = [l.strip() for l in open(os.path.join(GOLDEN, "fd_weights_m4.txt"))
            if l.strip() and not l.startswith("#")]
    want = [Fraction(r) for r in rows]
    assert stencil.fd_weights_exact(4) == want
    # lower orders reproduce the classic 3-, 5- and 7-point rules
    assert stencil.fd_weights_exact(1) == [Fraction(-2), Fraction(1)]
    assert stencil.fd_weights_exact(2) == [Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)]
    c = stencil.fd_weights_exact(4)
    assert c[0] + 2 * sum(c[1:]) == 0


def _box(n=24, h=0.3):
    return grid.build_grid("box", h, n=n)


def test_polynomial_exactness():
    """T is exact on x^a y^b z^c (each power <= 9) away from the faces;
    a 10th power is not reproduced."""
    g = _box()
    L = g.n * g.h
    x, y, z = (g.xyz / L).T
    u = g.inner
    far = np.all((u >= 4) & (u < g.n - 4), axis=1)
    s = 1.0 / L      # d/dx of the scaled coordinate
    for (a, b, c) in [(9, 0, 0), (0, 9, 0), (0, 0, 9), (4, 5, 3), (9, 9, 9), (2, 7, 8)]:
        f = x ** a * y ** b * z ** c
        lap = 0.0
        if a >= 2:
            lap = lap + a * (a - 1) * x ** (a - 2) * y ** b * z ** c * s * s
        if b >= 2:
            lap = lap + b * (b - 1) * x ** a * y ** (b - 2) * z ** c * s * s
        if c >= 2:
            lap = lap + c * (c - 1) * x ** a * y ** b * z ** (c - 2) * s * s
        want = -0.5 * lap
        got = stencil.apply_kinetic(g, f)
        scale = np.max(np.abs(f[far])) / g.h ** 2
        err = np.max(np.abs(got[far] - want[far] if np.ndim(want) else got[far]))
        assert err <= 1e-12 * scale, (a, b, c, err / scale)
    f = x ** 10
    want = -0.5 * 90 * x ** 8 * s * s
    got = stencil.apply_kinetic(g, f)
    scale = np.max(np.abs(f[far])) / g.h ** 2
    assert np.max(np.abs(got[far] - want[far])) > 1e-9 * scale


def test_plane_wave_symbol_and_continuum_limit():
    n, h = 16, 0.25
    g = grid.build_grid("periodic", h, n=n)
    L = n * h
    r = g.xyz
    for nvec in [(1, 0, 0), (0, 2, 3), (8, 0, 0), (5, 7, 8), (8, 8, 8)]:
        k = 2 * np.pi * np.array(nvec) / L
        for f in (np.cos(r @ k), np.sin(r @ k)):
            got = stencil.apply_kinetic(g, f)
            sym = stencil.kinetic_symbol(k, h)
            assert np.max(np.abs(got - sym * f)) <= 1e-12 * max(abs(sym), 1.0)
    # small k: symbol -> |k|^2/2 with an O((kh)^8) error
    k = np.array([0.05, 0.03, 0.02]) / h
    sym = stencil.kinetic_symbol(k, h)
    assert abs(sym - 0.5 * k @ k) <= 1e-3 * (0.05 ** 8) / h ** 2
    # Nyquist value per axis
    ny = stencil.kinetic_symbol(np.array([np.pi / h, 0, 0]), h)
    c = stencil.fd_weights(4)
    assert abs(ny * h * h + 0.5 * (c[0] + 2 * (-c[1] + c[2] - c[3] + c[4]))) < 1e-14
    assert abs(ny * h * h - 3.2507936507936506) < 1e-12


def _one_d_harmonic(n=32, h=0.3):
    """1-D Dirichlet cell-centred problem -1/2 d2/dx2 + x^2/2, banded form,
    solved with LAPACK's banded symmetric eigensolver."""
    c = stencil.fd_weights(4)
    x = (np.arange(n) - 0.5 * (n - 1)) * h
    ab = np.zeros((5, n))
    ab[0] = -0.5 * c[0] / h ** 2 + 0.5 * x * x
    for m in range(1, 5):
        ab[m, : n - m] = -0.5 * c[m] / h ** 2
    e, v = scipy.linalg.eig_banded(ab, lower=True)
    return e, v


def test_config1_separable_operator():
    """The star stencil and V = r^2/2 are sums of 1-D operators: products of
    1-D eigenvectors are eigenvectors of the 3-D operator with summed
    eigenvalues."""
    w = synthetic.WORKLOADS["box32_harmonic"]
    g, _, H = hamiltonian.build_system(w)
    e, v = _one_d_harmonic()
    u = g.inner          # integer coordinates 0..31 per axis
    for (i, j, k) in [(0, 0, 0), (1, 0, 0), (0, 2, 1), (3, 1, 2)]:
        f = v[u[:, 0], i] * v[u[:, 1], j] * v[u[:, 2], k]
        got = H.apply(f)
        lam = e[i] + e[j] + e[k]
        assert np.max(np.abs(got - lam * f)) < 1e-12 * (abs(lam) + 1 / g.h ** 2)
    # lowest 3-D levels of the 32^3 box
    lev = np.sort((e[:6, None, None] + e[None, :6, None] + e[None, None, :6]).ravel())[:10]
    want = [1.4999991750, 2.4999964915, 2.4999964915, 2.4999964915,
            3.4999835553, 3.4999835553, 3.4999835553,
            3.4999938080, 3.4999938080, 3.4999938080]
    assert np.allclose(lev, want, atol=2e-10)
    assert np.allclose(lev[:4], [1.5, 2.5, 2.5, 2.5], atol=2e-5)


def test_local_at_matches_full():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=2.0, nat=0)
    g, _, H = hamiltonian.build_system(w)
    rng = np.random.default_rng(0)
    psi = rng.uniform(-1, 1, size=(3, g.np))
    full = H.apply(psi)
    pts = rng.choice(g.np, 40, replace=False)
    part = stencil.apply_local_at(g, H.vloc, psi, pts)
    assert np.max(np.abs(part - full[:, pts])) < 1e-12 * np.max(np.abs(full))


def test_hermitian_local():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=2.2, nat=0)
    g, _, H = hamiltonian.build_system(w)
    rng = np.random.default_rng(1)
    a, b = rng.uniform(-1, 1, size=(2, g.np))
    lhs = a @ H.apply(b)
    rhs = H.apply(a) @ b
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.linalg.norm(a) * np.linalg.norm(b) / g.h ** 2)
