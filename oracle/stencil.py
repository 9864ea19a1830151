"""Oracle: finite-difference kinetic operator and local potential
(TEST INFRASTRUCTURE ONLY).

Sec. 5.1: the kinetic energy -1/2 nabla^2 is a high-order finite-difference
stencil, a weighted sum of neighbour values; the paper's "fourth-order"
approximation has 25 points in 3-D, read as a star with 4 neighbours per side
on each axis (1 + 3*2*4 = 25).  Sec. 5.2: the local potential is a pointwise
product with one summed potential field.

Weights are the unique central weights that make the 1-D rule exact for
polynomials of the highest possible degree; they are derived here from the
Taylor-moment equations in exact rational arithmetic.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence

import numpy as np

from .grid import Grid, neighbour_table


def fd_weights_exact(M: int) -> List[Fraction]:
    """c_0..c_M with f''(0) h^2 ~ c_0 f(0) + sum_m c_m (f(mh) + f(-mh)).

    Conditions: for f = x^(2k), k = 0..M, the rule reproduces the exact
    second derivative at 0, i.e. sum_{m=-M..M} c_|m| m^(2k) = 2 [k == 1].
    Solved by Gauss-Jordan elimination over the rationals.
    """
    n = M + 1
    A = [[Fraction(0)] * n for _ in range(n)]
    b = [Fraction(0)] * n
    for k in range(n):
        A[k][0] = Fraction(1 if k == 0 else 0)       # the centre, m = 0
        for m in range(1, M + 1):
            A[k][m] = Fraction(2 * m ** (2 * k))
        b[k] = Fraction(2 if k == 1 else 0)
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        inv = 1 / A[col][col]
        A[col] = [a * inv for a in A[col]]
        b[col] *= inv
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [a - f * c for a, c in zip(A[r], A[col])]
                b[r] -= f * b[col]
    return b


def fd_weights(M: int = 4) -> np.ndarray:
    return np.array([float(c) for c in fd_weights_exact(M)])


def kinetic_symbol(k: np.ndarray, h: float, M: int = 4) -> np.ndarray:
    """Eigenvalue of the discrete -1/2 nabla^2 on a plane wave exp(i k.r),
    k [..., 3]: -1/(2h^2) sum_a [c_0 + 2 sum_m c_m cos(m k_a h)]."""
    c = fd_weights(M)
    tot = 0.0
    for a in range(3):
        s = c[0] + sum(2.0 * c[m] * np.cos(m * k[..., a] * h)
                       for m in range(1, M + 1))
        tot = tot + s
    return -0.5 * tot / h ** 2


def apply_kinetic(g: Grid, psi: np.ndarray, nbr: np.ndarray = None) -> np.ndarray:
    """T psi for state-major psi [N, np] (or [np]); values outside the
    domain are zero (Dirichlet) or wrap (periodic)."""
    if nbr is None:
        nbr = neighbour_table(g)
    c = fd_weights(g.M)
    x = np.atleast_2d(psi)
    N = x.shape[0]
    xp = np.concatenate([x, np.zeros((N, 1))], axis=1)   # index -1 -> 0
    idx = np.where(nbr < 0, g.np, nbr)
    lap = 3.0 * c[0] * x
    for a in range(3):
        for m in range(1, g.M + 1):
            lap = lap + c[m] * (xp[:, idx[:, a, 0, m - 1]]
                                + xp[:, idx[:, a, 1, m - 1]])
    out = -0.5 / g.h ** 2 * lap
    return out if psi.ndim == 2 else out[0]


def apply_local(g: Grid, vloc: np.ndarray, psi: np.ndarray,
                nbr: np.ndarray = None) -> np.ndarray:
    """(T + V) psi: the kinetic stencil plus the local-potential product."""
    return apply_kinetic(g, psi, nbr) + vloc * psi


def apply_local_at(g: Grid, vloc: np.ndarray, psi: np.ndarray,
                   points: Sequence[int]) -> np.ndarray:
    """(T + V) psi evaluated only at the given point indices, one point at a
    time (for sampling outputs of very large grids).  Returns [N, len(points)]."""
    c = fd_weights(g.M)
    x = np.atleast_2d(psi)
    out = np.empty((x.shape[0], len(points)))
    for j, p in enumerate(points):
        u = g.inner[p] - g.lo
        acc = 3.0 * c[0] * x[:, p]
        for a in range(3):
            for m in range(1, g.M + 1):
                for sgn in (1, -1):
                    v = u.copy()
                    v[a] += sgn * m
                    if g.periodic:
                        v[a] %= g.L[a]
                    q = g.lookup[v[2], v[1], v[0]]
                    if q >= 0:
                        acc = acc + c[m] * x[:, q]
        out[:, j] = -0.5 / g.h ** 2 * acc + vloc[p] * x[:, p]
    return out
