"""Oracle: Kleinman-Bylander non-local potential (TEST INFRASTRUCTURE ONLY).

Eq. (6), Sec. 5.3: V_nl phi(r) = sum_A sum_lm gamma_A,lm(r - R_A)
integral_{r' < r_c} gamma_A,lm(r' - R_A) phi(r') dr'.  Read with a diagonal
coupling D_A,i (the eq. writes it folded into gamma): V_nl = sum_A sum_i
|gamma_A,i> D_A,i <gamma_A,i|, the integral being h^3 times a sum over grid
points inside the projector sphere.  The paper computes it in two parts: the
projections (one integral per atom, projector and state) and the scatter
(multiply the stored integrals by the projector functions and sum); atoms
are split into groups whose spheres do not overlap (Fig. "colors").

Projector shapes: gamma_lm(r) = N_l r^l Y_lm(r/|r|) exp(-r^2/2s^2) for l = 0..l_max
(Sec. 5.3 lets l run to l_max, usually 3, and m from -l to l), with Y_lm the
real spherical harmonics, unit-normalised on the sphere, and N_l chosen so
that the continuum integral of gamma_lm^2 is one:
  int_0^inf r^(2l+2) exp(-r^2/s^2) dr = Gamma(l + 3/2) s^(2l+3) / 2.
r^l Y_lm is a harmonic polynomial of degree l (a solid harmonic).  Order of
the (l_max+1)^2 projectors of an atom: l ascending; within l = 1 the order
x, y, z; within l = 2: xy, yz, 3z^2 - r^2, xz, x^2 - y^2; within l = 3:
y(3x^2 - y^2), xyz, y(5z^2 - r^2), z(5z^2 - 3r^2), x(5z^2 - r^2),
z(x^2 - y^2), x(x^2 - 3y^2).  l <= 1 gives the s and p_x, p_y, p_z set of
the synthetic workloads: N_s exp(-r^2/2s^2), N_p x_a exp(-r^2/2s^2) with
N_s = (pi^1.5 s^3)^-1/2, N_p = (pi^1.5 s^5 / 2)^-1/2.  The sphere is inclusive,
|r_p - R_A|^2 <= r_c^2, with the squared distance formed as
((dx*dx + dy*dy) + dz*dz) without fused multiply-add; periodic grids use the
minimum image.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from .grid import Grid


def projector_norms(sigma: float):
    """(N_s, N_p) such that the continuum integrals of gamma^2 are one."""
    ns = (math.pi ** 1.5 * sigma ** 3) ** -0.5
    npn = (math.pi ** 1.5 * sigma ** 5 / 2.0) ** -0.5
    return ns, npn


def nproj(lmax: int) -> int:
    return (lmax + 1) ** 2


def radial_norm(l: int, sigma: float) -> float:
    """N_l: one over the square root of int_0^inf r^(2l+2) exp(-r^2/s^2) dr."""
    return (math.gamma(l + 1.5) * sigma ** (2 * l + 3) / 2.0) ** -0.5


def solid_harmonics(d: np.ndarray, lmax: int) -> np.ndarray:
    """r^l Y_lm(d/|d|) for l <= lmax at displacements d [n, 3]: the real
    spherical harmonics' Cartesian forms, [n, (lmax+1)^2] in the order of
    the module docstring."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    r2 = x * x + y * y + z * z
    pi = math.pi
    cols = [np.full_like(x, 0.5 / math.sqrt(pi))]
    if lmax >= 1:
        c1 = math.sqrt(3.0 / (4.0 * pi))
        cols += [c1 * x, c1 * y, c1 * z]
    if lmax >= 2:
        c2 = 0.5 * math.sqrt(15.0 / pi)
        cols += [c2 * x * y, c2 * y * z,
                 0.25 * math.sqrt(5.0 / pi) * (3.0 * z * z - r2),
                 c2 * x * z,
                 0.25 * math.sqrt(15.0 / pi) * (x * x - y * y)]
    if lmax >= 3:
        a = 0.25 * math.sqrt(35.0 / (2.0 * pi))
        b = 0.25 * math.sqrt(21.0 / (2.0 * pi))
        cols += [a * y * (3.0 * x * x - y * y),
                 0.5 * math.sqrt(105.0 / pi) * x * y * z,
                 b * y * (5.0 * z * z - r2),
                 0.25 * math.sqrt(7.0 / pi) * z * (5.0 * z * z - 3.0 * r2),
                 b * x * (5.0 * z * z - r2),
                 0.25 * math.sqrt(105.0 / pi) * z * (x * x - y * y),
                 a * x * (x * x - 3.0 * y * y)]
    return np.stack(cols, axis=1)


def projector_values(d: np.ndarray, lmax: int, sigma: float) -> np.ndarray:
    """gamma_lm at displacements d [n, 3] (no cut-off): [n, (lmax+1)^2]."""
    r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    e = np.exp(-r2 / (2.0 * sigma * sigma))
    S = solid_harmonics(d, lmax)
    out = np.empty_like(S)
    for l in range(lmax + 1):
        out[:, l * l:(l + 1) ** 2] = radial_norm(l, sigma) * S[:, l * l:(l + 1) ** 2] * e[:, None]
    return out


@dataclasses.dataclass
class ProjectorSet:
    idx: List[np.ndarray]      # per atom: inner-point indices in the sphere
    gamma: List[np.ndarray]    # per atom: [n_A, (l_max+1)^2]
    D: np.ndarray              # [nat, (l_max+1)^2]
    colour: np.ndarray         # [nat] colour group of each atom
    dv: float                  # h^3

    lmax: int = 1

    @property
    def nat(self) -> int:
        return len(self.idx)

    @property
    def nproj(self) -> int:
        return nproj(self.lmax)


def displacement(xyz: np.ndarray, X: np.ndarray,
                 box_length: Optional[float]) -> np.ndarray:
    d = xyz - X
    if box_length is not None:
        d = d - box_length * np.rint(d / box_length)
    return d


def colour_atoms(pos: np.ndarray, rc: float,
                 box_length: Optional[float] = None) -> np.ndarray:
    """Greedy colouring in atom order: each atom takes the smallest colour not
    used by an earlier atom whose sphere overlaps its own (|R_A - R_B| <= 2 r_c)."""
    nat = pos.shape[0]
    colour = np.full(nat, -1, dtype=np.int64)
    lim = (2.0 * rc) * (2.0 * rc)
    for a in range(nat):
        used = set()
        for b in range(a):
            d = displacement(pos[a][None, :], pos[b], box_length)[0]
            if (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2] <= lim:
                used.add(int(colour[b]))
        c = 0
        while c in used:
            c += 1
        colour[a] = c
    return colour


def build_projectors(g: Grid, pos: np.ndarray, D: np.ndarray, rc: float,
                     sigma: float, lmax: int = 1) -> ProjectorSet:
    """Sphere lists and projector values of every atom; D [nat, (lmax+1)^2]."""
    if not 0 <= lmax <= 3:
        raise ValueError("lmax must be 0..3")
    D = np.asarray(D, dtype=np.float64).reshape(pos.shape[0], nproj(lmax))
    xyz = g.xyz
    rc2 = rc * rc
    idx, gam = [], []
    for a in range(pos.shape[0]):
        d = displacement(xyz, pos[a], g.box_length)
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        sel = np.nonzero(r2 <= rc2)[0]
        idx.append(sel)
        gam.append(projector_values(d[sel], lmax, sigma))
    return ProjectorSet(idx=idx, gamma=gam, D=D, lmax=lmax,
                        colour=colour_atoms(pos, rc, g.box_length), dv=g.dv)


def project(ps: ProjectorSet, psi: np.ndarray) -> np.ndarray:
    """First part: P[k, A, i] = h^3 sum_{p in sphere A} gamma_A,i(p) psi_k(p)
    (psi may be complex; the projectors are real)."""
    x = np.atleast_2d(psi)
    P = np.zeros((x.shape[0], ps.nat, ps.nproj), dtype=np.result_type(x, np.float64))
    for a in range(ps.nat):
        P[:, a, :] = ps.dv * (x[:, ps.idx[a]] @ ps.gamma[a])
    return P


def apply_projections(ps: ProjectorSet, P: np.ndarray, npoints: int) -> np.ndarray:
    """Second part: sum_A sum_i gamma_A,i(r) D_A,i P[k, A, i], done one colour
    group at a time (within a group the spheres are disjoint)."""
    out = np.zeros((P.shape[0], npoints), dtype=np.result_type(P, np.float64))
    for col in range(int(ps.colour.max()) + 1 if ps.nat else 0):
        for a in np.nonzero(ps.colour == col)[0]:
            out[:, ps.idx[a]] += (P[:, a, :] * ps.D[a]) @ ps.gamma[a].T
    return out


def apply_nonlocal(ps: ProjectorSet, psi: np.ndarray) -> np.ndarray:
    x = np.atleast_2d(psi)
    out = apply_projections(ps, project(ps, x), x.shape[1])
    return out if psi.ndim == 2 else out[0]
