"""Oracle: Kleinman-Bylander non-local potential (TEST INFRASTRUCTURE ONLY).

Eq. (6), Sec. 5.3: V_nl phi(r) = sum_A sum_lm gamma_A,lm(r - R_A)
integral_{r' < r_c} gamma_A,lm(r' - R_A) phi(r') dr'.  Read with a diagonal
coupling D_A,i (the eq. writes it folded into gamma): V_nl = sum_A sum_i
|gamma_A,i> D_A,i <gamma_A,i|, the integral being h^3 times a sum over grid
points inside the projector sphere.  The paper computes it in two parts: the
projections (one integral per atom, projector and state) and the scatter
(multiply the stored integrals by the projector functions and sum); atoms
are split into groups whose spheres do not overlap (Fig. "colors").

Projector shapes of the synthetic workloads (l <= 1): s = N_s exp(-r^2/2s^2),
p_a = N_p x_a exp(-r^2/2s^2), continuum-normalised.  The sphere is inclusive,
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


@dataclasses.dataclass
class ProjectorSet:
    idx: List[np.ndarray]      # per atom: inner-point indices in the sphere
    gamma: List[np.ndarray]    # per atom: [n_A, 4] (s, p_x, p_y, p_z)
    D: np.ndarray              # [nat, 4]
    colour: np.ndarray         # [nat] colour group of each atom
    dv: float                  # h^3

    @property
    def nat(self) -> int:
        return len(self.idx)


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
                     sigma: float) -> ProjectorSet:
    xyz = g.xyz
    ns, npn = projector_norms(sigma)
    rc2 = rc * rc
    idx, gam = [], []
    for a in range(pos.shape[0]):
        d = displacement(xyz, pos[a], g.box_length)
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        sel = np.nonzero(r2 <= rc2)[0]
        e = np.exp(-r2[sel] / (2.0 * sigma * sigma))
        ga = np.empty((sel.size, 4))
        ga[:, 0] = ns * e
        ga[:, 1] = npn * d[sel, 0] * e
        ga[:, 2] = npn * d[sel, 1] * e
        ga[:, 3] = npn * d[sel, 2] * e
        idx.append(sel)
        gam.append(ga)
    return ProjectorSet(idx=idx, gamma=gam, D=np.asarray(D, dtype=np.float64),
                        colour=colour_atoms(pos, rc, g.box_length), dv=g.dv)


def project(ps: ProjectorSet, psi: np.ndarray) -> np.ndarray:
    """First part: P[k, A, i] = h^3 sum_{p in sphere A} gamma_A,i(p) psi_k(p)."""
    x = np.atleast_2d(psi)
    P = np.zeros((x.shape[0], ps.nat, 4))
    for a in range(ps.nat):
        P[:, a, :] = ps.dv * (x[:, ps.idx[a]] @ ps.gamma[a])
    return P


def apply_projections(ps: ProjectorSet, P: np.ndarray, npoints: int) -> np.ndarray:
    """Second part: sum_A sum_i gamma_A,i(r) D_A,i P[k, A, i], done one colour
    group at a time (within a group the spheres are disjoint)."""
    out = np.zeros((P.shape[0], npoints))
    for col in range(int(ps.colour.max()) + 1 if ps.nat else 0):
        for a in np.nonzero(ps.colour == col)[0]:
            out[:, ps.idx[a]] += (P[:, a, :] * ps.D[a]) @ ps.gamma[a].T
    return out


def apply_nonlocal(ps: ProjectorSet, psi: np.ndarray) -> np.ndarray:
    x = np.atleast_2d(psi)
    out = apply_projections(ps, project(ps, x), x.shape[1])
    return out if psi.ndim == 2 else out[0]
