"""Seeded synthetic workloads shared by the CPU oracle and the GPU path.

This module only draws random numbers and evaluates the *given* external
fields (the local potential) at coordinates handed to it.  It holds none of
the method's arithmetic: no grid construction, no stencil, no projector
evaluation, no linear algebra.  Both the oracle and the HIP path receive the
same arrays from here.

The paper's molecules (union-of-spheres grids, norm-conserving
pseudopotentials, Sec. "Computational methods") are not available, so the
workloads are synthetic stand-ins with the same structure: a uniform grid
restricted to a sphere (or a box), atoms carrying Gaussian local wells and
one s plus three p Kleinman-Bylander projectors, and blocks of real states.

Random draws use ``numpy.random.default_rng(seed)`` in a fixed order:
atom positions, well depths, well widths, D_s, D_p, then initial states.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "make_workload", "draw_atoms", "draw_states",
    "wells_potential", "harmonic_potential",
]


@dataclasses.dataclass
class Workload:
    """Description of one synthetic system.

    grid_kind: "box" (zero Dirichlet outside an n^3 cell-centred box),
               "periodic" (n^3 periodic box), "sphere" (all points within
               ``radius`` of the centre) or "union" (all points within
               ``radius`` of some atom: the molecular grid).
    """
    name: str
    grid_kind: str
    h: float
    n: int = 0               # box edge in points (box / periodic)
    radius: float = 0.0      # sphere radius in bohr
    nstates: int = 8
    block: int = 8
    seed: int = 0
    potential: str = "wells"  # "harmonic" or "wells"
    nat: int = 0
    atom_layout: str = "ball"  # "ball", "box", "cage"
    atom_radius: float = 8.0   # ball radius or cage radius (bohr)
    rc: float = 2.5            # projector cutoff radius (bohr)
    sigma: float = 0.7         # projector Gaussian width (bohr)
    depth: tuple = (2.0, 6.0)  # well depth U(a, b) in Ha
    width: tuple = (0.6, 1.2)  # well width U(a, b) in bohr (standard deviation)
    d_s: tuple = (1.0, 3.0)    # KB coupling for s, U(a, b) Ha
    d_p: tuple = (0.5, 1.5)    # KB coupling for p, U(a, b) Ha

    @property
    def box_length(self) -> float:
        return self.n * self.h


# The workloads, by name: a harmonic box, a sphere in FP64, the same sphere
# in FP32 / split precision, a periodic box for the learned preconditioner,
# a large sphere with a cage of atoms, and a molecular grid (union of 5.5
# bohr spheres at h 0.41, the paper's grid parameters) around a 60-atom
# cage.
WORKLOADS = {w.name: w for w in (
    Workload("box32_harmonic", "box", 0.3, n=32, nstates=8, block=8, seed=1,
             potential="harmonic"),
    Workload("sphere_r12_h0.2", "sphere", 0.2, radius=12.0, nstates=128,
             block=32, seed=2, nat=16, atom_layout="ball", atom_radius=8.0),
    Workload("sphere_r12_h0.2_fp32", "sphere", 0.2, radius=12.0, nstates=128,
             block=32, seed=2, nat=16, atom_layout="ball", atom_radius=8.0),
    Workload("periodic96_h0.25", "periodic", 0.25, n=96, nstates=256,
             block=32, seed=4, nat=32, atom_layout="box"),
    Workload("sphere_r18_h0.18_cage60", "sphere", 0.18, radius=18.0,
             nstates=240, block=64, seed=5, nat=60, atom_layout="cage",
             atom_radius=6.7),
    Workload("union_cage60_r5.5_h0.41", "union", 0.41, radius=5.5,
             nstates=128, block=32, seed=6, nat=60, atom_layout="cage",
             atom_radius=6.7),
)}


def make_workload(name: str, **overrides) -> Workload:
    """Return a copy of workload ``name`` with fields overridden (for small
    test-sized variants of the same recipe)."""
    return dataclasses.replace(WORKLOADS[name], **overrides)


@dataclasses.dataclass
class Atoms:
    pos: np.ndarray     # [nat, 3] bohr
    depth: np.ndarray   # [nat]  Ha
    width: np.ndarray   # [nat]  bohr
    D: np.ndarray       # [nat, 4] Ha: (D_s, D_p, D_p, D_p)


def _fibonacci_cage(rng, nat, radius):
    """``nat`` points on a near-uniform spherical shell, randomly rotated and
    jittered by N(0, 0.1 bohr) per coordinate (a synthetic cage)."""
    k = np.arange(nat) + 0.5
    z = 1.0 - 2.0 * k / nat
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    pts = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1) * radius
    # random rotation from a normalised quaternion
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    rot = np.array([
        [a*a + b*b - c*c - d*d, 2*(b*c - a*d), 2*(b*d + a*c)],
        [2*(b*c + a*d), a*a - b*b + c*c - d*d, 2*(c*d - a*b)],
        [2*(b*d - a*c), 2*(c*d + a*b), a*a - b*b - c*c + d*d]])
    pts = pts @ rot.T
    pts += rng.normal(scale=0.1, size=pts.shape)
    return pts


def draw_atoms(w: Workload, rng: Optional[np.random.Generator] = None) -> Atoms:
    """Atom positions, well depths/widths and KB couplings, in the fixed draw
    order.  ``rng`` defaults to ``default_rng(w.seed)``."""
    if rng is None:
        rng = np.random.default_rng(w.seed)
    nat = w.nat
    if w.atom_layout == "ball":
        pos = np.empty((nat, 3))
        i = 0
        while i < nat:                      # rejection sampling in the ball
            p = rng.uniform(-w.atom_radius, w.atom_radius, size=3)
            if p @ p <= w.atom_radius ** 2:
                pos[i] = p
                i += 1
    elif w.atom_layout == "box":
        pos = rng.uniform(0.0, w.box_length, size=(nat, 3))
    elif w.atom_layout == "cage":
        pos = _fibonacci_cage(rng, nat, w.atom_radius)
    else:
        raise ValueError(w.atom_layout)
    depth = rng.uniform(*w.depth, size=nat)
    width = rng.uniform(*w.width, size=nat)
    ds = rng.uniform(*w.d_s, size=nat)
    dp = rng.uniform(*w.d_p, size=nat)
    D = np.stack([ds, dp, dp, dp], axis=1)
    return Atoms(pos=pos, depth=depth, width=width, D=D)


def couplings_lmax(w: Workload, atoms: Atoms, lmax: int) -> np.ndarray:
    """KB couplings for projectors up to lmax, [nat, (lmax+1)^2]: the
    workload's s and p values, then one value per atom and l >= 2 shared by
    its 2l + 1 projectors, drawn U(0.3, 1.0) Ha from default_rng(seed + 7)."""
    nat = atoms.D.shape[0]
    cols = [atoms.D[:, :1]] + ([atoms.D[:, 1:4]] if lmax >= 1 else [])
    rng = np.random.default_rng(w.seed + 7)
    for l in range(2, lmax + 1):
        d = rng.uniform(0.3, 1.0, size=nat)
        cols.append(np.repeat(d[:, None], 2 * l + 1, axis=1))
    return np.concatenate(cols, axis=1)


def draw_states(rng: np.random.Generator, nstates: int, npoints: int,
                dtype=np.float64) -> np.ndarray:
    """Initial states, uniform[-1, 1], state-major [nstates, npoints]."""
    return rng.uniform(-1.0, 1.0, size=(nstates, npoints)).astype(dtype)


def rng_after_atoms(w: Workload) -> np.random.Generator:
    """The generator positioned after the atom draws (for drawing states)."""
    rng = np.random.default_rng(w.seed)
    if w.nat:
        draw_atoms(w, rng)
    return rng


def harmonic_potential(xyz: np.ndarray) -> np.ndarray:
    """V = r^2 / 2 about the origin, at physical coordinates ``xyz`` [n, 3]."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return 0.5 * ((x * x + y * y) + z * z)


def wells_potential(xyz: np.ndarray, atoms: Atoms,
                    box_length: Optional[float] = None) -> np.ndarray:
    """V(r) = -sum_A U_A exp(-|r - R_A|^2 / (2 w_A^2)); minimum image when
    ``box_length`` is given (periodic)."""
    v = np.zeros(xyz.shape[0])
    for a in range(atoms.pos.shape[0]):
        d = xyz - atoms.pos[a]
        if box_length is not None:
            d = d - box_length * np.rint(d / box_length)
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        v -= atoms.depth[a] * np.exp(-r2 / (2.0 * atoms.width[a] ** 2))
    return v


def potential_for(w: Workload, xyz: np.ndarray, atoms: Optional[Atoms]) -> np.ndarray:
    if w.potential == "harmonic":
        return harmonic_potential(xyz)
    if atoms is None or atoms.pos.shape[0] == 0:
        return np.zeros(xyz.shape[0])
    return wells_potential(xyz, atoms,
                           w.box_length if w.grid_kind == "periodic" else None)
