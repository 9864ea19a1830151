"""Oracle: the real-space Kohn-Sham Hamiltonian in operator form
(TEST INFRASTRUCTURE ONLY).

Sec. 5: H is applied as three independent terms, the kinetic stencil, the
local potential and the non-local projectors.  ``dense`` assembles the
matrix column by column for tiny grids (brute-force checks only).
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import kb, stencil
from .grid import Grid, grid_for, neighbour_table


class Hamiltonian:
    def __init__(self, g: Grid, vloc: np.ndarray,
                 proj: Optional[kb.ProjectorSet] = None):
        self.g = g
        self.vloc = np.asarray(vloc, dtype=np.float64)
        self.proj = proj
        self.nbr = neighbour_table(g)

    @property
    def dv(self) -> float:
        return self.g.dv

    def apply(self, psi: np.ndarray) -> np.ndarray:
        out = stencil.apply_local(self.g, self.vloc, psi, self.nbr)
        if self.proj is not None and self.proj.nat:
            out = out + kb.apply_nonlocal(self.proj, psi)
        return out

    def apply_kinetic(self, psi: np.ndarray) -> np.ndarray:
        return stencil.apply_kinetic(self.g, psi, self.nbr)

    def dense(self) -> np.ndarray:
        n = self.g.np
        if n > 6000:
            raise ValueError("dense assembly is for tiny grids only")
        return self.apply(np.eye(n)).T.copy()


def build_system(w, brick=(4, 4, 4), with_projectors=True):
    """Grid, atoms, potential and Hamiltonian of a synthetic workload."""
    import synthetic
    g = grid_for(w, brick)
    atoms = synthetic.draw_atoms(w) if w.nat else None
    v = synthetic.potential_for(w, g.xyz, atoms)
    proj = None
    if atoms is not None and with_projectors:
        proj = kb.build_projectors(g, atoms.pos, atoms.D, w.rc, w.sigma)
    return g, atoms, Hamiltonian(g, v, proj)
