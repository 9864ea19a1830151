"""Oracle: real-space grid and its index map (TEST INFRASTRUCTURE ONLY).

Follows Sec. 2 (uniform grid restricted to a shape that avoids points where
the density is negligible) and Sec. 5.1 (the 3-D to 1-D map enumerates the
grid by small parallelepipedic sub-grids, Fig. "locality" (b)).

Readings taken where the paper is silent:
  * a molecular grid is the union of spheres of radius R around the atoms
    (Sec. 2, Fig. "struct"): point (i,j,k) at (i h, j h, k h) is inner iff
    ((x - X)^2 + (y - Y)^2) + (z - Z)^2 <= R^2 for some atom (X, Y, Z), in
    FP64 rounded as written;
  * sphere membership is decided in integer arithmetic (point (i,j,k) at
    i*h from the centre is inner iff i^2+j^2+k^2 <= Q, Q = q^2 when R/h is an
    integer q to 1e-9 relative, else floor((R/h)^2));
  * the Dirichlet box is cell-centred, x_i = (i - (n-1)/2) h;
  * sub-grids ("bricks") are enumerated x fastest, then y, then z over the
    brick lattice; inside a brick x is fastest; inner points come first and
    boundary points (outside the domain but within the stencil's reach
    along one axis) follow in the same order;
  * only bricks that hold at least one inner point are numbered.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np


def sphere_bound(radius: float, h: float) -> Tuple[int, int]:
    """Integer sphere rule: returns (q, Q) with inner <=> i^2+j^2+k^2 <= Q."""
    x = radius / h
    q = int(round(x))
    if abs(x - q) <= 1e-9 * max(q, 1):
        return q, q * q
    return int(math.floor(x)), int(math.floor(x * x))


@dataclasses.dataclass
class Grid:
    kind: str                 # "box", "periodic", "sphere", "union"
    h: float
    n: int                    # box edge (box/periodic), 0 for sphere
    M: int                    # stencil half-width (neighbours per side)
    brick: Tuple[int, int, int]
    lo: np.ndarray            # integer coordinate of lattice origin [3]
    L: np.ndarray             # lattice dims [3]
    nb: np.ndarray            # brick counts [3]
    inner: np.ndarray         # int64 [np, 3] integer coordinates, in map order
    boundary: np.ndarray      # int64 [nbnd, 3]
    brick_map: np.ndarray     # int32 [nbz, nby, nbx], -1 = absent
    lookup: np.ndarray        # int64 [Lz, Ly, Lx] lattice -> point index, -1
    centre: float             # coordinate offset c: x = (i - c) h

    @property
    def np(self) -> int:
        return self.inner.shape[0]

    @property
    def nbnd(self) -> int:
        return self.boundary.shape[0]

    @property
    def periodic(self) -> bool:
        return self.kind == "periodic"

    @property
    def box_length(self) -> Optional[float]:
        return self.n * self.h if self.periodic else None

    @property
    def xyz(self) -> np.ndarray:
        """Physical coordinates of the inner points (bohr)."""
        return (self.inner.astype(np.float64) - self.centre) * self.h

    @property
    def dv(self) -> float:
        """Volume element h^3 of the grid sums that replace integrals."""
        return self.h ** 3


def _brick_key(u: np.ndarray, brick, nb) -> np.ndarray:
    """Sort key of lattice coordinates u [n, 3] (x, y, z order): brick index
    (x fastest) then slot inside the brick (x fastest)."""
    bx, by, bz = brick
    b = u // np.array(brick)
    s = u % np.array(brick)
    bid = (b[:, 2] * nb[1] + b[:, 1]) * nb[0] + b[:, 0]
    sid = (s[:, 2] * by + s[:, 1]) * bx + s[:, 0]
    return bid * (bx * by * bz) + sid


def union_inside(centres: np.ndarray, radius: float, h: float, lo: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Membership [z, y, x] of the lattice points lo + (i, j, k) in the union
    of the spheres of radius `radius` around `centres` [nat, 3]: written out
    atom by atom over the whole lattice (brute force)."""
    ax = [(np.arange(L[d]) + lo[d]).astype(np.float64) * h for d in range(3)]
    inside = np.zeros((L[2], L[1], L[0]), dtype=bool)
    r2 = radius * radius
    for c in np.asarray(centres, dtype=np.float64):
        dx = ax[0] - c[0]
        dy = ax[1] - c[1]
        dz = ax[2] - c[2]
        d2 = (dx[None, None, :] * dx[None, None, :] + dy[None, :, None] * dy[None, :, None]) \
            + dz[:, None, None] * dz[:, None, None]
        inside |= d2 <= r2
    return inside


def build_grid(kind: str, h: float, n: int = 0, radius: float = 0.0,
               brick=(4, 4, 4), M: int = 4, centres: Optional[np.ndarray] = None) -> Grid:
    """Enumerate inner and boundary points in sub-grid order (Sec. 5.1).
    kind "union": the union of spheres of `radius` around `centres`."""
    brick = tuple(int(b) for b in brick)
    if kind == "sphere":
        q, Q = sphere_bound(radius, h)
        lo_in = np.array([-q] * 3)
        ext = 2 * q + 1
        pad = M
        centre = 0.0
    elif kind == "union":
        c = np.asarray(centres, dtype=np.float64)
        lo_in = np.floor((c.min(axis=0) - radius) / h).astype(np.int64)
        ext = np.ceil((c.max(axis=0) + radius) / h).astype(np.int64) - lo_in + 1
        pad = M
        centre = 0.0
    elif kind == "box":
        lo_in = np.zeros(3, dtype=np.int64)
        ext = n
        pad = M
        centre = 0.5 * (n - 1)
    elif kind == "periodic":
        lo_in = np.zeros(3, dtype=np.int64)
        ext = n
        pad = 0
        centre = 0.0
        if any(n % b for b in brick):
            raise ValueError("periodic edge must be a multiple of the brick")
    else:
        raise ValueError(kind)
    L = np.broadcast_to(np.asarray(ext) + 2 * pad, (3,)).astype(np.int64)
    lo = lo_in - pad
    nb = -(-L // np.array(brick))

    # dense membership over the lattice, indexed [z, y, x]
    ax = [np.arange(L[d]) + lo[d] for d in range(3)]
    if kind == "sphere":
        r2 = (ax[2][:, None, None] ** 2 + ax[1][None, :, None] ** 2
              + ax[0][None, None, :] ** 2)
        inside = r2 <= Q
    elif kind == "union":
        inside = union_inside(c, radius, h, lo, L)
    else:
        inside = np.zeros((L[2], L[1], L[0]), dtype=bool)
        inside[pad:pad + ext, pad:pad + ext, pad:pad + ext] = True

    # boundary: not inside, but an inside point within M steps along one axis
    near = np.zeros_like(inside)
    if kind != "periodic":
        for axis in range(3):
            for m in range(1, M + 1):
                for sgn in (1, -1):
                    near |= np.roll(inside, sgn * m, axis=axis)
        # np.roll wraps, but the M-deep padding keeps wrapped rows empty
    bnd = near & ~inside

    def ordered(mask):
        z, y, x = np.nonzero(mask)
        u = np.stack([x, y, z], axis=1).astype(np.int64)
        key = _brick_key(u, brick, nb)
        order = np.argsort(key, kind="stable")
        return u[order]

    u_in = ordered(inside)
    u_bd = ordered(bnd)

    lookup = np.full((L[2], L[1], L[0]), -1, dtype=np.int64)
    lookup[u_in[:, 2], u_in[:, 1], u_in[:, 0]] = np.arange(u_in.shape[0])

    bidx = u_in // np.array(brick)
    bid = (bidx[:, 2] * nb[1] + bidx[:, 1]) * nb[0] + bidx[:, 0]
    present = np.unique(bid)
    brick_map = np.full(int(nb[0] * nb[1] * nb[2]), -1, dtype=np.int32)
    brick_map[present] = np.arange(present.size, dtype=np.int32)
    brick_map = brick_map.reshape(nb[2], nb[1], nb[0])

    return Grid(kind=kind, h=h, n=n, M=M, brick=brick, lo=lo, L=L, nb=nb,
                inner=u_in + lo, boundary=u_bd + lo, brick_map=brick_map,
                lookup=lookup, centre=centre)


def grid_for(workload, brick=(4, 4, 4)) -> Grid:
    w = workload
    if w.grid_kind == "sphere":
        return build_grid("sphere", w.h, radius=w.radius, brick=brick)
    if w.grid_kind == "union":
        import synthetic
        return build_grid("union", w.h, radius=w.radius, brick=brick, centres=synthetic.draw_atoms(w).pos)
    return build_grid(w.grid_kind, w.h, n=w.n, brick=brick)


def neighbour_table(g: Grid) -> np.ndarray:
    """int64 [np, 3, 2, M]: index of the point m steps along +/- each axis,
    or -1 when it lies outside the domain (its value is zero)."""
    u = g.inner - g.lo
    out = np.empty((g.np, 3, 2, g.M), dtype=np.int64)
    for a in range(3):
        for si, sgn in enumerate((1, -1)):
            for m in range(1, g.M + 1):
                v = u.copy()
                v[:, a] += sgn * m
                if g.periodic:
                    v[:, a] %= g.L[a]
                out[:, a, si, m - 1] = g.lookup[v[:, 2], v[:, 1], v[:, 0]]
    return out


def brick_csr(g: Grid):
    """Per-brick point ranges of the inner points (brick_start [nbricks+1])
    and the brick lattice coordinate of every numbered brick."""
    u = g.inner - g.lo
    bidx = u // np.array(g.brick)
    bid = (bidx[:, 2] * g.nb[1] + bidx[:, 1]) * g.nb[0] + bidx[:, 0]
    present, counts = np.unique(bid, return_counts=True)
    start = np.zeros(present.size + 1, dtype=np.int64)
    start[1:] = np.cumsum(counts)
    return start, present
