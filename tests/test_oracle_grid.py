"""Pins of the oracle's grid / index map (CPU only).

The counts are checked against an independent closed-form count (a sum over
grid columns of the integer square root), the ordering and boundary set
against pure-Python brute force on small grids.
"""
import math

import numpy as np
import pytest

from oracle import grid


def column_count(Q: int, q: int) -> int:
    """Number of integer points with i^2+j^2+k^2 <= Q, counted per (j, k)
    column as 2*isqrt(Q - j^2 - k^2) + 1."""
    tot = 0
    for j in range(-q, q + 1):
        for k in range(-q, q + 1):
            r = Q - j * j - k * k
            if r >= 0:
                tot += 2 * math.isqrt(r) + 1
    return tot


def test_sphere_rule_integer_radius():
    # R/h = 12/0.2 is 60 up to rounding: the surface points are included
    assert grid.sphere_bound(12.0, 0.2) == (60, 3600)
    assert grid.sphere_bound(18.0, 0.18) == (100, 10000)
    # non-integer ratio: floor of the squared ratio
    q, Q = grid.sphere_bound(1.05, 0.5)
    assert Q == math.floor((1.05 / 0.5) ** 2) == 4


@pytest.mark.parametrize("R,h,expect", [(12.0, 0.2, 904089)])
def test_sphere_count_closed_form(R, h, expect):
    q, Q = grid.sphere_bound(R, h)
    assert column_count(Q, q) == expect
    g = grid.build_grid("sphere", h, radius=R)
    assert g.np == expect
    # every inner point satisfies the integer rule, every boundary point fails it
    assert np.all((g.inner ** 2).sum(1) <= Q)
    assert np.all((g.boundary ** 2).sum(1) > Q)


def test_large_sphere_count_closed_form():
    q, Q = grid.sphere_bound(18.0, 0.18)
    assert column_count(Q, q) == 4187857


def _brute(kind, h, n=0, radius=0.0, brick=(4, 4, 4), M=4):
    """Pure-Python enumeration: membership, star reach, sort by tuple key."""
    if kind == "sphere":
        q, Q = grid.sphere_bound(radius, h)
        rng = range(-q - M, q + M + 1)
        inside = lambda p: p[0] ** 2 + p[1] ** 2 + p[2] ** 2 <= Q
        lo = -q - M
    else:
        rng = range(-M, n + M)
        inside = lambda p: all(0 <= c < n for c in p)
        lo = -M
    pts = [(i, j, k) for k in rng for j in rng for i in rng]
    inner = [p for p in pts if inside(p)]
    bnd = []
    for p in pts:
        if inside(p):
            continue
        hit = False
        for a in range(3):
            for m in range(1, M + 1):
                for s in (1, -1):
                    qq = list(p)
                    qq[a] += s * m
                    hit |= inside(qq)
        if hit:
            bnd.append(p)

    def key(p):
        u = [c - lo for c in p]
        b = [u[d] // brick[d] for d in range(3)]
        s = [u[d] % brick[d] for d in range(3)]
        return (b[2], b[1], b[0], s[2], s[1], s[0])

    return sorted(inner, key=key), sorted(bnd, key=key)


@pytest.mark.parametrize("args", [
    dict(kind="sphere", h=0.5, radius=2.6),
    dict(kind="sphere", h=0.25, radius=1.0),
    dict(kind="box", h=0.3, n=6),
    dict(kind="sphere", h=0.5, radius=2.6, brick=(2, 3, 4)),
])
def test_order_and_boundary_bruteforce(args):
    brick = args.pop("brick", (4, 4, 4))
    g = grid.build_grid(args["kind"], args["h"], n=args.get("n", 0),
                        radius=args.get("radius", 0.0), brick=brick)
    inner, bnd = _brute(args["kind"], args["h"], args.get("n", 0),
                        args.get("radius", 0.0), brick)
    assert [tuple(p) for p in g.inner.tolist()] == inner
    assert [tuple(p) for p in g.boundary.tolist()] == bnd


def test_box_counts():
    g = grid.build_grid("box", 0.3, n=32)
    assert g.np == 32 ** 3
    assert g.nbnd == 6 * 32 * 32 * 4       # four planes beyond each face
    p = grid.build_grid("periodic", 0.25, n=16)
    assert p.np == 16 ** 3 and p.nbnd == 0


def test_neighbours_resolve_to_inner_or_boundary():
    g = grid.build_grid("sphere", 0.2, radius=2.0)
    nbr = grid.neighbour_table(g)
    inner = set(map(tuple, g.inner.tolist()))
    bnd = set(map(tuple, g.boundary.tolist()))
    assert not inner & bnd
    for p in range(0, g.np, 7):
        for a in range(3):
            for si, s in enumerate((1, -1)):
                for m in range(1, 5):
                    q = list(g.inner[p])
                    q[a] += s * m
                    q = tuple(q)
                    idx = nbr[p, a, si, m - 1]
                    if idx >= 0:
                        assert tuple(g.inner[idx]) == q
                    else:
                        assert q in bnd


def test_periodic_wrap():
    g = grid.build_grid("periodic", 0.25, n=8)
    nbr = grid.neighbour_table(g)
    for p in range(g.np):
        for a in range(3):
            for si, s in enumerate((1, -1)):
                for m in range(1, 5):
                    q = g.inner[p].copy()
                    q[a] = (q[a] + s * m) % 8
                    assert tuple(g.inner[nbr[p, a, si, m - 1]]) == tuple(q)


def test_brick_map_numbering():
    g = grid.build_grid("sphere", 0.2, radius=3.0)
    start, present = grid.brick_csr(g)
    flat = g.brick_map.reshape(-1)
    assert np.array_equal(np.nonzero(flat >= 0)[0], present)
    assert np.array_equal(flat[present], np.arange(present.size))
    assert start[-1] == g.np
    # points of brick b occupy exactly [start[b], start[b+1])
    u = g.inner - g.lo
    b = u // 4
    bid = (b[:, 2] * g.nb[1] + b[:, 1]) * g.nb[0] + b[:, 0]
    assert np.all(np.diff(bid) >= 0)


def _union_brute(centres, radius, h, brick, M=4):
    """Union-of-spheres grid by plain loops: every lattice point near any
    sphere, inside iff within radius of some centre (Python floats, the
    same rounding order), boundary by the one-axis reach rule, sub-grid
    order."""
    c = [tuple(map(float, x)) for x in centres]
    lo = [int(np.floor((min(p[a] for p in c) - radius) / h)) - M for a in range(3)]
    hi = [int(np.ceil((max(p[a] for p in c) + radius) / h)) + M for a in range(3)]

    def inside(p):
        for X, Y, Z in c:
            dx, dy, dz = p[0] * h - X, p[1] * h - Y, p[2] * h - Z
            if (dx * dx + dy * dy) + dz * dz <= radius * radius:
                return True
        return False

    pts = [(i, j, k) for k in range(lo[2], hi[2] + 1) for j in range(lo[1], hi[1] + 1)
           for i in range(lo[0], hi[0] + 1)]
    ins = {p for p in pts if inside(p)}
    bnd = [p for p in pts if p not in ins and any(
        tuple(p[d] + (s * m if d == a else 0) for d in range(3)) in ins
        for a in range(3) for m in range(1, M + 1) for s in (1, -1))]

    def key(p):
        u = [p[d] - lo[d] for d in range(3)]
        b = [u[d] // brick[d] for d in range(3)]
        s = [u[d] % brick[d] for d in range(3)]
        return (b[2], b[1], b[0], s[2], s[1], s[0])

    return sorted(ins, key=key), sorted(bnd, key=key)


@pytest.mark.parametrize("brick", [(4, 4, 4), (2, 3, 5)])
def test_union_of_spheres_bruteforce(brick):
    """The molecular grid (Sec. 2, Fig. "struct"): three overlapping and one
    separate sphere around off-lattice centres."""
    centres = np.array([[0.13, -0.41, 0.27], [1.37, 0.52, -0.33], [0.61, 1.44, 0.95], [4.9, -2.2, 0.4]])
    g = grid.build_grid("union", 0.45, radius=1.6, brick=brick, centres=centres)
    inner, bnd = _union_brute(centres, 1.6, 0.45, brick)
    assert [tuple(p) for p in g.inner.tolist()] == inner
    assert [tuple(p) for p in g.boundary.tolist()] == bnd
    # each atom's sphere is inside the grid, and the union has fewer points
    # than the spheres' separate counts (they overlap)
    d2 = ((g.xyz[:, None, :] - centres[None]) ** 2).sum(-1)
    assert np.all(d2.min(axis=1) <= 1.6 ** 2 + 1e-12)
    per = [(((g.xyz - c) ** 2).sum(-1) <= 1.6 ** 2).sum() for c in centres]
    assert g.np < sum(per)
