"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol the header declares, and its host-built index map and projector sets
match the oracle bit for bit."""
import os
import re

import numpy as np
import pytest

import synthetic
from oracle import grid as ogrid
from oracle import kb as okb

rsd = pytest.importorskip("paper_1306_2953_amd")
from paper_1306_2953_amd import _abi  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "rsdft.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = _abi.lib()
    syms = header_symbols()
    assert len(syms) >= 10
    for name in syms:
        assert hasattr(L, name), name
    assert sorted(_abi.SIGNATURES) == syms
    assert L.rs_version() >= 1


def test_bad_arguments_are_reported():
    with pytest.raises(_abi.RsError) as e:
        rsd.Grid("sphere", -0.2, radius=1.0, host_only=True)
    assert e.value.code == _abi.RS_EINVAL
    with pytest.raises(_abi.RsError):
        rsd.Grid("periodic", 0.25, n=10, host_only=True)   # not a multiple of 4


GRIDS = [
    dict(kind="sphere", h=0.2, radius=12.0),
    dict(kind="sphere", h=0.2, radius=2.0),
    dict(kind="sphere", h=0.5, radius=2.6, brick=(2, 3, 4)),
    dict(kind="sphere", h=0.3, radius=1.05),
    dict(kind="box", h=0.3, n=32),
    dict(kind="box", h=0.3, n=6, brick=(4, 4, 4)),
    dict(kind="periodic", h=0.25, n=16),
    dict(kind="sphere", h=0.2, radius=3.0, brick=(64, 64, 64)),   # standard order
]


@pytest.mark.parametrize("args", GRIDS, ids=lambda a: "-".join(str(v) for v in a.values()))
def test_index_map_bit_exact(args):
    args = dict(args)
    brick = args.pop("brick", (4, 4, 4))
    og = ogrid.build_grid(args["kind"], args["h"], n=args.get("n", 0),
                          radius=args.get("radius", 0.0), brick=brick)
    g = rsd.Grid(args["kind"], args["h"], n=args.get("n", 0), radius=args.get("radius", 0.0),
                 brick=brick, host_only=True)
    assert g.np == og.np and g.nbnd == og.nbnd
    ex = g.export()
    assert np.array_equal(ex["inner"], og.inner)
    assert np.array_equal(ex["boundary"], og.boundary.reshape(-1, 3))
    assert np.array_equal(ex["brick_map"], og.brick_map)
    assert np.array_equal(ex["xyz"], og.xyz)          # same rounding of (i - c) h
    assert tuple(g.lo) == tuple(og.lo)


@pytest.mark.parametrize("brick", [(4, 4, 4), (2, 3, 5), (8, 8, 8), (128, 128, 128)])
def test_union_index_map_bit_exact(brick):
    """The molecular grid of the 60-atom cage workload (union of 5.5-bohr
    spheres at h 0.41) in several sub-grid shapes, the largest being the
    standard (lexicographic) order."""
    w = synthetic.WORKLOADS["union_cage60_r5.5_h0.41"]
    og = ogrid.grid_for(w, brick=brick)
    g = rsd.Grid.for_workload(w, host_only=True, brick=brick)
    assert g.np == og.np and g.nbnd == og.nbnd
    ex = g.export()
    assert np.array_equal(ex["inner"], og.inner)
    assert np.array_equal(ex["boundary"], og.boundary.reshape(-1, 3))
    assert np.array_equal(ex["brick_map"], og.brick_map)
    assert np.array_equal(ex["xyz"], og.xyz)
    assert tuple(g.lo) == tuple(og.lo)


def test_union_grid_bad_arguments():
    for kw in (dict(centres=None), dict(centres=np.array([[0.0, 0.0, np.nan]])),
               dict(centres=np.zeros((2, 3)), radius=0.0)):
        kw = dict(dict(radius=2.0), **kw)
        with pytest.raises(_abi.RsError) as e:
            rsd.Grid("union", 0.3, host_only=True, **kw)
        assert e.value.code == _abi.RS_EINVAL


@pytest.mark.parametrize("cfg", [
    dict(name="sphere_r12_h0.2", radius=4.0, nat=5, atom_radius=2.5),
    dict(name="sphere_r12_h0.2"),
    dict(name="periodic96_h0.25", n=24, nat=6),
    dict(name="sphere_r18_h0.18_cage60", radius=9.0, nat=60, atom_radius=6.7, rc=1.2),
    dict(name="union_cage60_r5.5_h0.41"),
])
def test_projector_sets_match_oracle(cfg):
    cfg = dict(cfg)
    name = cfg.pop("name")
    w = synthetic.make_workload(name, **cfg)
    og = ogrid.grid_for(w)
    atoms = synthetic.draw_atoms(w)
    ops = okb.build_projectors(og, atoms.pos, atoms.D, w.rc, w.sigma)
    g = rsd.Grid.for_workload(w, host_only=True)
    nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=64)
    ex = nl.export()
    lens = np.diff(ex["sph_ptr"])
    assert list(lens) == [len(i) for i in ops.idx]
    assert np.array_equal(ex["sph_idx"], np.concatenate(ops.idx))
    gam = np.concatenate(ops.gamma)
    assert np.max(np.abs(ex["gamma"] - gam)) <= 1e-14 * np.max(np.abs(gam))
    assert np.array_equal(ex["colour"], ops.colour)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; a request for more exits with status 2
    and a JSON error line before touching any device."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], cwd=root,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "--gpus must be 1" in msg["error"]


@pytest.mark.parametrize("lmax", [0, 2, 3])
def test_projector_sets_lmax_match_oracle(lmax):
    """(lmax+1)^2 projectors per atom: the same sphere lists, and projector
    values within a few ulps of the oracle's (the constants are folded in a
    different order), for a sphere and a periodic box."""
    for name, cfg in (("sphere_r12_h0.2", dict(radius=4.0, nat=5, atom_radius=2.5)),
                      ("periodic96_h0.25", dict(n=24, nat=6))):
        w = synthetic.make_workload(name, **cfg)
        og = ogrid.grid_for(w)
        atoms = synthetic.draw_atoms(w)
        npj = (lmax + 1) ** 2
        D = np.random.default_rng(40 + lmax).uniform(0.2, 2.0, size=(atoms.pos.shape[0], npj))
        ops = okb.build_projectors(og, atoms.pos, D, w.rc, w.sigma, lmax=lmax)
        g = rsd.Grid.for_workload(w, host_only=True)
        nl = rsd.NonLocal(g, atoms.pos, D, w.rc, w.sigma, max_states=64, lmax=lmax)
        assert nl.nproj == npj
        ex = nl.export()
        assert np.array_equal(ex["sph_idx"], np.concatenate(ops.idx))
        gam = np.concatenate(ops.gamma)
        assert ex["gamma"].shape == gam.shape
        assert np.max(np.abs(ex["gamma"] - gam)) <= 1e-14 * np.max(np.abs(gam))
        assert np.array_equal(ex["colour"], ops.colour)


def test_projector_set_refuses_bad_lmax_and_D():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=3.0, nat=2, atom_radius=1.0)
    atoms = synthetic.draw_atoms(w)
    g = rsd.Grid.for_workload(w, host_only=True)
    with pytest.raises(ValueError):
        rsd.NonLocal(g, atoms.pos, np.ones((2, 25)), w.rc, w.sigma, max_states=8, lmax=4)
    with pytest.raises(ValueError):
        rsd.NonLocal(g, atoms.pos, np.ones((2, 4)), w.rc, w.sigma, max_states=8, lmax=2)
    # the C ABI refuses lmax outside 0..3 on its own
    import ctypes
    h = ctypes.c_void_p()
    pos = np.ascontiguousarray(atoms.pos)
    D = np.ones(2 * 25)
    L = _abi.lib()
    rc = L.rs_nl_create(g.handle, 2, pos.ctypes.data_as(ctypes.c_void_p), D.ctypes.data_as(ctypes.c_void_p),
                        float(w.rc), float(w.sigma), 4, 8, ctypes.byref(h))
    assert rc == _abi.RS_EINVAL and not h.value
    assert b"lmax" in L.rs_last_error()
