"""GPU parity of H psi, the projections and the scatter against the FP64
oracle, through the C ABI.  Tolerances: FP64 1e-12 relative, FP32 1e-5
relative (max-norm over all outputs, relative to the largest output)."""
import numpy as np
import pytest

import synthetic
from oracle import hamiltonian, kb, stencil

torch = pytest.importorskip("torch")
import paper_1306_2953_amd as rsd  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"


def _system(w, max_states=256):
    og, atoms, H = hamiltonian.build_system(w)
    g = rsd.Grid.for_workload(w)
    assert g.np == og.np
    nl = None
    if atoms is not None:
        nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=max_states)
    return og, H, g, nl


def _states(w, N, npts, dtype):
    rng = synthetic.rng_after_atoms(w)
    return synthetic.draw_states(rng, N, npts).astype(dtype)


def _gpu_hpsi(g, nl, v, psi_sm, B, dtype):
    blk = rsd.to_blocks(psi_sm, B)
    tp = torch.from_numpy(blk).to(DEV)
    th = torch.empty_like(tp)
    tv = torch.from_numpy(np.ascontiguousarray(v.astype(dtype))).to(DEV)
    rsd.hpsi_block(g, nl, tv, tp, th)
    torch.cuda.synchronize()
    return rsd.from_blocks(th.cpu().numpy())


def _relerr(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


SMALL = synthetic.make_workload("sphere_r12_h0.2", radius=3.0, nat=5, atom_radius=2.0)


@pytest.mark.parametrize("B", [1, 2, 4, 8, 16, 32, 64])
def test_hpsi_fp64_sphere_all_block_sizes(B):
    og, H, g, nl = _system(SMALL)
    psi = _states(SMALL, 2 * B, og.np, np.float64)
    got = _gpu_hpsi(g, nl, H.vloc, psi, B, np.float64)
    assert _relerr(got, H.apply(psi)) < 1e-12


@pytest.mark.parametrize("B", [1, 8, 32, 64])
def test_hpsi_fp32_sphere(B):
    og, H, g, nl = _system(SMALL)
    psi = _states(SMALL, 2 * B, og.np, np.float32)
    v32 = H.vloc.astype(np.float32)
    Hq = hamiltonian.Hamiltonian(og, v32.astype(np.float64), H.proj)
    want = Hq.apply(psi.astype(np.float64))
    got = _gpu_hpsi(g, nl, v32, psi, B, np.float32)
    assert _relerr(got, want) < 1e-5
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-6


def test_hpsi_box_harmonic_and_periodic():
    w = synthetic.WORKLOADS["box32_harmonic"]
    og, H, g, nl = _system(w)
    psi = _states(w, 8, og.np, np.float64)
    got = _gpu_hpsi(g, nl, H.vloc, psi, 8, np.float64)
    assert _relerr(got, H.apply(psi)) < 1e-12
    wp = synthetic.make_workload("periodic96_h0.25", n=24, nat=4)
    og, H, g, nl = _system(wp)
    psi = _states(wp, 64, og.np, np.float64)
    got = _gpu_hpsi(g, nl, H.vloc, psi, 32, np.float64)
    assert _relerr(got, H.apply(psi)) < 1e-12


@pytest.mark.parametrize("kind,n,nat", [("periodic", 4, 0), ("periodic", 12, 0), ("periodic", 20, 2),
                                         ("box", 13, 0)])
def test_hpsi_fp64_march_lattice_edges(kind, n, nat):
    """FP64 blocks of 16 and 32 states run the z-marching kernel.  Periodic
    edges of 1, 3 and 5 bricks leave the last 2 x 2 tile half outside the
    lattice (its second column wraps onto bricks another tile writes: they
    are read as neighbours, never written); the Dirichlet box has partial
    bricks on every face."""
    if kind == "periodic":
        w = synthetic.make_workload("periodic96_h0.25", n=n, nat=nat, rc=1.5)
    else:
        w = synthetic.make_workload("box32_harmonic", n=n)
    og, H, g, nl = _system(w)
    psi = _states(w, 64, og.np, np.float64)
    want = H.apply(psi)
    for B in (16, 32):
        got = _gpu_hpsi(g, nl, H.vloc, psi, B, np.float64)
        assert _relerr(got, want) < 1e-12, (kind, n, B)


def test_overlapping_spheres_no_race():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=2.4, nat=8, atom_radius=0.8, rc=1.5)
    og, H, g, nl = _system(w)
    assert nl.ncolours >= 3
    psi = _states(w, 32, og.np, np.float64)
    a = _gpu_hpsi(g, nl, H.vloc, psi, 32, np.float64)
    b = _gpu_hpsi(g, nl, H.vloc, psi, 32, np.float64)
    assert np.array_equal(a, b)                      # bitwise repeatable
    assert _relerr(a, H.apply(psi)) < 1e-12


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-12), (np.float32, 1e-5)])
def test_project_and_apply_nl(dtype, tol):
    og, H, g, nl = _system(SMALL)
    B, nblk = 16, 3
    psi = _states(SMALL, nblk * B, og.np, dtype)
    P = kb.project(H.proj, psi.astype(np.float64))               # [N, nat, 4]
    tp = torch.from_numpy(rsd.to_blocks(psi, B)).to(DEV)
    proj = torch.empty((nblk, nl.nat, 4, B), dtype=tp.dtype, device=DEV)
    rsd.project_nl(g, nl, tp, proj)
    got = proj.cpu().numpy().transpose(0, 3, 1, 2).reshape(nblk * B, nl.nat, 4)
    assert _relerr(got, P) < tol
    # scatter on top of an arbitrary field
    base = _states(SMALL, nblk * B, og.np, dtype)
    th = torch.from_numpy(rsd.to_blocks(base, B)).to(DEV)
    rsd.apply_nl(g, nl, proj, th)
    torch.cuda.synchronize()
    want = base.astype(np.float64) + kb.apply_projections(H.proj, got.astype(np.float64), og.np)
    assert _relerr(rsd.from_blocks(th.cpu().numpy()), want) < tol


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-12), (np.float32, 1e-5)])
def test_full_size_sphere_sampled(dtype, tol):
    """Config-2 grid (0.9M points, 16 atoms), all 128 states in blocks of 32,
    checked at sampled points computed one by one by the oracle."""
    w = synthetic.WORKLOADS["sphere_r12_h0.2"]
    og, atoms, H = hamiltonian.build_system(w)
    g = rsd.Grid.for_workload(w)
    nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=128)
    psi = _states(w, 128, og.np, dtype)
    v = H.vloc.astype(dtype)
    got = _gpu_hpsi(g, nl, v, psi, 32, dtype)
    x64 = psi.astype(np.float64)
    rng = np.random.default_rng(11)
    pts = rng.choice(og.np, 300, replace=False)
    sph = np.concatenate(H.proj.idx)
    pts = np.unique(np.concatenate([pts, rng.choice(sph, 200, replace=False)]))
    want = stencil.apply_local_at(og, v.astype(np.float64), x64, pts)
    P = kb.project(H.proj, x64)
    want += kb.apply_projections(H.proj, P, og.np)[:, pts]
    assert _relerr(got[:, pts], want) < tol


@pytest.mark.parametrize("name,seed,N,B", [("periodic96_h0.25", 4, 64, 32), ("sphere_r18_h0.18_cage60", 5, 64, 64)])
def test_full_size_periodic_and_cage_sampled(name, seed, N, B):
    """The periodic 96^3 box (32 atoms, minimum image) and the sphere R 18 at
    h 0.18 (4.19M points, 60 atoms on a cage) in FP32, N states, checked at
    sampled points (grid-wide and inside projector spheres)."""
    w = synthetic.WORKLOADS[name]
    og, atoms, H = hamiltonian.build_system(w)
    g = rsd.Grid.for_workload(w)
    assert g.np == og.np
    nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=N)
    psi = _states(w, N, og.np, np.float32)
    v = H.vloc.astype(np.float32)
    got = _gpu_hpsi(g, nl, v, psi, B, np.float32)
    x64 = psi.astype(np.float64)
    rng = np.random.default_rng(seed)
    pts = rng.choice(og.np, 300, replace=False)
    sph = np.concatenate(H.proj.idx)
    pts = np.unique(np.concatenate([pts, rng.choice(sph, 200, replace=False)]))
    want = stencil.apply_local_at(og, v.astype(np.float64), x64, pts)
    P = kb.project(H.proj, x64)
    want += kb.apply_projections(H.proj, P, og.np)[:, pts]
    assert _relerr(got[:, pts], want) < 1e-5


def test_bad_block_size_rejected():
    """B = 3 is refused by the binding (ValueError) and, called directly, by
    the C entry point (RS_EINVAL) before any kernel runs."""
    og, H, g, nl = _system(SMALL)
    t = torch.zeros((1, og.np, 3), dtype=torch.float64, device=DEV)
    v = torch.zeros(og.np, dtype=torch.float64, device=DEV)
    out = torch.empty_like(t)
    with pytest.raises(ValueError):
        rsd.hpsi_block(g, nl, v, t, out)
    st = rsd.lib().rs_hpsi_block(g.handle, nl.handle, rsd._dev(v, "v"), rsd._dev(t, "psi"), rsd._dev(out, "hpsi"),
                                 1, 3, rsd.RS_F64, None)
    assert st == rsd._abi.RS_EINVAL


UNION_SMALL = synthetic.make_workload("union_cage60_r5.5_h0.41", nat=6, atom_radius=2.0, radius=2.5, h=0.3)


@pytest.mark.parametrize("dtype,B,tol", [(np.float64, 16, 1e-12), (np.float64, 32, 1e-12), (np.float64, 8, 1e-12),
                                         (np.float32, 32, 1e-5), (np.float32, 4, 1e-5)])
def test_hpsi_union_of_spheres(dtype, B, tol):
    """The molecular grid (union of spheres around 6 atoms on a small cage):
    FP64 blocks of 16 and 32 run the z-marching kernel over the irregular
    brick columns, B = 8 and FP32 the per-brick kernel."""
    og, H, g, nl = _system(UNION_SMALL)
    assert og.kind == "union" and g.np == og.np
    psi = _states(UNION_SMALL, 2 * B, og.np, dtype)
    v = H.vloc.astype(dtype)
    Hq = hamiltonian.Hamiltonian(og, v.astype(np.float64), H.proj)
    got = _gpu_hpsi(g, nl, v, psi, B, dtype)
    assert _relerr(got, Hq.apply(psi.astype(np.float64))) < tol


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-12), (np.float32, 1e-5)])
def test_full_size_union_sampled(dtype, tol):
    """The 60-atom molecular grid (103k points, h 0.41, 5.5-bohr spheres),
    all 128 states in blocks of 32, at sampled points."""
    w = synthetic.WORKLOADS["union_cage60_r5.5_h0.41"]
    og, atoms, H = hamiltonian.build_system(w)
    g = rsd.Grid.for_workload(w)
    nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=128)
    psi = _states(w, 128, og.np, dtype)
    v = H.vloc.astype(dtype)
    got = _gpu_hpsi(g, nl, v, psi, 32, dtype)
    x64 = psi.astype(np.float64)
    rng = np.random.default_rng(13)
    pts = rng.choice(og.np, 400, replace=False)
    sph = np.concatenate(H.proj.idx)
    pts = np.unique(np.concatenate([pts, rng.choice(sph, 200, replace=False)]))
    want = stencil.apply_local_at(og, v.astype(np.float64), x64, pts)
    P = kb.project(H.proj, x64)
    want += kb.apply_projections(H.proj, P, og.np)[:, pts]
    assert _relerr(got[:, pts], want) < tol
