"""GPU parity of the projector terms with l up to 3 and of complex states
(eq. (6) with l_max = 3; eq. (1b) conjugates complex states) against the
FP64 oracle, through the C ABI.  Tolerances as for the real s/p path: FP64
1e-12 and FP32 1e-5 relative to the largest output; the complex FP32
overlap against the split-BF16 bound 2^-16 h^3 sum_p |x_p| |y_p| of each of
the two real products forming a complex element."""
import numpy as np
import pytest

import synthetic
from oracle import hamiltonian, kb, linalg

torch = pytest.importorskip("torch")
import paper_1306_2953_amd as rsd  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SMALL = synthetic.make_workload("sphere_r12_h0.2", radius=3.0, nat=5, atom_radius=2.0)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"


def _system(w, lmax, max_states=256):
    og, atoms, H0 = hamiltonian.build_system(w, with_projectors=False)
    npj = (lmax + 1) ** 2
    D = np.random.default_rng(50 + lmax).uniform(-1.5, 2.0, size=(atoms.pos.shape[0], npj))
    ps = kb.build_projectors(og, atoms.pos, D, w.rc, w.sigma, lmax=lmax)
    H = hamiltonian.Hamiltonian(og, H0.vloc, ps)
    g = rsd.Grid.for_workload(w)
    nl = rsd.NonLocal(g, atoms.pos, D, w.rc, w.sigma, max_states=max_states, lmax=lmax)
    return og, H, g, nl


def _states(w, N, npts, seed_shift=0):
    rng = synthetic.rng_after_atoms(w)
    for _ in range(seed_shift):
        rng.random()
    return synthetic.draw_states(rng, N, npts)


def _cstates(w, N, npts):
    a = _states(w, 2 * N, npts)
    return a[:N] + 1j * a[N:]


def _relerr(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _hpsi(g, nl, v, psi_sm, B, dtype, vdtype):
    tp = torch.from_numpy(rsd.to_blocks(psi_sm.astype(dtype), B)).to(DEV)
    th = torch.empty_like(tp)
    tv = torch.from_numpy(np.ascontiguousarray(v.astype(vdtype))).to(DEV)
    rsd.hpsi_block(g, nl, tv, tp, th)
    torch.cuda.synchronize()
    return rsd.from_blocks(th.cpu().numpy())


@pytest.mark.parametrize("lmax", [0, 2, 3])
@pytest.mark.parametrize("B", [8, 32])
def test_hpsi_fp64_lmax(lmax, B):
    """B = 32 runs the z-marching kernel, B = 8 the per-brick kernel; both
    then the point-centric projector add (the per-brick kernel fuses the
    projector term only for the 4-projector s and p set)."""
    og, H, g, nl = _system(SMALL, lmax)
    psi = _states(SMALL, 2 * B, og.np)
    got = _hpsi(g, nl, H.vloc, psi, B, np.float64, np.float64)
    assert _relerr(got, H.apply(psi)) < 1e-12


@pytest.mark.parametrize("lmax", [0, 3])
def test_hpsi_fp32_lmax(lmax):
    og, H, g, nl = _system(SMALL, lmax)
    psi = _states(SMALL, 32, og.np).astype(np.float32)
    v32 = H.vloc.astype(np.float32)
    Hq = hamiltonian.Hamiltonian(og, v32.astype(np.float64), H.proj)
    got = _hpsi(g, nl, v32, psi, 16, np.float32, np.float32)
    assert _relerr(got, Hq.apply(psi.astype(np.float64))) < 1e-5


@pytest.mark.parametrize("lmax", [0, 2, 3])
@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-12), (np.float32, 1e-5)])
def test_project_and_apply_lmax(lmax, dtype, tol):
    og, H, g, nl = _system(SMALL, lmax)
    npj = (lmax + 1) ** 2
    assert nl.nproj == npj
    B, nblk = 16, 3
    psi = _states(SMALL, nblk * B, og.np).astype(dtype)
    P = kb.project(H.proj, psi.astype(np.float64))               # [N, nat, npj]
    tp = torch.from_numpy(rsd.to_blocks(psi, B)).to(DEV)
    proj = torch.empty((nblk, nl.nat, npj, B), dtype=tp.dtype, device=DEV)
    rsd.project_nl(g, nl, tp, proj)
    got = proj.cpu().numpy().transpose(0, 3, 1, 2).reshape(nblk * B, nl.nat, npj)
    assert _relerr(got, P) < tol
    base = _states(SMALL, nblk * B, og.np, seed_shift=1).astype(dtype)
    th = torch.from_numpy(rsd.to_blocks(base, B)).to(DEV)
    rsd.apply_nl(g, nl, proj, th)
    torch.cuda.synchronize()
    want = base.astype(np.float64) + kb.apply_projections(H.proj, got.astype(np.float64), og.np)
    assert _relerr(rsd.from_blocks(th.cpu().numpy()), want) < tol


@pytest.mark.parametrize("B", [4, 16])
def test_hpsi_complex128(B):
    """Complex states: B = 16 complex (32 real columns) runs the z-marching
    kernel, B = 4 the per-brick kernel.  Oracle: H applied to the complex
    array."""
    og, H, g, nl = _system(SMALL, 2)
    z = _cstates(SMALL, 2 * B, og.np)
    got = _hpsi(g, nl, H.vloc, z, B, np.complex128, np.float64)
    assert got.dtype == np.complex128
    assert _relerr(got, H.apply(z)) < 1e-12


def test_hpsi_complex64():
    og, H, g, nl = _system(SMALL, 3)
    z = _cstates(SMALL, 16, og.np).astype(np.complex64)
    v32 = H.vloc.astype(np.float32)
    Hq = hamiltonian.Hamiltonian(og, v32.astype(np.float64), H.proj)
    got = _hpsi(g, nl, v32, z, 8, np.complex64, np.float32)
    assert _relerr(got, Hq.apply(z.astype(np.complex128))) < 1e-5


@pytest.mark.parametrize("dtype,tol", [(np.complex128, 1e-12), (np.complex64, 1e-5)])
def test_project_and_apply_complex(dtype, tol):
    og, H, g, nl = _system(SMALL, 3)
    B, nblk = 8, 2
    z = _cstates(SMALL, nblk * B, og.np).astype(dtype)
    P = kb.project(H.proj, z.astype(np.complex128))
    tp = torch.from_numpy(rsd.to_blocks(z, B)).to(DEV)
    proj = torch.empty((nblk, nl.nat, nl.nproj, B), dtype=tp.dtype, device=DEV)
    rsd.project_nl(g, nl, tp, proj)
    got = proj.cpu().numpy().transpose(0, 3, 1, 2).reshape(nblk * B, nl.nat, nl.nproj)
    assert _relerr(got, P) < tol
    th = torch.zeros_like(tp)
    rsd.apply_nl(g, nl, proj, th)
    torch.cuda.synchronize()
    want = kb.apply_projections(H.proj, got.astype(np.complex128), og.np)
    assert _relerr(rsd.from_blocks(th.cpu().numpy()), want) < tol


@pytest.mark.parametrize("same", [True, False])
def test_overlap_complex128(same):
    og, H, g, nl = _system(SMALL, 1)
    B, nblk = 16, 3
    x = _cstates(SMALL, nblk * B, og.np)
    y = x if same else np.conj(x[::-1]) * (1.0 + 0.5j)
    ctx = rsd.Context(g, 2 * nblk * B)
    tx = torch.from_numpy(rsd.to_blocks(x, B)).to(DEV)
    ty = tx if same else torch.from_numpy(rsd.to_blocks(np.ascontiguousarray(y), B)).to(DEV)
    S = ctx.overlap(tx, ty).cpu().numpy()
    want = linalg.overlap(x, og.dv, y)
    assert S.dtype == np.complex128
    assert np.max(np.abs(S - want)) < 1e-12 * np.max(np.abs(want))
    if same:
        assert np.array_equal(S, S.conj().T)


def test_overlap_complex64_bound():
    og, H, g, nl = _system(SMALL, 1)
    B, nblk = 8, 2
    x = _cstates(SMALL, nblk * B, og.np).astype(np.complex64)
    y = (_cstates(SMALL, nblk * B, og.np)[::-1] * 0.7).astype(np.complex64)
    ctx = rsd.Context(g, 2 * nblk * B)
    tx = torch.from_numpy(rsd.to_blocks(x, B)).to(DEV)
    ty = torch.from_numpy(rsd.to_blocks(np.ascontiguousarray(y), B)).to(DEV)
    S = ctx.overlap(tx, ty).cpu().numpy()
    x64, y64 = x.astype(np.complex128), y.astype(np.complex128)
    want = linalg.overlap(x64, og.dv, y64)
    ax = np.abs(x64.real) + np.abs(x64.imag)
    ay = np.abs(y64.real) + np.abs(y64.imag)
    bound = 2.0 ** -16 * og.dv * ax @ ay.T
    assert np.all(np.abs(S.real - want.real) <= bound)
    assert np.all(np.abs(S.imag - want.imag) <= bound)


def test_complex_block_limits_at_the_c_abi():
    """The C ABI refuses complex blocks of more than 32 states and a complex
    overlap whose 2N real columns exceed the context."""
    import ctypes
    from paper_1306_2953_amd import _abi
    og, H, g, nl = _system(SMALL, 0)
    L = _abi.lib()
    t = torch.zeros((1, og.np, 64), dtype=torch.complex128, device=DEV)
    v = torch.zeros(og.np, dtype=torch.float64, device=DEV)
    o = torch.zeros_like(t)
    rc = L.rs_hpsi_block(g.handle, None, ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                         ctypes.c_void_p(o.data_ptr()), 1, 64, _abi.RS_C128, None)
    assert rc == _abi.RS_EINVAL and b"32" in L.rs_last_error()
    ctx = rsd.Context(g, 16)
    x = torch.zeros((1, og.np, 16), dtype=torch.complex128, device=DEV)
    S = torch.zeros((16, 16), dtype=torch.complex128, device=DEV)
    rc = L.rs_overlap(ctx.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                      ctypes.c_void_p(S.data_ptr()), 1, 16, _abi.RS_C128, _abi.RS_PREC_NATIVE, None)
    assert rc == _abi.RS_EINVAL
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-12), (np.float32, 1e-5)])
def test_full_size_sphere_lmax3_sampled(dtype, tol):
    """The 904k-point sphere with 16 atoms carrying 16 projectors each (l <= 3),
    all 128 states in blocks of 32 (FP64: z-marching kernel and projector
    add; FP32: per-brick kernel and projector add), checked at sampled points
    computed one by one by the oracle."""
    from oracle import stencil
    w = synthetic.WORKLOADS["sphere_r12_h0.2"]
    og, atoms, H0 = hamiltonian.build_system(w, with_projectors=False)
    D = synthetic.couplings_lmax(w, atoms, 3)
    ps = kb.build_projectors(og, atoms.pos, D, w.rc, w.sigma, lmax=3)
    g = rsd.Grid.for_workload(w)
    nl = rsd.NonLocal(g, atoms.pos, D, w.rc, w.sigma, max_states=128, lmax=3)
    psi = _states(w, 128, og.np).astype(dtype)
    v = H0.vloc.astype(dtype)
    got = _hpsi(g, nl, v, psi, 32, dtype, dtype)
    x64 = psi.astype(np.float64)
    rng = np.random.default_rng(13)
    pts = rng.choice(og.np, 300, replace=False)
    sph = np.concatenate(ps.idx)
    pts = np.unique(np.concatenate([pts, rng.choice(sph, 200, replace=False)]))
    want = stencil.apply_local_at(og, v.astype(np.float64), x64, pts)
    want += kb.apply_projections(ps, kb.project(ps, x64), og.np)[:, pts]
    assert _relerr(got[:, pts], want) < tol
