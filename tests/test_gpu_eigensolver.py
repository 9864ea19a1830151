"""GPU eigensolver (RMM-DIIS step, filter, block stop) against the oracle's
step, and converged eigenvalues against the exact discrete spectra."""
import numpy as np
import pytest

import synthetic
from oracle import hamiltonian, linalg, rmmdiis

torch = pytest.importorskip("torch")
import paper_1306_2953_amd as rsd  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"


def _setup(w, N, B, dtype=np.float64, **kw):
    og, atoms, H = hamiltonian.build_system(w)
    g = rsd.Grid.for_workload(w)
    nl = None
    if atoms is not None:
        nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=-(-N // B) * B)
    v = torch.from_numpy(H.vloc.astype(dtype)).to(DEV)
    solver = rsd.Eigensolver(g, nl, v, N, B, **kw)
    psi = synthetic.draw_states(synthetic.rng_after_atoms(w), N, og.np)
    psi, _, _ = linalg.orthonormalize(psi, og.dv)
    return og, H, g, solver, psi


@pytest.mark.parametrize("m", [1, 2, 3])
def test_one_step_matches_oracle(m):
    """The same step on the same orthonormal input: eigenvalues, residual norms
    and the updated states agree with the oracle's implementation."""
    w = synthetic.make_workload("sphere_r12_h0.2", radius=2.4, nat=3, atom_radius=1.2)
    N, B = 16, 8
    og, H, g, solver, psi = _setup(w, N, B, m=m, tol=1e-12)
    # a few oracle steps first so the states are not random noise
    opts = rmmdiis.Options(m=m, block=B, tol=1e-12)
    for _ in range(3):
        psi = rmmdiis.rmmdiis_step(H, psi, opts)["psi"]
    want = rmmdiis.rmmdiis_step(H, psi, opts)
    t = torch.from_numpy(rsd.to_blocks(psi, B)).to(DEV)
    eig, res, nconv = solver.step(t)
    got = rsd.from_blocks(t.cpu().numpy())
    assert np.max(np.abs(eig - want["eig"])) < 1e-10 * np.max(np.abs(want["eig"]))
    assert np.max(np.abs(res - want["resnorm"])) < 1e-8 * np.max(want["resnorm"])
    assert np.max(np.abs(got - want["psi"])) < 1e-7 * np.max(np.abs(want["psi"]))


def test_block_stop_freezes_converged_blocks():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=2.4, nat=3, atom_radius=1.2)
    N, B = 16, 8
    og, H, g, solver, psi = _setup(w, N, B, tol=1e9)
    t = torch.from_numpy(rsd.to_blocks(psi, B)).to(DEV)
    eig, res, nconv = solver.step(t)
    assert nconv == N
    lam, xi, p2, _ = linalg.rayleigh_ritz(psi, H.apply(psi), og.dv)
    p2, _, _ = linalg.orthonormalize(p2, og.dv)
    got = rsd.from_blocks(t.cpu().numpy())
    assert np.max(np.abs(got - p2)) < 1e-9 * np.max(np.abs(p2))


def test_converges_harmonic_box():
    """Lowest four levels of the 32^3 harmonic box from random states."""
    w = synthetic.make_workload("box32_harmonic", nstates=4)
    og, H, g, solver, psi = _setup(w, 4, 4, tol=1e-9)
    t = torch.from_numpy(rsd.to_blocks(psi, 4)).to(DEV)
    want = np.array([1.4999991750, 2.4999964915, 2.4999964915, 2.4999964915])
    for it in range(150):
        eig, res, nconv = solver.step(t)
        if nconv == 4:
            break
    assert np.max(np.abs(eig - want)) < 1e-9
    assert np.max(res) < 1e-9


@pytest.mark.parametrize("dtype,etol", [(np.float64, 1e-10), (np.float32, 1e-6)])
def test_converges_dense_bruteforce(dtype, etol):
    """Tiny sphere with wells and projectors: lowest eigenvalues of the dense
    matrix; the FP32 / split-precision solve reaches them to 1e-6 Ha."""
    w = synthetic.make_workload("sphere_r12_h0.2", radius=1.6, h=0.2, nat=2, atom_radius=0.6, rc=1.0)
    og, H, g, solver, psi = _setup(w, 8, 8, dtype=dtype, tol=1e-9 if dtype == np.float64 else 1e-5)
    ev = np.linalg.eigvalsh(H.dense())[:8]
    t = torch.from_numpy(rsd.to_blocks(psi.astype(dtype), 8)).to(DEV)
    best = np.inf
    for it in range(300):
        eig, res, nconv = solver.step(t)
        best = np.max(np.abs(eig - ev))
        if best < etol / 10:
            break
    assert best < etol


def test_partial_last_block_step_matches_oracle():
    """12 states in blocks of 8: the last block holds 4 zero padding states.
    The step agrees with the oracle's on the 12 states (whose stopping rule
    sees a block of 4), and the padding stays exactly zero."""
    w = synthetic.make_workload("sphere_r12_h0.2", radius=2.4, nat=3, atom_radius=1.2)
    N, B = 12, 8
    og, H, g, solver, psi = _setup(w, N, B, tol=1e-12)
    opts = rmmdiis.Options(m=3, block=B, tol=1e-12)
    for _ in range(3):
        psi = rmmdiis.rmmdiis_step(H, psi, opts)["psi"]
    want = rmmdiis.rmmdiis_step(H, psi, opts)
    t = torch.from_numpy(rsd.to_blocks(psi, B)).to(DEV)
    assert tuple(t.shape) == (2, og.np, B)
    eig, res, nconv = solver.step(t)
    assert eig.shape == (N,) and res.shape == (N,)
    full = rsd.from_blocks(t.cpu().numpy())
    assert np.all(full[N:] == 0.0)
    got = full[:N]
    assert np.max(np.abs(eig - want["eig"])) < 1e-10 * np.max(np.abs(want["eig"]))
    assert np.max(np.abs(res - want["resnorm"])) < 1e-8 * np.max(want["resnorm"])
    assert np.max(np.abs(got - want["psi"])) < 1e-7 * np.max(np.abs(want["psi"]))


@pytest.mark.parametrize("dtype,etol", [(np.float64, 1e-10), (np.float32, 1e-6)])
def test_partial_last_block_converges(dtype, etol):
    """6 states in blocks of 4 (two padding states) reach the lowest six
    eigenvalues of the dense matrix of a tiny sphere."""
    w = synthetic.make_workload("sphere_r12_h0.2", radius=1.6, h=0.2, nat=2, atom_radius=0.6, rc=1.0)
    og, H, g, solver, psi = _setup(w, 6, 4, dtype=dtype, tol=1e-9 if dtype == np.float64 else 1e-5)
    ev = np.linalg.eigvalsh(H.dense())[:6]
    t = torch.from_numpy(rsd.to_blocks(psi.astype(dtype), 4)).to(DEV)
    best = np.inf
    for it in range(300):
        eig, res, nconv = solver.step(t)
        best = np.max(np.abs(eig - ev))
        if best < etol / 10:
            break
    assert best < etol
    assert np.all(rsd.from_blocks(t.cpu().numpy())[6:] == 0.0)


def test_cage_workload_full_size_steps():
    """The largest workload (sphere R 18 at h 0.18, 4.19M points, 60 atoms on
    a cage), 240 FP32 states in blocks of 64 (one padded block): three steps
    run, keep the padding zero, and lower every Rayleigh-Ritz value."""
    w = synthetic.WORKLOADS["sphere_r18_h0.18_cage60"]
    g = rsd.Grid.for_workload(w)
    atoms = synthetic.draw_atoms(w)
    v = synthetic.potential_for(w, g.xyz(), atoms)
    nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=256)
    tv = torch.from_numpy(v.astype(np.float32)).to(DEV)
    psi = synthetic.draw_states(synthetic.rng_after_atoms(w), w.nstates, g.np).astype(np.float32)
    t = torch.from_numpy(rsd.to_blocks(psi, w.block)).to(DEV)
    del psi
    assert tuple(t.shape) == (4, g.np, 64)
    solver = rsd.Eigensolver(g, nl, tv, w.nstates, w.block)
    solver.orthonormalize(t)
    eigs = [solver.step(t)[0] for _ in range(3)]
    assert all(e.shape == (240,) and np.all(np.isfinite(e)) for e in eigs)
    assert np.all(eigs[2] <= eigs[0] + 1e-6 * np.abs(eigs[0]))
    assert torch.count_nonzero(t[3, :, 48:]).item() == 0


def test_bad_solver_arguments_raise():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=2.4, nat=3, atom_radius=1.2)
    g = rsd.Grid.for_workload(w)
    v = torch.zeros(g.np, dtype=torch.float64, device=DEV)
    for n, B in ((0, 8), (257, 8), (16, 3), (16, 128)):
        with pytest.raises(rsd.RsError) as e:
            rsd.Eigensolver(g, None, v, n, B)
        assert e.value.code == rsd._abi.RS_EINVAL
