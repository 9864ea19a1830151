"""GPU SCF loop (Sec. 3) against the oracle's loop on the same start, and
its converged result against the dense eigenproblem of its own effective
Hamiltonian."""
import numpy as np
import pytest

import synthetic
from oracle import hamiltonian, linalg, rmmdiis, scf as oscf

torch = pytest.importorskip("torch")
import paper_1306_2953_amd as rsd  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"


W = synthetic.make_workload("sphere_r12_h0.2", radius=2.4, h=0.3, nat=2, atom_radius=0.8, rc=1.0, nstates=8)


def _setup():
    og, atoms, H = hamiltonian.build_system(W)
    g = rsd.Grid.for_workload(W)
    nl = rsd.NonLocal(g, atoms.pos, atoms.D, W.rc, W.sigma, max_states=8)
    psi = synthetic.draw_states(synthetic.rng_after_atoms(W), 8, og.np)
    return og, H, g, nl, psi


def test_scf_matches_oracle_and_is_self_consistent():
    og, H, g, nl, psi = _setup()
    opts = oscf.ScfOptions(nocc=1, eig_steps=3, mix=0.3, history=5, tol=1e-9)
    want_psi, want = oscf.scf(H, psi, opts, rmmdiis.Options(m=3, block=8, tol=1e-12), max_iter=40)
    s = rsd.Scf(g, nl, torch.from_numpy(H.vloc).cuda(), 8, 8, nocc=1, eig_steps=3, mix=0.3, history=5, tol=1e-12)
    t = torch.from_numpy(rsd.to_blocks(psi, 8)).cuda()
    s.start(t)
    got = []
    for it in range(len(want)):
        eig, res, dr = s.iterate(t)
        got.append((dr, eig))
    # the occupied state and the next three follow the oracle to 1e-8 Ha;
    # the upper states of the set (a near-degenerate cluster at 2.56-2.61 Ha
    # that three eigensolver steps per iteration never converge) drift
    # apart by rounding order, and are held to 1e-6 Ha
    for it, ((dg, eg), (dw, ew)) in enumerate(zip(got, want)):
        print(f"iter {it}: density residual {dg:.6e} (oracle {dw:.6e}), eig0 {eg[0]:.12f} ({ew[0]:.12f}), "
              f"max eig difference {np.max(np.abs(eg - ew)):.2e}")
        assert abs(dg - dw) <= 1e-6 * dw + 1e-12
        assert np.max(np.abs(eg[:4] - ew[:4])) < 1e-8
        assert np.max(np.abs(eg - ew)) < 1e-6
    assert got[-1][0] < 1e-9
    # self-consistency: the GPU's final density is the ground-state density
    # of the dense effective Hamiltonian built from it
    n_in, n_out = s.densities()
    n = n_out.cpu().numpy()
    Heff = hamiltonian.Hamiltonian(og, oscf.effective_potential(og, H.vloc, n), H.proj)
    ev, vec = np.linalg.eigh(Heff.dense())
    n_dense = oscf.density((vec / np.sqrt(og.dv)).T, 1)
    assert np.max(np.abs(n_dense - n)) < 1e-6 * np.max(n)
    assert np.max(np.abs(got[-1][1][:4] - ev[:4])) < 1e-7


def test_scf_split_precision_converges_to_the_fp64_result():
    og, H, g, nl, psi = _setup()
    res = {}
    for dt in (torch.float64, torch.float32):
        s = rsd.Scf(g, nl, torch.from_numpy(H.vloc).cuda(), 8, 8, nocc=1, dtype=dt, tol=1e-12)
        npdt = np.float64 if dt == torch.float64 else np.float32
        t = torch.from_numpy(rsd.to_blocks(psi.astype(npdt), 8)).cuda()
        s.start(t)
        for it in range(40):
            eig, r, dr = s.iterate(t)
            if dr < (1e-9 if dt == torch.float64 else 1e-5):
                break
        res[dt] = (eig, dr)
        print(f"{dt}: {it + 1} iterations, density residual {dr:.2e}, eig0 {eig[0]:.10f}")
    assert res[torch.float32][1] < 1e-5
    assert np.max(np.abs(res[torch.float32][0][:4] - res[torch.float64][0][:4])) < 1e-5


def test_scf_bad_options_raise():
    og, H, g, nl, psi = _setup()
    v = torch.from_numpy(H.vloc).cuda()
    for kw in (dict(nocc=0), dict(nocc=9), dict(history=9), dict(mix=0.0), dict(eig_steps=0)):
        args = dict(nocc=1)
        args.update(kw)
        with pytest.raises(rsd.RsError) as e:
            rsd.Scf(g, nl, v, 8, 8, **args)
        assert e.value.code == rsd._abi.RS_EINVAL
