"""What the trained network gains over the filter (A/B on the same seeds).

The network is trained on the GPU by the library's own kernels on pairs the
method generates (residuals of plain filter steps and their shifted-kinetic
CG solutions), then both preconditioners run the same number of RMM-DIIS
steps from the same start on a small periodic system (32^3 points, h 0.25,
four wells with projectors, 32 FP32 states).  The gain has no pin in the
paper: the assertion is the measured improvement, with a wide margin.  The
run is deterministic (fixed seeds, fixed-order reductions).  A shorter
schedule (8 000 steps) gave a network whose solve stalled, so the test
trains for 20 000 steps and asks for a validation loss below 0.05."""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
import paper_1306_2953_amd as rsd  # noqa: E402
from paper_1306_2953_amd import learned  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"


def _system():
    w = synthetic.make_workload("periodic96_h0.25", n=32, nat=4, nstates=32, block=32)
    g = rsd.Grid.for_workload(w)
    atoms = synthetic.draw_atoms(w)
    v = synthetic.potential_for(w, g.xyz(), atoms)
    nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=w.nstates)
    tv = torch.from_numpy(v.astype(np.float32)).cuda()
    psi = synthetic.draw_states(synthetic.rng_after_atoms(w), w.nstates, g.np).astype(np.float32)
    tp = torch.from_numpy(rsd.to_blocks(psi, w.block)).cuda()
    rsd.Context(g, w.nstates).orthonormalize(tp)
    return w, g, nl, tv, tp


def _solve(w, g, nl, tv, psi0, net, steps):
    s = rsd.Eigensolver(g, nl, tv, w.nstates, w.block, tol=1e-4)
    if net is not None:
        s.set_precond(net)
    x = psi0.clone()
    for _ in range(steps):
        eig, res, _ = s.step(x)
    return eig, res


def test_trained_network_beats_filter():
    w, g, nl, tv, psi0 = _system()
    net = rsd.Cnn(32, g.np)
    net.set_params(learned.init_params(0))
    rng = np.random.default_rng(0)
    rec = rsd.Eigensolver(g, nl, tv, w.nstates, w.block, tol=1e-4, record=True)
    pairs = learned.collect_pairs(g, rec, psi0.clone(), net, steps=30, crops_per_state=2, crop=16, rng=rng,
                                  cg_tol=1e-5)
    val = pairs.subset(pairs.state % 10 == 9)
    tr = pairs.subset(pairs.state % 10 != 9)
    iters = 20000
    learned.train(net, tr, g.h, iters=iters, batch=32, lr=learned.cosine_lr(3e-3, 1e-5, iters), margin=3,
                  rng=rng)
    vloss = learned.evaluate(net, val, g.h, 3, 32)
    print(f"validation energy-norm loss {vloss:.3e}")
    assert vloss < 0.05
    steps = 80
    ef, rf = _solve(w, g, nl, tv, psi0, None, steps)
    ec, rc = _solve(w, g, nl, tv, psi0, net, steps)
    print(f"after {steps} steps: median residual filter {np.median(rf):.3e} network {np.median(rc):.3e}; "
          f"lowest eigenvalue filter {ef[0]:.8f} network {ec[0]:.8f}")
    assert np.all(np.isfinite(ec)) and np.all(np.isfinite(rc))
    assert np.median(rc) < 0.25 * np.median(rf)
    # the lowest eigenvalue is an upper bound: the better solve is lower
    assert ec[0] < ef[0]
