"""The stored reference eigenvalues (tests/golden/*_eigs.txt): written by
tests/golden/make_eigs.py from the oracle's FP64 operator with scipy's
LOBPCG, a route independent of the RMM-DIIS iteration (Sec. 3) whose
converged result they pin.  Checks here: the file's own consistency, and the
stored values against a fresh Rayleigh-Ritz bound that needs no eigensolver.
"""
import os

import numpy as np
import pytest

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    path = os.path.join(HERE, f"{name}_eigs.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    idx = np.array([int(r[0]) for r in rows])
    lam = np.array([float(r[1]) for r in rows])
    res = np.array([float(r[2]) for r in rows])
    return idx, lam, res


@pytest.mark.parametrize("name,n", [("sphere_r12_h0.2", 128), ("periodic96_h0.25", 256)])
def test_golden_eigenvalues_consistent(name, n):
    idx, lam, res = _load(name)
    assert np.array_equal(idx, np.arange(n))
    assert np.all(np.diff(lam) >= 0.0)
    # residual norms of normalised eigenvectors: the eigenvalue error is
    # bounded by the residual (and by residual^2 / gap away from clusters)
    assert np.all(res < 1e-6)
    assert np.all(np.isfinite(lam))


def test_golden_sphere_below_harmonic_like_bounds():
    """Cheap independent bounds on the sphere workload's lowest eigenvalue:
    it lies above min(V) (T is positive semi-definite and the projectors are
    repulsive, D > 0) and below the Rayleigh quotient of a Gaussian centred
    on the deepest well's atom."""
    import synthetic
    from oracle import hamiltonian
    _, lam, _ = _load("sphere_r12_h0.2")
    w = synthetic.WORKLOADS["sphere_r12_h0.2"]
    g, atoms, H = hamiltonian.build_system(w)
    assert lam[0] > H.vloc.min()
    a = int(np.argmax(atoms.depth))
    d2 = np.sum((g.xyz - atoms.pos[a]) ** 2, axis=1)
    best = np.inf
    for width in (0.5, 0.7, 1.0, 1.4):
        x = np.exp(-d2 / (2 * width * width))
        best = min(best, float(x @ H.apply(x)) / float(x @ x))
    assert lam[0] <= best
