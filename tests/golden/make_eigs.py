#!/usr/bin/env python3
"""Writes the reference eigenvalues of a workload into tests/golden/.

The stored values are the lowest ``nev`` eigenvalues of the FP64 operator
H = T + V + V_nl of the named synthetic workload (Sec. 5 and eq. (6)), computed
by scipy's LOBPCG on the oracle's operator (``oracle.lobpcg_ref``).  Only
``oracle/`` and ``synthetic/`` are used.  One line per eigenvalue: index,
eigenvalue (Ha), residual norm |H v - lambda v| of the normalised vector.

Usage: python tests/golden/make_eigs.py [--workload sphere_r12_h0.2]
           [--nev 128] [--nguard 32] [--tol 1e-7] [--maxiter 400]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synthetic  # noqa: E402
from oracle import cpu_hpsi, hamiltonian, lobpcg_ref  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="sphere_r12_h0.2")
    ap.add_argument("--nev", type=int, default=128)
    ap.add_argument("--nguard", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--maxiter", type=int, default=400)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    cpu_hpsi.build()
    w = synthetic.WORKLOADS[a.workload]
    t0 = time.perf_counter()
    og, atoms, H = hamiltonian.build_system(w)
    print(f"system: {og.np} points, {w.nat} atoms ({time.perf_counter() - t0:.0f} s)", flush=True)
    lam, res, _, el = lobpcg_ref.lowest_eigs(H, a.nev, a.nguard, a.tol, a.maxiter,
                                             log=lambda s: print(s, flush=True))
    out = a.out or os.path.join(HERE, f"{w.name}_eigs.txt")
    with open(out, "w") as f:
        f.write(f"# lowest {a.nev} eigenvalues (Ha) of the FP64 H = T + V + V_nl of workload {w.name}\n")
        f.write(f"# ({og.np} grid points, {w.nat} atoms, seed {w.seed}): scipy.sparse.linalg.lobpcg with "
                f"{a.nev + a.nguard} vectors,\n")
        f.write("# H applied by the C oracle, preconditioner (T + 1)^-1 on an enclosing periodic box "
                "(oracle/lobpcg_ref.py);\n")
        f.write(f"# written by tests/golden/make_eigs.py, tol {a.tol:g}, {el:.0f} s.\n")
        f.write("# columns: index, eigenvalue, residual norm of the normalised eigenvector\n")
        for k in range(a.nev):
            f.write(f"{k} {lam[k]:.15e} {res[k]:.3e}\n")
    print(f"wrote {out}: max residual {res.max():.2e}", flush=True)


if __name__ == "__main__":
    main()
