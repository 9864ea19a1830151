"""Oracle: lowest eigenvalues of the discrete H by an independent route
(TEST INFRASTRUCTURE ONLY).

The converged result of any eigensolver of Sec. 3 is the lowest N eigenvalues
of the discrete operator H = T + V + V_nl (Sec. 5, eq. (6)), a plain
definition that does not depend on the RMM-DIIS iteration.  Here they are
computed with scipy's block LOBPCG (Knyazev 2001), a library routine unrelated
to RMM-DIIS, on the oracle's operator:

  * H is applied by the C/OpenMP oracle (``cpu_hpsi``), FP64, which the
    Python oracle pins (polynomial exactness, plane-wave symbol, dense brute
    force);
  * the preconditioner is (T + c)^-1 of the same 25-point stencil on a
    periodic box that holds the domain (diagonal in Fourier space with the
    closed-form symbol of ``stencil.kinetic_symbol``), restricted to the
    domain's points.  It only changes how fast LOBPCG converges: a restricted
    inverse of a positive definite operator is positive definite, so the
    limit is the same.

Grid inner products are h^3-weighted sums; LOBPCG works in the Euclidean
inner product, which has the same eigenvalues (the weight is a constant).
"""
from __future__ import annotations

import time
from typing import Optional

import numpy as np
import scipy.fft
import scipy.sparse.linalg

from . import cpu_hpsi, stencil


class _Operator:
    """X [np, k] -> H X through the C oracle (blocks of at most 32 states)."""

    def __init__(self, H, log=None):
        self.ch = cpu_hpsi.CpuHamiltonian(H)
        self.np = H.g.np
        self.calls = 0
        self.log = log
        self.t0 = time.perf_counter()

    def __call__(self, X: np.ndarray) -> np.ndarray:
        X = np.asarray(X, dtype=np.float64)
        one = X.ndim == 1
        X2 = X.reshape(self.np, -1)
        out = np.empty_like(X2)
        for j0 in range(0, X2.shape[1], 32):
            j1 = min(j0 + 32, X2.shape[1])
            blk = np.ascontiguousarray(X2[:, j0:j1])[None]
            out[:, j0:j1] = self.ch.hpsi_blocks(blk)[0]
        self.calls += X2.shape[1]
        if self.log and X2.shape[1] > 1:
            self.log(f"  H applied to {X2.shape[1]} columns ({self.calls} in total, "
                     f"{time.perf_counter() - self.t0:.0f} s)")
        return out[:, 0] if one else out


class _KineticPreconditioner:
    """r -> restriction of (T + c)^-1 on a periodic box of edge n >= the
    domain's extent + 2M, embedding the domain's points by their integer
    coordinates."""

    def __init__(self, g, shift: float, workers: int = 8):
        ext = (g.inner.max(axis=0) - g.inner.min(axis=0)) + 1
        n = scipy.fft.next_fast_len(int(ext.max()) + 2 * g.M, real=True)
        if g.periodic:
            n = int(g.L[0])
        self.n = n
        u = g.inner - g.inner.min(axis=0)
        if not g.periodic:
            u = u + (n - ext) // 2
        self.flat = np.ravel_multi_index((u[:, 2], u[:, 1], u[:, 0]), (n, n, n))
        k1 = 2.0 * np.pi * np.fft.fftfreq(n, d=g.h)
        kz = k1[:, None, None]
        ky = k1[None, :, None]
        kx = 2.0 * np.pi * np.fft.rfftfreq(n, d=g.h)[None, None, :]
        k = np.stack(np.broadcast_arrays(kx, ky, kz), axis=-1)
        self.inv = 1.0 / (stencil.kinetic_symbol(k, g.h, g.M) + shift)
        self.workers = workers
        self.np = g.np

    def __call__(self, R: np.ndarray) -> np.ndarray:
        R = np.asarray(R, dtype=np.float64)
        one = R.ndim == 1
        R2 = R.reshape(self.np, -1)
        out = np.empty_like(R2)
        n = self.n
        for j0 in range(0, R2.shape[1], 8):
            j1 = min(j0 + 8, R2.shape[1])
            box = np.zeros((j1 - j0, n * n * n))
            box[:, self.flat] = R2[:, j0:j1].T
            f = scipy.fft.rfftn(box.reshape(j1 - j0, n, n, n), axes=(1, 2, 3), workers=self.workers)
            f *= self.inv[None]
            x = scipy.fft.irfftn(f, s=(n, n, n), axes=(1, 2, 3), workers=self.workers)
            out[:, j0:j1] = x.reshape(j1 - j0, -1)[:, self.flat].T
        return out[:, 0] if one else out


def lowest_eigs(H, nev: int, nguard: int, tol: float, maxiter: int, seed: int = 12345,
                shift: float = 1.0, log: Optional[callable] = None):
    """Lowest ``nev`` eigenvalues of H (FP64) by LOBPCG with nev + nguard
    vectors.  Returns (eigenvalues [nev], residual norms [nev] of the
    normalised eigenvectors, eigenvectors [np, nev], seconds)."""
    g = H.g
    op = _Operator(H, log)
    A = scipy.sparse.linalg.LinearOperator((g.np, g.np), matvec=op, matmat=op, dtype=np.float64)
    P = _KineticPreconditioner(g, shift)
    M = scipy.sparse.linalg.LinearOperator((g.np, g.np), matvec=P, matmat=P, dtype=np.float64)
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(g.np, nev + nguard))
    X = P(P(X))                               # smooth the random start
    t0 = time.perf_counter()
    lam, V = scipy.sparse.linalg.lobpcg(A, X, M=M, tol=tol, maxiter=maxiter, largest=False,
                                        verbosityLevel=0)
    el = time.perf_counter() - t0
    order = np.argsort(lam)
    lam, V = lam[order], V[:, order]
    V = V / np.linalg.norm(V, axis=0)
    R = op(V[:, :nev]) - V[:, :nev] * lam[None, :nev]
    res = np.linalg.norm(R, axis=0)
    if log:
        log(f"lobpcg: {nev + nguard} vectors, {el:.0f} s, {op.calls} column applications, "
            f"max residual of the lowest {nev}: {res.max():.2e}")
    return lam[:nev], res, V[:, :nev], el
