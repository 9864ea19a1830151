"""Training driver for the learned preconditioner (rs_cnn).

Pairs come from the method itself: the residuals R0 of plain (filter)
eigensolver steps, their shifts sigma_k = -<psi_k|T|psi_k>, and targets
x = (T - sigma)^-1 R0 from the library's conjugate-gradient solve.  They are
stored as random cubic crops of the whole-grid fields, scaled by the rms of
the residual, and the network is trained with the library's loss/gradient
and Adam kernels.  Every computation runs in the library; this module only
orders the calls and picks the random crops and batches (host RNG).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import Cnn, Eigensolver, Grid, shifted_solve


def init_params(seed: int) -> np.ndarray:
    """Scaled normal weights (std 1/sqrt(fan-in)); gain a = 0, b = -1, so
    g = softplus(-log(-sigma h^2)) starts near the scale of (T - sigma)^-1."""
    rng = np.random.default_rng(seed)
    p = np.zeros(Cnn.NPARAM)
    p[0:216] = rng.normal(scale=1.0 / np.sqrt(27.0), size=216)
    p[216:1944] = rng.normal(scale=1.0 / np.sqrt(216.0), size=1728)
    p[1944:2160] = rng.normal(scale=1.0 / np.sqrt(216.0), size=216)
    p[2160], p[2161] = 0.0, -1.0
    return p.astype(np.float32)


@dataclasses.dataclass
class Pairs:
    u: object          # device float32 [n, C, C, C]   r / s
    t: object          # device float32 [n, C, C, C]   x / s
    sigma: object      # device float64 [n]
    state: np.ndarray  # host int [n], the state each crop came from

    @property
    def n(self) -> int:
        return int(self.u.shape[0])

    def subset(self, keep: np.ndarray) -> "Pairs":
        import torch
        idx = torch.from_numpy(np.nonzero(keep)[0]).to(self.u.device)
        return Pairs(self.u[idx], self.t[idx], self.sigma[idx], self.state[keep])


def collect_pairs(grid: Grid, solver: Eigensolver, psi, net: Cnn, steps: int, crops_per_state: int,
                  crop: int, rng: np.random.Generator, cg_tol: float = 1e-6, cg_maxit: int = 4000,
                  log=None) -> Pairs:
    """Runs `steps` solver steps on psi (in place; the solver must record)
    and cuts crops_per_state crops of edge `crop` per state and step."""
    import torch
    dims = net.box(grid)                      # (Z, Y, X)
    us, ts, ss, st = [], [], [], []
    for k in range(steps):
        solver.step(psi)
        R, sig = solver.residuals()
        X, it = shifted_solve(grid, R, sig, tol=cg_tol, maxit=cg_maxit)
        N = solver.nstates
        n = N * crops_per_state
        desc = np.empty((n, 4), dtype=np.int32)
        desc[:, 0] = np.repeat(np.arange(N), crops_per_state)
        for a, d in zip((1, 2, 3), (dims[2], dims[1], dims[0])):
            desc[:, a] = rng.integers(0, d, size=n)
        u, t = net.crops(grid, R, X, desc, (crop, crop, crop))
        us.append(u)
        ts.append(t)
        ss.append(sig[torch.from_numpy(desc[:, 0].astype(np.int64)).to(sig.device)])
        st.append(desc[:, 0].copy())
        if log is not None:
            log(f"collect step {k}: cg iterations {it}")
    return Pairs(torch.cat(us), torch.cat(ts), torch.cat(ss), np.concatenate(st))


def cosine_lr(lr0: float, lr1: float, iters: int):
    """Learning rate falling from lr0 to lr1 along half a cosine."""
    return lambda it: lr1 + 0.5 * (lr0 - lr1) * (1.0 + np.cos(np.pi * min(it, iters) / iters))


def train(net: Cnn, pairs: Pairs, h: float, iters: int, batch: int, lr, margin: int,
          rng: np.random.Generator, val: Optional[Pairs] = None, log_every: int = 0, log=None) -> List[float]:
    """Adam on random batches (lr: a number or a function of the iteration);
    returns the training-loss history (and logs the validation loss every
    log_every iterations when val is given)."""
    import torch
    hist = []
    dev = pairs.u.device
    lr_at = lr if callable(lr) else (lambda it: lr)
    for it in range(iters):
        idx = torch.from_numpy(rng.integers(0, pairs.n, size=batch)).to(dev)
        hist.append(net.train_step(pairs.u[idx], pairs.t[idx], pairs.sigma[idx], h, margin, float(lr_at(it))))
        if log is not None and log_every and (it + 1) % log_every == 0:
            msg = f"train iter {it + 1}: loss {hist[-1]:.4e}"
            if val is not None:
                msg += f", validation {evaluate(net, val, h, margin, batch):.4e}"
            log(msg)
    return hist


def evaluate(net: Cnn, pairs: Pairs, h: float, margin: int, batch: int) -> float:
    """Mean loss over all pairs (in batches of at most `batch`)."""
    tot, n = 0.0, pairs.n
    for i in range(0, n, batch):
        j = min(n, i + batch)
        loss, _, _ = net.loss_grad(pairs.u[i:j], pairs.t[i:j], pairs.sigma[i:j], h, margin)
        tot += loss * (j - i)
    return tot / n
