"""Oracle: the self-consistent field loop (TEST INFRASTRUCTURE ONLY).

Sec. 3 (Fig. "groundstate"): each SCF iteration builds the Kohn-Sham
potential from the current density, runs a fixed number of eigensolver
iterations, computes the new density (eq. 1b) and mixes it with the old one
(Broyden).  Readings taken where the paper only cites:

  * density: n(r) = sum_k f_k psi_k(r)^2 over the nocc lowest states with
    f_k = 2 (closed shell, real states), psi_k normalised with h^3 sum = 1;
  * potential: V_eff = V_ion + V_H[n] + V_xc[n]; V_ion is the workload's
    local potential (wells), the projectors stay in H; V_H from the FFT
    solve of Sec. 7 (oracle.poisson);
  * exchange-correlation: the local density approximation, unpolarised:
    Dirac exchange eps_x = -(3/4)(3 n / pi)^(1/3), and the Ceperley-Alder
    correlation in the parametrisation of Perdew and Zunger (1981) (their
    published constants, below), with v_xc = d(n eps_xc)/dn;
  * mixing: Broyden's second method in Anderson's form on the density: with
    F = n_out - n_in and the differences dn_j, dF_j of the last m iterates,
    gamma minimises ||F - sum_j gamma_j dF_j|| (h^3-weighted) and
    n_in' = n_in + a F - sum_j gamma_j (dn_j + a dF_j), a the mixing weight;
  * the eigensolver steps are those of oracle.rmmdiis (filter
    preconditioner), iterated k times per SCF iteration on the same states.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import hamiltonian, poisson, rmmdiis
from .linalg import orthonormalize

# Perdew-Zunger (1981) unpolarised correlation: rs >= 1 and rs < 1 branches
PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116


def lda_xc(n: np.ndarray):
    """(v_xc, eps_xc) per point for the density n (points with n <= 0 give
    0, 0)."""
    n = np.asarray(n, dtype=np.float64)
    v = np.zeros_like(n)
    e = np.zeros_like(n)
    pos = n > 0.0
    x = n[pos]
    c13 = (3.0 * x / np.pi) ** (1.0 / 3.0)
    ex = -0.75 * c13
    vx = -c13
    rs = (3.0 / (4.0 * np.pi * x)) ** (1.0 / 3.0)
    ec = np.empty_like(x)
    vc = np.empty_like(x)
    hi = rs >= 1.0
    sr = np.sqrt(rs[hi])
    den = 1.0 + PZ_BETA1 * sr + PZ_BETA2 * rs[hi]
    ec[hi] = PZ_GAMMA / den
    vc[hi] = ec[hi] * (1.0 + (7.0 / 6.0) * PZ_BETA1 * sr + (4.0 / 3.0) * PZ_BETA2 * rs[hi]) / den
    lo = ~hi
    r, lr = rs[lo], np.log(rs[lo])
    ec[lo] = PZ_A * lr + PZ_B + PZ_C * r * lr + PZ_D * r
    vc[lo] = PZ_A * lr + (PZ_B - PZ_A / 3.0) + (2.0 / 3.0) * PZ_C * r * lr + (2.0 * PZ_D - PZ_C) / 3.0 * r
    v[pos] = vx + vc
    e[pos] = ex + ec
    return v, e


def density(psi: np.ndarray, nocc: int) -> np.ndarray:
    """n = 2 sum_{k < nocc} psi_k^2 (psi state-major [N, np])."""
    return 2.0 * np.sum(psi[:nocc] ** 2, axis=0)


@dataclasses.dataclass
class ScfOptions:
    nocc: int = 4
    eig_steps: int = 3       # eigensolver iterations per SCF iteration
    mix: float = 0.3         # mixing weight a
    history: int = 5         # Broyden / Anderson history length m
    tol: float = 1e-6        # ||n_out - n_in|| (h^3-weighted) for convergence


class Mixer:
    """Broyden's second method in Anderson's form on the density."""

    def __init__(self, dv: float, mix: float, history: int):
        self.dv, self.a, self.m = dv, mix, history
        self.prev = None      # (n_in, F) of the previous iteration
        self.dn, self.dF = [], []

    def __call__(self, n_in: np.ndarray, F: np.ndarray) -> np.ndarray:
        if self.prev is not None:
            self.dn.append(n_in - self.prev[0])
            self.dF.append(F - self.prev[1])
            if len(self.dn) > self.m:
                self.dn.pop(0)
                self.dF.pop(0)
        self.prev = (n_in.copy(), F.copy())
        out = n_in + self.a * F
        if self.dF:
            A = np.array([[self.dv * (x @ y) for y in self.dF] for x in self.dF])
            b = np.array([self.dv * (x @ F) for x in self.dF])
            gam = np.linalg.lstsq(A, b, rcond=None)[0]
            for g, dn, dF in zip(gam, self.dn, self.dF):
                out = out - g * (dn + self.a * dF)
        return out


def effective_potential(g, vion: np.ndarray, n: np.ndarray, rc=None, nbox=None) -> np.ndarray:
    vh = poisson.hartree(g, n, rc, nbox)
    vxc, _ = lda_xc(n)
    return vion + vh + vxc


def scf(H: hamiltonian.Hamiltonian, psi: np.ndarray, opts: ScfOptions, eig_opts: rmmdiis.Options,
        max_iter: int, apply=None):
    """Iterates from the states psi [N, np]; returns (psi, history of
    (||F||, eigenvalues)).  apply(Heff): an optional factory that returns an
    object with the Hamiltonian interface for a given effective potential
    (to use a faster H psi); by default the numpy operator."""
    g = H.g
    vion = H.vloc.copy()
    psi, _, _ = orthonormalize(psi, g.dv)
    n_in = density(psi, opts.nocc)
    mixer = Mixer(g.dv, opts.mix, opts.history)
    hist = []
    for it in range(max_iter):
        Heff = hamiltonian.Hamiltonian(g, effective_potential(g, vion, n_in), H.proj)
        Hop = apply(Heff) if apply is not None else Heff
        for _ in range(opts.eig_steps):
            out = rmmdiis.rmmdiis_step(Hop, psi, eig_opts)
            psi = out["psi"]
        n_out = density(psi, opts.nocc)
        F = n_out - n_in
        res = float(np.sqrt(g.dv * (F @ F)))
        hist.append((res, out["eig"].copy()))
        if res < opts.tol:
            break
        n_in = mixer(n_in, F)
    return psi, hist
