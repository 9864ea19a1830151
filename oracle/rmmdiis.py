"""Oracle: one RMM-DIIS eigensolver step with the filter preconditioner
(TEST INFRASTRUCTURE ONLY).

Sec. 3: each SCF iteration runs a fixed number of RMM-DIIS iterations on the
Kohn-Sham Hamiltonian, preconditioned with a low-pass filter; the method needs
H psi, orthogonalisation and subspace diagonalisation (Sec. 6).  Sec. 9: a
block of states stops iterating only when every state of the block is below
the threshold.  The RMM-DIIS body itself is only cited by the paper; the
reading taken here is:

  1. H psi for all states; Rayleigh-Ritz (eqs. 9-10) gives eps_k.
  2. Per state: R0 = H psi0 - eps0 psi0 (eps0 the Rayleigh quotient),
     d = K R0; the trial step lambda minimises the Rayleigh quotient of
     psi0 + lambda d (lowest eigenpair (x, y) of the 2x2 problem in the
     basis {psi0, d/||d||}, lambda = y / (x ||d||)); psi1 = psi0 + lambda d,
     H psi1 = H psi0 + lambda H d.  (Minimising the residual norm along d
     instead moves random starting states up the spectrum.)
  3. For j = 1 .. m-1: with residuals R_i = H psi_i - eps_i psi_i of every
     iterate so far, minimise ||sum c R|| / ||sum c psi|| over the history
     (generalised eigenproblem A c = mu B c, lowest mu).  The history is
     expressed in the basis {psi_L, psi_i - psi_L} (L the latest iterate), and
     c is normalised so its first component is one (coefficients on the
     original iterates then sum to one).  psibar, H psibar and Rbar follow
     from c; d = K Rbar; psi_{j+1} = psibar + lambda d (lambda from step 2),
     H psi_{j+1} = H psibar + lambda H d.
  4. Orthonormalise all states (Cholesky, eq. 8).
A state whose lambda is exactly zero keeps psi0.  The filter is
K r_p = alpha r_p + (1 - alpha)/6 sum of the six nearest neighbours (zero
outside the domain), alpha = 0.52.  Its symbol alpha + (1 - alpha)/3 sum_a
cos(k_a h) is 1 at k = 0 and 2 alpha - 1 at the Nyquist corner; with
alpha = 1/2 it vanishes there, and on a periodic grid with an even number of
points per edge the alternating vector (-1)^(i+j+k) is then an exact null
vector of K: no update can change the states' components along it, and the
random start's share of it stays in the residuals as a floor (~1e-2 on a
periodic 48^3 box).  Any alpha > 1/2 keeps the symbol positive; 0.52
(corner symbol 0.04) keeps the filter close to the smoothing it is meant to
be: the closer alpha is to 1, the more the filter acts like the identity and
the slower the high-energy residual decays.

With a learned preconditioner K_n (the project's addition, ``oracle.cnn``)
the network does not replace the filter K_f: it adds a second direction.
The trial step minimises the Rayleigh quotient over span{psi0, d_f, d_n},
d_f = K_f R0, d_n = K_n R0 (lowest eigenpair of the 3x3 generalised problem
in the basis {psi0, d_f/|d_f|, d_n/|d_n|}, first component scaled to one),
which gives per state the coefficients (a, b) of K = a K_f + b K_n.  That K
is the state's preconditioner for the rest of the step, with lambda = 1:
psi1 = psi0 + K R0 and psi_{j+1} = psibar + K Rbar.  The filter is always in
the trial subspace, so a useless network gets b ~ 0 and the step is the
filter's; when the 3x3 problem is singular (d_n parallel to d_f, zero or not
finite) the state takes the filter step of step 2 (b = 0).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.linalg

from .grid import Grid, neighbour_table
from .linalg import dots, orthonormalize, rayleigh_ritz


@dataclasses.dataclass
class Options:
    m: int = 3               # iterates built per step (H d applications)
    alpha: float = 0.52      # filter centre weight
    tol: float = 1e-6        # residual-norm threshold
    block: int = 32          # block size for the stopping rule
    block_stop: bool = True


def filter_precond(g: Grid, r: np.ndarray, nbr: Optional[np.ndarray] = None,
                   alpha: float = 0.52) -> np.ndarray:
    """K r = alpha r + (1 - alpha)/6 (sum of the 6 nearest neighbours)."""
    if nbr is None:
        nbr = neighbour_table(g)
    x = np.atleast_2d(r)
    # point-major copy with a zero row for "outside": neighbour gathers are
    # row gathers
    xt = np.concatenate([x.T, np.zeros((1, x.shape[0]))], axis=0)
    idx = np.where(nbr[:, :, :, 0] < 0, g.np, nbr[:, :, :, 0])   # m = 1
    s = np.zeros_like(xt[:-1])
    for a in range(3):
        s = s + (xt[idx[:, a, 0]] + xt[idx[:, a, 1]])
    out = alpha * x + (1.0 - alpha) / 6.0 * s.T
    return out if r.ndim == 2 else out[0]


def diis_coefficients(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Lowest generalised eigenvector of A c = mu B c with c[0] = 1;
    falls back to c = e_0 when B is not positive definite."""
    try:
        mu, vec = scipy.linalg.eigh(A, B)
    except np.linalg.LinAlgError:
        vec = None
    c = np.zeros(A.shape[0])
    c[0] = 1.0
    if vec is None:
        return c
    v = vec[:, 0]
    if not np.isfinite(v).all() or v[0] == 0.0:
        return c
    return v / v[0]


def trial_lambda(a11, a12, a22, b11, b12, b22) -> float:
    """Step length minimising the Rayleigh quotient on span{psi, d}; the
    entries are <psi|H psi>, <psi|H d>, <d|H d>, <psi|psi>, <psi|d>, <d|d>."""
    if not b22 > 0.0:
        return 0.0
    s = 1.0 / np.sqrt(b22)
    A = np.array([[a11, a12 * s], [a12 * s, a22 * s * s]])
    B = np.array([[b11, b12 * s], [b12 * s, 1.0]])
    try:
        mu, vec = scipy.linalg.eigh(A, B)
    except np.linalg.LinAlgError:
        return 0.0
    x, y = vec[0, 0], vec[1, 0]
    if x == 0.0 or not np.isfinite(x) or not np.isfinite(y):
        return 0.0
    return float(y / x * s)


def trial_mix(A: np.ndarray, Bm: np.ndarray):
    """Coefficients (a, b) of the filter and network directions minimising
    the Rayleigh quotient of psi + a d_f + b d_n; A, Bm [3, 3] are
    <v_i|H|v_j> and <v_i|v_j> for v = (psi, d_f, d_n).  None when the
    problem is singular."""
    n = np.sqrt(np.diag(Bm))
    if not (n[1] > 0.0 and n[2] > 0.0) or not np.all(np.isfinite(A)) or not np.all(np.isfinite(Bm)):
        return None
    D = np.array([1.0, 1.0 / n[1], 1.0 / n[2]])
    try:
        mu, vec = scipy.linalg.eigh(A * np.outer(D, D), Bm * np.outer(D, D))
    except np.linalg.LinAlgError:
        return None
    v = vec[:, 0]
    if v[0] == 0.0 or not np.all(np.isfinite(v)):
        return None
    return float(v[1] / v[0] * D[1]), float(v[2] / v[0] * D[2])


def kinetic_shifts(H, psi: np.ndarray) -> np.ndarray:
    """sigma_k = -<psi_k|T psi_k> / <psi_k|psi_k> (the learned
    preconditioner's shifts)."""
    dv = H.dv
    return -dots(psi, H.apply_kinetic(psi), dv) / dots(psi, psi, dv)


def rmmdiis_step(H, psi: np.ndarray, opts: Options, net: Optional[np.ndarray] = None):
    """One eigensolver step.  psi [N, np] orthonormal on entry; net: the
    learned preconditioner's parameters (oracle.cnn), or None for the filter
    alone.  Returns dict(psi, eig, resnorm, active, lam, mix)."""
    dv = H.dv
    g = H.g
    nbr = H.nbr
    hpsi = H.apply(psi)
    eig, _, psi, hpsi = rayleigh_ritz(psi, hpsi, dv)
    N = psi.shape[0]

    eps0 = dots(psi, hpsi, dv) / dots(psi, psi, dv)
    R0 = hpsi - eps0[:, None] * psi
    res = np.sqrt(dots(R0, R0, dv))

    active = np.ones(N, dtype=bool)
    if opts.block_stop:
        for b0 in range(0, N, opts.block):
            if np.all(res[b0:b0 + opts.block] < opts.tol):
                active[b0:b0 + opts.block] = False
    lam = np.zeros(N)
    mix = np.zeros((N, 2))
    if active.any():
        A = np.nonzero(active)[0]
        p0, h0, r0, e0 = psi[A], hpsi[A], R0[A], eps0[A]
        d = filter_precond(g, r0, nbr, opts.alpha)
        hd = H.apply(d)
        a11 = dots(p0, h0, dv)
        a12 = 0.5 * (dots(p0, hd, dv) + dots(d, h0, dv))
        a22 = dots(d, hd, dv)
        b11 = dots(p0, p0, dv)
        b12 = dots(p0, d, dv)
        b22 = dots(d, d, dv)
        lm = np.array([trial_lambda(a11[s], a12[s], a22[s], b11[s], b12[s], b22[s])
                       for s in range(len(A))])
        cf, cn = lm.copy(), np.zeros(len(A))
        if net is not None:
            from . import cnn
            sig = kinetic_shifts(H, psi)[A]
            dn = cnn.precondition(net, g, r0, sig)
            hdn = H.apply(dn)
            for s in range(len(A)):
                v = (p0[s], d[s], dn[s])
                hv = (h0[s], hd[s], hdn[s])
                Am = np.empty((3, 3))
                Bq = np.empty((3, 3))
                for i in range(3):
                    for j in range(i, 3):
                        Am[i, j] = Am[j, i] = 0.5 * dv * (v[i] @ hv[j] + v[j] @ hv[i])
                        Bq[i, j] = Bq[j, i] = dv * (v[i] @ v[j])
                ab = trial_mix(Am, Bq)
                if ab is not None:
                    cf[s], cn[s] = ab
            lm = np.where(cn != 0.0, 1.0, lm)
            d = np.where((cn != 0.0)[:, None], cf[:, None] * d + cn[:, None] * dn, d)
            hd = np.where((cn != 0.0)[:, None], cf[:, None] * hd + cn[:, None] * hdn, hd)
        lam[A] = lm
        mix[A, 0], mix[A, 1] = cf, cn
        hist_p = [p0, p0 + lm[:, None] * d]
        hist_h = [h0, h0 + lm[:, None] * hd]
        moving = lm != 0.0
        for _ in range(1, opts.m):
            L = len(hist_p) - 1
            eps = [dots(p, hh, dv) / dots(p, p, dv) for p, hh in zip(hist_p, hist_h)]
            R = [hh - e[:, None] * p for p, hh, e in zip(hist_p, hist_h, eps)]
            ev = [hist_p[L]] + [hist_p[i] - hist_p[L] for i in range(L)]
            hv = [hist_h[L]] + [hist_h[i] - hist_h[L] for i in range(L)]
            rv = [R[L]] + [R[i] - R[L] for i in range(L)]
            n = L + 1
            Am = np.empty((len(A), n, n))
            Bm = np.empty((len(A), n, n))
            for a in range(n):
                for b in range(a, n):
                    Am[:, a, b] = Am[:, b, a] = dots(rv[a], rv[b], dv)
                    Bm[:, a, b] = Bm[:, b, a] = dots(ev[a], ev[b], dv)
            c = np.zeros((len(A), n))
            for s in range(len(A)):
                if moving[s]:
                    c[s] = diis_coefficients(Am[s], Bm[s])
                else:
                    c[s, 0] = 1.0
            pbar = sum(c[:, a, None] * ev[a] for a in range(n))
            hbar = sum(c[:, a, None] * hv[a] for a in range(n))
            rbar = sum(c[:, a, None] * rv[a] for a in range(n))
            d = filter_precond(g, rbar, nbr, opts.alpha)
            if net is not None and np.any(cn != 0.0):
                from . import cnn
                use = cn != 0.0
                dn = cnn.precondition(net, g, rbar, sig)
                d = np.where(use[:, None], cf[:, None] * d + cn[:, None] * dn, d)
            hd = H.apply(d)
            hist_p.append(pbar + lm[:, None] * d)
            hist_h.append(hbar + lm[:, None] * hd)
        psi = psi.copy()
        psi[A] = hist_p[-1]
    psi, _, _ = orthonormalize(psi, dv)
    return dict(psi=psi, eig=eig, resnorm=res, active=active, lam=lam, mix=mix)


def eigensolve(H, psi: np.ndarray, opts: Options, max_steps: int,
               eref: Optional[np.ndarray] = None, etol: float = 1e-6, net: Optional[np.ndarray] = None):
    """Iterate rmmdiis_step from orthonormalised psi until every residual is
    below opts.tol (or, with eref, each of the lowest len(eref) eigenvalues
    is within etol of it)."""
    psi, _, _ = orthonormalize(psi, H.dv)
    hist = []
    for it in range(max_steps):
        out = rmmdiis_step(H, psi, opts, net)
        psi = out["psi"]
        hist.append((out["eig"].copy(), out["resnorm"].copy()))
        if eref is not None:
            if np.max(np.abs(out["eig"][:len(eref)] - eref)) < etol:
                break
        elif np.all(out["resnorm"] < opts.tol):
            break
    return psi, hist
