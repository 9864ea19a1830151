"""Oracle: Hartree potential by FFT on an enlarged cubic grid
(TEST INFRASTRUCTURE ONLY).

Sec. 7, eq. (5): the Hartree potential solves the Poisson equation
nabla^2 V = -4 pi n; for a finite system V(r) = int n(r') / |r - r'| d^3r'.
The paper's GPU method copies the density into a cubic grid, transforms it,
multiplies by the Coulomb kernel in reciprocal space, transforms back and
copies the result out; free (non-periodic) boundaries come from an enlarged
cell and a modified kernel.  The reading taken here (the kernel is only
cited): the Coulomb interaction cut off at a radius R_c,
    v(r) = 1/|r| for |r| <= R_c, 0 beyond,
whose Fourier transform is
    v(k) = 4 pi / k^2 (1 - cos(k R_c)),   v(0) = 2 pi R_c^2.
If every pair of domain points is at most R_c apart and the periodic cell
is longer than the domain's span plus R_c along each axis, no periodic image
of the density comes within R_c of a domain point, so the periodic
convolution with v equals the free-space one with the cut-off kernel, which
on the domain is the free-space Coulomb potential.  Discretely: the density
on the domain's points is placed on an N^3 box (zeros elsewhere), and

    V = IDFT( v(k) DFT(n) ),  k = 2 pi m / (N h),  m the DFT frequencies,

(the lattice sum h^3 sum_j n_j v(r - r_j) has the DFT h^3 DFT(n) DFT(v_m),
and DFT(v_m) = v(k) / h^3 for the sampled kernel v_m = v(m h)),
read back at the domain's points.  R_c = twice the largest distance of a
domain point from the centre of the domain's bounding box (an upper bound
of every pair distance); N = the smallest power of two with
N > (extent - 1) + R_c / h on every axis.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid


def cutoff_radius(g: Grid) -> float:
    """Twice the largest distance of an inner point from the centre of the
    inner points' bounding box (bohr)."""
    lo = g.inner.min(axis=0)
    hi = g.inner.max(axis=0)
    c = 0.5 * (lo + hi)
    d = g.inner - c
    return 2.0 * g.h * float(np.sqrt(np.max(np.sum(d * d, axis=1))))


def box_size(g: Grid, rc: float) -> int:
    ext = int((g.inner.max(axis=0) - g.inner.min(axis=0)).max()) + 1
    n = 2
    while not n > (ext - 1) + rc / g.h:
        n *= 2
    return n


def kernel(n: int, h: float, rc: float) -> np.ndarray:
    """v(k) on the N^3 DFT frequencies, indexed [z, y, x]."""
    k1 = 2.0 * np.pi * np.fft.fftfreq(n, d=h)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    k = np.sqrt((kx * kx + ky * ky) + kz * kz)
    out = np.empty_like(k)
    nz = k > 0.0
    out[nz] = 4.0 * np.pi / (k[nz] * k[nz]) * (1.0 - np.cos(k[nz] * rc))
    out[~nz] = 2.0 * np.pi * rc * rc
    return out


def hartree(g: Grid, rho: np.ndarray, rc: float = None, n: int = None) -> np.ndarray:
    """V_H at the inner points for the density rho [np] (FP64)."""
    if g.periodic:
        raise ValueError("the free-boundary solve is for finite systems")
    rc = cutoff_radius(g) if rc is None else rc
    n = box_size(g, rc) if n is None else n
    lo = g.inner.min(axis=0)
    u = g.inner - lo
    box = np.zeros((n, n, n))
    box[u[:, 2], u[:, 1], u[:, 0]] = rho
    f = np.fft.fftn(box)
    v = np.fft.ifftn(f * kernel(n, g.h, rc))
    return np.real(v)[u[:, 2], u[:, 1], u[:, 0]]
