"""Pins of the oracle's Hartree potential (Sec. 7, eq. (5)): the FFT solve on
an enlarged box with the cut-off Coulomb kernel against closed forms."""
import numpy as np
import pytest
import scipy.integrate
from scipy.special import erf

from oracle import grid, poisson


def _gauss(g, s, c=(0.0, 0.0, 0.0), q=1.0):
    d = g.xyz - np.asarray(c)
    r2 = np.sum(d * d, axis=1)
    return q * (2 * np.pi * s * s) ** -1.5 * np.exp(-r2 / (2 * s * s)), np.sqrt(r2)


def _erf_potential(r, s, q=1.0):
    out = np.empty_like(r)
    nz = r > 0
    out[nz] = q * erf(r[nz] / (np.sqrt(2) * s)) / r[nz]
    out[~nz] = q * np.sqrt(2 / np.pi) / s
    return out


@pytest.mark.parametrize("h", [0.4, 0.25])
def test_gaussian_charge_gives_erf_over_r(h):
    """A normalised Gaussian charge of width s has the potential
    erf(r / (sqrt(2) s)) / r (Gauss's law); the discrete solve on a sphere of
    radius 6 reproduces it to round-off (the density is resolved and the
    cut-off kernel is exact)."""
    g = grid.build_grid("sphere", h, radius=6.0)
    rho, r = _gauss(g, 0.8)
    V = poisson.hartree(g, rho)
    assert np.max(np.abs(V - _erf_potential(r, 0.8))) < 1e-10


def test_two_charges_on_a_molecular_grid():
    """Superposition and far field on a union-of-spheres grid: two Gaussian
    charges (+1 and -0.5) give the sum of their erf potentials."""
    c = np.array([[-2.1, 0.3, 0.2], [2.4, -0.5, 0.9]])
    g = grid.build_grid("union", 0.3, radius=4.5, centres=c)
    rho1, r1 = _gauss(g, 0.7, c[0], 1.0)
    rho2, r2 = _gauss(g, 0.6, c[1], -0.5)
    V = poisson.hartree(g, rho1 + rho2)
    want = _erf_potential(r1, 0.7, 1.0) + _erf_potential(r2, 0.6, -0.5)
    # the grid cuts the Gaussians' tails: the charge it misses (about 5e-9)
    # bounds the difference
    missing = abs(0.5 - (rho1 + rho2).sum() * g.h ** 3)
    assert missing < 1e-8
    assert np.max(np.abs(V - want)) < 1e-9 + missing


def test_kernel_is_the_transform_of_the_cut_off_coulomb():
    """v(k) = int_{|r|<=R} e^{-ik.r} / |r| d^3r = 4 pi int_0^R sin(kr)/(kr) r dr,
    by quadrature, at a few k (and 2 pi R^2 at k = 0)."""
    R = 7.3
    for k in (0.0, 0.11, 0.9, 3.7):
        if k == 0.0:
            want = 4 * np.pi * R * R / 2
        else:
            want = 4 * np.pi * scipy.integrate.quad(lambda r: np.sin(k * r) / k, 0.0, R, limit=400)[0]
        n = 8
        h = 2 * np.pi / (n * k) if k > 0 else 1.0    # put k on the first DFT frequency
        got = poisson.kernel(n, h, R)[0, 0, 1 if k > 0 else 0]
        assert abs(got - want) <= 1e-10 * max(1.0, abs(want))


def test_box_is_large_enough_and_symmetric_operator():
    """The box exceeds the domain's span plus R_c, R_c bounds the pair
    distances, and the potential operator is symmetric:
    <a|V[b]> = <b|V[a]>."""
    g = grid.build_grid("sphere", 0.35, radius=3.0)
    rc = poisson.cutoff_radius(g)
    n = poisson.box_size(g, rc)
    span = (g.inner.max(axis=0) - g.inner.min(axis=0)).max()
    assert n > span + rc / g.h
    d = g.xyz[:, None, :][::37] - g.xyz[None, :, :][:, ::41]
    assert np.sqrt((d * d).sum(-1)).max() <= rc + 1e-12
    rng = np.random.default_rng(4)
    a, b = rng.normal(size=(2, g.np))
    lhs, rhs = a @ poisson.hartree(g, b), b @ poisson.hartree(g, a)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
