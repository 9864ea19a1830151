"""Pins for the learned-preconditioner oracle: library and adjoint identities
for the convolutions, finite differences for the gradients, closed forms for
Adam's first steps and for the periodic shifted-kinetic solve."""
import numpy as np
import pytest
import scipy.ndimage

from oracle import cnn, grid, stencil


def _params(rng, scale=0.3):
    p = rng.normal(scale=scale, size=cnn.NP)
    p[cnn.NW] = 0.2          # a
    p[cnn.NW + 1] = -0.9     # b
    return p


@pytest.mark.parametrize("pad,mode", [("zero", "constant"), ("wrap", "wrap")])
def test_conv_matches_library_correlate(pad, mode):
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 6, 7))
    w = rng.normal(size=(3, 2, 3, 3, 3))
    got = cnn.conv(x, w, pad)
    for co in range(3):
        want = sum(scipy.ndimage.correlate(x[ci], w[co, ci], mode=mode, cval=0.0) for ci in range(2))
        assert np.allclose(got[co], want, rtol=0, atol=1e-12)


def test_conv_delta_orientation():
    """A unit impulse at p0 gives out[p0 - (t - 1)] = w[t]."""
    w = np.arange(27, dtype=np.float64).reshape(1, 1, 3, 3, 3) + 1.0
    x = np.zeros((1, 7, 7, 7))
    x[0, 3, 3, 3] = 1.0
    out = cnn.conv(x, w, "zero")[0]
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                assert out[3 - (dz - 1), 3 - (dy - 1), 3 - (dx - 1)] == w[0, 0, dz, dy, dx]
    assert np.count_nonzero(out) == 27


@pytest.mark.parametrize("pad", ["zero", "wrap"])
def test_conv_adjoint_and_weight_gradient(pad):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 6, 5, 4))
    d = rng.normal(size=(2, 6, 5, 4))
    w = rng.normal(size=(2, 3, 3, 3, 3))
    lhs = np.sum(cnn.conv(x, w, pad) * d)
    assert lhs == pytest.approx(np.sum(x * cnn.conv_transpose(d, w, pad)), rel=1e-12)
    assert lhs == pytest.approx(np.sum(w * cnn.conv_weight_grad(x, d, pad)), rel=1e-12)


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(2)
    p = _params(rng)
    u = rng.normal(size=(2, 7, 6, 8))
    t = rng.normal(size=(2, 7, 6, 8))
    sigma = np.array([-1.3, -4.0])
    h, margin = 0.25, 1
    loss, grad, du = cnn.loss_and_grad(p, u, t, sigma, h, margin)
    eps = 1e-6
    picks = [0, 100, 215, 216, 900, 1943, 1944, 2000, 2159, cnn.NW, cnn.NW + 1]
    for j in picks:
        e = np.zeros(cnn.NP)
        e[j] = eps
        lp = cnn.loss_and_grad(p + e, u, t, sigma, h, margin)[0]
        lm = cnn.loss_and_grad(p - e, u, t, sigma, h, margin)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grad[j]) <= 1e-7 * max(1.0, abs(grad[j])), j
    for idx in [(0, 3, 3, 3), (1, 0, 0, 0), (1, 6, 5, 7)]:
        e = np.zeros_like(u)
        e[idx] = eps
        lp = cnn.loss_and_grad(p, u + e, t, sigma, h, margin)[0]
        lm = cnn.loss_and_grad(p, u - e, t, sigma, h, margin)[0]
        assert abs((lp - lm) / (2 * eps) - du[idx]) <= 1e-7 * max(1.0, abs(du[idx]))


def test_loss_zero_at_exact_fit():
    """The loss vanishes when the target is the gained network output, and
    equals one for a zero network (w3 = 0)."""
    rng = np.random.default_rng(3)
    p = _params(rng)
    u = rng.normal(size=(1, 6, 6, 6))
    f, _ = cnn.forward(p, u[0], np.ones((6, 6, 6)), "zero")
    g = cnn.gain(p, -2.0, 0.25)
    loss, _, _ = cnn.loss_and_grad(p, u, (g * f)[None], np.array([-2.0]), 0.25, 1)
    assert loss < 1e-28
    p0 = p.copy()
    p0[1944:2160] = 0.0
    t = rng.normal(size=(2, 6, 6, 6))
    loss, _, _ = cnn.loss_and_grad(p0, rng.normal(size=(2, 6, 6, 6)), t, np.array([-2.0, -1.0]), 0.25, 1)
    assert loss == pytest.approx(1.0, rel=1e-13)


def test_box_kinetic_matches_grid_stencil():
    """The dense-box kinetic operator of the loss equals the oracle's grid
    stencil on a Dirichlet box of the same size (points mapped by their
    integer coordinates)."""
    g = grid.build_grid("box", 0.25, n=9)
    rng = np.random.default_rng(11)
    x = rng.normal(size=g.np)
    want = stencil.apply_kinetic(g, x)
    box = np.zeros((9, 9, 9))
    u = g.inner - g.inner.min(axis=0)
    box[u[:, 2], u[:, 1], u[:, 0]] = x
    got = cnn.box_kinetic(box, 0.25)[u[:, 2], u[:, 1], u[:, 0]]
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.max(np.abs(want)))


def test_energy_norm_loss_weights_short_waves():
    """For a zero network the loss is one; an error made of a short wave
    costs more than the same L2 error made of a long wave."""
    rng = np.random.default_rng(12)
    p = _params(rng)
    p0 = p.copy()
    p0[1944:2160] = 0.0
    t = rng.normal(size=(1, 12, 12, 12))
    loss, _, _ = cnn.loss_and_grad(p0, rng.normal(size=(1, 12, 12, 12)), t, np.array([-1.0]), 0.25, 2)
    assert loss == pytest.approx(1.0, rel=1e-13)
    zz = np.arange(12)[:, None, None] * np.ones((1, 12, 12))
    slow = np.cos(2 * np.pi * zz / 12.0)
    fast = np.cos(np.pi * zz)
    e_slow = cnn.box_kinetic(slow, 0.25) + 1.0 * slow
    e_fast = cnn.box_kinetic(fast, 0.25) + 1.0 * fast
    inner = (slice(4, 8),) * 3
    assert np.sum(fast[inner] * e_fast[inner]) > 10 * np.sum(slow[inner] * e_slow[inner])


def test_adam_first_steps_closed_form():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2, so every step moves each parameter by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(4)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = p0
    for step in (1, 2, 3):
        p, m, v = cnn.adam_step(p, g, m, v, step, lr=1e-2)
        want = p0 - step * 1e-2 * g / (np.abs(g) + 1e-8)
        assert np.allclose(p, want, rtol=0, atol=1e-13)


def test_gain_softplus_values():
    p = np.zeros(cnn.NP)
    assert cnn.gain(p, -3.0, 0.3) == pytest.approx(np.log(2.0), rel=1e-15)
    p[cnn.NW], p[cnn.NW + 1] = 1.5, -1.0
    sig, h = -2.0, 0.25
    assert cnn.gain(p, sig, h) == pytest.approx(np.log1p(np.exp(1.5) / (2.0 * h * h)), rel=1e-14)


def test_preconditioner_odd_and_homogeneous():
    g = grid.build_grid("sphere", 0.3, radius=1.6)
    rng = np.random.default_rng(5)
    p = _params(rng)
    r = rng.normal(size=(2, g.np))
    sig = np.array([-1.0, -2.5])
    k = cnn.precondition(p, g, r, sig)
    assert np.allclose(cnn.precondition(p, g, -r, sig), -k, rtol=0, atol=1e-14)
    assert np.allclose(cnn.precondition(p, g, 3.0 * r, sig), 3.0 * k, rtol=1e-13, atol=1e-14)
    assert np.all(cnn.precondition(p, g, np.zeros_like(r), sig) == 0.0)


def test_box_of_sphere_and_periodic():
    g = grid.build_grid("sphere", 0.2, radius=1.0)
    lo, dims, idx, mask = cnn.box_of(g)
    assert dims == (11, 11, 11) and tuple(lo) == (-5, -5, -5)
    assert mask.sum() == g.np and len(np.unique(idx)) == g.np
    gp = grid.build_grid("periodic", 0.25, n=8)
    _, dims, idx, mask = cnn.box_of(gp)
    assert dims == (8, 8, 8) and mask.all()


def test_shifted_inverse_periodic_solves_stencil_system():
    """(T - sigma) x = r with T applied by the stencil (independent of the
    Fourier symbol used in the solve)."""
    g = grid.build_grid("periodic", 0.25, n=16)
    rng = np.random.default_rng(6)
    r = rng.normal(size=(3, g.np))
    sig = np.array([-0.5, -2.0, -7.0])
    x = cnn.shifted_inverse_periodic(g, r, sig)
    back = stencil.apply_kinetic(g, x) - sig[:, None] * x
    assert np.max(np.abs(back - r)) < 1e-12 * np.max(np.abs(r))
