"""Oracle: learned 3-D convolutional preconditioner (TEST INFRASTRUCTURE ONLY).

Not part of the paper: the paper's eigensolver (Sec. 3, RMM-DIIS with a
filter preconditioner) leaves the preconditioner open, and this is the
project's learned replacement for the filter.  Everything here is plain
FP64 numpy written from the definitions below.

Network f (one input channel, three layers, 3x3x3 kernels, 8 channels):

    a1 = mask * tanh(conv(u,  w1))      w1 [8][1][3][3][3]
    a2 = mask * tanh(conv(a1, w2))      w2 [8][8][3][3][3]
    f  = mask * conv(a2, w3)            w3 [1][8][3][3][3]

conv is a cross-correlation without bias,
    out[co, z, y, x] = sum_{ci, dz, dy, dx} w[co, ci, dz, dy, dx]
                       * in[ci, z + dz - 1, y + dy - 1, x + dx - 1],
with values outside the box either zero ("zero") or wrapped ("wrap").
mask is 1 on the domain's points and 0 elsewhere in the box (all ones on a
periodic box); masking every layer keeps the preconditioner supported on the
domain (Dirichlet problem).  No bias and an odd activation make f odd.

Preconditioner for a residual r of a state with shift sigma < 0:
    s    = rms of r over the domain points,
    K(r) = s * g(sigma) * f(r / s),   g = softplus(a + b log(-sigma h^2)),
so K(-r) = -K(r) and K(c r) = c K(r) for c > 0.  Training pairs are
(r, x = (T - sigma)^-1 r) with sigma = -<psi|T|psi>.  The loss of a batch
measures the error in the energy norm of A_i = T - sigma_i (the norm in which
a preconditioner is measured: an error at wave number k weighs k^2/2 - sigma,
so wrong short-wavelength output, which the plain L2 norm of the smooth
target barely sees, is penalised):
    L = sum_i <e_i|A_i|e_i> / sum_i <t_i|A_i|t_i>,  e_i = M (g_i f(u_i) - t_i),
t_i masked by M too, M the points at least `margin` from the crop faces
(u = r/s, t = x/s), A_i applied on the crop with zero outside it.  The ratio
is over the whole batch: per-crop ratios are unbounded on crops where a
localised state's target nearly vanishes.

Parameters are one flat vector: w1 (216), w2 (1728), w3 (216), a, b.
"""
from __future__ import annotations

import numpy as np

from .stencil import fd_weights, kinetic_symbol

SHAPES = ((8, 1, 3, 3, 3), (8, 8, 3, 3, 3), (1, 8, 3, 3, 3))
NW = sum(int(np.prod(s)) for s in SHAPES)      # 2160
NP = NW + 2                                     # + gain parameters a, b


def unpack(params: np.ndarray):
    ws, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        ws.append(params[o:o + n].reshape(s))
        o += n
    return ws, params[NW], params[NW + 1]


def shift(x: np.ndarray, dz: int, dy: int, dx: int, pad: str) -> np.ndarray:
    """y[..., z, y, x] = x[..., z + dz, y + dy, x + dx] (zero or wrapped
    outside); x has the three spatial axes last."""
    if pad == "wrap":
        return np.roll(x, (-dz, -dy, -dx), axis=(-3, -2, -1))
    out = np.zeros_like(x)
    Z, Y, X = x.shape[-3:]
    def rng(d, n):
        return slice(max(0, -d), min(n, n - d)), slice(max(0, d), min(n, n + d))
    (oz, iz), (oy, iy), (ox, ix) = rng(dz, Z), rng(dy, Y), rng(dx, X)
    out[..., oz, oy, ox] = x[..., iz, iy, ix]
    return out


def conv(x: np.ndarray, w: np.ndarray, pad: str) -> np.ndarray:
    """x [C_in, Z, Y, X], w [C_out, C_in, 3, 3, 3] -> [C_out, Z, Y, X]."""
    out = np.zeros((w.shape[0],) + x.shape[1:])
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                xs = shift(x, dz - 1, dy - 1, dx - 1, pad)
                out += np.einsum("oi,izyx->ozyx", w[:, :, dz, dy, dx], xs)
    return out


def conv_transpose(d: np.ndarray, w: np.ndarray, pad: str) -> np.ndarray:
    """Adjoint of conv with respect to its input: d [C_out, ...] ->
    [C_in, ...], in[ci, q] collects w[co, ci, t] d[co, q - (t - 1)]."""
    out = np.zeros((w.shape[1],) + d.shape[1:])
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                ds = shift(d, 1 - dz, 1 - dy, 1 - dx, pad)
                out += np.einsum("oi,ozyx->izyx", w[:, :, dz, dy, dx], ds)
    return out


def conv_weight_grad(x: np.ndarray, d: np.ndarray, pad: str) -> np.ndarray:
    """dL/dw[co, ci, t] = sum_p d[co, p] x[ci, p + t - 1]."""
    g = np.zeros((d.shape[0], x.shape[0], 3, 3, 3))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                xs = shift(x, dz - 1, dy - 1, dx - 1, pad)
                g[:, :, dz, dy, dx] = np.einsum("ozyx,izyx->oi", d, xs)
    return g


def forward(params: np.ndarray, u: np.ndarray, mask: np.ndarray, pad: str):
    """u [Z, Y, X] -> (f, cache)."""
    (w1, w2, w3), _, _ = unpack(params)
    a1 = mask * np.tanh(conv(u[None], w1, pad))
    a2 = mask * np.tanh(conv(a1, w2, pad))
    f = mask * conv(a2, w3, pad)[0]
    return f, (u, a1, a2)


def backward(params: np.ndarray, cache, df: np.ndarray, mask: np.ndarray, pad: str):
    """Gradients of a scalar loss given df = dL/df: returns (dw flat [NW], du)."""
    (w1, w2, w3), _, _ = unpack(params)
    u, a1, a2 = cache
    d3 = (mask * df)[None]
    g3 = conv_weight_grad(a2, d3, pad)
    d2 = conv_transpose(d3, w3, pad) * mask * (1.0 - a2 ** 2)
    g2 = conv_weight_grad(a1, d2, pad)
    d1 = conv_transpose(d2, w2, pad) * mask * (1.0 - a1 ** 2)
    g1 = conv_weight_grad(u[None], d1, pad)
    du = conv_transpose(d1, w1, pad)[0]
    return np.concatenate([g1.ravel(), g2.ravel(), g3.ravel()]), du


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def gain(params: np.ndarray, sigma, h: float):
    a, b = params[NW], params[NW + 1]
    return softplus(a + b * np.log(-np.asarray(sigma) * h * h))


def box_kinetic(x: np.ndarray, h: float) -> np.ndarray:
    """T x on a dense box [Z, Y, X] with zero outside: the 25-point star of
    Sec. 5.1, -1/(2h^2) sum_axes sum_m c_m (x_{p+m} + x_{p-m} - 2 x_p)."""
    c = fd_weights(4)
    out = np.zeros_like(x)
    for m in range(1, 5):
        for d in ((m, 0, 0), (0, m, 0), (0, 0, m)):
            out += c[m] * (shift(x, *d, "zero") + shift(x, *(-v for v in d), "zero") - 2.0 * x)
    return -0.5 / (h * h) * out


def loss_and_grad(params: np.ndarray, u: np.ndarray, t: np.ndarray, sigma: np.ndarray,
                  h: float, margin: int, pad: str = "zero"):
    """Batch u, t [n, Z, Y, X], sigma [n]; crops are whole boxes (mask 1).
    Returns (loss, grad [NP], du [n, Z, Y, X])."""
    n = u.shape[0]
    a, b = params[NW], params[NW + 1]
    inner = np.zeros(u.shape[1:])
    Z, Y, X = u.shape[1:]
    inner[margin:Z - margin, margin:Y - margin, margin:X - margin] = 1.0
    mask = np.ones(u.shape[1:])

    def A(i, x):
        return box_kinetic(x, h) - sigma[i] * x

    den = sum(np.sum((inner * t[i]) * A(i, inner * t[i])) for i in range(n))
    grad = np.zeros(NP)
    du = np.zeros_like(u)
    loss = 0.0
    for i in range(n):
        f, cache = forward(params, u[i], mask, pad)
        ell = np.log(-sigma[i] * h * h)
        z = a + b * ell
        g = softplus(z)
        e = inner * (g * f - t[i])
        Ae = A(i, e)
        loss += np.sum(e * Ae) / den
        dpred = 2.0 * inner * Ae / den
        dw, du[i] = backward(params, cache, g * dpred, mask, pad)
        grad[:NW] += dw
        dg = np.sum(dpred * f)
        grad[NW] += dg * sigmoid(z)
        grad[NW + 1] += dg * sigmoid(z) * ell
    return loss, grad, du


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1); step counts from 1.
    Returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------ on a grid
def box_of(g):
    """Smallest axis-aligned box holding every inner point: (lo [3] in x, y,
    z order, dims (Z, Y, X), flat box index of each inner point, mask)."""
    lo = g.inner.min(axis=0)
    hi = g.inner.max(axis=0)
    X, Y, Z = (hi - lo + 1).tolist()
    u = g.inner - lo
    idx = (u[:, 2] * Y + u[:, 1]) * X + u[:, 0]
    mask = np.zeros(Z * Y * X)
    mask[idx] = 1.0
    return lo, (Z, Y, X), idx, mask.reshape(Z, Y, X)


def precondition(params: np.ndarray, g, r: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """K applied to state-major residuals r [N, np] on grid g, shifts
    sigma [N]; a zero residual maps to zero."""
    _, dims, idx, mask = box_of(g)
    pad = "wrap" if g.periodic else "zero"
    r2 = np.atleast_2d(r)
    out = np.zeros_like(r2)
    for k in range(r2.shape[0]):
        s = np.sqrt(np.mean(r2[k] ** 2))
        if s == 0.0:
            continue
        box = np.zeros(int(np.prod(dims)))
        box[idx] = r2[k] / s
        f, _ = forward(params, box.reshape(dims), mask, pad)
        out[k] = s * gain(params, sigma[k], g.h) * f.ravel()[idx]
    return out if r.ndim == 2 else out[0]


def shifted_inverse_periodic(g, r: np.ndarray, sigma) -> np.ndarray:
    """x = (T - sigma)^-1 r on a periodic box: T is diagonal on plane waves
    with the finite-difference symbol, so the solve is a division in
    Fourier space (closed form)."""
    if not g.periodic:
        raise ValueError("closed form needs a periodic box")
    lo, dims, idx, _ = box_of(g)
    n = dims[0]
    kk = 2.0 * np.pi * np.fft.fftfreq(n, d=g.h)
    KZ, KY, KX = np.meshgrid(kk, kk, kk, indexing="ij")
    sym = kinetic_symbol(np.stack([KX, KY, KZ], axis=-1), g.h, g.M)
    r2 = np.atleast_2d(r)
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (r2.shape[0],))
    out = np.empty_like(r2)
    for k in range(r2.shape[0]):
        box = np.zeros(n ** 3)
        box[idx] = r2[k]
        xf = np.fft.fftn(box.reshape(dims)) / (sym - sig[k])
        out[k] = np.real(np.fft.ifftn(xf)).ravel()[idx]
    return out if r.ndim == 2 else out[0]
