"""GPU parity of the orthogonalisation / subspace stage (Sec. 6) against the
FP64 oracle and LAPACK, through the C ABI."""
import numpy as np
import pytest

import synthetic
from oracle import hamiltonian, linalg

torch = pytest.importorskip("torch")
import paper_1306_2953_amd as rsd  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"


@pytest.fixture(scope="module")
def small():
    w = synthetic.make_workload("sphere_r12_h0.2", radius=3.0, nat=5, atom_radius=2.0)
    og, atoms, H = hamiltonian.build_system(w)
    g = rsd.Grid.for_workload(w)
    ctx = rsd.Context(g, 256)
    return w, og, H, g, ctx


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _blk(states, B):
    return _dev(rsd.to_blocks(states, B))


@pytest.mark.parametrize("nblk,B", [(4, 32), (3, 32), (1, 8), (5, 8), (2, 64), (16, 16)])
def test_overlap_fp64(small, nblk, B):
    """(4, 32) runs the register-fed products (chunks of 16 points here, the
    last one ragged); the other shapes the LDS-staged ones."""
    w, og, H, g, ctx = small
    rng = np.random.default_rng(B + nblk)
    x = rng.uniform(-1, 1, (nblk * B, og.np))
    y = rng.uniform(-1, 1, (nblk * B, og.np))
    S = ctx.overlap(_blk(x, B), _blk(x, B)).cpu().numpy()
    want = linalg.overlap(x, og.dv)
    assert np.max(np.abs(S - want)) <= 1e-12 * np.max(np.abs(want))
    assert np.array_equal(S, S.T)
    # one tensor for both operands: the symmetric (upper blocks) product
    tx = _blk(x, B)
    Ss = ctx.overlap(tx, tx).cpu().numpy()
    assert np.max(np.abs(Ss - want)) <= 1e-12 * np.max(np.abs(want))
    assert np.array_equal(Ss, Ss.T)
    M = ctx.overlap(_blk(x, B), _blk(y, B)).cpu().numpy()
    want = og.dv * x @ y.T
    assert np.max(np.abs(M - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("nblk,B", [(4, 32), (1, 8), (3, 16)])
def test_overlap_bf16x3_error_bound(small, nblk, B):
    """Split-BF16 products: |error| <= 2^-16 h^3 sum_p |x_p y_p| elementwise
    (two-term splits leave 2^-17 |x y| per product; each MFMA step sums at
    most 32 points in FP32, the steps are accumulated in FP64)."""
    w, og, H, g, ctx = small
    rng = np.random.default_rng(7 + B)
    x = rng.uniform(-1, 1, (nblk * B, og.np)).astype(np.float32)
    y = rng.uniform(-1, 1, (nblk * B, og.np)).astype(np.float32)
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    for a, b, same in ((x, x, True), (x, x, False), (x, y, False)):
        ta = _blk(a, B)
        got = ctx.overlap(ta, ta if same else _blk(b, B)).cpu().numpy()
        want = og.dv * a.astype(np.float64) @ b.astype(np.float64).T
        bound = 2.0 ** -16 * og.dv * np.abs(a.astype(np.float64)) @ np.abs(b.astype(np.float64)).T
        assert np.all(np.abs(got - want) <= bound)


@pytest.mark.parametrize("N", [1, 37, 100, 128, 200])
def test_cholesky_and_pivot(small, N):
    """N <= 130 keeps the working matrix in LDS, 200 runs it in global memory."""
    w, og, H, g, ctx = small
    rng = np.random.default_rng(3)
    A = rng.normal(size=(N, N))
    S = A @ A.T + N * np.eye(N)
    U, info = ctx.cholesky(_dev(S))
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Ug = U.cpu().numpy()
    assert np.all(np.tril(Ug, -1) == 0.0)
    assert np.allclose(Ug, np.linalg.cholesky(S).T, atol=1e-12 * np.max(np.abs(S)))
    # a state repeated at column k (beyond the LDS limit of 130 for N = 200):
    # its pivot is not positive; rows from it on are not computed
    k = {1: 0, 37: 20, 100: 60, 128: 127, 200: 150}[N]
    psi = rng.uniform(-1, 1, (N, 4 * N + 16))
    if k > 0:
        psi[k] = psi[k - 1]
    else:
        psi[0] = 0.0
    S2 = linalg.overlap(psi, 1.0)
    if k > 0:
        S2[k, k] -= 1e-9 * S2[k - 1, k - 1]
    U, info = ctx.cholesky(_dev(S2))
    assert int(info.item()) == k + 1
    Ug = U.cpu().numpy()
    assert np.all(Ug[k:] == 0.0)
    if k > 0:
        Lk = np.linalg.cholesky(S2[:k, :k])
        assert np.allclose(Ug[:k, :k], Lk.T, atol=1e-12 * np.max(np.abs(S2)))


@pytest.mark.parametrize("N", [8, 37, 128, 200, 256])
def test_eigh_jacobi(small, N):
    w, og, H, g, ctx = small
    rng = np.random.default_rng(N)
    A = rng.normal(size=(N, N))
    A = 0.5 * (A + A.T)
    ev, V = ctx.eigh(_dev(A))
    ev, V = ev.cpu().numpy(), V.cpu().numpy()
    lam, X = np.linalg.eigh(A)
    X = X * linalg.fix_signs(X)
    nrm = np.linalg.norm(A, 2)
    assert np.max(np.abs(ev - lam)) < 1e-13 * N * nrm
    assert np.allclose(V.T @ V, np.eye(N), atol=1e-13 * N)
    assert np.max(np.abs(A @ V - V * ev)) < 1e-12 * N * nrm
    gap = np.min(np.diff(lam))
    assert np.max(np.abs(V - X)) < 1e-13 * N * nrm / gap


@pytest.mark.parametrize("dtype,nblk,B", [(np.float64, 3, 32), (np.float64, 5, 8), (np.float32, 4, 32),
                                          (np.float32, 2, 8), (np.float64, 5, 32), (np.float64, 3, 16),
                                          (np.float32, 5, 32), (np.float32, 3, 16), (np.float64, 4, 32),
                                          (np.float64, 8, 16)])
def test_rotate(small, dtype, nblk, B):
    """N <= 128 with B a multiple of 16 (FP64) or 8 (FP32) runs the
    persistent kernels (48 states: an odd count of 16-state blocks, a padded
    last 32-row slice; 128 states: eight column blocks, X filling the LDS as
    in the benchmark); N = 160 the tiled ones."""
    w, og, H, g, ctx = small
    N = nblk * B
    rng = np.random.default_rng(N)
    x = rng.uniform(-1, 1, (N, og.np)).astype(dtype)
    X = rng.normal(size=(N, N))
    t = _blk(x, B)
    ctx.rotate(t, _dev(X))
    got = rsd.from_blocks(t.cpu().numpy())
    want = X.T @ x.astype(np.float64)
    if dtype == np.float64:
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    else:
        bound = 2.0 ** -21 * np.abs(X.T) @ np.abs(x.astype(np.float64)) + 2.0 ** -22 * np.abs(want)
        assert np.all(np.abs(got - want) <= bound)


@pytest.mark.parametrize("dtype,nblk,B", [(np.float64, 3, 32), (np.float64, 1, 8), (np.float32, 4, 32)])
def test_orthonormalize(small, dtype, nblk, B):
    w, og, H, g, ctx = small
    N = nblk * B
    x = synthetic.draw_states(np.random.default_rng(N), N, og.np).astype(dtype)
    want, U, S = linalg.orthonormalize(x.astype(np.float64), og.dv)
    t = _blk(x, B)
    info = ctx.orthonormalize(t)
    assert info == 0
    got = rsd.from_blocks(t.cpu().numpy()).astype(np.float64)
    G = og.dv * got @ got.T
    if dtype == np.float64:
        assert np.max(np.abs(got - want)) < 1e-11 * np.max(np.abs(want))
        assert np.max(np.abs(G - np.eye(N))) < 1e-12
    else:
        assert np.max(np.abs(got - want)) < 1e-5 * np.max(np.abs(want))
        assert np.max(np.abs(G - np.eye(N))) < 1e-6


def test_orthonormalize_singular_reports_pivot(small):
    w, og, H, g, ctx = small
    x = synthetic.draw_states(np.random.default_rng(1), 8, og.np)
    x[5] = 0.0                              # a zero state: pivot 6 is exactly zero
    t = _blk(x, 8)
    before = t.clone()
    with pytest.raises(rsd.RsError) as e:
        ctx.orthonormalize(t)
    assert e.value.code == rsd._abi.RS_ENOTPOSDEF
    assert torch.equal(t, before)          # psi left unchanged


def test_subspace_diag_fp64(small):
    w, og, H, g, ctx = small
    N, B = 64, 32
    x, _, _ = linalg.orthonormalize(synthetic.draw_states(np.random.default_rng(5), N, og.np), og.dv)
    hx = H.apply(x)
    lam, xi, p2, h2 = linalg.rayleigh_ritz(x, hx, og.dv)
    tp, th = _blk(x, B), _blk(hx, B)
    ev = ctx.subspace_diag(tp, th).cpu().numpy()
    nrm = np.max(np.abs(lam))
    assert np.max(np.abs(ev - lam)) < 1e-13 * N * nrm
    gp = rsd.from_blocks(tp.cpu().numpy())
    gh = rsd.from_blocks(th.cpu().numpy())
    # an eigenvector is determined to (rounding x |h|) / (gap to its
    # neighbours): the rotated states inherit that bound
    gap = np.min(np.diff(lam))
    tol = 1e-13 * N * nrm / gap
    print(f"gap {gap:.2e}, bound {tol:.2e}, psi err {np.max(np.abs(gp - p2)) / np.max(np.abs(p2)):.2e}")
    assert np.max(np.abs(gp - p2)) < tol * np.max(np.abs(p2))
    assert np.max(np.abs(gh - h2)) < tol * np.max(np.abs(h2))


def test_full_size_overlap():
    """Config-2 grid (0.9M points), 128 states: FP64 overlap and the split
    BF16 overlap of the FP32 copy."""
    w = synthetic.WORKLOADS["sphere_r12_h0.2"]
    g = rsd.Grid.for_workload(w)
    ctx = rsd.Context(g, 128)
    x = synthetic.draw_states(synthetic.rng_after_atoms(w), 128, g.np)
    want = linalg.overlap(x, g.dv)
    tx = _blk(x, 32)
    for a, b in ((tx, _blk(x, 32)), (tx, tx)):          # general, then symmetric
        S = ctx.overlap(a, b).cpu().numpy()
        assert np.max(np.abs(S - want)) <= 1e-12 * np.max(np.abs(want))
    x32 = x.astype(np.float32)
    x64 = x32.astype(np.float64)
    want32 = linalg.overlap(x64, g.dv)
    bound = 2.0 ** -16 * g.dv * np.abs(x64) @ np.abs(x64).T
    t32 = _blk(x32, 32)
    for a, b in ((t32, _blk(x32, 32)), (t32, t32)):
        S32 = ctx.overlap(a, b).cpu().numpy()
        assert np.all(np.abs(S32 - want32) <= bound)


@pytest.mark.parametrize("radius", [0.3, 0.7])
def test_overlap_tiny_grid_4x32(radius):
    """128 states in blocks of 32 (the register-fed products) on grids of a
    few dozen points: one ragged chunk, most of a k-step past the end."""
    g = rsd.Grid("sphere", 0.2, radius=radius)
    assert 0 < g.np < 1000
    ctx = rsd.Context(g, 128)
    rng = np.random.default_rng(int(radius * 10))
    for dtype in (np.float64, np.float32):
        x = rng.uniform(-1, 1, (128, g.np)).astype(dtype)
        y = rng.uniform(-1, 1, (128, g.np)).astype(dtype)
        x64, y64 = x.astype(np.float64), y.astype(np.float64)
        tx = _blk(x, 32)
        for a, b, want, scale in ((tx, tx, x64 @ x64.T, np.abs(x64) @ np.abs(x64).T),
                                  (tx, _blk(y, 32), x64 @ y64.T, np.abs(x64) @ np.abs(y64).T)):
            S = ctx.overlap(a, b).cpu().numpy() / g.dv
            if dtype == np.float64:
                assert np.max(np.abs(S - want)) <= 1e-13 * np.max(scale)
            else:
                assert np.all(np.abs(S - want) <= 2.0 ** -16 * scale)
