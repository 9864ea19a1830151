"""rs_overlap_noalloc (the overlap product on the library's fixed device
scratch) against rs_overlap on the same inputs, through the C ABI: two calls
in a row, the second on a smaller grid with fewer states."""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
import paper_1306_2953_amd as rsd  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(radius, N, B, dtype, seed):
    w = synthetic.make_workload("sphere_r12_h0.2", radius=radius, nat=0)
    g = rsd.Grid.for_workload(w)
    x = np.random.default_rng(seed).uniform(-1.0, 1.0, size=(N // B, g.np, B)).astype(dtype)
    y = np.random.default_rng(seed + 1).uniform(-1.0, 1.0, size=(N // B, g.np, B)).astype(dtype)
    return g, torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV)


def _flat(t):
    return t.double().cpu().permute(1, 0, 2).reshape(t.shape[1], -1).numpy()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_noalloc_overlap_matches_context_overlap(dtype):
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    for radius, N, B, seed in ((6.0, 128, 32, 11), (4.0, 40, 8, 12)):
        print(f"noalloc overlap: radius {radius} N {N} B {B} {np.dtype(dtype).name}", flush=True)
        g, x, y = _case(radius, N, B, dtype, seed)
        ctx = rsd.Context(g, N)
        for a, b in ((x, y), (x, x)):
            want = ctx.overlap(a, b)
            S = torch.full((N, N), float("nan"), dtype=torch.float64, device=DEV)
            got = rsd.overlap_noalloc(g, a, b, S)
            torch.cuda.synchronize()
            want, got = want.cpu().numpy(), got.cpu().numpy()
            A, Bm = _flat(a), _flat(b)
            dv = g.h ** 3
            scale = dv * (np.abs(A).T @ np.abs(Bm))           # sum |a b| per entry
            if dtype == np.float64:
                assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
                assert np.max(np.abs(got - dv * (A.T @ Bm))) <= 1e-12 * np.max(np.abs(want))
            else:
                # both are split-BF16 products (FP32 sums of at most 32 points,
                # accumulated in FP64): each within 2^-16 sum|ab| of the exact
                # product of the FP32 inputs
                exact = dv * (A.T @ Bm)
                assert np.all(np.abs(got - exact) <= 2.0 ** -16 * scale)
                assert np.all(np.abs(got - want) <= 2.0 ** -15 * scale)


def test_noalloc_overlap_refuses_too_many_states():
    g, x, y = _case(3.0, 512, 64, np.float64, 3)
    S = torch.empty((512, 512), dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        rsd.overlap_noalloc(g, x, y, S)
    # the C entry point itself refuses it too
    st = rsd.lib().rs_overlap_noalloc(g.handle, rsd._dev(x, "x"), rsd._dev(y, "y"), rsd._dev(S, "S"),
                                      8, 64, rsd.RS_F64, rsd.RS_PREC_NATIVE, None)
    assert st == rsd._abi.RS_EINVAL
