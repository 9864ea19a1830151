"""The Python binding refuses tensors whose shape, dtype or device differ from
what the C call reads or writes (the C ABI only sees pointers).  Runs on the
CPU: every refusal happens before any device call."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_1306_2953_amd as rsd  # noqa: E402


@pytest.fixture(scope="module")
def grid():
    return rsd.Grid("sphere", 0.2, radius=1.2, host_only=True)


def _ctx(grid, max_states=64):
    c = rsd.Context.__new__(rsd.Context)      # no device handle: checks only
    c.grid, c.max_states, c._h = grid, max_states, None
    return c


def _solver(grid, nstates=16, B=8, dtype=torch.float64):
    s = rsd.Eigensolver.__new__(rsd.Eigensolver)
    s.grid, s.nstates, s.B, s.nblk, s.dtype, s._h = grid, nstates, B, -(-nstates // B), dtype, None
    s.vloc = torch.zeros(grid.np, dtype=dtype)
    return s


def f64(*shape):
    return torch.zeros(*shape, dtype=torch.float64)


def test_field_shape_dtype_and_block(grid):
    n = grid.np
    with pytest.raises(ValueError, match="np="):
        rsd.hpsi_block(grid, None, f64(n), f64(1, n + 1, 8), f64(1, n + 1, 8))
    with pytest.raises(ValueError, match="float32 or float64"):
        rsd.hpsi_block(grid, None, f64(n), torch.zeros(1, n, 8, dtype=torch.float16), f64(1, n, 8))
    with pytest.raises(ValueError, match="power of two"):
        rsd.hpsi_block(grid, None, f64(n), f64(1, n, 6), f64(1, n, 6))
    with pytest.raises(ValueError, match="hpsi must be torch.float64"):
        rsd.hpsi_block(grid, None, f64(n), f64(1, n, 8), torch.zeros(1, n, 8))
    with pytest.raises(ValueError, match="hpsi must have shape"):
        rsd.hpsi_block(grid, None, f64(n), f64(1, n, 8), f64(2, n, 8))
    with pytest.raises(ValueError, match="vloc must have"):
        rsd.hpsi_block(grid, None, f64(n - 1), f64(1, n, 8), f64(1, n, 8))
    with pytest.raises(ValueError, match="vloc must be torch.float64"):
        rsd.hpsi_block(grid, None, torch.zeros(n), f64(1, n, 8), f64(1, n, 8))
    x = f64(1, n, 8)
    with pytest.raises(ValueError, match="alias"):
        rsd.hpsi_block(grid, None, f64(n), x, x)
    # correct shapes and dtypes, host memory: refused as not on the device
    with pytest.raises(ValueError, match="device tensor"):
        rsd.hpsi_block(grid, None, f64(n), f64(1, n, 8), f64(1, n, 8))


def test_projection_buffers(grid):
    class NL:
        nat, nproj, max_states, handle = 3, 4, 64, None
    n = grid.np
    with pytest.raises(ValueError, match="proj must have shape"):
        rsd.project_nl(grid, NL, f64(2, n, 8), f64(2, 3, 4, 4))
    with pytest.raises(ValueError, match="proj must be torch.float64"):
        rsd.apply_nl(grid, NL, torch.zeros(2, 3, 4, 8), f64(2, n, 8))

    class NL16(NL):
        nproj = 16
    with pytest.raises(ValueError, match=r"proj must have shape \(2, 3, 16, 8\)"):
        rsd.project_nl(grid, NL16, f64(2, n, 8), f64(2, 3, 4, 8))
    # complex states: two real columns each, at most 32 per block
    c128 = torch.zeros(2, n, 32, dtype=torch.complex128)
    with pytest.raises(ValueError, match="real columns exceed"):
        rsd.project_nl(grid, NL, c128, torch.zeros(2, 3, 4, 32, dtype=torch.complex128))
    with pytest.raises(ValueError, match=r"power of two in \[1, 32\]"):
        rsd.project_nl(grid, NL, torch.zeros(1, n, 64, dtype=torch.complex128),
                       torch.zeros(1, 3, 4, 64, dtype=torch.complex128))
    with pytest.raises(ValueError, match="proj must be torch.complex64"):
        rsd.project_nl(grid, NL, torch.zeros(1, n, 8, dtype=torch.complex64), f64(1, 3, 4, 8))


def test_complex_fields(grid):
    n = grid.np
    z = torch.zeros(1, n, 8, dtype=torch.complex128)
    with pytest.raises(ValueError, match="vloc must be torch.float64"):
        rsd.hpsi_block(grid, None, torch.zeros(n, dtype=torch.complex128), z, torch.zeros_like(z))
    with pytest.raises(ValueError, match="device tensor"):
        rsd.hpsi_block(grid, None, f64(n), z, torch.zeros_like(z))
    c = _ctx(grid, max_states=16)
    with pytest.raises(ValueError, match="real columns exceed"):
        c.overlap(torch.zeros(2, n, 8, dtype=torch.complex128), torch.zeros(2, n, 8, dtype=torch.complex128))
    c = _ctx(grid, max_states=64)
    with pytest.raises(ValueError, match="S must be torch.complex128"):
        c.overlap(z, z, S=f64(8, 8))
    # only H psi, the projections and the overlap take complex states
    with pytest.raises(ValueError, match="float32 or float64, got"):
        c.rotate(z, f64(8, 8))
    with pytest.raises(ValueError, match="float32 or float64, got"):
        rsd.overlap_noalloc(grid, z, z, f64(8, 8))


def test_context_refusals(grid):
    c = _ctx(grid, max_states=64)
    n = grid.np
    with pytest.raises(ValueError, match="max_states"):
        c.overlap(f64(9, n, 8), f64(9, n, 8))
    with pytest.raises(ValueError, match="y must be torch.float64"):
        c.overlap(f64(2, n, 8), torch.zeros(2, n, 8))
    with pytest.raises(ValueError, match="S must have shape"):
        c.overlap(f64(2, n, 8), f64(2, n, 8), S=f64(8, 8))
    with pytest.raises(ValueError, match="S must be torch.float64"):
        c.overlap(torch.zeros(2, n, 8), torch.zeros(2, n, 8), S=torch.zeros(16, 16))
    with pytest.raises(ValueError, match="X must have shape"):
        c.rotate(f64(2, n, 8), f64(8, 8))
    with pytest.raises(ValueError, match="X must be torch.float64"):
        c.rotate(torch.zeros(2, n, 8), torch.zeros(16, 16))
    with pytest.raises(ValueError, match="square"):
        c.cholesky(f64(4, 5))
    with pytest.raises(ValueError, match="S must be torch.float64"):
        c.cholesky(torch.zeros(4, 4))
    with pytest.raises(ValueError, match="N must be in"):
        c.cholesky(f64(65, 65))
    with pytest.raises(ValueError, match="square"):
        c.eigh(f64(3))
    with pytest.raises(ValueError, match="A must be torch.float64"):
        c.eigh(torch.zeros(4, 4))
    with pytest.raises(ValueError, match="np="):
        c.orthonormalize(f64(2, n - 1, 8))
    with pytest.raises(ValueError, match="S_out must have shape"):
        c.orthonormalize(f64(2, n, 8), S_out=f64(8, 8))
    with pytest.raises(ValueError, match="hpsi must have shape"):
        c.subspace_diag(f64(2, n, 8), f64(1, n, 8))


def test_solver_refusals(grid):
    s = _solver(grid, nstates=16, B=8, dtype=torch.float64)
    n = grid.np
    with pytest.raises(ValueError, match="blocks"):
        s.step(f64(3, n, 8))
    with pytest.raises(ValueError, match="psi must be torch.float64"):
        s.step(torch.zeros(2, n, 8))
    with pytest.raises(ValueError, match="psi must be torch.float64"):
        s.orthonormalize(torch.zeros(2, n, 8))
    with pytest.raises(ValueError, match="blocks"):
        s.orthonormalize(f64(2, n, 4))
    with pytest.raises(ValueError, match="vloc must have"):
        rsd.Eigensolver(grid, None, f64(n + 1), 16, 8)
    with pytest.raises(ValueError, match="one-dimensional"):
        rsd.Eigensolver(grid, None, f64(1, n), 16, 8)


def test_network_refusals(grid):
    net = rsd.Cnn.__new__(rsd.Cnn)
    net._h = None
    u = torch.zeros(4, 8, 8, 8)
    with pytest.raises(ValueError, match="u must be torch.float32"):
        net.forward(u.double())
    with pytest.raises(ValueError, match="t must have shape"):
        net.loss_grad(u, torch.zeros(4, 8, 8, 9), f64(4), 0.25, 2)
    with pytest.raises(ValueError, match="sigma must have 4"):
        net.loss_grad(u, u, f64(3), 0.25, 2)
    with pytest.raises(ValueError, match="sigma must be torch.float64"):
        net.train_step(u, u, torch.zeros(4), 0.25, 2, 1e-3)
    with pytest.raises(ValueError, match=r"\[n, Z, Y, X\]"):
        net.loss_grad(torch.zeros(4, 8, 8), torch.zeros(4, 8, 8), f64(4), 0.25, 2)
    n = grid.np
    with pytest.raises(ValueError, match="sigma must have 16"):
        net.precondition(grid, f64(2, n, 8), f64(8))
    with pytest.raises(ValueError, match="x must be torch.float64"):
        net.crops(grid, f64(2, n, 8), torch.zeros(2, n, 8), np.zeros((1, 4)), (4, 4, 4))
    with pytest.raises(ValueError, match="desc"):
        net.crops(grid, f64(2, n, 8), f64(2, n, 8), np.zeros((1, 3)), (4, 4, 4))
    with pytest.raises(ValueError, match="sigma must have 16"):
        rsd.shifted_solve(grid, f64(2, n, 8), f64(15))
