"""MI355X-native real-space Kohn-Sham hot path (Andrade & Aspuru-Guzik,
arXiv 1306.2953): H psi on blocks of states over an irregular grid,
orthogonalisation, subspace diagonalisation and an RMM-DIIS step.

This module is the thin Python binding of librsdft.so: it converts torch
tensors (device memory and the current HIP stream) into the pointers and
sizes of the C ABI declared in include/rsdft.h.  No arithmetic of the method
happens here.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from . import _abi
from ._abi import (RS_C64, RS_C128, RS_F32, RS_F64, RS_GRID_BOX, RS_GRID_HOST_ONLY, RS_GRID_PERIODIC,
                   RS_GRID_SPHERE, RS_GRID_UNION, RS_PREC_BF16X3, RS_PREC_NATIVE, RsError, check, lib)

_KINDS = {"box": RS_GRID_BOX, "periodic": RS_GRID_PERIODIC, "sphere": RS_GRID_SPHERE, "union": RS_GRID_UNION}


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Grid:
    """Index map of a uniform grid restricted to a box, a sphere or a union
    of spheres around atom centres (rs_grid)."""

    def __init__(self, kind: str, h: float, n: int = 0, radius: float = 0.0,
                 brick: Sequence[int] = (4, 4, 4), host_only: bool = False, centres=None):
        d = _abi.GridDesc()
        d.kind = _KINDS[kind]
        d.h = float(h)
        d.n = int(n)
        d.radius = float(radius)
        for a in range(3):
            d.brick[a] = int(brick[a])
        d.flags = RS_GRID_HOST_ONLY if host_only else 0
        c = None
        if centres is not None:
            c = np.ascontiguousarray(centres, dtype=np.float64)
            if c.ndim != 2 or c.shape[1] != 3:
                raise ValueError("centres must be [natoms, 3]")
            d.natoms = c.shape[0]
            d.centres = c.ctypes.data_as(ctypes.c_void_p)
        self.kind, self.h, self.n, self.radius = kind, float(h), int(n), float(radius)
        self.host_only = host_only
        self._h = ctypes.c_void_p()
        check(lib().rs_grid_create(ctypes.byref(d), ctypes.byref(self._h)))
        np_, nb_, nbr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        nb = (ctypes.c_int32 * 3)()
        lo = (ctypes.c_int32 * 3)()
        check(lib().rs_grid_info(self._h, ctypes.byref(np_), ctypes.byref(nb_),
                                 ctypes.byref(nbr), nb, lo))
        self.np, self.nbnd, self.nbricks = np_.value, nb_.value, nbr.value
        self.nb = tuple(nb)
        self.lo = tuple(lo)

    @classmethod
    def for_workload(cls, w, host_only: bool = False, brick: Sequence[int] = (4, 4, 4)) -> "Grid":
        if w.grid_kind == "sphere":
            return cls("sphere", w.h, radius=w.radius, host_only=host_only, brick=brick)
        if w.grid_kind == "union":
            import synthetic
            return cls("union", w.h, radius=w.radius, host_only=host_only, brick=brick,
                       centres=synthetic.draw_atoms(w).pos)
        return cls(w.grid_kind, w.h, n=w.n, host_only=host_only, brick=brick)

    @property
    def handle(self):
        return self._h

    @property
    def dv(self) -> float:
        return self.h ** 3

    def export(self):
        inner = np.empty((self.np, 3), dtype=np.int32)
        bnd = np.empty((max(self.nbnd, 1), 3), dtype=np.int32)
        bmap = np.empty((self.nb[2], self.nb[1], self.nb[0]), dtype=np.int32)
        xyz = np.empty((self.np, 3), dtype=np.float64)
        check(lib().rs_grid_export(self._h, _ptr(inner), _ptr(bnd), _ptr(bmap), _ptr(xyz)))
        return dict(inner=inner, boundary=bnd[: self.nbnd], brick_map=bmap, xyz=xyz)

    def xyz(self) -> np.ndarray:
        xyz = np.empty((self.np, 3), dtype=np.float64)
        check(lib().rs_grid_export(self._h, None, None, None, _ptr(xyz)))
        return xyz

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(_abi, "_lib", None) if _abi is not None else None
        if h and L is not None:
            L.rs_grid_destroy(h)
            self._h = None


class NonLocal:
    """Kleinman-Bylander projector set (rs_nl)."""

    def __init__(self, grid: Grid, pos: np.ndarray, D: np.ndarray, rc: float,
                 sigma: float, max_states: int, lmax: int = 1):
        """D [nat, (lmax+1)^2]; max_states counts real columns (a complex
        state takes two)."""
        if not 0 <= int(lmax) <= 3:
            raise ValueError(f"lmax must be 0..3, got {lmax}")
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        npj = (int(lmax) + 1) ** 2
        D = np.ascontiguousarray(D, dtype=np.float64)
        if D.size != pos.shape[0] * npj:
            raise ValueError(f"D must hold {npj} values per atom for lmax {lmax}, got shape {D.shape}")
        D = D.reshape(-1, npj)
        self.grid = grid
        self.nat = pos.shape[0]
        self.lmax = int(lmax)
        self.max_states = int(max_states)
        self._h = ctypes.c_void_p()
        check(lib().rs_nl_create(grid.handle, self.nat, _ptr(pos), _ptr(D), float(rc),
                                 float(sigma), self.lmax, int(max_states), ctypes.byref(self._h)))
        nnz, ncol, npr = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().rs_nl_info(self._h, ctypes.byref(nnz), ctypes.byref(ncol), ctypes.byref(npr)))
        self.nnz, self.ncolours, self.nproj = nnz.value, ncol.value, npr.value

    @property
    def handle(self):
        return self._h

    def export(self):
        ptr = np.empty(self.nat + 1, dtype=np.int64)
        idx = np.empty(max(self.nnz, 1), dtype=np.int64)
        gam = np.empty((max(self.nnz, 1), self.nproj), dtype=np.float64)
        col = np.empty(max(self.nat, 1), dtype=np.int32)
        check(lib().rs_nl_export(self._h, _ptr(ptr), _ptr(idx), _ptr(gam), _ptr(col)))
        return dict(sph_ptr=ptr, sph_idx=idx[: self.nnz], gamma=gam[: self.nnz],
                    colour=col[: self.nat])

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(_abi, "_lib", None) if _abi is not None else None
        if h and L is not None:
            L.rs_nl_destroy(h)
            self._h = None


# ------------------------------------------------------------ torch glue
def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return RS_F64
    if t.dtype == torch.float32:
        return RS_F32
    if t.dtype == torch.complex128:
        return RS_C128
    if t.dtype == torch.complex64:
        return RS_C64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _real_dtype(t):
    """float64 for float64/complex128 fields, float32 for float32/complex64."""
    torch = _torch()
    return torch.float64 if t.dtype in (torch.float64, torch.complex128) else torch.float32


def _columns(psi) -> int:
    """Real columns per state: 2 for complex states."""
    return 2 if psi.is_complex() else 1


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check(t, name: str, shape=None, dtype=None, like=None, numel=None):
    """Refuses a tensor whose shape, dtype or device differs from what the C
    call will read or write (the C side only sees a pointer)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if like is not None:
        shape = tuple(like.shape) if shape is None else shape
        dtype = like.dtype if dtype is None else dtype
        if t.device != like.device:
            raise ValueError(f"{name} must be on {like.device}, got {t.device}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _blocks(psi, grid: Grid, complex_ok: bool = False):
    torch = _torch()
    if not isinstance(psi, torch.Tensor):
        raise TypeError("fields must be torch tensors")
    if psi.dim() != 3 or psi.shape[1] != grid.np:
        raise ValueError(f"psi must be [nblk, np={grid.np}, B], got {tuple(psi.shape)}")
    ok = (torch.float32, torch.float64) + ((torch.complex64, torch.complex128) if complex_ok else ())
    if psi.dtype not in ok:
        extra = " (or complex64, complex128)" if complex_ok else ""
        raise ValueError(f"fields must be float32 or float64{extra}, got {psi.dtype}")
    B = psi.shape[2]
    bmax = 32 if psi.is_complex() else 64
    if B < 1 or B > bmax or (B & (B - 1)):
        raise ValueError(f"B must be a power of two in [1, {bmax}], got {B}")
    return psi.shape[0], B


def hpsi_block(grid: Grid, nl: Optional[NonLocal], vloc, psi, hpsi, stream=None):
    """hpsi = (T + V + V_nl) psi for psi [nblk, np, B] (rs_hpsi_block); psi
    real or complex, vloc real of the same precision."""
    nblk, B = _blocks(psi, grid, complex_ok=True)
    _check(hpsi, "hpsi", like=psi)
    _check(vloc, "vloc", dtype=_real_dtype(psi), numel=grid.np)
    if nl is not None and nblk * B * _columns(psi) > nl.max_states:
        raise ValueError(f"{nblk * B * _columns(psi)} real columns exceed the projector set's max_states")
    if vloc.device != psi.device:
        raise ValueError("vloc must be on psi's device")
    if hpsi.data_ptr() == psi.data_ptr():
        raise ValueError("hpsi must not alias psi")
    check(lib().rs_hpsi_block(grid.handle, nl.handle if nl is not None else None,
                              _dev(vloc, "vloc"), _dev(psi, "psi"), _dev(hpsi, "hpsi"),
                              nblk, B, _dtype_code(psi), _stream(stream)))
    return hpsi


def project_nl(grid: Grid, nl: NonLocal, psi, proj, stream=None):
    """proj [nblk, nat, nproj, B] = h^3 <gamma_A,i|psi> (rs_project_nl)."""
    nblk, B = _blocks(psi, grid, complex_ok=True)
    _check(proj, "proj", shape=(nblk, nl.nat, nl.nproj, B), dtype=psi.dtype)
    if nblk * B * _columns(psi) > nl.max_states:
        raise ValueError(f"{nblk * B * _columns(psi)} real columns exceed the projector set's max_states")
    check(lib().rs_project_nl(grid.handle, nl.handle, _dev(psi, "psi"), _dev(proj, "proj"),
                              nblk, B, _dtype_code(psi), _stream(stream)))
    return proj


def apply_nl(grid: Grid, nl: NonLocal, proj, hpsi, stream=None):
    """hpsi += sum gamma D proj (rs_apply_nl)."""
    nblk, B = _blocks(hpsi, grid, complex_ok=True)
    _check(proj, "proj", shape=(nblk, nl.nat, nl.nproj, B), dtype=hpsi.dtype)
    if proj.device != hpsi.device:
        raise ValueError("proj must be on hpsi's device")
    if nblk * B * _columns(hpsi) > nl.max_states:
        raise ValueError(f"{nblk * B * _columns(hpsi)} real columns exceed the projector set's max_states")
    check(lib().rs_apply_nl(grid.handle, nl.handle, _dev(proj, "proj"), _dev(hpsi, "hpsi"),
                            nblk, B, _dtype_code(hpsi), _stream(stream)))
    return hpsi


def overlap_noalloc(grid: Grid, x, y, S, prec=None, stream=None):
    """S [N, N] (float64, caller-allocated) = h^3 X^T Y with the library's
    fixed device scratch (rs_overlap_noalloc): N <= 256, no allocation."""
    torch = _torch()
    nblk, B = _blocks(x, grid)
    _check(y, "y", like=x)
    N = nblk * B
    if N > 256:
        raise ValueError(f"rs_overlap_noalloc handles at most 256 states, got {N}")
    _check(S, "S", shape=(N, N), dtype=torch.float64)
    if S.device != x.device:
        raise ValueError("S must be on x's device")
    check(lib().rs_overlap_noalloc(grid.handle, _dev(x, "x"), _dev(y, "y"), _dev(S, "S"), nblk, B,
                                   _dtype_code(x), Context._prec(x, prec), _stream(stream)))
    return S


class Poisson:
    """Hartree potential of a density on a finite grid by FFT on an enlarged
    box with the cut-off Coulomb kernel (rs_poisson)."""

    def __init__(self, grid: Grid):
        self.grid = grid
        self._h = ctypes.c_void_p()
        check(lib().rs_poisson_create(grid.handle, ctypes.byref(self._h)))
        n, rc = ctypes.c_int32(), ctypes.c_double()
        check(lib().rs_poisson_info(self._h, ctypes.byref(n), ctypes.byref(rc)))
        self.nbox, self.rc = n.value, rc.value

    def solve(self, rho, out=None, stream=None):
        """V_H [np] (float64, on rho's device) for the density rho [np]."""
        torch = _torch()
        _check(rho, "rho", dtype=torch.float64, numel=self.grid.np)
        if not rho.is_cuda:
            raise ValueError("rho must be a device tensor")
        if out is None:
            out = torch.empty_like(rho)
        _check(out, "out", like=rho)
        if out.data_ptr() == rho.data_ptr():
            raise ValueError("out must not alias rho")
        check(lib().rs_poisson_solve(self._h, _dev(rho, "rho"), _dev(out, "out"), _stream(stream)))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(_abi, "_lib", None) if _abi is not None else None
        if h and L is not None:
            L.rs_poisson_destroy(h)
            self._h = None


class Context:
    """Workspaces of the orthogonalisation / subspace stage (rs_ctx)."""

    def __init__(self, grid: Grid, max_states: int):
        self.grid = grid
        self.max_states = max_states
        self._h = ctypes.c_void_p()
        check(lib().rs_ctx_create(grid.handle, int(max_states), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(_abi, "_lib", None) if _abi is not None else None
        if h and L is not None:
            L.rs_ctx_destroy(h)
            self._h = None

    def _fields(self, psi, complex_ok: bool = False):
        nblk, B = _blocks(psi, self.grid, complex_ok)
        if nblk * B * _columns(psi) > self.max_states:
            raise ValueError(f"{nblk * B * _columns(psi)} real columns exceed the context's max_states "
                             f"{self.max_states}")
        return nblk, B

    def _square(self, A, name):
        torch = _torch()
        if A.dim() != 2 or A.shape[0] != A.shape[1]:
            raise ValueError(f"{name} must be square [N, N], got {tuple(A.shape)}")
        N = A.shape[0]
        if N < 1 or N > self.max_states:
            raise ValueError(f"{name}: N must be in [1, {self.max_states}]")
        _check(A, name, dtype=torch.float64)
        return N

    @staticmethod
    def _prec(t, prec):
        if prec is not None:
            return prec
        return RS_PREC_NATIVE if _dtype_code(t) in (RS_F64, RS_C128) else RS_PREC_BF16X3

    def overlap(self, x, y, S=None, prec=None, stream=None):
        """S [N, N] = h^3 X^H Y (rs_overlap): float64, or complex128 for
        complex states."""
        nblk, B = self._fields(x, complex_ok=True)
        _check(y, "y", like=x)
        torch = _torch()
        N = nblk * B
        sdt = torch.complex128 if x.is_complex() else torch.float64
        if S is None:
            S = torch.empty((N, N), dtype=sdt, device=x.device)
        _check(S, "S", shape=(N, N), dtype=sdt)
        if S.device != x.device:
            raise ValueError("S must be on x's device")
        check(lib().rs_overlap(self._h, _dev(x, "x"), _dev(y, "y"), _dev(S, "S"), nblk, B,
                               _dtype_code(x), self._prec(x, prec), _stream(stream)))
        return S

    def rotate(self, psi, X, prec=None, stream=None):
        """psi <- psi X in place (rs_rotate)."""
        nblk, B = self._fields(psi)
        N = nblk * B
        _check(X, "X", shape=(N, N), dtype=_torch().float64)
        check(lib().rs_rotate(self._h, _dev(psi, "psi"), _dev(X, "X"), nblk, B,
                              _dtype_code(psi), self._prec(psi, prec), _stream(stream)))
        return psi

    def cholesky(self, S, stream=None):
        """(U, info) with S = U^T U (rs_cholesky); info is a device int32."""
        torch = _torch()
        N = self._square(S, "S")
        U = torch.empty_like(S)
        info = torch.zeros(1, dtype=torch.int32, device=S.device)
        check(lib().rs_cholesky(self._h, _dev(S, "S"), _dev(U, "U"), N, _dev(info, "info"),
                                _stream(stream)))
        return U, info

    def eigh(self, A, stream=None):
        """(evals, V) of symmetric A (rs_eigh); A is copied, not destroyed."""
        torch = _torch()
        N = self._square(A, "A")
        W = A.clone()
        V = torch.empty_like(A)
        ev = torch.empty(N, dtype=torch.float64, device=A.device)
        check(lib().rs_eigh(self._h, _dev(W, "A"), _dev(V, "V"), _dev(ev, "evals"), N,
                            _stream(stream)))
        return ev, V

    def orthonormalize(self, psi, S_out=None, prec=None, stream=None):
        """psi <- psi U^-1 in place (rs_orthonormalize_block); returns info."""
        nblk, B = self._fields(psi)
        if S_out is not None:
            _check(S_out, "S_out", shape=(nblk * B, nblk * B), dtype=_torch().float64)
        info = ctypes.c_int32(0)
        check(lib().rs_orthonormalize_block(
            self._h, _dev(psi, "psi"), nblk, B, _dtype_code(psi), self._prec(psi, prec),
            _dev(S_out, "S_out") if S_out is not None else None, ctypes.byref(info),
            _stream(stream)))
        return info.value

    def subspace_diag(self, psi, hpsi, prec=None, stream=None):
        """Rayleigh-Ritz in place (rs_subspace_diag); returns eigenvalues."""
        nblk, B = self._fields(psi)
        _check(hpsi, "hpsi", like=psi)
        torch = _torch()
        ev = torch.empty(nblk * B, dtype=torch.float64, device=psi.device)
        check(lib().rs_subspace_diag(self._h, _dev(psi, "psi"), _dev(hpsi, "hpsi"), _dev(ev, "eig"),
                                     nblk, B, _dtype_code(psi), self._prec(psi, prec),
                                     _stream(stream)))
        return ev


class Scf:
    """The self-consistent field loop (rs_scf): effective potential from the
    density (Hartree by FFT, LDA), eig_steps eigensolver steps, output
    density, Broyden/Anderson mixing."""

    def __init__(self, grid: Grid, nl: Optional[NonLocal], vion, nstates: int, B: int, nocc: int,
                 dtype=None, eig_steps: int = 3, mix: float = 0.3, history: int = 5,
                 m: int = 3, alpha: float = 0.52, tol: float = 1e-6, block_stop: bool = True):
        torch = _torch()
        _check(vion, "vion", dtype=torch.float64, numel=grid.np)
        if not vion.is_cuda:
            raise ValueError("vion must be a device tensor")
        self.grid, self.nstates, self.B = grid, nstates, B
        self.nblk = -(-nstates // B)
        self.dtype = torch.float64 if dtype is None else dtype
        o = _abi.ScfOpts()
        o.nocc, o.eig_steps, o.history, o.mix = int(nocc), int(eig_steps), int(history), float(mix)
        o.solver.m, o.solver.alpha, o.solver.tol = int(m), float(alpha), float(tol)
        o.solver.block_stop, o.solver.record, o.solver.rr_sweeps = int(block_stop), 0, 0
        code = RS_F64 if self.dtype == torch.float64 else RS_F32
        self._h = ctypes.c_void_p()
        check(lib().rs_scf_create(grid.handle, nl.handle if nl is not None else None, _dev(vion, "vion"),
                                  int(nstates), int(B), code, ctypes.byref(o), ctypes.byref(self._h)))

    def _own(self, psi):
        _check(psi, "psi", shape=(self.nblk, self.grid.np, self.B), dtype=self.dtype)

    def start(self, psi, stream=None):
        self._own(psi)
        check(lib().rs_scf_start(self._h, _dev(psi, "psi"), _stream(stream)))

    def iterate(self, psi, stream=None):
        """One SCF iteration in place; returns (eig, resnorm, density residual)."""
        self._own(psi)
        eig = np.empty(self.nstates)
        res = np.empty(self.nstates)
        dr = ctypes.c_double(0.0)
        check(lib().rs_scf_iterate(self._h, _dev(psi, "psi"), eig.ctypes.data_as(_abi.PF64),
                                   res.ctypes.data_as(_abi.PF64), ctypes.byref(dr), _stream(stream)))
        return eig, res, dr.value

    def densities(self, stream=None):
        """(n_in, n_out) device float64 [np] copies."""
        torch = _torch()
        a = torch.empty(self.grid.np, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        check(lib().rs_scf_density(self._h, _dev(a, "n_in"), _dev(b, "n_out"), _stream(stream)))
        return a, b

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(_abi, "_lib", None) if _abi is not None else None
        if h and L is not None:
            L.rs_scf_destroy(h)
            self._h = None


class Eigensolver:
    """RMM-DIIS eigensolver over the states of one grid (rs_solver)."""

    def __init__(self, grid: Grid, nl: Optional[NonLocal], vloc, nstates: int, B: int,
                 m: int = 3, alpha: float = 0.52, tol: float = 1e-6, block_stop: bool = True,
                 record: bool = False, rr_sweeps: int = 0):
        _check(vloc, "vloc", numel=grid.np)
        if vloc.dim() != 1:
            raise ValueError("vloc must be one-dimensional [np]")
        self.grid, self.nl, self.vloc = grid, nl, vloc     # vloc kept alive here
        self.nstates, self.B = nstates, B
        self.nblk = -(-nstates // B)          # the last block may be zero-padded
        self.dtype = vloc.dtype
        self.precond = None
        o = _abi.SolverOpts()
        o.m, o.alpha, o.tol, o.block_stop = int(m), float(alpha), float(tol), int(block_stop)
        o.record = int(record)
        o.rr_sweeps = int(rr_sweeps)
        self._h = ctypes.c_void_p()
        check(lib().rs_eigensolve_create(grid.handle, nl.handle if nl is not None else None,
                                         _dev(vloc, "vloc"), int(nstates), int(B),
                                         _dtype_code(vloc), ctypes.byref(o), ctypes.byref(self._h)))

    def step(self, psi, stream=None):
        """One step in place; returns (eig, resnorm, nconv) on the host."""
        self._own(psi)
        eig = np.empty(self.nstates)
        res = np.empty(self.nstates)
        nconv = ctypes.c_int32(0)
        check(lib().rs_eigensolve_step(
            self._h, _dev(psi, "psi"), eig.ctypes.data_as(_abi.PF64),
            res.ctypes.data_as(_abi.PF64), ctypes.byref(nconv), _stream(stream)))
        return eig, res, nconv.value

    def orthonormalize(self, psi, stream=None):
        """Orthonormalise the states (padding states stay zero)."""
        self._own(psi)
        check(lib().rs_eigensolve_orthonormalize(self._h, _dev(psi, "psi"), _stream(stream)))

    def stats(self) -> dict:
        """Counters of the last step: steps, rr_sweeps (Jacobi sweeps of its
        Rayleigh-Ritz problem), frozen_blocks, net_states."""
        st = _abi.SolverStats()
        check(lib().rs_eigensolve_stats(self._h, ctypes.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in _abi.SolverStats._fields_}

    def _own(self, psi):
        """psi must be the solver's [nblk, np, B] blocks in its dtype."""
        nblk, B = _blocks(psi, self.grid)
        if nblk != self.nblk or B != self.B:
            raise ValueError("psi does not match the solver's blocks")
        if psi.dtype != self.dtype:
            raise ValueError(f"psi must be {self.dtype}, got {psi.dtype}")
        if psi.device != self.vloc.device:
            raise ValueError("psi must be on the solver's device")

    def set_precond(self, cnn: Optional["Cnn"]):
        """Use the network as preconditioner (None: the filter)."""
        check(lib().rs_eigensolve_set_precond(self._h, cnn.handle if cnn is not None else None))
        self.precond = cnn          # kept alive while in use

    def residuals(self, stream=None):
        """(R0 [nblk, np, B], sigma [N]) of the last step (needs record=True)."""
        torch = _torch()
        R = torch.empty((self.nblk, self.grid.np, self.B), dtype=self.dtype, device="cuda")
        sig = torch.empty(self.nblk * self.B, dtype=torch.float64, device="cuda")
        check(lib().rs_eigensolve_residuals(self._h, _dev(R, "R"), _dev(sig, "sigma"), _stream(stream)))
        return R, sig

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(_abi, "_lib", None) if _abi is not None else None
        if h and L is not None:
            L.rs_eigensolve_destroy(h)
            self._h = None


class Cnn:
    """Learned preconditioner network (rs_cnn): parameters, forward,
    training loss/gradient, Adam, and application to grid fields."""

    NPARAM = _abi.RS_CNN_NPARAM

    def __init__(self, max_batch: int, max_box: int):
        self._h = ctypes.c_void_p()
        check(lib().rs_cnn_create(int(max_batch), int(max_box), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (self.NPARAM,):
            raise ValueError(f"params must have {self.NPARAM} values")
        check(lib().rs_cnn_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p)))

    def get_params(self) -> np.ndarray:
        p = np.empty(self.NPARAM, dtype=np.float32)
        check(lib().rs_cnn_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p)))
        return p

    def save(self, path: str):
        """Parameters, Adam moments and step count to a file (rs_cnn_save)."""
        check(lib().rs_cnn_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        """Restores a checkpoint written by save (rs_cnn_load)."""
        check(lib().rs_cnn_load(self._h, os.fsencode(path)))

    @staticmethod
    def _dims(t):
        if t.dim() != 4:
            raise ValueError("boxes must be [n, Z, Y, X]")
        return (ctypes.c_int32 * 3)(*[int(v) for v in t.shape[1:]])

    def forward(self, u, periodic: bool = False, stream=None):
        torch = _torch()
        _check(u, "u", dtype=torch.float32)
        f = torch.empty_like(u)
        check(lib().rs_cnn_forward(self._h, _dev(u, "u"), _dev(f, "f"), int(u.shape[0]), self._dims(u),
                                   int(periodic), _stream(stream)))
        return f

    def loss_grad(self, u, t, sigma, h: float, margin: int, want_du: bool = False, stream=None):
        """Returns (loss, grad [NPARAM] float32, du or None)."""
        torch = _torch()
        self._batch(u, t, sigma)
        loss = ctypes.c_double(0.0)
        grad = np.empty(self.NPARAM, dtype=np.float32)
        du = torch.empty_like(u) if want_du else None
        check(lib().rs_cnn_loss_grad(self._h, _dev(u, "u"), _dev(t, "t"), _dev(sigma, "sigma"),
                                     int(u.shape[0]), self._dims(u), float(h), int(margin),
                                     ctypes.byref(loss), grad.ctypes.data_as(ctypes.c_void_p),
                                     _dev(du, "du") if du is not None else None, _stream(stream)))
        return loss.value, grad, du

    def train_step(self, u, t, sigma, h: float, margin: int, lr: float, stream=None) -> float:
        """Loss and gradient, then one Adam update; returns the loss."""
        self._batch(u, t, sigma)
        loss = ctypes.c_double(0.0)
        check(lib().rs_cnn_loss_grad(self._h, _dev(u, "u"), _dev(t, "t"), _dev(sigma, "sigma"),
                                     int(u.shape[0]), self._dims(u), float(h), int(margin),
                                     ctypes.byref(loss), None, None, _stream(stream)))
        self.adam_step(lr, stream=stream)
        return loss.value

    @staticmethod
    def _batch(u, t, sigma):
        torch = _torch()
        _check(u, "u", dtype=torch.float32)
        Cnn._dims(u)
        _check(t, "t", like=u)
        _check(sigma, "sigma", dtype=torch.float64, numel=int(u.shape[0]))

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                  stream=None):
        check(lib().rs_cnn_adam_step(self._h, lr, beta1, beta2, eps, _stream(stream)))

    def box(self, grid: Grid):
        d = (ctypes.c_int32 * 3)()
        check(lib().rs_cnn_box(self._h, grid.handle, d))
        return tuple(d)

    def precondition(self, grid: Grid, r, sigma, stream=None):
        nblk, B = _blocks(r, grid)
        _check(sigma, "sigma", dtype=_torch().float64, numel=nblk * B)
        out = _torch().empty_like(r)
        check(lib().rs_cnn_precondition(self._h, grid.handle, _dev(r, "r"), _dev(sigma, "sigma"),
                                        _dev(out, "out"), nblk, B, _dtype_code(r), _stream(stream)))
        return out

    def crops(self, grid: Grid, r, x, desc: np.ndarray, dims, stream=None):
        """desc [ncrops, 4] = (state, x0, y0, z0); returns (u, t) [ncrops, *dims]."""
        torch = _torch()
        nblk, B = _blocks(r, grid)
        _check(x, "x", like=r)
        d = np.ascontiguousarray(desc, dtype=np.int32)
        if d.ndim != 2 or d.shape[1] != 4:
            raise ValueError("desc must be [ncrops, 4]")
        if len(dims) != 3:
            raise ValueError("dims must be (Z, Y, X)")
        n = d.shape[0]
        u = torch.empty((n,) + tuple(dims), dtype=torch.float32, device="cuda")
        t = torch.empty_like(u)
        cd = (ctypes.c_int32 * 3)(*[int(v) for v in dims])
        check(lib().rs_cnn_crops(self._h, grid.handle, _dev(r, "r"), _dev(x, "x"), nblk, B, _dtype_code(r),
                                 n, d.ctypes.data_as(ctypes.c_void_p), cd, _dev(u, "u"), _dev(t, "t"),
                                 _stream(stream)))
        return u, t

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(_abi, "_lib", None) if _abi is not None else None
        if h and L is not None:
            L.rs_cnn_destroy(h)
            self._h = None


def shifted_solve(grid: Grid, r, sigma, tol: float = 1e-8, maxit: int = 2000, stream=None):
    """x = (T - sigma)^-1 r per state by conjugate gradients; returns (x, iterations)."""
    nblk, B = _blocks(r, grid)
    _check(sigma, "sigma", dtype=_torch().float64, numel=nblk * B)
    x = _torch().empty_like(r)
    it = ctypes.c_int32(0)
    check(lib().rs_shifted_solve(grid.handle, _dev(r, "r"), _dev(sigma, "sigma"), _dev(x, "x"), nblk, B,
                                 _dtype_code(r), float(tol), int(maxit), ctypes.byref(it), _stream(stream)))
    return x, it.value


def to_blocks(states: np.ndarray, B: int) -> np.ndarray:
    """State-major [N, np] -> block layout [ceil(N/B), np, B] (host-side
    reshuffle); a partial last block is padded with zero states."""
    N, npts = states.shape
    nblk = -(-N // B)
    if nblk * B != N:
        states = np.concatenate([states, np.zeros((nblk * B - N, npts), dtype=states.dtype)])
    return np.ascontiguousarray(states.reshape(nblk, B, npts).transpose(0, 2, 1))


def from_blocks(blocks: np.ndarray, n: Optional[int] = None) -> np.ndarray:
    """Block layout [nblk, np, B] -> state-major [n, np] (default all
    nblk*B states; n drops the padding)."""
    nblk, npts, B = blocks.shape
    out = np.ascontiguousarray(blocks.transpose(0, 2, 1).reshape(nblk * B, npts))
    return out if n is None else out[:n]
