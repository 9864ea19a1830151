"""ctypes wrapper of the C/OpenMP oracle H psi (TEST INFRASTRUCTURE ONLY).

``build()`` compiles ``cpu_hpsi.c`` with gcc; ``hpsi_blocks`` applies the
operator to states in the block layout [nblk, np, B] for CPU timing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import stencil
from .grid import neighbour_table

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpu_hpsi.c")
_LIB = os.path.join(_HERE, "libcpu_hpsi.so")


def build() -> str:
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-o", _LIB, _SRC]
    subprocess.run(cmd, check=True)
    return _LIB


def _lib():
    if not os.path.exists(_LIB):
        raise RuntimeError(f"{_LIB} not built; run oracle.cpu_hpsi.build()")
    lib = ctypes.CDLL(_LIB)
    f = lib.oracle_hpsi_f64
    P = ctypes.c_void_p
    f.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P,
                  ctypes.c_double, P, P, P, ctypes.c_int, P, P, P, P, P]
    f.restype = None
    return f


def threads() -> int:
    """OpenMP threads the C oracle's parallel loops use."""
    if not os.path.exists(_LIB):
        raise RuntimeError(f"{_LIB} not built; run oracle.cpu_hpsi.build()")
    f = ctypes.CDLL(_LIB).oracle_threads
    f.restype = ctypes.c_int
    return int(f())


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or 'unknown'."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class CpuHamiltonian:
    """Holds the flattened tables of an oracle Hamiltonian for the C kernel."""

    def __init__(self, H):
        g = H.g
        self.np = g.np
        self.M = g.M
        self.h = g.h
        self.nbr = np.ascontiguousarray(neighbour_table(g).reshape(g.np, -1))
        self.c = stencil.fd_weights(g.M)
        self.vloc = np.ascontiguousarray(H.vloc, dtype=np.float64)
        ps = H.proj
        if ps is not None and ps.nat:
            if ps.nproj != 4:
                raise ValueError("the C kernel takes the s and p projectors (lmax 1) only")
            self.nat = ps.nat
            lens = [len(i) for i in ps.idx]
            self.sph_ptr = np.zeros(self.nat + 1, dtype=np.int64)
            self.sph_ptr[1:] = np.cumsum(lens)
            self.sph_idx = np.ascontiguousarray(np.concatenate(ps.idx).astype(np.int64))
            self.gamma = np.ascontiguousarray(np.concatenate(ps.gamma, axis=0))
            self.D = np.ascontiguousarray(ps.D, dtype=np.float64)
        else:
            self.nat = 0
            self.sph_ptr = np.zeros(1, dtype=np.int64)
            self.sph_idx = np.zeros(1, dtype=np.int64)
            self.gamma = np.zeros((1, 4))
            self.D = np.zeros((1, 4))
        self._f = _lib()

    def hpsi_blocks(self, psi_blk: np.ndarray) -> np.ndarray:
        nblk, np_, B = psi_blk.shape
        assert np_ == self.np and B <= 64
        x = np.ascontiguousarray(psi_blk, dtype=np.float64)
        y = np.empty_like(x)
        proj = np.empty((max(self.nat, 1), 4, B))
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._f(self.np, nblk, B, ptr(self.nbr), self.M, ptr(self.c), self.h,
                ptr(self.vloc), ptr(x), ptr(y), self.nat, ptr(self.sph_ptr),
                ptr(self.sph_idx), ptr(self.gamma), ptr(self.D), ptr(proj))
        return y


class FastHamiltonian:
    """The oracle Hamiltonian's interface (g, dv, nbr, vloc, proj, apply,
    apply_kinetic) with ``apply`` done by the C kernel above, for oracle
    iterations on grids where the numpy operator is slow.  Same operator,
    same FP64 arithmetic (the C kernel is checked against the numpy one)."""

    def __init__(self, H):
        self.H = H
        self.g, self.vloc, self.proj, self.nbr = H.g, H.vloc, H.proj, H.nbr
        self.ch = CpuHamiltonian(H)

    @property
    def dv(self) -> float:
        return self.H.dv

    def apply(self, psi: np.ndarray) -> np.ndarray:
        x = np.atleast_2d(psi)
        N = x.shape[0]
        out = np.empty_like(x, dtype=np.float64)
        for j0 in range(0, N, 32):
            j1 = min(j0 + 32, N)
            blk = np.ascontiguousarray(x[j0:j1].T)[None]
            out[j0:j1] = self.ch.hpsi_blocks(blk)[0].T
        return out if psi.ndim == 2 else out[0]

    def apply_kinetic(self, psi: np.ndarray) -> np.ndarray:
        return self.H.apply_kinetic(psi)
