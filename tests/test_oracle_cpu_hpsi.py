"""The C/OpenMP oracle H psi (used for the CPU baseline) agrees with the
Python oracle (CPU only)."""
import numpy as np
import pytest

import synthetic
from oracle import cpu_hpsi, hamiltonian


@pytest.fixture(scope="module")
def lib():
    cpu_hpsi.build()


@pytest.mark.parametrize("B", [1, 4, 32])
def test_cpu_hpsi_matches_python(lib, B):
    w = synthetic.make_workload("sphere_r12_h0.2", radius=2.4, nat=3, atom_radius=1.0)
    g, _, H = hamiltonian.build_system(w)
    rng = np.random.default_rng(B)
    nblk = 2
    psi = rng.uniform(-1, 1, size=(nblk * B, g.np))
    want = H.apply(psi)
    blk = psi.reshape(nblk, B, g.np).transpose(0, 2, 1)
    got = cpu_hpsi.CpuHamiltonian(H).hpsi_blocks(blk)
    got = got.transpose(0, 2, 1).reshape(nblk * B, g.np)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
