"""GPU Hartree potential (Sec. 7, eq. (5): FFT on an enlarged box with the
cut-off Coulomb kernel) against the oracle's numpy-FFT solve of the same
definition, through the C ABI.  FP64; tolerance 1e-12 of the largest value
(round-off of two 3-D FFTs of up to 256^3 points)."""
import numpy as np
import pytest

import synthetic
from oracle import grid as ogrid, poisson as opoisson

torch = pytest.importorskip("torch")
import paper_1306_2953_amd as rsd  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"


CASES = [
    ("sphere", dict(h=0.4, radius=3.0)),                       # small box (32^3)
    ("sphere", dict(h=0.3, radius=5.0)),                       # 64^3
    ("box", dict(h=0.3, n=13)),                                # Dirichlet box
    ("union", dict(h=0.41, radius=5.5, nat=8, atom_radius=3.0)),
]


@pytest.mark.parametrize("kind,kw", CASES, ids=[c[0] + str(i) for i, c in enumerate(CASES)])
def test_hartree_matches_oracle(kind, kw):
    if kind == "union":
        w = synthetic.make_workload("union_cage60_r5.5_h0.41", h=kw["h"], radius=kw["radius"], nat=kw["nat"],
                                    atom_radius=kw["atom_radius"])
        og = ogrid.grid_for(w)
        g = rsd.Grid.for_workload(w)
    elif kind == "sphere":
        og = ogrid.build_grid("sphere", kw["h"], radius=kw["radius"])
        g = rsd.Grid("sphere", kw["h"], radius=kw["radius"])
    else:
        og = ogrid.build_grid("box", kw["h"], n=kw["n"])
        g = rsd.Grid("box", kw["h"], n=kw["n"])
    rng = np.random.default_rng(21)
    rho = rng.uniform(0.0, 1.0, size=og.np)
    want = opoisson.hartree(og, rho)
    ps = rsd.Poisson(g)
    rc = opoisson.cutoff_radius(og)
    assert ps.nbox == opoisson.box_size(og, rc)
    assert ps.rc == rc
    got = ps.solve(torch.from_numpy(rho).cuda()).cpu().numpy()
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    print(f"{kind}: {og.np} points, box {ps.nbox}^3, rel err {err:.2e}")
    assert err < 1e-12


def test_full_size_sphere_hartree_of_a_gaussian():
    """The 904k-point sphere (box 256^3): a Gaussian charge's potential
    against erf(r / (sqrt(2) s)) / r, and against the oracle at sampled
    points (the full oracle solve of a 256^3 box runs on the host)."""
    from scipy.special import erf
    w = synthetic.WORKLOADS["sphere_r12_h0.2"]
    og = ogrid.grid_for(w)
    g = rsd.Grid.for_workload(w)
    s = 1.3
    r = np.sqrt(np.sum(og.xyz ** 2, axis=1))
    rho = (2 * np.pi * s * s) ** -1.5 * np.exp(-r * r / (2 * s * s))
    ps = rsd.Poisson(g)
    assert ps.nbox == 256
    got = ps.solve(torch.from_numpy(rho).cuda()).cpu().numpy()
    want = np.where(r > 0, erf(r / (np.sqrt(2) * s)) / np.where(r > 0, r, 1.0), np.sqrt(2 / np.pi) / s)
    assert np.max(np.abs(got - want)) < 1e-10
    ref = opoisson.hartree(og, rho)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_periodic_grid_refused():
    g = rsd.Grid("periodic", 0.25, n=16)
    with pytest.raises(rsd.RsError) as e:
        rsd.Poisson(g)
    assert e.value.code == rsd._abi.RS_EINVAL
