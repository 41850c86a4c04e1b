"""The batch engine's autotune (rcell_autotune: the neighbour-bin factor by timed rebuilds of every
cell, then the lanes per atom) and the bin factor itself.

rcell_autotune copies the state aside, rebuilds every cell with each bin factor, and copies the state
back: afterwards the state must be bit for bit the state of an untuned twin, and the trajectory
that follows must equal the twin's once the twin is given the same lanes and bin factor by hand.
The second call on a batch of the same kind takes the cached choice.  With the bin factor 2 (bins
of (rc + skin) / 2, a +-2-bin stencil) forces and trajectories match the FP64 oracle at the usual
bounds, including cells with fewer than five bins along a dimension (then every bin is scanned),
and both rebuild-preparation paths give the same results bit for bit."""
import numpy as np
import pytest

from oracle import core
from synth import configs, fcc_lattice, maxwell_boltzmann

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rc():
    from paper_1902_09171_amd import rcell
    rcell.load()
    return rcell


def cu_cells(n, ncell=6, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        x, H = fcc_lattice(ncell)
        x = x + rng.normal(0, 0.05, x.shape)
        v = maxwell_boltzmann(len(x), 300.0, 63.546, configs.KB_EV, configs.MVV2E_METAL_FS, rng)
        out.append(dict(x=x, v=v, bonds=np.zeros((0, 2), np.int32), H0=H))
    return out


def batch(pot):
    if pot == "kg":
        return configs.kg_params(precision="mixed", skin=0.7), [configs.kg_cell([100] * 50, 950 + k) for k in range(4)]
    return configs.cu_params(precision="mixed"), cu_cells(3)


@pytest.mark.parametrize("pot", ["kg", "cu"])
def test_autotune_leaves_the_state_and_matches_a_hand_set_twin(rc, pot):
    p, cells = batch(pot)
    a, b = rc.RCellBatch(p, cells), rc.RCellBatch(p, cells)
    F = np.stack([configs.uniaxial_isochoric(0.01 * (k + 1)) for k in range(len(cells))])
    for g in (a, b):
        g.set_deformation(F)
        g.run(23)
    lanes, f = a.autotune(use_cache=False)
    print(pot, "autotune chose", lanes, "lanes per atom, bin factor", f, flush=True)
    assert lanes in (1, 2, 4, 8, 16) and f in (1, 2)
    for k in range(len(cells)):
        sa, sb = a.get_state(k), b.get_state(k)
        for key in ("x", "v", "H", "Rprev"):
            assert np.array_equal(sa[key], sb[key]), (k, key)
        assert sa["step"] == sb["step"]
        assert np.array_equal(a.get_forces(k), b.get_forces(k))
    assert a.rebuilds() == b.rebuilds()
    b.set_lanes(lanes)
    b.set_bin_factor(f)
    for g in (a, b):
        g.run(60)
    assert np.array_equal(a.get_stress(), b.get_stress())
    for k in range(len(cells)):
        assert np.array_equal(a.get_state(k)["x"], b.get_state(k)["x"])
    assert a.rebuilds() == b.rebuilds()
    assert np.all(a.status() == 0)
    # a batch of the same kind takes the cached choice
    c = rc.RCellBatch(p, cells)
    assert c.autotune(use_cache=True) == (lanes, f)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_bin_factor_two_matches_the_oracle(rc, prec):
    p = configs.kg_params(precision=prec, skin=0.7)
    # L = 10.6, 4.2 and 3.7 sigma: 11, 4 and 4 half-width bins per dimension
    cells = [configs.kg_cell([50] * 20, 960), configs.kg_cell([10] * 6, 961), configs.kg_cell([11] * 4, 962)]
    g = rc.RCellBatch(p, cells)
    g.set_bin_factor(2)
    assert g.bin_factor() == 2
    F = np.stack([configs.uniaxial_isochoric(0.02), np.eye(3) + 0.01 * np.ones((3, 3)), np.eye(3)])
    o = core.OracleBatch(dict(p, precision="fp64"), cells)
    g.set_deformation(F)        # rebuilds with the half-width bins
    o.set_deformation(F)
    tol = 1e-11 if prec == "fp64" else 1e-5
    for k in range(len(cells)):
        fg, fo = g.get_forces(k), o.get_forces(k)
        err = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
        print(prec, "cell", k, "force rel", err, flush=True)
        assert err <= tol
    g.get_stress()
    o.get_stress()
    for g_ in (g, o):
        g_.run(100)
    sg, so = g.get_stress(), o.get_stress()
    fro = np.sqrt((so[:, :3] ** 2).sum(1) + 2 * (so[:, 3:] ** 2).sum(1))
    err = np.abs(sg - so).max(1) / fro
    print(prec, "100-step window stress rel", err, "rebuilds", g.rebuilds(), flush=True)
    assert err.max() <= (1e-9 if prec == "fp64" else 1e-4)
    assert g.rebuilds() > len(cells)


def test_bin_factor_two_rebuild_paths_are_bitwise_equal(rc):
    p = configs.kg_params(precision="mixed", skin=0.7)
    cells = [configs.kg_cell([50] * 20, 970 + k) for k in range(3)]
    F = np.stack([configs.uniaxial_isochoric(0.02 * (k + 1)) for k in range(3)])
    res = []
    for mode in (1, 2):
        g = rc.RCellBatch(p, cells)
        g.set_build_mode(mode)
        g.set_bin_factor(2)
        g.set_deformation(F)
        g.run(150)
        res.append((g.get_stress(), [g.get_state(k)["x"] for k in range(3)], g.rebuilds()))
    (s1, x1, r1), (s2, x2, r2) = res
    assert r1 == r2 and r1 > 3
    assert np.array_equal(s1, s2)
    for a, b in zip(x1, x2):
        assert np.array_equal(a, b)
