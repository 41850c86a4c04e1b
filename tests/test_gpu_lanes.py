"""The lanes-per-atom autotune (rcell_set_lanes(0)) times the MD step's force pass on copies of the
positions, velocities and forces: it must leave the state (positions, velocities, stored forces,
box, step counter) and the trajectory that follows bit for bit as they were, for both potentials."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("pot", ["kg", "cu"])
def test_autotune_advances_no_state(rc, pot):
    if pot == "kg":
        p = configs.kg_params(precision="mixed")
        cells = [configs.kg_cell([40] * 25, 900 + k) for k in range(3)]
    else:
        p = configs.cu_params(precision="mixed")
        cells = cu_cells(3)
    a, b = rc.RCellBatch(p, cells), rc.RCellBatch(p, cells)
    F = np.stack([configs.uniaxial_isochoric(0.01 * (k + 1)) for k in range(3)])
    for g in (a, b):
        g.set_deformation(F)
        g.run(7)
    lanes = b.lanes()
    chosen = a.set_lanes(0)
    print(pot, "autotune chose", chosen, "lanes per atom", flush=True)
    assert chosen in (1, 2, 4, 8, 16)
    for k in range(3):
        sa, sb = a.get_state(k), b.get_state(k)
        for key in ("x", "v", "H"):
            assert np.array_equal(sa[key], sb[key]), (k, key)
        assert sa["step"] == sb["step"]
        assert np.array_equal(a.get_forces(k), b.get_forces(k))
    a.set_lanes(lanes)
    for g in (a, b):
        g.run(30)
    assert np.array_equal(a.get_stress(), b.get_stress())
    for k in range(3):
        assert np.array_equal(a.get_state(k)["x"], b.get_state(k)["x"])
    assert np.all(a.status() == 0)
