"""A cell above 65 536 atoms in mixed precision takes 32-bit neighbour-list entries (batches of
smaller cells use 16-bit ones): forces, stress and a short trajectory against the FP64 oracle, at
the mixed-precision bounds of the other parity tests, beside a small cell of the same batch."""
import numpy as np
import pytest

from oracle import core
from synth import configs

pytestmark = pytest.mark.gpu


def fro(s6):
    return np.sqrt((s6[..., :3] ** 2).sum(-1) + 2 * (s6[..., 3:] ** 2).sum(-1))


def large_batch():
    p = configs.kg_params(precision="mixed")
    cells = [configs.kg_cell([100] * 700, 4242), configs.kg_cell([20] * 10, 4243)]   # 70 000 and 200 beads
    F = np.stack([configs.uniaxial_isochoric(0.02), configs.uniaxial_isochoric(0.01)])
    return p, cells, F


def test_mixed_precision_cell_above_65536_atoms():
    from paper_1902_09171_amd import rcell
    rcell.load()
    p, cells, F = large_batch()
    assert len(cells[0]["x"]) > 65536
    g = rcell.RCellBatch(p, cells)
    o = core.OracleBatch(p, cells)
    g.set_deformation(F)
    o.set_deformation(F)
    for k in range(2):
        fg, fo = g.get_forces(k), o.get_forces(k)
        err = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
        err_a = np.abs(fg - fo).max() / np.sqrt((fo ** 2).sum(1).mean())
        print(f"cell {k}: force rel {err:.2e}, per-atom {err_a:.2e}", flush=True)
        assert err <= 1e-5 and err_a <= 1e-4
    sg, so = g.get_stress(), o.get_stress()
    assert (np.abs(sg - so).max(-1) / fro(so)).max() <= 1e-5
    g.run(10)
    o.run(10)
    sg, so = g.get_stress(), o.get_stress()
    err = (np.abs(sg - so).max(-1) / fro(so)).max()
    print(f"window stress after 10 steps: rel {err:.2e}", flush=True)
    assert err <= 1e-4
    assert np.all(g.status() == 0)
