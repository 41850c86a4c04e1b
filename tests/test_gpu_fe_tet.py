"""The FE driver on the paper's element (C3D4 tetrahedra, one r-cell per element; Sec. 3.2) with
GPU r-cells, against the same driver with FP64 oracle r-cells: a bar of 10 tetrahedra pulled for
a few load steps, in FP64 (the nodal motion feeds back into the next load step's F, so the two
runs agree only if every step does), and in mixed precision at the trajectory tolerance."""
import numpy as np
import pytest

from oracle import core
from synth import configs

pytestmark = pytest.mark.gpu

MD_STEPS, NLOAD = 20, 4
TOL = {"fp64": 1e-9, "mixed": 1e-4}


def fro(s6):
    return np.sqrt((s6[..., :3] ** 2).sum(-1) + 2 * (s6[..., 3:] ** 2).sum(-1))


class OracleStress:
    """The FE stress provider backed by oracle r-cells (the same protocol as fe.MDStress)."""

    def __init__(self, params, cells, md_steps):
        self.o = core.OracleBatch(params, cells)
        self.md_steps = md_steps

    def __call__(self, F):
        self.o.set_deformation(F)
        self.o.run(self.md_steps)
        s, P = self.o.get_stress(with_P=True)
        return P, s


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tet_bar_with_gpu_cells_matches_oracle_cells(prec):
    from paper_1902_09171_amd import fe
    params = configs.kg_params(precision=prec)
    mesh = fe.Tet4Bar(nel=(2, 1, 1), size=(40.0, 20.0, 20.0), rho0=0.85)
    assert mesh.ngp == 10
    cells = [configs.kg_cell([20] * 10, 700 + g) for g in range(mesh.ngp)]
    dt = MD_STEPS * params["dt"]
    vpull = 0.02 * mesh.size[0] / dt
    bars = []
    for provider in (fe.MDStress(params, cells, MD_STEPS), OracleStress(params, cells, MD_STEPS)):
        bar = fe.ExplicitBar(mesh, provider, dt=dt, pull_velocity=vpull, damping=0.2)
        for _ in range(NLOAD):
            bar.step()
        bars.append(bar)
    g, o = bars
    for k in range(NLOAD):
        sg, so = g.history[k]["sigma"], o.history[k]["sigma"]
        err = (np.abs(sg - so).max(1) / fro(so)).max()
        print(f"{prec} load step {k}: strain {g.history[k]['strain']:.3f}, stress rel {err:.2e}", flush=True)
        assert err <= TOL[prec], (k, err)
    assert np.abs(g.u - o.u).max() <= TOL[prec] * np.abs(o.u).max()
    assert np.all(bars[0].provider.g.status() == 0)
