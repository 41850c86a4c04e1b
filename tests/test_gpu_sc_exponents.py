"""Sutton-Chen with exponents other than (9, 6) runs the kernels' general power path (the exponents
taken at run time): gold (n = 10, m = 8, a = 4.08 A, eps = 1.2793e-2 eV, c = 34.408, the published
Sutton-Chen parameter set) in mixed precision against the FP64 oracle - forces and stress of a
deformed, perturbed lattice, then the window stress of a short Langevin run."""
import numpy as np
import pytest

from oracle import core
from synth import configs, fcc_lattice, maxwell_boltzmann

pytestmark = pytest.mark.gpu

A_AU, M_AU = 4.08, 196.967


def fro(s6):
    return np.sqrt((s6[..., :3] ** 2).sum(-1) + 2 * (s6[..., 3:] ** 2).sum(-1))


def gold():
    p = configs.cu_params(sc_eps=1.2793e-2, sc_a=A_AU, sc_c=34.408, sc_n=10, sc_m=8, mass=M_AU,
                          rc=1.95 * A_AU, precision="mixed")
    rng = np.random.default_rng(21)
    cells = []
    for _ in range(2):
        x, H = fcc_lattice(6, A_AU)
        x = x + rng.normal(0, 0.05, x.shape)
        v = maxwell_boltzmann(len(x), 300.0, M_AU, configs.KB_EV, configs.MVV2E_METAL_FS, rng)
        cells.append(dict(x=x, v=v, bonds=np.zeros((0, 2), np.int32), H0=H))
    F = np.stack([configs.uniaxial_isochoric(0.02), configs.uniaxial_isochoric(0.03, axis=1)])
    return p, cells, F


def test_general_exponents_match_the_oracle():
    from paper_1902_09171_amd import rcell
    rcell.load()
    p, cells, F = gold()
    g = rcell.RCellBatch(p, cells)
    o = core.OracleBatch(p, cells)
    g.set_deformation(F)
    o.set_deformation(F)
    for k in range(2):
        fg, fo = g.get_forces(k), o.get_forces(k)
        err = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
        print(f"cell {k}: force rel {err:.2e}", flush=True)
        assert err <= 1e-5
    sg, so = g.get_stress(), o.get_stress()
    assert (np.abs(sg - so).max(-1) / fro(so)).max() <= 1e-5
    pe_g, _ = g.get_energy()
    pe_o, _ = o.get_energy()
    assert np.abs(pe_g - pe_o).max() <= 1e-6 * np.abs(pe_o).max()
    g.run(10)
    o.run(10)
    sg, so = g.get_stress(), o.get_stress()
    err = (np.abs(sg - so).max(-1) / fro(so)).max()
    print(f"window stress after 10 steps: rel {err:.2e}", flush=True)
    assert err <= 1e-4
    assert np.all(g.status() == 0)
