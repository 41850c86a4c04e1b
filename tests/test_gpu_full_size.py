"""Parity at the full sizes of the batched workloads, in the launch configuration the benchmark
times (one batch holding every cell, autotuned lanes per atom, graph-captured MD steps): a sample
of cells, from the smallest to the largest, against the FP64 oracle run on those cells alone
from the same initial state.  Cells are independent, so the oracle needs only the sample.

  * 512 uneven Kremer-Grest cells (2k-20k beads, ~5.6 M beads), each under its own rotation x
    symmetric stretch;
  * the FE bar's 256 Kremer-Grest cells of 400 x 100 beads (~10.2 M beads) under a uniaxial
    stretch with lateral contraction;
  * the single FP64 Kremer-Grest cell under its whole ramp: a new F before each of 1000 MD steps,
    the stress read every 100 steps (all of it, not a sample).  MD is chaotic: FP64 rounding-order
    differences (1e-16) grow by about a decade per 100 steps, so the stress must agree to 1e-9 over
    the first 500 steps and to 1e-4 (with positions to 1e-4) at the end of the ramp;
  * the 100 r-cells of the paper's tetrahedral specimen (100 x 100 beads, 10^6 beads) and the 100
    glassy cells (LJ to 2.5 sigma, T = 0.1), each batch under its own stretches.

Checks: static forces and stress right after the deformation (mixed-precision tolerances), and
the window stress after 20 MD steps (trajectory tolerance)."""
import numpy as np
import pytest

from oracle import core
from synth import configs

pytestmark = pytest.mark.gpu

TOL_F, TOL_FA, TOL_S, TOL_S20 = 1e-5, 1e-4, 1e-5, 1e-4


def fro(s):
    return np.sqrt((s[..., :3] ** 2).sum(-1) + 2 * (s[..., 3:] ** 2).sum(-1))


def check_sample(g, params, cells, F, sample, what):
    sub = [cells[c] for c in sample]
    o = core.OracleBatch(params, sub, cell_ids=sample)     # the noise the cells draw in the batch
    o.set_deformation(F[sample])
    for k, c in enumerate(sample):
        fg, fo = g.get_forces(c), o.get_forces(k)
        err = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
        err_a = np.abs(fg - fo).max() / np.sqrt((fo ** 2).sum(1).mean())
        print(f"{what} cell {c} ({len(fo)} beads): force rel {err:.2e} per-atom {err_a:.2e}", flush=True)
        assert err <= TOL_F and err_a <= TOL_FA, (c, err, err_a)
    sg, so = g.get_stress()[sample], o.get_stress()
    e0 = (np.abs(sg - so).max(1) / fro(so)).max()
    g.run(20)
    o.run(20)
    sg, so = g.get_stress()[sample], o.get_stress()
    e20 = (np.abs(sg - so).max(1) / fro(so)).max()
    print(f"{what}: static stress rel {e0:.2e}, window stress after 20 steps {e20:.2e}", flush=True)
    assert e0 <= TOL_S and e20 <= TOL_S20
    assert np.all(g.status() == 0)


@pytest.mark.timeout(900)
def test_kg_batched_full_size_sampled():
    from paper_1902_09171_amd import rcell
    cfg = configs.kg_batched()
    cells, F, params = cfg["cells"], cfg["F"], cfg["params"]
    sizes = np.array([len(c["x"]) for c in cells])
    print(f"512 cells, {sizes.sum()} beads", flush=True)
    g = rcell.RCellBatch(params, cells)
    g.set_deformation(F)
    g.set_lanes(0)
    order = np.argsort(sizes)
    sample = sorted({int(order[0]), int(order[1]), int(order[len(order) // 2]), int(order[-1]), 0, 511})
    check_sample(g, params, cells, F, sample, "kg_batched")


@pytest.mark.timeout(900)
def test_fe_bar_full_size_sampled():
    from paper_1902_09171_amd import rcell
    cfg = configs.fe_bar_cells()
    cells, params = cfg["cells"], cfg["params"]
    print(f"{len(cells)} cells, {sum(len(c['x']) for c in cells)} beads", flush=True)
    F = np.stack([np.diag([1.02, 0.99, 0.99])] * len(cells))
    g = rcell.RCellBatch(params, cells)
    g.set_deformation(F)
    g.set_lanes(0)
    check_sample(g, params, cells, F, [0, 127, 255], "fe_bar")


@pytest.mark.timeout(600)
def test_kg_single_full_ramp():
    from paper_1902_09171_amd import rcell
    cfg = configs.kg_single()
    params, cells, F_path = cfg["params"], cfg["cells"], cfg["F_path"]
    g = rcell.RCellBatch(params, cells)
    g.set_lanes(0)
    o = core.OracleBatch(params, cells)
    worst, early = 0.0, 0.0
    for k in range(len(F_path)):
        g.set_deformation(F_path[k])
        o.set_deformation(F_path[k])
        g.run(1)
        o.run(1)
        if (k + 1) % cfg["stress_every"] == 0:
            sg, so = g.get_stress(), o.get_stress()
            err = float((np.abs(sg - so).max(1) / fro(so)).max())
            worst = max(worst, err)
            if k < 500:
                early = max(early, err)
            print(f"step {k + 1}: stress rel {err:.2e}", flush=True)
    sg, so = g.get_state(0), o.get_state(0)
    d = sg["x"] - so["x"]                                   # minimum image in the oracle's box
    H = so["H"]
    d -= (np.rint(d @ np.linalg.inv(H).T)) @ H.T
    rms = float(np.sqrt((d ** 2).sum(1).mean()))
    print(f"after {len(F_path)} steps: worst stress rel {worst:.2e} ({early:.2e} over the first 500), "
          f"rms dx {rms:.2e}", flush=True)
    assert early <= 1e-9
    assert worst <= 1e-4 and rms <= 1e-4
    assert np.all(g.status() == 0)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("which", ["fe_tet", "kg_glassy"])
def test_paper_sized_batches_sampled(which):
    from paper_1902_09171_amd import rcell
    if which == "fe_tet":
        cfg = configs.fe_tet_cells()
        cells, params = cfg["cells"], cfg["params"]
        F = np.stack([configs.uniaxial_isochoric(0.01 * (1 + c % 3)) for c in range(len(cells))])
    else:
        cfg = configs.kg_glassy()
        cells, params, F = cfg["cells"], cfg["params"], cfg["F"]
    print(f"{which}: {len(cells)} cells, {sum(len(c['x']) for c in cells)} beads", flush=True)
    g = rcell.RCellBatch(params, cells)
    g.set_deformation(F)
    g.set_lanes(0)
    check_sample(g, params, cells, F, [0, len(cells) // 2, len(cells) - 1], which)
