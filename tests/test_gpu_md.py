"""Parity of the HIP r-cell MD library (through its C ABI) with the FP64 oracle.

Tolerances (forces and stresses, cell-global metrics):
  mixed precision (FP32 pair forces, FP64 positions / integration / stress reduction):
      |f_gpu - f_ora|_2 / |f_ora|_2 <= 1e-5 over a cell; per atom max |df_i| / rms |f_ora| <= 1e-4;
      max |d sigma| / |sigma_ora|_F <= 1e-5
  FP64 mode: the same metrics at 1e-11.
Trajectories from an identical state with bit-identical noise: RMS |dx| after 1 step <= 1e-7,
after 100 steps <= 1e-4 (mixed); window-averaged stress over 100 steps within 1e-4 relative.
"""
import numpy as np
import pytest

from oracle import core
from synth import TABLE1_F, configs, fcc_lattice, kg_melt, maxwell_boltzmann

pytestmark = pytest.mark.gpu

TOL = {"mixed": dict(f=1e-5, fa=1e-4, s=1e-5, x1=1e-7, x100=1e-4, s100=1e-4),
       "fp64": dict(f=1e-11, fa=1e-10, s=1e-11, x1=1e-12, x100=1e-9, s100=1e-9)}


@pytest.fixture(scope="module")
def rc():
    from paper_1902_09171_amd import rcell
    rcell.load()
    return rcell


def fro(s6):
    s6 = np.asarray(s6)
    return np.sqrt((s6[..., :3] ** 2).sum(-1) + 2 * (s6[..., 3:] ** 2).sum(-1))


def check_forces(fg, fo, tol, what=""):
    err = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
    rms = np.sqrt((fo ** 2).sum(1).mean())
    err_a = np.abs(fg - fo).max() / rms
    print(f"{what} force rel {err:.3e} per-atom {err_a:.3e}", flush=True)
    assert err <= tol["f"], (what, err)
    assert err_a <= tol["fa"], (what, err_a)


def check_stress(sg, so, tol, key="s", what=""):
    err = np.abs(sg - so).max(-1) / fro(so)
    print(f"{what} stress rel {np.max(err):.3e}", flush=True)
    assert np.all(err <= tol[key]), (what, err)


def min_image(d, H):
    S = np.linalg.solve(H, d.T).T
    return (S - np.rint(S)) @ H.T


def kg_cells(sizes, seed0=100):
    out = []
    for k, lens in enumerate(sizes):
        out.append(configs.kg_cell(lens, seed0 + k))
    return out


def cu_cells(ncells, ncell=10, disp=0.1, seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(ncells):
        x, H = fcc_lattice(ncell)
        x = x + rng.normal(0, disp, x.shape)
        v = maxwell_boltzmann(len(x), 300.0, 63.546, configs.KB_EV, configs.MVV2E_METAL_FS, rng)
        out.append(dict(x=x, v=v, bonds=np.zeros((0, 2), np.int32), H0=H))
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_static_kg_forces_energy_stress(rc, prec):
    cells = kg_cells([[50] * 20, [37] * 21])
    p = configs.kg_params(precision=prec)
    g = rc.RCellBatch(p, cells)
    o = core.OracleBatch(p, cells)
    for k in range(2):
        check_forces(g.get_forces(k), o.get_forces(k), TOL[prec], f"kg cell {k}")
    peg, keg = g.get_energy()
    peo, keo = o.get_energy()
    assert np.allclose(peg, peo, rtol=TOL[prec]["f"])
    assert np.allclose(keg, keo, rtol=1e-13)
    check_stress(g.get_stress(), o.get_stress(), TOL[prec], what="kg")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_static_cu_forces_energy_stress(rc, prec):
    cells = cu_cells(2, ncell=6)
    p = configs.cu_params(precision=prec)
    g = rc.RCellBatch(p, cells)
    o = core.OracleBatch(p, cells)
    for k in range(2):
        check_forces(g.get_forces(k), o.get_forces(k), TOL[prec], f"cu cell {k}")
    peg, _ = g.get_energy()
    peo, _ = o.get_energy()
    assert np.allclose(peg, peo, rtol=TOL[prec]["f"])
    check_stress(g.get_stress(), o.get_stress(), TOL[prec], what="cu")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_deformation_qr_remap_parity(rc, prec):
    # Table 1's four deformation gradients plus a general one, one per cell
    rng = np.random.default_rng(3)
    Fs = list(TABLE1_F.values()) + [np.eye(3) + 0.08 * rng.standard_normal((3, 3))]
    cells = kg_cells([[50] * 20] * len(Fs))
    p = configs.kg_params(precision=prec)
    g = rc.RCellBatch(p, cells)
    o = core.OracleBatch(p, cells)
    for rep in range(2):                       # second call exercises Delta R = R R_prev^-1
        F = np.stack(Fs) if rep == 0 else np.stack([f @ (np.eye(3) + 0.02 * rng.standard_normal((3, 3))) for f in Fs])
        g.set_deformation(F)
        o.set_deformation(F)
        for k in range(len(Fs)):
            Hg, Qg, Rg, Jg = g.get_box(k)
            Ho, Qo, Ro, Jo = o.get_box(k)
            assert np.abs(Qg - Qo).max() < 1e-14 and np.abs(Rg - Ro).max() < 1e-14
            assert np.abs(Hg - Ho).max() < 1e-12 * np.abs(Ho).max() and abs(Jg - Jo) < 1e-14
            check_forces(g.get_forces(k), o.get_forces(k), TOL[prec], f"deformed cell {k}")
        sg, Pg = g.get_stress(with_P=True)
        so, Po = o.get_stress(with_P=True)
        check_stress(sg, so, TOL[prec], what="deformed")
        assert np.all(np.abs(Pg - Po).max((1, 2)) <= TOL[prec]["s"] * 3 * fro(so))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_glassy_kg_forces_stress_and_trajectory(rc, prec):
    # attractive LJ kept to 2.5 sigma (~60 listed neighbours per bead) at T = 0.1: static forces and
    # stress after a deformation, then the window stress and positions after 100 Langevin steps
    cells = [configs.kg_cell([50] * 20, 900 + k, T=0.1) for k in range(2)]
    p = configs.kg_glassy_params(precision=prec)
    g = rc.RCellBatch(p, cells)
    o = core.OracleBatch(p, cells)
    F = np.stack([configs.uniaxial_isochoric(0.02), np.eye(3)])
    g.set_deformation(F)
    o.set_deformation(F)
    for k in range(2):
        check_forces(g.get_forces(k), o.get_forces(k), TOL[prec], f"glassy cell {k}")
    check_stress(g.get_stress(), o.get_stress(), TOL[prec], what="glassy static")
    g.run(100)
    o.run(100)
    check_stress(g.get_stress(), o.get_stress(), TOL[prec], key="s100", what="glassy 100 steps")
    for k in range(2):
        d = min_image(g.get_state(k)["x"] - o.get_state(k)["x"], o.get_state(k)["H"])
        rms = np.sqrt((d ** 2).sum(1).mean())
        print(f"glassy cell {k} rms dx after 100 steps {rms:.2e}", flush=True)
        assert rms <= TOL[prec]["x100"]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_trajectory_kg_with_langevin(rc, prec):
    cells = kg_cells([[50] * 20])
    p = configs.kg_params(precision=prec)
    g = rc.RCellBatch(p, cells)
    o = core.OracleBatch(p, cells)
    F = configs.uniaxial_isochoric(0.05)[None]
    g.set_deformation(F)
    o.set_deformation(F)
    g.get_stress(); o.get_stress()
    g.run(1); o.run(1)
    sg, so = g.get_state(0), o.get_state(0)
    d = min_image(sg["x"] - so["x"], so["H"])
    rms1 = np.sqrt((d ** 2).sum(1).mean())
    print("rms after 1 step", rms1)
    assert rms1 <= TOL[prec]["x1"]
    g.run(99); o.run(99)
    sg, so = g.get_state(0), o.get_state(0)
    d = min_image(sg["x"] - so["x"], so["H"])
    rms = np.sqrt((d ** 2).sum(1).mean())
    print("rms after 100 steps", rms, "rebuilds", g.rebuilds())
    assert rms <= TOL[prec]["x100"]
    assert sg["step"] == so["step"] == 100
    check_stress(g.get_stress(), o.get_stress(), TOL[prec], key="s100", what="100-step window")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_langevin_noise_is_bit_identical(rc, prec):
    # no interactions: after one step from rest, v = h * xi exactly on both sides
    rng = np.random.default_rng(1)
    n, L = 300, 12.0
    p = configs.kg_params(precision=prec, lj_eps=0.0, gamma=0.7, temperature=1.3, rc=1.0, skin=0.3)
    x = rng.uniform(0, L, (n, 3))
    cells = [dict(x=x, v=np.zeros_like(x), bonds=np.zeros((0, 2), np.int32), H0=np.eye(3) * L)] * 3
    g = rc.RCellBatch(p, cells)
    o = core.OracleBatch(p, cells)
    g.run(1); o.run(1)
    for k in range(3):
        assert np.array_equal(g.get_state(k)["v"], o.get_state(k)["v"]), k


def test_batch_invariance_and_run_split_are_bitwise(rc):
    cells = kg_cells([[50] * 20, [40] * 10, [60] * 30])
    p = configs.kg_params(precision="mixed")
    big = rc.RCellBatch(p, cells)
    one = rc.RCellBatch(p, cells[:1])
    big.run(30)
    one.run(10); one.run(20)
    a, b = big.get_state(0), one.get_state(0)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["v"], b["v"])
    assert np.array_equal(big.get_stress()[0], one.get_stress()[0])
    # without noise the cell index does not matter: the last cell alone equals the batched one
    pn = dict(p, gamma=0.0)
    big = rc.RCellBatch(pn, cells)
    last = rc.RCellBatch(pn, cells[2:])
    big.run(25); last.run(25)
    assert np.array_equal(big.get_state(2)["x"], last.get_state(0)["x"])


def test_checkpoint_resume_is_bitwise(rc):
    cells = kg_cells([[50] * 20, [30] * 20])
    p = configs.kg_params(precision="mixed")
    a = rc.RCellBatch(p, cells)
    a.set_deformation(np.stack([configs.uniaxial_isochoric(0.03)] * 2))
    a.run(17)
    st = [a.get_state(k) for k in range(2)]
    a.run(13)
    b = rc.RCellBatch(p, cells)
    for k in range(2):
        b.set_state(k, st[k]["x"], st[k]["v"], st[k]["H"], st[k]["Rprev"], st[k]["step"])
    # forces after a restore are the conservative ones: restart both from the same restored state
    a2 = rc.RCellBatch(p, cells)
    for k in range(2):
        a2.set_state(k, st[k]["x"], st[k]["v"], st[k]["H"], st[k]["Rprev"], st[k]["step"])
    a2.run(13); b.run(5); b.run(8)
    for k in range(2):
        assert np.array_equal(a2.get_state(k)["x"], b.get_state(k)["x"])
        assert b.get_state(k)["step"] == st[k]["step"] + 13


def test_errors_leave_state_untouched(rc):
    cells = kg_cells([[50] * 20, [50] * 20])
    p = configs.kg_params(precision="mixed")
    g = rc.RCellBatch(p, cells)
    before = g.get_state(0)
    with pytest.raises(rc.RCellError) as e:
        g.set_deformation(np.stack([np.eye(3), np.diag([1.0, 1.0, -1.0])]))
    assert e.value.code == rc.ERR_BAD_F
    with pytest.raises(rc.RCellError) as e:
        g.set_deformation(np.stack([np.eye(3), np.diag([1.0, 1.0, 0.2])]))
    assert e.value.code == rc.ERR_BOX
    after = g.get_state(0)
    assert np.array_equal(before["x"], after["x"]) and np.array_equal(before["H"], after["H"])
    g.run(3)                                       # still usable
    assert np.all(g.status() == 0)
    with pytest.raises(rc.RCellError) as e:        # box too small at create
        rc.RCellBatch(p, [dict(x=np.zeros((1, 3)), v=None, bonds=np.zeros((0, 2), np.int32), H0=np.eye(3) * 2.5)])
    assert e.value.code == rc.ERR_BOX
    with pytest.raises(rc.RCellError) as e:        # initial FENE bond beyond R0
        rc.RCellBatch(p, [dict(x=np.array([[1.0, 1, 1], [2.6, 1, 1]]), v=None, bonds=np.array([[0, 1]], np.int32),
                               H0=np.eye(3) * 8.0)])
    assert e.value.code == rc.ERR_BOND


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_maxwell_boltzmann_velocities_match_the_oracle(rc, prec):
    # cells created without velocities draw Maxwell-Boltzmann velocities from the seed on the
    # device (zero total momentum, kinetic energy exactly (3N - 3) kB T / 2); the oracle draws them
    # from the same Philox stream with the host's libm, so they agree to rounding
    p = configs.kg_params(precision=prec)
    cells = [dict(configs.kg_cell(lens, 4300 + k), v=None) for k, lens in enumerate(([50] * 20, [30] * 10))]
    g = rc.RCellBatch(p, cells)
    o = core.OracleBatch(dict(p, precision="fp64"), cells)
    _, ke = g.get_energy()
    for k, c in enumerate(cells):
        vg, vo = g.get_state(k)["v"], o.get_state(k)["v"]
        print(prec, "cell", k, "max |dv|", np.abs(vg - vo).max(), flush=True)
        assert np.abs(vg - vo).max() <= 1e-12 * np.abs(vo).max()
        assert np.abs(vg.sum(0)).max() <= 1e-11 * np.abs(vg).sum()
        n = len(c["x"])
        assert ke[k] == pytest.approx(0.5 * (3 * n - 3) * p["kB"] * p["temperature"], rel=1e-12)
    g.get_stress()
    o.get_stress()
    g.run(50)
    o.run(50)
    check_stress(g.get_stress(), o.get_stress(), TOL[prec], key="s100", what=f"{prec} 50 steps from drawn velocities")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_one_and_two_atom_cells_from_the_seed(rc, prec):
    # the smallest cells the method admits, created without velocities beside a normal cell: a single
    # atom has no degree of freedom left once the momentum is fixed (zero velocity, and the per-cell
    # noise, whose mean is removed, is exactly zero), a bonded dimer has three
    p = configs.kg_params(precision=prec)
    box = np.eye(3) * 3.5
    one = dict(x=np.array([[0.3, 0.2, 0.1]]), v=None, bonds=np.zeros((0, 2), np.int32), H0=box)
    dimer = dict(x=np.array([[1.0, 1.0, 1.0], [1.97, 1.0, 1.0]]), v=None, bonds=np.array([[0, 1]], np.int32), H0=box)
    cells = [one, dimer, dict(configs.kg_cell([20] * 10, 4400), v=None)]
    g = rc.RCellBatch(p, cells)
    o = core.OracleBatch(dict(p, precision="fp64"), cells)
    _, ke = g.get_energy()
    assert ke[0] == 0.0 and np.all(g.get_state(0)["v"] == 0.0)
    assert ke[1] == pytest.approx(0.5 * 3 * p["kB"] * p["temperature"], rel=1e-12)
    for k in (1, 2):
        vg, vo = g.get_state(k)["v"], o.get_state(k)["v"]
        assert np.abs(vg - vo).max() <= 1e-12 * np.abs(vo).max()
        check_forces(g.get_forces(k), o.get_forces(k), TOL[prec], f"{prec} small cell {k}")
    g.get_stress(); o.get_stress()
    g.run(50); o.run(50)
    sg, so = g.get_stress(), o.get_stress()
    assert np.all(g.status() == 0)
    assert np.all(g.get_state(0)["v"] == 0.0) and np.all(sg[0] == 0.0) and np.all(so[0] == 0.0)
    check_stress(sg[1:], so[1:], TOL[prec], key="s100", what=f"{prec} dimer and 200 beads, 50 steps")


def test_injected_allocation_failures_leave_nothing_behind(rc, monkeypatch):
    # RCELL_FAULT_ALLOC=n makes the n-th device allocation of a context fail as if the device were
    # out of memory: create must report RCELL_ERR_OOM, free what it had allocated, and a create
    # without the fault must then work normally
    p = configs.kg_params(precision="mixed")
    cells = kg_cells([[20] * 10, [30] * 10], seed0=4200)
    for n in (1, 9, 33, 37):
        monkeypatch.setenv("RCELL_FAULT_ALLOC", str(n))
        with pytest.raises(rc.RCellError) as e:
            rc.RCellBatch(p, cells)
        assert e.value.code == -6 and "injected" in str(e.value), (n, str(e.value))
    monkeypatch.delenv("RCELL_FAULT_ALLOC")
    g = rc.RCellBatch(p, cells)
    g.run(20)
    assert np.all(g.status() == 0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ragged_cells_and_few_bins(rc, prec):
    # uneven cells, ragged last tiles (1000, 777, 130 atoms, 1 atom) and a box with < 3 bins per edge
    cells = kg_cells([[50] * 20, [37] * 21, [13] * 10])
    cells.append(dict(x=np.array([[0.3, 0.2, 0.1]]), v=np.array([[0.1, -0.2, 0.3]]), bonds=np.zeros((0, 2), np.int32),
                      H0=np.eye(3) * 3.5))
    p = configs.kg_params(precision=prec)
    g = rc.RCellBatch(p, cells)
    o = core.OracleBatch(p, cells)
    rng = np.random.default_rng(9)
    F = np.stack([np.eye(3) + 0.05 * rng.standard_normal((3, 3)) for _ in cells])
    g.set_deformation(F); o.set_deformation(F)
    for k in range(3):
        check_forces(g.get_forces(k), o.get_forces(k), TOL[prec], f"ragged {k}")
    g.get_stress(); o.get_stress()
    g.run(20); o.run(20)
    sg, so = g.get_stress(), o.get_stress()
    check_stress(sg[:3], so[:3], TOL[prec], key="s100", what="ragged 20 steps")
    assert np.allclose(sg[3], so[3], rtol=1e-9, atol=1e-12)


def test_full_cu_element_parity(rc):
    # the copper element workload: 8 cells x 4000 atoms, mixed precision, rotated uniaxial F.
    # The cells start as perfect lattices, where every net force vanishes by symmetry: there the
    # force check is absolute (1e-5 eV/A, against ~1 eV/A single-pair forces).
    cfg = configs.cu_element()
    p = cfg["params"]
    g = rc.RCellBatch(p, cfg["cells"])
    g.set_lanes(0)                       # the benchmark's launch configuration: autotuned lanes
    o = core.OracleBatch(p, cfg["cells"])
    F = cfg["F_path"][3]
    g.set_deformation(F); o.set_deformation(F)
    for k in range(8):
        assert np.abs(g.get_forces(k) - o.get_forces(k)).max() < 1e-5
    check_stress(g.get_stress(), o.get_stress(), TOL["mixed"], what="cu element static")
    g.run(10); o.run(10)
    check_stress(g.get_stress(), o.get_stress(), TOL["mixed"], key="s100", what="cu element 10 steps")
    for k in range(8):
        check_forces(g.get_forces(k), o.get_forces(k), TOL["mixed"], f"cu element cell {k} after 10 steps")


def test_neighbour_rebuilds_keep_parity(rc):
    # plain Verlet (gamma = 0): the stored force is the conservative one at the current positions,
    # evaluated with a list that has been rebuilt several times
    cells = kg_cells([[50] * 20])
    p = configs.kg_params(precision="mixed", gamma=0.0)
    g = rc.RCellBatch(p, cells)
    g.run(60)
    assert g.rebuilds() >= 2
    s = g.get_state(0)
    fo = core.forces(p, s["H"], s["x"], cells[0]["bonds"])[0]
    check_forces(g.get_forces(0), fo, TOL["mixed"], "after rebuilds")


def test_small_deformations_keep_the_list_exact(rc):
    # load steps of 0.4 % strain leave the neighbour list in place while the skin still covers the
    # affine change plus the thermal displacement; the forces after every load step and after the
    # MD between them must still equal an exact pair enumeration of the same state
    cfg = configs.cu_element()
    cells = cfg["cells"][:2]
    p = cfg["params"]
    g = rc.RCellBatch(p, cells)
    g.run(20)
    n0 = g.rebuilds()
    F = np.eye(3)
    nload = 6
    for k in range(nload):
        F = F @ np.diag([1.004, 0.998, 0.998])
        g.set_deformation(np.stack([F, F]))
        for c in range(2):
            s = g.get_state(c)
            fo = core.forces(p, s["H"], s["x"], cells[c]["bonds"])[0]
            check_forces(g.get_forces(c), fo, TOL["mixed"], f"load step {k} cell {c}")
        g.run(10)
    print("rebuilds over", nload, "load steps of 2 cells:", g.rebuilds() - n0, flush=True)
    assert g.rebuilds() - n0 < 2 * nload


def test_deformation_rebuilds_when_the_atoms_already_moved_past_the_new_threshold(rc):
    # A deformation keeps the list only while the skin still covers the affine change plus the
    # displacement the atoms already have since the last build.  Here a run ends with a largest
    # displacement above 0.17 sigma (below skin / 2 = 0.2), and a 5 % stretch lowers the kept-list
    # threshold to 0.163 sigma: the deformation must rebuild, and the forces of its prime pass must
    # equal an exact pair enumeration of the remapped state.
    p = configs.kg_params(precision="mixed")
    cell = configs.kg_cell([50] * 20, 4100)
    g = rc.RCellBatch(p, [cell])
    rcs = p["rc"] + p["skin"]
    xb = g.get_state(0)["x"]                   # create builds the list at the initial positions
    nreb = g.rebuilds()
    u = 0.0
    for _ in range(400):
        g.run(1)
        st = g.get_state(0)
        if g.rebuilds() != nreb:               # this step rebuilt: the reference is the new state
            nreb, xb = g.rebuilds(), st["x"]
            continue
        u = np.sqrt((min_image(st["x"] - xb, st["H"]) ** 2).sum(1)).max()
        if u > 0.17:
            break
    print("largest displacement since the last build", u, flush=True)
    assert 0.17 < u < 0.5 * p["skin"]
    F = np.diag([1.04, 0.98, 0.98])
    e = np.linalg.norm(F - np.eye(3))
    assert 0.5 * ((1.0 - e) * rcs - p["rc"]) < u
    g.set_deformation(F[None])
    assert g.rebuilds() == nreb + 1
    st = g.get_state(0)
    fo = core.forces(p, st["H"], st["x"], cell["bonds"])[0]
    check_forces(g.get_forces(0), fo, TOL["mixed"], "prime after the deformation")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_rebuild_preparation_paths_are_bitwise_equal(rc, prec):
    # one block per cell (the default for small cells) and the six phase kernels order the bins and
    # the atoms identically, so the lists, forces and trajectories are the same bit for bit
    cells = kg_cells([[50] * 20, [30] * 30, [40] * 40], seed0=400)
    p = configs.kg_params(precision=prec)
    F = np.stack([configs.uniaxial_isochoric(0.02 * (k + 1)) for k in range(3)])
    res = []
    for mode in (1, 2):
        g = rc.RCellBatch(p, cells)
        g.set_build_mode(mode)
        g.set_deformation(F)
        g.run(200)
        res.append((g.get_stress(), [g.get_state(k)["x"] for k in range(3)], g.rebuilds(), g.status()))
    (s1, x1, r1, st1), (s2, x2, r2, st2) = res
    print("rebuilds", r1, r2, flush=True)
    assert r1 > 0 and r1 == r2
    assert np.array_equal(s1, s2)
    assert all(np.array_equal(a, b) for a, b in zip(x1, x2))
    assert np.all(st1 == 0) and np.all(st2 == 0)
    with pytest.raises(rc.RCellError):
        rc.RCellBatch(p, kg_cells([[100] * 50], seed0=500)).set_build_mode(1)   # 5000 beads
    with pytest.raises(rc.RCellError):
        g.set_build_mode(3)


def test_one_lane_and_eight_lane_list_builds_agree(rc):
    # a rebuild covering at least 4096 tiles takes the one-lane-per-atom list build, a smaller one the
    # eight-lane build: the first build of 72 cells of 4100 beads at once (4680 tiles) and of the
    # same cells in batches of 8 (520 tiles) must give the same lists, hence the same forces and
    # stresses bit for bit (each atom sums its pairs in list order)
    cells = kg_cells([[100] * 41] * 72, seed0=800)
    p = configs.kg_params(precision="mixed", skin=0.7)
    big = rc.RCellBatch(p, cells)
    sig_big = big.get_stress()
    for b in range(0, 72, 8):
        small = rc.RCellBatch(p, cells[b:b + 8])
        assert np.array_equal(small.get_stress(), sig_big[b:b + 8]), b
        for k in range(8):
            assert np.array_equal(small.get_forces(k), big.get_forces(b + k)), (b, k)
    assert np.all(big.status() == 0)


@pytest.mark.parametrize("pot", ["kg", "cu"])
def test_graph_replay_equals_eager_launches(rc, pot):
    # replays of the captured MD-step graphs (with neighbour rebuilds inside) give bit-identical
    # states, stresses and rebuild counts to launching every kernel individually
    if pot == "kg":
        cells, p = kg_cells([[50] * 20, [40] * 10]), configs.kg_params()
    else:
        cells, p = cu_cells(2, ncell=6), configs.cu_params()
    a = rc.RCellBatch(p, cells)
    a.set_graph_steps(0)
    b = rc.RCellBatch(p, cells)
    b.set_graph_steps(4)
    for n in (1, 9, 23, 40):
        a.run(n)
        b.run(n)
        assert np.array_equal(a.get_stress(), b.get_stress()), n
    for k in range(len(cells)):
        sa, sb = a.get_state(k), b.get_state(k)
        assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["v"], sb["v"])
    assert a.rebuilds() == b.rebuilds()


def test_stateless_qr_and_stress_return_match_the_oracle(rc):
    import torch
    rng = np.random.default_rng(12)
    Fs = list(TABLE1_F.values()) + [np.eye(3) + 0.2 * rng.standard_normal((3, 3)) for _ in range(60)]
    Fs = [F for F in Fs if np.linalg.det(F) > 0.05] + [np.diag([1.0, 1.0, -1.0])]
    n = len(Fs)
    F = torch.tensor(np.stack(Fs).reshape(n, 9), dtype=torch.float64, device="cuda:0")
    Q = torch.zeros_like(F); R = torch.zeros_like(F)
    st = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    smd = torch.tensor(rng.standard_normal((n, 6)), dtype=torch.float64, device="cuda:0")
    sf = torch.zeros_like(smd); P = torch.zeros_like(F)
    rc.qr_dev(F.data_ptr(), n, Q.data_ptr(), R.data_ptr(), st.data_ptr())
    rc.stress_return_dev(F.data_ptr(), smd.data_ptr(), n, sf.data_ptr(), P.data_ptr())
    torch.cuda.synchronize()
    Qh, Rh, sth = Q.cpu().numpy().reshape(n, 3, 3), R.cpu().numpy().reshape(n, 3, 3), st.cpu().numpy()
    sfh, Ph, smh = sf.cpu().numpy(), P.cpu().numpy().reshape(n, 3, 3), smd.cpu().numpy()
    for k in range(n - 1):
        Qo, Ro = core.qr(Fs[k])
        assert sth[k] == 0 and np.abs(Qh[k] - Qo).max() < 1e-14 and np.abs(Rh[k] - Ro).max() < 1e-14
        so, Po = core.stress_to_fem(Fs[k], smh[k])
        assert np.abs(sfh[k] - so).max() < 1e-13 * np.abs(so).max() and np.abs(Ph[k] - Po).max() < 1e-12 * np.abs(Po).max()
    assert sth[-1] == rc.ERR_BAD_F and np.all(np.isnan(sfh[-1]))
