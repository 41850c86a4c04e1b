"""Pins for the oracle's time integration: velocity Verlet (energy conservation, time
reversibility, momentum), the Langevin thermostat (equipartition, exact zero-mean noise, the
Ornstein-Uhlenbeck closed forms for free particles) and the stress window with rotation."""
import numpy as np
import pytest

from conftest import unvoigt
from oracle import core
from synth import configs


@pytest.fixture(scope="module")
def relaxed_kg():
    c1 = configs.kg_single()
    ob = core.OracleBatch(c1["params"], c1["cells"])
    ob.run(3000)                     # the synthetic start relaxes to T = 1 within ~2000 steps
    st = ob.get_state(0)
    return c1["params"], dict(x=st["x"], v=st["v"], bonds=c1["cells"][0]["bonds"], H0=st["H"])


def _nve_energy(p, cell, dt, t_total=10.0, samples=200):
    ob = core.OracleBatch(dict(p, gamma=0.0, dt=dt), [cell])
    every = int(round(t_total / dt / samples))
    E = []
    for _ in range(samples):
        ob.run(every)
        pe, ke = ob.get_energy()
        E.append(float(pe[0] + ke[0]) / len(cell["x"]))
    return np.array(E)


def test_nve_energy_drift_and_second_order(relaxed_kg):
    p, cell = relaxed_kg
    E = _nve_energy(p, cell, 0.005)
    slope = np.polyfit(np.arange(len(E)), E, 1)[0]       # per 10 steps
    assert abs(slope * 100) < 1e-4                         # drift per atom per 1000 steps
    # velocity Verlet is second order: the shadow-energy fluctuation scales as dt^2
    E2 = _nve_energy(p, cell, 0.0025)
    ratio = E.std() / E2.std()
    assert 3.0 < ratio < 5.5, ratio


def test_time_reversibility_and_momentum(relaxed_kg):
    p, cell = relaxed_kg
    pn = dict(p, gamma=0.0)
    ob = core.OracleBatch(pn, [cell])
    st0 = ob.get_state(0)
    p0 = st0["v"].sum(0)
    ob.run(100)
    st = ob.get_state(0)
    assert np.abs(st["v"].sum(0) - p0).max() < 1e-11
    # negate velocities, keep the forces of the last step, run back
    f = ob.get_forces(0)
    ob2 = core.OracleBatch(pn, [dict(cell, x=st["x"], v=-st["v"], H0=st["H"])])
    assert np.abs(ob2.get_forces(0) - f).max() < 1e-9 * np.abs(f).max()
    ob2.run(100)
    back = ob2.get_state(0)
    d = back["x"] - st0["x"]
    S = np.linalg.solve(st0["H"], d.T).T
    d = (S - np.rint(S)) @ st0["H"].T
    assert np.abs(d).max() < 1e-9
    assert np.abs(back["v"] + st0["v"]).max() < 1e-9


def test_langevin_equipartition_and_zero_momentum(relaxed_kg):
    p, cell = relaxed_kg
    ob = core.OracleBatch(p, [cell])
    n = len(cell["x"])
    T = []
    for _ in range(150):
        ob.run(20)
        T.append(2 * ob.get_energy()[1][0] / (3 * n - 3))
        st = ob.get_state(0)
        assert np.abs(st["v"].sum(0)).max() < 1e-9      # noise mean removed exactly per cell
    blocks = np.array(T).reshape(6, 25).mean(1)         # 500-step blocks
    se = blocks.std(ddof=1) / np.sqrt(len(blocks))
    assert abs(np.mean(T) - p["temperature"]) < max(3 * se, 0.015)


def test_free_particle_ornstein_uhlenbeck():
    # No interactions: velocity Verlet + Langevin is a discretised OU process with
    # <v^2> -> kB T / m and velocity autocorrelation exp(-gamma t).
    rng = np.random.default_rng(0)
    n, L = 3000, 60.0
    p = configs.kg_params(lj_eps=0.0, gamma=0.5, temperature=1.0, rc=1.0, skin=0.3)
    x = rng.uniform(0, L, (n, 3))
    ob = core.OracleBatch(p, [dict(x=x, v=np.zeros_like(x), bonds=np.zeros((0, 2), np.int32),
                                   H0=np.eye(3) * L)])
    ob.run(2000)                                     # t = 10 = 5 relaxation times
    ob.get_stress()
    ob.run(400)
    # ideal gas: the window-averaged stress is -rho kB T on the diagonal (tension positive)
    s = ob.get_stress()[0]
    assert np.allclose(s[:3], -n / L ** 3 * 1.0, rtol=0.05)
    assert np.abs(s[3:]).max() < 0.05 * n / L ** 3
    v0 = ob.get_state(0)["v"]
    v2 = (v0 ** 2).mean()
    assert v2 == pytest.approx(1.0, abs=0.05)
    k = 200                                          # t = 1
    ob.run(k)
    v1 = ob.get_state(0)["v"]
    c = (v0 * v1).mean() / v2
    assert c == pytest.approx(np.exp(-0.5 * k * p["dt"]), abs=0.03)


def test_kinetic_stress_in_metal_units():
    # a non-interacting copper cell (eps = 0) created without velocities: the velocities drawn from
    # the seed carry exactly (3N - 3) kB T of kinetic energy twice over (Sum m v.v), so the trace of
    # the instantaneous stress is -(3N - 3) kB T / V in eV / A^3, whatever the units of m v^2: a
    # kinetic tensor or a draw that drops the amu A^2 / fs^2 -> eV conversion is off by ~104x
    p = configs.cu_params(precision="fp64", sc_eps=0.0)
    cell = dict(configs.cu_cell(3, ncell=5), v=None)
    ob = core.OracleBatch(p, [cell])
    s = ob.get_stress()[0]
    n, V = len(cell["x"]), abs(np.linalg.det(np.asarray(cell["H0"], float)))
    assert s[:3].sum() == pytest.approx(-(3 * n - 3) * configs.KB_EV * p["temperature"] / V, rel=1e-12)


def test_noise_is_keyed_by_seed_cell_step():
    rng = np.random.default_rng(1)
    n, L = 50, 20.0
    p = configs.kg_params(lj_eps=0.0, gamma=1.0, temperature=1.0, rc=1.0, skin=0.3)
    x = rng.uniform(0, L, (n, 3))
    cell = dict(x=x, v=np.zeros_like(x), bonds=np.zeros((0, 2), np.int32), H0=np.eye(3) * L)
    a = core.OracleBatch(p, [cell, cell])
    a.run(3)
    va0, va1 = a.get_state(0)["v"], a.get_state(1)["v"]
    assert not np.array_equal(va0, va1)                     # different cell index, different noise
    b = core.OracleBatch(p, [cell])
    b.run(3)
    assert np.array_equal(b.get_state(0)["v"], va0)         # batch invariance of the noise
    c = core.OracleBatch(dict(p, seed=p["seed"] + 1), [cell])
    c.run(3)
    assert not np.array_equal(c.get_state(0)["v"], va0)
    d = core.OracleBatch(p, [cell])
    d.run(1)
    d.run(2)
    assert np.array_equal(d.get_state(0)["v"], va0)         # run(1) + run(2) == run(3)


def test_window_average_then_rotate(relaxed_kg):
    # sigma_FEM of the window average equals the average of per-step rotated stresses (linear, Q fixed)
    p, cell = relaxed_kg
    F = np.array([[1.05, 0.02, -0.01], [0.03, 0.97, 0.02], [-0.02, 0.01, 1.01]])
    ob = core.OracleBatch(p, [cell])
    ob.set_deformation(F[None])
    ob.get_stress()
    per_step = []
    for _ in range(5):
        ob.run(1)
        per_step.append(ob.get_stress()[0])
    ob2 = core.OracleBatch(p, [cell])
    ob2.set_deformation(F[None])
    ob2.get_stress()
    ob2.run(5)
    avg, P = ob2.get_stress(with_P=True)
    assert np.abs(avg[0] - np.mean(per_step, 0)).max() < 1e-12 * np.abs(avg).max()
    J = np.linalg.det(F)
    assert np.abs(P[0] @ F.T / J - unvoigt(avg[0])).max() < 1e-12 * np.abs(avg).max()


def test_a_deformation_empties_the_window(relaxed_kg):
    # the window holds the steps since the last get_stress or set_deformation: right after a
    # deformation it is empty and get_stress returns the instantaneous stress of the remapped state,
    # (W - sum m v v) / V with W from the pinned force routine, rotated by the Q of F (Eq. 7; Q from
    # numpy's QR with R_ii > 0), not an average over the steps run before the deformation
    p, cell = relaxed_kg
    ob = core.OracleBatch(p, [cell])
    ob.run(20)
    F = np.array([[1.04, 0.03, 0.00], [-0.02, 0.98, 0.01], [0.01, 0.02, 1.02]])
    ob.set_deformation(F[None])
    st = ob.get_state(0)
    _, _, W = core.forces(p, st["H"], st["x"], cell["bonds"])
    K = p["mass"] * p["mvv2e"] * st["v"].T @ st["v"]
    sig_md = (W - K) / abs(np.linalg.det(st["H"]))
    Q, R = np.linalg.qr(F)
    Q = Q * np.sign(np.diag(R))
    expected = Q @ sig_md @ Q.T
    got = unvoigt(ob.get_stress()[0])
    assert np.abs(got - expected).max() < 1e-10 * np.abs(expected).max()


def test_set_deformation_is_atomic_on_error():
    c1 = configs.kg_single()
    ob = core.OracleBatch(c1["params"], c1["cells"] * 2)
    st_before = ob.get_state(1)
    bad = np.stack([np.eye(3), np.diag([1.0, 1.0, -1.0])])
    with pytest.raises(core.OracleError) as e:
        ob.set_deformation(bad)
    assert e.value.code == core.ERR_BAD_F
    st_after = ob.get_state(0)
    assert np.array_equal(st_after["H"], st_before["H"])
    squash = np.stack([np.eye(3), np.diag([1.0, 1.0, 0.2])])    # 2.1 sigma box < 2 (rc + skin)
    with pytest.raises(core.OracleError) as e:
        ob.set_deformation(squash)
    assert e.value.code == core.ERR_BOX
    assert np.array_equal(ob.get_state(0)["x"], st_before["x"])


def test_maxwell_boltzmann_initial_velocities():
    """Cells created without velocities draw them from the seed: zero total momentum, kinetic energy
    exactly (3N - 3) kB T / 2, each component normally distributed with the variance that this
    kinetic energy leaves, components uncorrelated, reproducible for a seed and different for
    another seed or another cell."""
    from scipy import stats
    p = dict(configs.kg_params(precision="fp64"), temperature=1.7, mass=2.0)
    n_side = 28
    g = np.arange(n_side) + 0.5
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) * 1.1      # 21952 atoms
    H = np.eye(3) * 1.1 * n_side
    cell = dict(x=x, v=None, bonds=np.zeros((0, 2), np.int32), H0=H)
    small = dict(x=x[:500] * 0.5, v=None, bonds=np.zeros((0, 2), np.int32), H0=H * 0.5)
    ob = core.OracleBatch(p, [cell, small])
    v = ob.get_state(0)["v"]
    n = len(v)
    assert np.abs(v.sum(0)).max() <= 1e-11 * np.abs(v).sum()
    ke2 = p["mass"] * (v * v).sum()
    assert ke2 == pytest.approx((3 * n - 3) * p["kB"] * p["temperature"], rel=1e-13)
    sd = np.sqrt(p["kB"] * p["temperature"] / p["mass"] * (3 * n - 3) / (3 * n))
    for q in range(3):
        assert stats.kstest(v[:, q] / sd, "norm").pvalue > 1e-3
    c = np.corrcoef(v.T)
    assert np.abs(c[np.triu_indices(3, 1)]).max() < 4.0 / np.sqrt(n)
    vs = ob.get_state(1)["v"]
    assert np.abs(vs.sum(0)).max() <= 1e-11 * np.abs(vs).sum()
    assert not np.allclose(vs, v[:500])
    again = core.OracleBatch(p, [cell, small]).get_state(0)["v"]
    assert np.array_equal(again, v)
    other = core.OracleBatch(dict(p, seed=p["seed"] + 1), [cell, small]).get_state(0)["v"]
    assert np.abs(other - v).max() > 0.1 * sd
