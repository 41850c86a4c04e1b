"""The seeded input generators produce the shapes the workloads promise."""
import numpy as np

from synth import configs, fcc_lattice, kg_melt, maxwell_boltzmann, random_rotation


def test_kg_melt_shape_density_bonds():
    x, b, H = kg_melt([50] * 20, seed=1)
    L = H[0, 0]
    assert x.shape == (1000, 3) and b.shape == (980, 2)
    assert 1000 / L ** 3 == np.float64(0.85) or abs(1000 / L ** 3 - 0.85) < 1e-12
    assert x.min() >= 0 and x.max() < L
    d = x[b[:, 1]] - x[b[:, 0]]
    d -= L * np.rint(d / L)
    assert np.allclose(np.linalg.norm(d, axis=1), 0.97, atol=1e-3)
    # soft excluded volume plus geometric relaxation: no two beads closer than 0.8 sigma
    dd = x[:, None] - x[None]
    dd -= L * np.rint(dd / L)
    r = np.linalg.norm(dd, axis=-1)
    np.fill_diagonal(r, 9)
    assert r.min() > 0.8
    x2, _, _ = kg_melt([50] * 20, seed=1)
    assert np.array_equal(x, x2)


def test_fcc_and_velocities():
    x, H = fcc_lattice(10)
    assert x.shape == (4000, 3) and np.allclose(H, np.eye(3) * 36.15)
    v = maxwell_boltzmann(4000, 300.0, 63.546, configs.KB_EV, configs.MVV2E_METAL_FS,
                          np.random.default_rng(0))
    assert np.abs(v.sum(0)).max() < 1e-10
    ke = 0.5 * 63.546 * configs.MVV2E_METAL_FS * (v * v).sum()
    assert abs(ke - 0.5 * (3 * 4000 - 3) * configs.KB_EV * 300.0) < 1e-9 * ke


def test_rotations_and_batched_sizes():
    rng = np.random.default_rng(3)
    for _ in range(20):
        Q = random_rotation(rng)
        assert np.abs(Q.T @ Q - np.eye(3)).max() < 1e-14 and abs(np.linalg.det(Q) - 1) < 1e-14
    sizes = configs.kg_batched_sizes(512)
    tot = [sum(s) for s in sizes]
    assert min(tot) >= 2000 and max(tot) <= 20000 + 200
    assert all(50 <= l <= 200 for s in sizes for l in s)
    assert 5.0e6 < sum(tot) < 6.2e6
