"""The surrogate's training pairs (history of the stretch R, window-averaged MD stress) produced by
batched MD on the GPU against the same pairs produced by the FP64 oracle, from the same cells,
deformation paths and Langevin noise: random stretch paths (generate_data) and FE bars stepped in
lockstep in one batch (generate_bars_data).  The features are rebuilt here from their definition:
the R of the current and the 16 previous load steps, newest first, 9 row-major floats each, R = I
before the first load step.  Bounds: FP64 mode 1e-9 relative for the stress (MD over a few hundred
steps diverges from the oracle's rounding by ~1e-12), 1e-13 for the features; mixed precision
1e-4 for the first load step's window (C26's 100-step trajectory bound)."""
import numpy as np
import pytest

from oracle import core
from synth import configs, stretch_paths
from synth.rng import generator

pytestmark = pytest.mark.gpu

MD_STEPS = 100
WARM = 100


def features(Rs):
    """Rs: (nload, n, 3, 3) stretches in load-step order -> (nload, n, 153)."""
    nload, n = Rs.shape[:2]
    out = np.zeros((nload, n, 17, 9))
    for k in range(nload):
        for j in range(17):
            out[k, :, j] = (Rs[k - j] if k - j >= 0 else np.broadcast_to(np.eye(3), (n, 3, 3))).reshape(n, 9)
    return out.reshape(nload, n, 153)


def fro(s):
    return np.sqrt((s[:, :3] ** 2).sum(1) + 2 * (s[:, 3:] ** 2).sum(1))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_random_path_pairs_match_the_oracle(prec):
    import torch
    from paper_1902_09171_amd import surrogate as SU
    params = configs.kg_params(precision=prec)
    cells = [configs.kg_cell([50] * 20, 5100 + k) for k in range(3)]
    nload = 3 if prec == "fp64" else 1
    paths = stretch_paths(3, nload, generator(5200, 0), rate_max=0.02, nu=(-0.5, 0.5))
    X, Y = SU.generate_data(torch, params, cells, paths, MD_STEPS, warmup_steps=WARM)
    o = core.OracleBatch(dict(params, precision="fp64"), cells)
    o.run(WARM)
    Yo = []
    for k in range(nload):
        o.set_deformation(paths[:, k])
        o.run(MD_STEPS)
        Yo.append(o.get_stress())         # F = R: Q = I, the FE-frame stress is the MD-frame stress
    # generate_data orders its rows by cell, then load step
    Yo = np.stack(Yo, 1).reshape(-1, 6)
    assert np.array_equal(X, features(paths.transpose(1, 0, 2, 3)).transpose(1, 0, 2).reshape(-1, 153))
    err = np.abs(Y - Yo).max(1) / fro(Yo)
    print(prec, "stress rel per pair", err, flush=True)
    assert err.max() <= (1e-9 if prec == "fp64" else 1e-4)


def test_bar_pairs_match_the_oracle():
    """Two small bars in lockstep, their r-cells in one batch; the same bars driven by oracle cells."""
    import torch
    from paper_1902_09171_amd import fe, surrogate as SU
    params = configs.kg_params(precision="fp64")
    meshes = [fe.Hex8Bar(nel=(1, 1, 1), size=(20.0, 20.0, 20.0), rho0=0.85),
              fe.Hex8Bar(nel=(1, 1, 1), size=(20.0, 20.0, 20.0), rho0=0.85, imperfection=1.0)]
    cells = [[configs.kg_cell([50] * 20, 5300 + 8 * b + g) for g in range(8)] for b in range(2)]
    rates = [0.02, 0.01]
    nload = 3
    X, Y, bars = SU.generate_bars_data(torch, params, meshes, cells, nload, MD_STEPS, rates, warmup_steps=WARM)
    # the same lockstep loop with the oracle's cells as the stress provider
    o = core.OracleBatch(params, [c for cs in cells for c in cs])
    o.run(WARM)
    dt = MD_STEPS * params["dt"]
    obars = [fe.ExplicitBar(m, None, dt=dt, pull_velocity=r * m.size[0] / dt, damping=0.2)
             for m, r in zip(meshes, rates)]
    Rs, Yo = [], []
    for k in range(nload):
        F = np.concatenate([b.begin_step() for b in obars])
        o.set_deformation(F)
        o.run(MD_STEPS)
        s, P = o.get_stress(with_P=True)
        for b, bar in enumerate(obars):
            bar.finish_step(F[8 * b:8 * b + 8], P[8 * b:8 * b + 8], s[8 * b:8 * b + 8])
        QR = [core.qr(f) for f in F]
        Rs.append(np.stack([r for _, r in QR]))
        # back to the MD frame: sigma_MD = Q^T sigma_FEM Q
        for i, (Q, _) in enumerate(QR):
            S = np.array([[s[i, 0], s[i, 3], s[i, 4]], [s[i, 3], s[i, 1], s[i, 5]], [s[i, 4], s[i, 5], s[i, 2]]])
            M = Q.T @ S @ Q
            s[i] = [M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]]
        Yo.append(s)
    Yo = np.concatenate(Yo)
    xerr = np.abs(X - features(np.stack(Rs)).reshape(-1, 153)).max()   # rows by load step, then point
    err = np.abs(Y - Yo).max(1) / fro(Yo)
    print("features", xerr, "stress rel", err.max(), flush=True)
    assert xerr <= 1e-13
    assert err.max() <= 1e-9
    assert np.abs(bars[0].u - obars[0].u).max() <= 1e-9 * np.abs(obars[0].u).max()
