"""Learned constitutive surrogate for the r-cells, with batched MD as its fallback (host
orchestration; every arithmetic step runs in the HIP library: QR of F and the stress return
through rcell, the network through rsur).

Features: the rotation-free stretch R of F = Q R (Eq. 4) at the current and the 16 previous load
steps, 9 floats each (153), so the network predicts the MD-frame stress sigma_MD from a
frame-indifferent history; sigma_FEM = Q sigma_MD Q^T and P = J sigma_FEM F^-T follow (Eqs. 7-8).
Before 17 load steps have passed the history is padded with R = I.  Targets: the window-averaged
MD stress of each load step (6 Voigt components).  The ensemble spread flags points outside the
training data (threshold: the largest spread met on held-out bars); those points take their
stress from MD r-cells that replay their deformation history.
"""
import numpy as np

from . import rcell as _rcell
from . import rsur as _rsur

HISTORY = 17
FEATURES = 9 * HISTORY


class History:
    """The last HISTORY stretches R of n points, newest first (host-side arrangement only)."""

    def __init__(self, n):
        self.R = np.tile(np.eye(3).reshape(1, 1, 9), (n, HISTORY, 1))

    def push(self, R):
        self.R = np.concatenate([np.asarray(R).reshape(-1, 1, 9), self.R[:, :-1]], axis=1)

    def features(self):
        return np.ascontiguousarray(self.R.reshape(len(self.R), FEATURES))


def qr_batch(torch, F):
    """Q, R of every F (n, 3, 3) computed on the GPU (Eq. 4)."""
    n = len(F)
    Fd = torch.tensor(np.ascontiguousarray(F).reshape(n, 9), dtype=torch.float64, device="cuda")
    Qd, Rd = torch.zeros_like(Fd), torch.zeros_like(Fd)
    _rcell.qr_dev(Fd.data_ptr(), n, Qd.data_ptr(), Rd.data_ptr())
    torch.cuda.synchronize()
    return Qd.cpu().numpy().reshape(n, 3, 3), Rd.cpu().numpy().reshape(n, 3, 3)


def generate_data(torch, params, cells, paths, md_steps, warmup_steps=0):
    """Batched MD under prescribed rotation-free paths: paths (ncells, nload, 3, 3) upper-triangular
    stretches applied one per load step.  Returns X (ncells * nload, 153) and Y (same, 6) with the
    MD-frame stress of each load step (F = R, so Q = I and sigma_FEM = sigma_MD)."""
    g = _rcell.RCellBatch(params, cells)
    if warmup_steps:
        g.run(warmup_steps)
    ncells, nload = paths.shape[:2]
    hist = History(ncells)
    X, Y = [], []
    for k in range(nload):
        g.set_deformation(paths[:, k])
        g.run(md_steps)
        s = g.get_stress()
        hist.push(paths[:, k])
        X.append(hist.features())
        Y.append(s)
    X = np.stack(X, 1).reshape(-1, FEATURES)
    Y = np.stack(Y, 1).reshape(-1, 6)
    return X, Y


def generate_bars_data(torch, params, meshes, cells, nload, md_steps, pull_strains, warmup_steps=0,
                       damping=0.2, stream=None, progress=None, wave_speed=None):
    """(history, sigma_MD) pairs at every Gauss point of several MD-driven FE bars stepped in
    lockstep, the r-cells of all bars in one batched MD context (one set_deformation, run and stress
    read per load step for every bar).  meshes[b], cells[b] (one r-cell per Gauss point) and
    pull_strains[b] (nominal strain per load step) describe bar b.  Returns X (nload * sum ngp, 153)
    and Y (same, 6, the MD-frame window stress), rows ordered by load step, bar, Gauss point, and the
    bars, each checked against the CFL limit when wave_speed is given."""
    from . import fe
    allcells = [c for cs in cells for c in cs]
    g = _rcell.RCellBatch(params, allcells, stream=stream)
    if warmup_steps:
        g.run(warmup_steps)
    dt = md_steps * params["dt"]
    bars = [fe.ExplicitBar(m, None, dt=dt, pull_velocity=r * m.size[0] / dt, damping=damping,
                           wave_speed=wave_speed) for m, r in zip(meshes, pull_strains)]
    off = np.cumsum([0] + [m.ngp for m in meshes])
    hist = History(len(allcells))
    X, Y = [], []
    for k in range(nload):
        F = np.concatenate([b.begin_step() for b in bars])
        g.set_deformation(F)
        g.run(md_steps)
        sig, P, smd = g.get_stress_ext()
        for b, bar in enumerate(bars):
            sl = slice(off[b], off[b + 1])
            bar.finish_step(F[sl], P[sl], sig[sl])
        _, R = qr_batch(torch, F)
        hist.push(R)
        X.append(hist.features())
        Y.append(smd)
        if progress:
            progress(k)
    g.close()
    return np.concatenate(X), np.concatenate(Y), bars


def train(torch, net, X, Y, steps, batch=1024, lr=1e-3, seed=0, lr_final=None, log_every=0):
    """Adam on minibatches drawn without replacement from a fresh device permutation every epoch
    (all members see the same batch); returns the loss history."""
    Xd = torch.tensor(np.asarray(X, np.float32), device="cuda")
    Yd = torch.tensor(np.asarray(Y, np.float32), device="cuda")
    net.fit_norm(Xd.data_ptr(), Yd.data_ptr(), len(X))
    gen = torch.Generator(device="cuda").manual_seed(int(seed))
    b = min(batch, len(X), net.max_batch)
    xb = torch.empty((b, X.shape[1]), dtype=torch.float32, device="cuda")
    yb = torch.empty((b, Y.shape[1]), dtype=torch.float32, device="cuda")
    per_epoch = len(X) // b
    perm = None
    losses = []
    for t in range(steps):
        if t % per_epoch == 0:
            perm = torch.randperm(len(X), generator=gen, device="cuda")
        idx = perm[(t % per_epoch) * b:(t % per_epoch + 1) * b]
        torch.index_select(Xd, 0, idx, out=xb)
        torch.index_select(Yd, 0, idx, out=yb)
        torch.cuda.synchronize()
        rate = lr if lr_final is None else lr * (lr_final / lr) ** (t / max(steps - 1, 1))
        want = log_every and (t % log_every == 0 or t == steps - 1)
        loss = net.train_step(xb.data_ptr(), yb.data_ptr(), b, rate, want_loss=bool(want))
        if want:
            losses.append((t, float(np.mean(loss))))
    torch.cuda.synchronize()
    return losses


def predict(torch, net, X):
    """Ensemble mean and variance (host arrays) for raw features X, in chunks of max_batch."""
    mean, var = [], []
    for lo in range(0, len(X), net.max_batch):
        xs = X[lo:lo + net.max_batch]
        Xd = torch.tensor(xs.astype(np.float32), device="cuda")
        m = torch.zeros((len(xs), net.dout), dtype=torch.float32, device="cuda")
        v = torch.zeros_like(m)
        net.forward(Xd.data_ptr(), len(xs), m.data_ptr(), v.data_ptr())
        torch.cuda.synchronize()
        mean.append(m.cpu().numpy())
        var.append(v.cpu().numpy())
    return np.concatenate(mean).astype(np.float64), np.concatenate(var).astype(np.float64)


def spread(var, y_sd):
    """Per-row out-of-distribution score: the largest ensemble standard deviation over the stress
    components, in units of each component's training standard deviation."""
    return (np.sqrt(np.maximum(var, 0.0)) / y_sd[None, :]).max(1)


class SurrogateStress:
    """FE stress provider: ensemble mean for in-distribution points, MD r-cells otherwise.

    fallback_cells[g]: the initial r-cell of Gauss point g (used only if g is ever flagged), warmed
    by warmup_steps MD steps before it replays the point's deformation history, as the MD cells the
    network was trained on were.  Each group of points flagged at the same load step keeps its own
    r-cell batch from then on, so an MD cell's trajectory is never interrupted."""

    def __init__(self, torch, net, y_sd, tau, params, fallback_cells, md_steps, warmup_steps=0):
        self.torch, self.net, self.y_sd, self.tau = torch, net, np.asarray(y_sd), tau
        self.params, self.cells, self.md_steps = params, fallback_cells, md_steps
        self.warmup_steps = warmup_steps
        self.hist = History(len(fallback_cells))
        self.F_hist = []               # every load step's F, for catching up fallback cells
        self.live = []                 # Gauss points whose MD r-cell is kept in sync
        self.groups = []               # (points, r-cell batch) per load step that flagged new points
        self.flag_log = []

    def _catch_up(self, new):
        """MD cells for the newly flagged points replay their whole deformation history."""
        g = _rcell.RCellBatch(self.params, [self.cells[i] for i in new])
        if self.warmup_steps:
            g.run(self.warmup_steps)
        for F in self.F_hist[:-1]:
            g.set_deformation(F[new])
            g.run(self.md_steps)
        self.live = self.live + list(new)
        self.groups.append((np.array(new), g))

    def __call__(self, F):
        torch = self.torch
        n = len(F)
        F = np.asarray(F)
        self.F_hist.append(F.copy())
        _, R = qr_batch(torch, F)
        self.hist.push(R)
        mean, var = predict(torch, self.net, self.hist.features())
        flagged = np.where(spread(var, self.y_sd) > self.tau)[0]
        self.flag_log.append(len(flagged))
        new = [int(i) for i in flagged if int(i) not in self.live]
        if new:
            self._catch_up(new)
        # network points: sigma_MD -> sigma_FEM, P through the library's stress return (Eqs. 7-8)
        Fd = torch.tensor(np.ascontiguousarray(F).reshape(n, 9), dtype=torch.float64, device="cuda")
        sd = torch.tensor(np.ascontiguousarray(mean), dtype=torch.float64, device="cuda")
        sf = torch.zeros((n, 6), dtype=torch.float64, device="cuda")
        Pd = torch.zeros((n, 9), dtype=torch.float64, device="cuda")
        _rcell.stress_return_dev(Fd.data_ptr(), sd.data_ptr(), n, sf.data_ptr(), Pd.data_ptr())
        torch.cuda.synchronize()
        sigma, P = sf.cpu().numpy(), Pd.cpu().numpy().reshape(n, 3, 3)
        for pts, g in self.groups:      # MD points, kept in sync once flagged
            g.set_deformation(F[pts])
            g.run(self.md_steps)
            s_md, P_md = g.get_stress(with_P=True)
            sigma[pts], P[pts] = s_md, P_md
        return P, sigma


def generate_bar_data(torch, params, mesh, cells, nload, md_steps, pull_strain_per_step, warmup_steps=0,
                      damping=0.2):
    """(history, sigma_MD) pairs recorded at every Gauss point of an MD-driven FE bar: the
    deformation paths the surrogate will meet when it drives the same kind of bar."""
    from . import fe
    md = fe.MDStress(params, cells, md_steps)
    if warmup_steps:
        md.g.run(warmup_steps)
    dt = md_steps * params["dt"]
    bar = fe.ExplicitBar(mesh, md, dt=dt, pull_velocity=pull_strain_per_step * mesh.size[0] / dt, damping=damping)
    hist = History(mesh.ngp)
    X, Y = [], []
    for _ in range(nload):
        F, _, _ = bar.step()
        _, R = qr_batch(torch, F)
        hist.push(R)
        X.append(hist.features())
        Y.append(md.last_md.copy())
    return np.concatenate(X), np.concatenate(Y), bar


def fro6(s6):
    """Frobenius norm of symmetric tensors in Voigt order (xx, yy, zz, xy, xz, yz), per row."""
    s6 = np.asarray(s6)
    return np.sqrt((s6[..., :3] ** 2).sum(-1) + 2.0 * (s6[..., 3:] ** 2).sum(-1))


def deviatoric6(s6):
    """The deviatoric part of Voigt rows (the mean of the diagonal removed)."""
    s6 = np.array(s6, dtype=np.float64)
    s6[..., :3] -= s6[..., :3].mean(-1, keepdims=True)
    return s6


def floored_error(s, ref, floor):
    """|s - ref|_F / max(|ref|_F, floor) per row: the relative error, with a stress-magnitude floor
    below which a window-averaged r-cell stress is dominated by its own fluctuations."""
    return fro6(np.asarray(s) - ref) / np.maximum(fro6(ref), floor)


def train_on_bars(torch, net, params, meshes, cells, nload, md_steps, pull_strains, warmup_steps, train_steps,
                  holdout, batch=4096, lr=2e-3, lr_final=1e-4, seed=0, progress=None, wave_speed=None):
    """Training data from MD-driven bars (generate_bars_data), the ensemble trained on all bars but the
    last `holdout`, and on those: the OOD threshold (the largest ensemble spread met) and the error
    against their own MD.  Returns a dict with X, Y, losses, y_sd, tau, err_ho, timings."""
    import time
    t0 = time.perf_counter()
    X, Y, _ = generate_bars_data(torch, params, meshes, cells, nload, md_steps, pull_strains,
                                 warmup_steps=warmup_steps, progress=progress, wave_speed=wave_speed)
    t_gen = time.perf_counter() - t0
    nbar = np.concatenate([np.full(m.ngp, b) for b, m in enumerate(meshes)])
    held = np.tile(nbar, nload) >= len(meshes) - holdout
    t0 = time.perf_counter()
    losses = train(torch, net, X[~held], Y[~held], steps=train_steps, batch=batch, lr=lr, lr_final=lr_final,
                   seed=seed, log_every=max(1, train_steps // 20))
    t_train = time.perf_counter() - t0
    y_sd = Y[~held].std(0)
    mho, vho = predict(torch, net, X[held])
    sp = spread(vho, y_sd)
    return dict(X=X, Y=Y, held=held, losses=losses, y_sd=y_sd, tau=float(sp.max()), spread_ho=sp,
                err_ho=fro6(mho - Y[held]) / fro6(Y[held]), t_gen=t_gen, t_train=t_train)


def shadow_evaluation(torch, provider, params, mesh, cells, md_steps, nload, pull_strain, warmup_steps, floor,
                      damping=0.2, wave_speed=None, progress=None):
    """Drive the bar with `provider` while two shadow MD batches of the same r-cells (the given
    Langevin seed and the next one, each warmed by warmup_steps) follow its deformation gradients.
    Per load step and Gauss point: the provider's floored error against shadow MD, the same measure
    between the two MD batches (the seed-to-seed spread), both also for the deviatoric parts, the MD
    stress magnitude, and the wall time of the provider and of one MD load step."""
    import time
    from . import fe
    shadow = []
    for sd in (params["seed"], params["seed"] + 1):
        sh = fe.MDStress(dict(params, seed=sd), cells, md_steps)
        if warmup_steps:
            sh.g.run(warmup_steps)
        shadow.append(sh)
    dt = md_steps * params["dt"]
    bar = fe.ExplicitBar(mesh, provider, dt=dt, pull_velocity=pull_strain * mesh.size[0] / dt, damping=damping,
                         wave_speed=wave_speed)
    out = {k: [] for k in ("rel", "floor", "dev", "dev_floor", "mags", "t_provider", "t_md")}
    for k in range(nload):
        F = bar.begin_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P, sig = provider(F)
        torch.cuda.synchronize()
        out["t_provider"].append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        _, sA = shadow[0](F)
        out["t_md"].append(time.perf_counter() - t0)
        _, sB = shadow[1](F)
        bar.finish_step(F, P, sig)
        out["rel"].append(floored_error(sig, sA, floor))
        out["floor"].append(floored_error(sB, sA, floor))
        out["dev"].append(floored_error(deviatoric6(sig), deviatoric6(sA), floor))
        out["dev_floor"].append(floored_error(deviatoric6(sB), deviatoric6(sA), floor))
        out["mags"].append(fro6(sA))
        if progress:
            progress(k, out)
    for sh in shadow:
        sh.g.close()
    res = {k: np.array(v) for k, v in out.items()}
    res["bar"] = bar
    return res
