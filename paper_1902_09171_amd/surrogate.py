"""Learned constitutive surrogate for the r-cells, with batched MD as its fallback (host
orchestration; every arithmetic step runs in the HIP library: QR of F and the stress return
through rcell, the network through rsur).

Features: the rotation-free stretch R of F = Q R (Eq. 4) at the current and the 16 previous load
steps, 9 floats each (153), so the network predicts the MD-frame stress sigma_MD from a
frame-indifferent history; sigma_FEM = Q sigma_MD Q^T and P = J sigma_FEM F^-T follow (Eqs. 7-8).
Before 17 load steps have passed the history is padded with R = I.  Targets: the window-averaged
MD stress of each load step (6 Voigt components).  The ensemble spread flags points outside the
training data (threshold: a high quantile of the spread on held-out data); those points take
their stress from MD r-cells that replay their deformation history.
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


def train(torch, net, X, Y, steps, batch=1024, lr=1e-3, seed=0, lr_final=None, log_every=0):
    """Adam on random minibatches (all members see the same batch); returns the loss history."""
    Xd = torch.tensor(X.astype(np.float32), device="cuda")
    Yd = torch.tensor(Y.astype(np.float32), device="cuda")
    net.fit_norm(Xd.data_ptr(), Yd.data_ptr(), len(X))
    rng = np.random.default_rng(seed)
    b = min(batch, len(X), net.max_batch)
    xb = torch.empty((b, X.shape[1]), dtype=torch.float32, device="cuda")
    yb = torch.empty((b, Y.shape[1]), dtype=torch.float32, device="cuda")
    losses = []
    for t in range(steps):
        idx = torch.tensor(rng.choice(len(X), b, replace=False), device="cuda")
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

    fallback_cells[g]: the initial r-cell of Gauss point g (used only if g is ever flagged)."""

    def __init__(self, torch, net, y_sd, tau, params, fallback_cells, md_steps):
        self.torch, self.net, self.y_sd, self.tau = torch, net, np.asarray(y_sd), tau
        self.params, self.cells, self.md_steps = params, fallback_cells, md_steps
        self.hist = History(len(fallback_cells))
        self.F_hist = []               # every load step's F, for catching up fallback cells
        self.live = []                 # Gauss points whose MD r-cell is kept in sync
        self.md = None
        self.flag_log = []

    def _catch_up(self, new):
        """MD cells for the newly flagged points replay their whole deformation history."""
        g = _rcell.RCellBatch(self.params, [self.cells[i] for i in new])
        for F in self.F_hist[:-1]:
            g.set_deformation(F[new])
            g.run(self.md_steps)
        states = [g.get_state(k) for k in range(len(new))]
        old = [] if self.md is None else [self.md.get_state(k) for k in range(len(self.live))]
        self.live = self.live + list(new)
        self.md = _rcell.RCellBatch(self.params, [self.cells[i] for i in self.live])
        for k, st in enumerate(old + states):
            self.md.set_state(k, st["x"], st["v"], st["H"], st["Rprev"], st["step"])

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
        if self.live:                   # MD points, kept in sync once flagged
            live = np.array(self.live)
            self.md.set_deformation(F[live])
            self.md.run(self.md_steps)
            s_live, P_live = self.md.get_stress(with_P=True)
            sigma[live], P[live] = s_live, P_live
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
