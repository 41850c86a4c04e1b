"""Independent numpy O(N^2) twin of the oracle's static force evaluation, for tiny cells.

Test infrastructure only.  Written separately from rcell_oracle.c: every pair (i, j) and every
periodic image n in a box of integers wide enough to reach the cutoff is scanned with array
operations; no cell list, no pair list.  Used to check the C oracle's pair set, forces, energy
and virial (Eq. 15 without the 1/Omega_0 factor) on cells of a few hundred atoms.
"""
import itertools

import numpy as np


def _images(H, rc):
    Hi = np.linalg.inv(H)
    w = 1.0 / np.linalg.norm(Hi, axis=1)          # perpendicular widths: 1 / |row k of H^-1|
    m = [int(np.ceil(rc / wk)) + 1 for wk in w]
    return np.array(list(itertools.product(*[range(-mk, mk + 1) for mk in m])), dtype=np.float64)


def pair_table(H, x, rc):
    """All (i, j, d) with |x_j + H n - x_i| < rc, i < j any n, or i == j with n in one half-space."""
    H = np.asarray(H, float)
    x = np.asarray(x, float)
    Hi = np.linalg.inv(H)
    S = x @ Hi.T
    out_i, out_j, out_d = [], [], []
    imgs = _images(H, rc)
    n = len(x)
    for i in range(n):
        j = np.arange(i, n)
        base = np.rint(S[j] - S[i])               # centre the image scan on the nearest image
        for im in imgs:
            nn = im[None, :] - base
            d = (x[j] - x[i]) + nn @ H.T
            r2 = (d * d).sum(1)
            keep = r2 < rc * rc
            self_ = j == i
            if self_.any():
                k = nn[self_][0]
                pos = (k[0] > 0) or (k[0] == 0 and (k[1] > 0 or (k[1] == 0 and k[2] > 0)))
                keep &= ~self_ | pos
            if keep.any():
                out_i.append(np.full(keep.sum(), i))
                out_j.append(j[keep])
                out_d.append(d[keep])
    if not out_i:
        return np.zeros(0, int), np.zeros(0, int), np.zeros((0, 3))
    return np.concatenate(out_i), np.concatenate(out_j), np.concatenate(out_d)


def forces(params, H, x, bonds=None):
    """Return (f [N,3], PE, W [3,3]) with W = sum over interactions of (dU/dr) d (x) d / r."""
    x = np.asarray(x, float)
    H = np.asarray(H, float)
    n = len(x)
    rc = params["rc"]
    i, j, d = pair_table(H, x, rc)
    r = np.linalg.norm(d, axis=1)
    f = np.zeros((n, 3))
    W = np.zeros((3, 3))
    pe = 0.0
    pot = params["potential"]
    if pot in ("kg", 1):
        e, s = params["lj_eps"], params["lj_sigma"]
        u = lambda rr: 4 * e * ((s / rr) ** 12 - (s / rr) ** 6)
        pe += float((u(r) - u(rc)).sum())
        g = 4 * e * (-12 * s ** 12 / r ** 13 + 6 * s ** 6 / r ** 7)
        if bonds is not None and len(bonds):
            b = np.asarray(bonds)
            Hi = np.linalg.inv(H)
            db = x[b[:, 1]] - x[b[:, 0]]
            db -= np.rint(db @ Hi.T) @ H.T
            rb = np.linalg.norm(db, axis=1)
            K, R0 = params["fene_K"], params["fene_R0"]
            pe += float((-0.5 * K * R0 ** 2 * np.log(1 - (rb / R0) ** 2)).sum())
            gb = K * rb / (1 - (rb / R0) ** 2)
            i = np.concatenate([i, b[:, 0]])
            j = np.concatenate([j, b[:, 1]])
            d = np.concatenate([d, db])
            r = np.concatenate([r, rb])
            g = np.concatenate([g, gb])
    elif pot in ("sc_eam", 2):
        e, a, c, nn, m = (params[k] for k in ("sc_eps", "sc_a", "sc_c", "sc_n", "sc_m"))
        rho_pair = (a / r) ** m - (a / rc) ** m
        rho = np.bincount(i, rho_pair, n) + np.bincount(j, rho_pair, n)
        pe += float((e * ((a / r) ** nn - (a / rc) ** nn)).sum() - (e * c * np.sqrt(rho)).sum())
        Fp = np.where(rho > 0, -e * c / (2 * np.sqrt(np.where(rho > 0, rho, 1.0))), 0.0)
        g = e * (-nn / r) * (a / r) ** nn + (Fp[i] + Fp[j]) * (-m / r) * (a / r) ** m
    else:
        raise ValueError(pot)
    fv = (g / r)[:, None] * d
    np.add.at(f, i, fv)
    np.add.at(f, j, -fv)
    W = np.einsum("k,ka,kb->ab", g / r, d, d)
    return f, pe, W
