"""Pins for the oracle's pair set, forces, energy and virial.

Independent checks: the numpy O(N^2) twin (oracle/brute.py), central finite differences of the
energy (forces = -dE/dx; virial = (dE/dF) F^T, the derivative form of Eq. 15), closed forms of
the LJ/FENE dimer, FCC lattice sums enumerated from integer coordinates, frame indifference
of the QR route (Sec. 2.1: stress of R H0 rotated by Q equals stress of F H0), and the cubic
symmetry of Table 1's deformations."""
import itertools

import numpy as np
import pytest

from conftest import unvoigt
from oracle import brute, core
from synth import TABLE1_F, fcc_lattice, kg_melt
from synth.configs import cu_params, kg_params

KG = kg_params(gamma=0.0, temperature=0.0, include_kinetic=0)
CU = cu_params(gamma=0.0, temperature=0.0, include_kinetic=0)


def _pairset(ij, d):
    return sorted((int(a), int(b), *np.round(v, 9)) for (a, b), v in zip(ij, d))


@pytest.mark.parametrize("box", ["cubic", "skewed", "skewed_bins", "tiny"])
def test_pair_set_matches_brute_force(box):
    rng = np.random.default_rng(1)
    if box == "cubic":
        H = np.eye(3) * 6.0
    elif box == "skewed":
        H = np.array([[6.0, 2.5, -1.7], [0.0, 5.5, 2.2], [0.0, 0.0, 6.3]])
    elif box == "skewed_bins":
        # wide enough for the cell list; the tilt makes the perpendicular width along x (6.57) a
        # whole bin narrower than the edge (8): 3 bins of >= rc, where the edge would allow 4
        H = np.array([[8.0, 3.6, -2.5], [0.0, 7.5, 3.2], [0.0, 0.0, 8.0]])
    else:   # rc larger than half the box: several images of the same pair, self images
        H = np.array([[2.0, 0.6, 0.3], [0.0, 2.2, -0.5], [0.0, 0.0, 1.9]])
    n = {"tiny": 5, "skewed_bins": 300}.get(box, 60)
    x = rng.uniform(0, 1, (n, 3)) @ H.T
    rc = 1.9
    ij, d = core.pairs(H, x, rc)
    i2, j2, d2 = brute.pair_table(H, x, rc)
    assert len(ij) == len(i2)
    assert _pairset(ij, d) == _pairset(np.stack([i2, j2], 1), d2)


@pytest.mark.parametrize("pot", ["kg", "cu"])
def test_forces_energy_virial_match_brute_force(pot):
    rng = np.random.default_rng(2)
    if pot == "kg":
        x, b, H = kg_melt([10] * 12, seed=9)
        L = H[0, 0]
        H = np.array([[L, 0.7, -0.4], [0, L * 0.95, 0.3], [0, 0, L * 1.04]])
        x = (x / L) @ H.T
        p = KG
    else:
        x, H = fcc_lattice(3)
        x = x + rng.normal(0, 0.08, x.shape)
        b, p = None, CU
    f, pe, W = core.forces(p, H, x, b)
    f2, pe2, W2 = brute.forces(p, H, x, b)
    assert np.abs(f - f2).max() <= 1e-12 * np.abs(f2).max()
    assert pe == pytest.approx(pe2, rel=1e-13)
    assert np.abs(W - W2).max() <= 1e-12 * np.abs(W2).max()
    assert np.abs(f.sum(0)).max() <= 1e-12 * np.abs(f).sum()


@pytest.mark.parametrize("pot", ["kg", "cu"])
def test_forces_are_minus_energy_gradient(pot):
    rng = np.random.default_rng(4)
    if pot == "kg":
        x, b, H = kg_melt([8] * 10, seed=21)
        p = KG
    else:
        x, H = fcc_lattice(3)
        x = x + rng.normal(0, 0.1, x.shape)
        b, p = None, CU
    f, _, _ = core.forces(p, H, x, b)
    h = 1e-6
    for i in rng.choice(len(x), 8, replace=False):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (core.forces(p, H, xp, b)[1] - core.forces(p, H, xm, b)[1]) / (2 * h)
            assert -g == pytest.approx(f[i, a], rel=2e-6, abs=2e-6 * np.abs(f).max())


@pytest.mark.parametrize("pot", ["kg", "cu"])
def test_virial_equals_energy_derivative_wrt_F(pot):
    # W = sum g d (x) d / r must equal (dE/dF) F^T for the energy of the affinely deformed cell
    # (positions F x0, box F H0), central differences over the nine components of F.
    rng = np.random.default_rng(6)
    if pot == "kg":
        x0, b, H0 = kg_melt([8] * 12, seed=5)
        p = KG
    else:
        x0, H0 = fcc_lattice(3)
        x0 = x0 + rng.normal(0, 0.1, x0.shape)
        b, p = None, CU
    F = np.eye(3) + 0.03 * rng.standard_normal((3, 3))
    E = lambda G: core.forces(p, G @ H0, x0 @ G.T, b)[1]
    _, _, W = core.forces(p, F @ H0, x0 @ F.T, b)
    h = 1e-6
    dEdF = np.zeros((3, 3))
    for a, c in itertools.product(range(3), range(3)):
        Fp, Fm = F.copy(), F.copy()
        Fp[a, c] += h
        Fm[a, c] -= h
        dEdF[a, c] = (E(Fp) - E(Fm)) / (2 * h)
    Wfd = dEdF @ F.T
    assert np.abs(W - Wfd).max() <= 1e-6 * np.abs(W).max()
    assert np.abs(Wfd - Wfd.T).max() <= 1e-6 * np.abs(W).max()   # rotational invariance


def test_lj_fene_dimer_closed_forms():
    H = np.eye(3) * 20.0
    for r in [0.9, 1.0, 1.05, 2 ** (1 / 6) - 1e-9]:
        x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
        f, pe, W = core.forces(KG, H, x)
        g = -24.0 * (2 * r ** -12 - r ** -6) / r
        assert f[1, 0] == pytest.approx(-g, rel=1e-13)
        assert pe == pytest.approx(4 * (r ** -12 - r ** -6) + 1.0, rel=1e-12, abs=1e-12)
        assert W[0, 0] == pytest.approx(g * r, rel=1e-13)
    # the truncated-shifted LJ force vanishes at rc = 2^(1/6) sigma
    x = np.array([[5.0, 5.0, 5.0], [5.0 + 2 ** (1 / 6) * (1 - 1e-12), 5.0, 5.0]])
    assert abs(core.forces(KG, H, x)[0][1, 0]) < 1e-9
    # bonded dimer: WCA + FENE, U = -K R0^2/2 ln(1 - (r/R0)^2)
    r = 0.97
    x = np.array([[5.0, 5.0, 5.0], [5.0, 5.0 + r, 5.0]])
    f, pe, _ = core.forces(KG, H, x, np.array([[0, 1]]))
    g = -24.0 * (2 * r ** -12 - r ** -6) / r + 30.0 * r / (1 - (r / 1.5) ** 2)
    assert f[1, 1] == pytest.approx(-g, rel=1e-13)
    assert pe == pytest.approx(4 * (r ** -12 - r ** -6) + 1 - 0.5 * 30 * 1.5 ** 2 * np.log(1 - (r / 1.5) ** 2), rel=1e-13)
    with pytest.raises(core.OracleError) as e:
        core.forces(KG, H, np.array([[5.0, 5, 5], [6.6, 5, 5]]), np.array([[0, 1]]))
    assert e.value.code == core.ERR_BOND


def _fcc_shells(a, rc):
    """Distances to all FCC lattice points within rc, from integer coordinates (i+j+k even)."""
    m = int(np.ceil(2 * rc / a)) + 1
    g = np.arange(-m, m + 1)
    ijk = np.array(list(itertools.product(g, g, g)))
    ijk = ijk[(ijk.sum(1) % 2 == 0) & np.any(ijk != 0, axis=1)]
    r = np.linalg.norm(ijk * (a / 2), axis=1)
    return r[r < rc]


# gold in the published Sutton-Chen parameter set: other exponents than copper's (9, 6)
AU = dict(CU, sc_eps=1.2793e-2, sc_a=4.08, sc_c=34.408, sc_n=10, sc_m=8, mass=196.967, rc=1.95 * 4.08)


@pytest.mark.parametrize("P", [CU, AU], ids=["cu_9_6", "au_10_8"])
def test_sutton_chen_perfect_lattice(P):
    a, rc = P["sc_a"], P["rc"]
    e, c, n, m = P["sc_eps"], P["sc_c"], P["sc_n"], P["sc_m"]

    def e_atom(scale):
        r = _fcc_shells(a * scale, rc)
        return 0.5 * e * ((a / r) ** n - (a / rc) ** n).sum() - e * c * np.sqrt(((a / r) ** m - (a / rc) ** m).sum())

    assert len(_fcc_shells(a, rc)) == 134            # shells up to 1.871a: 12+6+24+12+24+8+48
    for ncell in (3, 6):                             # brute-force image path and cell-list path
        x, H = fcc_lattice(ncell, a)
        f, pe, W = core.forces(P, H, x)
        assert pe / len(x) == pytest.approx(e_atom(1.0), rel=1e-12)
        assert np.abs(f).max() < 1e-12                # inversion symmetry of a Bravais lattice
        # hydrostatic stress = dE/dV per atom, V_atom = a^3/4, from a central difference in a
        h = 1e-6
        dEda = (e_atom(1 + h) - e_atom(1 - h)) / (2 * h * a)
        sig_h = dEda / (3 * a * a / 4)
        V = np.linalg.det(H)
        assert np.allclose(np.diag(W) / V, sig_h, rtol=1e-7)
        assert np.abs(W - np.diag(np.diag(W))).max() < 1e-10
    if P is CU:
        assert e_atom(1.0) == pytest.approx(-3.3997, abs=5e-5)


@pytest.mark.parametrize("pot", ["kg", "cu"])
def test_frame_indifference_of_qr_route(pot):
    # Stress of the general box F H0 (positions F H0 S) equals Q sigma(R H0) Q^T (Sec. 2.1).
    rng = np.random.default_rng(8)
    if pot == "kg":
        x0, b, H0 = kg_melt([10] * 20, seed=13)
        p = KG
    else:
        x0, H0 = fcc_lattice(6)
        x0 = x0 + rng.normal(0, 0.05, x0.shape)
        b, p = None, CU
    S = np.linalg.solve(H0, x0.T).T
    for F in [TABLE1_F["C(t)"], np.eye(3) + 0.08 * rng.standard_normal((3, 3))]:
        Q, R = core.qr(F)
        fF, eF, WF = core.forces(p, F @ H0, S @ (F @ H0).T, b)
        fR, eR, WR = core.forces(p, R @ H0, S @ (R @ H0).T, b)
        assert eF == pytest.approx(eR, rel=1e-12)
        assert np.abs(WF - Q @ WR @ Q.T).max() <= 1e-12 * np.abs(WR).max()
        assert np.abs(fF - fR @ Q.T).max() <= 1e-11 * np.abs(fR).max()


def test_cubic_symmetry_of_table1_deformations():
    # B(t)/B(c): F is invariant under (x, y, z) -> (-z, y, -x), so sigma_xx = sigma_zz and
    # sigma_xy = -sigma_yz; C(t)/C(c): F is symmetric under permutations, so equal diagonal and
    # equal off-diagonal components (as printed in Table 1).  Perfect FCC copper, 0 K, static.
    x, H0 = fcc_lattice(10)
    cells = [dict(x=x, v=np.zeros_like(x), bonds=np.zeros((0, 2), np.int32), H0=H0)]
    for case, F in TABLE1_F.items():
        ob = core.OracleBatch(CU, cells)
        ob.set_deformation(F[None])
        s = unvoigt(ob.get_stress()[0])
        tol = 1e-10 * np.abs(s).max()
        if case.startswith("B"):
            assert abs(s[0, 0] - s[2, 2]) < tol and abs(s[0, 1] + s[1, 2]) < tol, case
        else:
            assert np.ptp(np.diag(s)) < tol and np.ptp([s[0, 1], s[0, 2], s[1, 2]]) < tol, case
