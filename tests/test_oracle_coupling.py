"""Pins for the oracle's coupling arithmetic: QR of F (Eq. 4), stress rotation (Eq. 7),
first Piola-Kirchhoff stress (Eq. 8) and the incremental box update (Eq. 9).

Pins come from Table 1 (printed values, tests/golden/table1.txt), from LAPACK, and from
identities that any correct implementation satisfies."""
import numpy as np
import pytest

from conftest import unvoigt, voigt
from oracle import core


def test_qr_reproduces_table1(table1):
    # Table 1 prints F, Q and R to three decimals: the QR of the printed F must round to them.
    for case, t in table1.items():
        Q, R = core.qr(t["F"])
        assert np.abs(Q - t["Q"]).max() <= 5e-4 + 1e-12, case
        assert np.abs(R - t["R"]).max() <= 5e-4 + 1e-12, case


def test_qr_matches_lapack_and_identities():
    rng = np.random.default_rng(7)
    for _ in range(200):
        F = np.eye(3) + 0.4 * rng.standard_normal((3, 3))
        if np.linalg.det(F) <= 0.05:
            continue
        Q, R = core.qr(F)
        q, r = np.linalg.qr(F)
        s = np.sign(np.diag(r))
        q, r = q * s[None, :], r * s[:, None]
        assert np.abs(Q - q).max() < 1e-13
        assert np.abs(R - r).max() < 1e-13
        assert np.abs(Q.T @ Q - np.eye(3)).max() < 1e-14
        assert np.abs(Q @ R - F).max() < 1e-14
        assert np.all(np.diag(R) > 0) and np.all(np.tril(R, -1) == 0)
        assert abs(np.linalg.det(Q) - 1.0) < 1e-14


@pytest.mark.parametrize("F", [np.diag([1.0, 1.0, -1.0]), np.zeros((3, 3)),
                               np.array([[1, 0, 0], [0, 1, 0], [np.nan, 0, 1.0]]),
                               np.array([[1, 1, 0], [1, 1, 0], [0, 0, 1.0]])])
def test_qr_rejects_bad_F(F):
    with pytest.raises(core.OracleError) as e:
        core.qr(F)
    assert e.value.code == core.ERR_BAD_F


def test_rotation_reproduces_table1(table1):
    # sigma_FEM = Q sigma_MD Q^T with the exact Q of the printed F reproduces the printed sigma_FEM
    # to the table's rounding; the reverse rotation Q^T sigma Q does not.
    for case, t in table1.items():
        s_fem, _ = core.stress_to_fem(t["F"], voigt(t["sig_MD"]))
        assert np.abs(unvoigt(s_fem) - t["sig_FEM"]).max() <= 1e-3, case
        Q, _ = core.qr(t["F"])
        wrong = Q.T @ t["sig_MD"] @ Q
        assert np.abs(wrong - t["sig_FEM"]).max() > 0.5, case


def test_table1_error_norm(table1):
    # The last row of Table 1 (spectral norm of sigma_IH - sigma_FEM) follows from the printed stresses.
    for case, t in table1.items():
        d = np.linalg.norm(t["sig_IH"] - t["sig_FEM"], 2)
        assert round(d, 3) == pytest.approx(t["dsig2"], abs=1e-9), case


def test_piola_kirchhoff_identities():
    rng = np.random.default_rng(3)
    for _ in range(50):
        F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
        if np.linalg.det(F) <= 0.2:
            continue
        A = rng.standard_normal((3, 3))
        s_md = voigt(A + A.T)
        s_fem, P = core.stress_to_fem(F, s_md)
        J = np.linalg.det(F)
        S = unvoigt(s_fem)
        # Eq. (8): P = J sigma F^-T, hence P F^T / J = sigma, symmetric
        assert np.abs(P @ F.T / J - S).max() < 1e-12
        # Eq. (7) is a similarity transform: eigenvalues are unchanged
        assert np.allclose(np.linalg.eigvalsh(S), np.linalg.eigvalsh(unvoigt(s_md)), atol=1e-12)


def test_incremental_box_equals_direct():
    # Eq. (9): successive Delta R = R(t) R(t-1)^-1 applied to the box compose to R(t) H0
    # (modulo the lattice-preserving tilt reduction, which keeps the same lattice).
    rng = np.random.default_rng(11)
    L = 30.0
    H0 = np.eye(3) * L
    x0 = rng.uniform(0, L, (40, 3))
    cells = [dict(x=x0, v=np.zeros_like(x0), bonds=np.zeros((0, 2), np.int32), H0=H0)]
    p = dict(core_params_kg())
    ob = core.OracleBatch(p, cells)
    Fs = [np.eye(3) + 0.05 * k * np.array([[0.1, 0.3, 0.2], [0.0, 0.2, -0.1], [0.1, 0.0, -0.1]])
          for k in range(1, 6)]
    for F in Fs:
        ob.set_deformation(F[None])
    H, Q, R, J = ob.get_box(0)
    Qd, Rd = core.qr(Fs[-1])
    assert np.abs(R - Rd).max() < 1e-14 and np.abs(Q - Qd).max() < 1e-14
    assert J == pytest.approx(np.linalg.det(Fs[-1]), rel=1e-14)
    # same lattice: H = Rd H0 U with U integer unimodular
    U = np.linalg.solve(Rd @ H0, H)
    assert np.abs(U - np.rint(U)).max() < 1e-10 and abs(abs(np.linalg.det(np.rint(U))) - 1) < 1e-12
    # positions: S preserved modulo the lattice
    st = ob.get_state(0)
    S_now = np.linalg.solve(Rd @ H0, st["x"].T).T
    dS = S_now - x0 / L
    assert np.abs(dS - np.rint(dS)).max() < 1e-12


def test_lattice_reduce_keeps_lattice():
    rng = np.random.default_rng(5)
    for _ in range(100):
        H = np.triu(rng.uniform(-3, 3, (3, 3)))
        H[np.diag_indices(3)] = rng.uniform(1, 2, 3)
        Hr = core.lattice_reduce(H)
        U = np.linalg.solve(H, Hr)
        assert np.abs(U - np.rint(U)).max() < 1e-10
        assert abs(abs(np.linalg.det(np.rint(U))) - 1) < 1e-12
        assert abs(Hr[1, 2]) <= 0.5 * Hr[1, 1] + 1e-12
        assert abs(Hr[0, 2]) <= 0.5 * Hr[0, 0] + 1e-12
        assert abs(Hr[0, 1]) <= 0.5 * Hr[0, 0] + 1e-12
        assert np.all(np.tril(Hr, -1) == 0)


def core_params_kg():
    from synth.configs import kg_params
    return kg_params(gamma=0.0, temperature=0.0)
