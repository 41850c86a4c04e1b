"""Pins for the host FE driver (Eqs. 10-14), for both meshes (hex8 bricks, C3D4 tetrahedra): the
patch test, internal forces as the exact gradient of the discrete strain energy, lumped mass, the
conformity of the tetrahedral mesh, and the closed-form uniaxial response of a neo-Hookean bar
reached quasi-statically by the explicit solver."""
from collections import Counter

import numpy as np
import pytest

from paper_1902_09171_amd import fe


MESHES = [fe.Hex8Bar, fe.Tet4Bar]


@pytest.mark.parametrize("mesh", MESHES)
def test_patch_test_homogeneous_motion(mesh):
    m = mesh(nel=(4, 2, 2), size=(40.0, 10.0, 12.0), imperfection=0.9)
    F0 = np.array([[1.1, 0.05, -0.02], [0.01, 0.95, 0.03], [0.0, -0.04, 1.02]])
    u = m.X @ (F0 - np.eye(3)).T
    F = m.deformation_gradients(u)
    assert np.abs(F - F0[None]).max() < 1e-13
    assert m.mass.sum() == pytest.approx(m.rho0 * m.volume, rel=1e-13)
    # a homogeneous stress is in equilibrium: interior nodes feel no net internal force
    P = np.broadcast_to(np.diag([2.0, -1.0, 0.5]) + 0.3, (m.ngp, 3, 3)).copy()
    f = m.internal_forces(P)
    interior = [m.node(i, j, k) for i in range(1, 4) for j in range(1, 2) for k in range(1, 2)]
    assert np.abs(f[interior]).max() < 1e-12
    assert np.abs(f.sum(0)).max() < 1e-11


@pytest.mark.parametrize("mesh", MESHES)
def test_internal_force_is_energy_gradient(mesh):
    m = mesh(nel=(2, 1, 1), size=(4.0, 2.0, 2.0), imperfection=0.9)
    mat = fe.neo_hookean(1.3, 2.1)
    rng = np.random.default_rng(0)
    u = 0.05 * rng.standard_normal((m.nnodes, 3))
    W = lambda uu: float((mat.energy(m.deformation_gradients(uu)) * m.wdet).sum())
    f = m.internal_forces(mat(m.deformation_gradients(u))[0])
    h = 1e-6
    for a in range(m.nnodes):
        for i in range(3):
            up, um = u.copy(), u.copy()
            up[a, i] += h
            um[a, i] -= h
            assert (W(up) - W(um)) / (2 * h) == pytest.approx(f[a, i], rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("mesh", MESHES)
def test_quasistatic_uniaxial_neo_hookean(mesh):
    mu, lam = 1.0, 1.5
    m = mesh(nel=(4, 1, 1), size=(8.0, 2.0, 2.0), rho0=1.0)
    mat = fe.neo_hookean(mu, lam)
    strain, steps = 0.02, 4000
    dt = 0.02
    bar = fe.ExplicitBar(m, mat, dt=dt, pull_velocity=strain * 8.0 / (steps * dt), damping=0.5)
    for _ in range(steps):
        bar.step()
    bar.vp = 0.0                                  # hold and let it settle
    for _ in range(3000):
        bar.step()
    F = m.deformation_gradients(bar.u)
    lam1 = 1.0 + strain
    # uniaxial stress: P_yy = mu (lt - 1/lt) + lam ln(J) / lt = 0 with J = lam1 lt^2
    lt = 1.0
    for _ in range(50):
        g = mu * (lt - 1 / lt) + lam * np.log(lam1 * lt * lt) / lt
        dg = mu * (1 + 1 / lt ** 2) + lam * (2 / lt ** 2 - np.log(lam1 * lt * lt) / lt ** 2)
        lt -= g / dg
    assert np.allclose(F[:, 0, 0], lam1, atol=2e-4)
    assert np.allclose(F[:, 1, 1], lt, atol=2e-4) and np.allclose(F[:, 2, 2], lt, atol=2e-4)
    Pxx = mu * (lam1 - 1 / lam1) + lam * np.log(lam1 * lt * lt) / lam1
    reaction = -m.internal_forces(mat(F)[0])[bar.right, 0].sum()
    assert -reaction == pytest.approx(Pxx * 2.0 * 2.0, rel=2e-3)
    assert fe.tensile_stress(bar.history[-1]["sigma"]) == pytest.approx(Pxx * lam1 / (lam1 * lt * lt), rel=2e-2)


def test_tetrahedral_mesh_is_conforming():
    """The paper's specimen: 100 C3D4 elements filling the cube, every interior face shared by
    exactly two elements and the surface covered by two triangles per brick face."""
    m = fe.Tet4Bar(nel=(5, 2, 2), size=(22.7, 22.7, 22.7))
    assert m.ngp == 100 and m.conn.shape == (100, 4)
    assert np.all(m.wdet > 0)
    assert m.volume == pytest.approx(22.7 ** 3, rel=1e-13)
    faces = Counter(tuple(sorted(np.delete(t, q))) for t in m.conn for q in range(4))
    assert set(faces.values()) == {1, 2}
    assert sum(1 for v in faces.values() if v == 1) == 2 * 2 * (5 * 2 + 5 * 2 + 2 * 2)
    # a uniaxial homogeneous stress: the pulled face carries P_xx times its area
    P = np.zeros((m.ngp, 3, 3))
    P[:, 0, 0] = 1.7
    f = m.internal_forces(P)
    assert f[m.face(0, 1), 0].sum() == pytest.approx(1.7 * 22.7 * 22.7, rel=1e-12)


@pytest.mark.parametrize("mesh", MESHES)
def test_cfl_check(mesh):
    """The explicit step is refused beyond 0.9 h / c: the neo-Hookean P-wave modulus lambda + 2 mu
    gives c, the smallest element length h (shortest brick edge, smallest tetrahedron altitude)."""
    m = mesh(nel=(4, 2, 2), size=(40.0, 10.0, 12.0))
    mu, lam, rho0 = 1.3, 2.1, m.rho0
    c = fe.wave_speed(lam + 2.0 * mu, rho0)
    assert c == pytest.approx(np.sqrt((lam + 2 * mu) / rho0), rel=1e-15)
    h = m.min_length()
    if mesh is fe.Hex8Bar:
        assert h == pytest.approx(5.0)                  # 10 / 2, the shortest brick edge
    else:
        assert 0.0 < h < 5.0                            # altitudes are shorter than the brick edges
    lim = fe.cfl_limit(m, c)
    assert lim == pytest.approx(0.9 * h / c)
    fe.ExplicitBar(m, fe.neo_hookean(mu, lam), dt=0.99 * lim, pull_velocity=0.01, wave_speed=c)
    with pytest.raises(ValueError, match="CFL"):
        fe.ExplicitBar(m, fe.neo_hookean(mu, lam), dt=1.01 * lim, pull_velocity=0.01, wave_speed=c)


def test_tet_altitude_of_the_unit_corner_tetrahedron():
    """The corner tetrahedron (0, e_x, e_y, e_z) has volume 1/6 and largest face sqrt(3)/2, so its
    smallest altitude is 3 (1/6) / (sqrt(3)/2) = 1/sqrt(3)."""
    class One(fe._Mesh):
        pass
    m = One()
    m.X = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    m.conn = np.array([[0, 1, 2, 3]])
    assert m.min_length() == pytest.approx(1.0 / np.sqrt(3.0), rel=1e-14)
