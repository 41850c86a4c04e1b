"""Host finite-element driver of the coupling (Sec. 2.2, Eqs. 10-14; Fig. 1): an explicit
total-Lagrangian bar whose quadrature points take their first Piola-Kirchhoff stress from a
stress provider - batched MD r-cells (rcell) or the learned surrogate.  Two meshes: trilinear
hex8 bricks with 2x2x2 Gauss points, and linear four-node tetrahedra (C3D4, one quadrature point
each), the element of the paper's polymer specimen (Sec. 3.2) and scaling test.

Per load step: F at every Gauss point from the nodal displacements (F = I + du/dX), P from the
provider, internal forces f_int = sum_gp B^T P w det J0 (Eq. 12), lumped mass (Eq. 11), and a
central-difference update of M d'' + f_int = f_ext (Eq. 10) with mass-proportional damping.
Loading: the face x = 0 is held in x, the face x = L moves at a prescribed velocity along x, the
lateral faces are free; two pins remove the remaining rigid-body motion.
"""
import numpy as np

_XI = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
_G = 1.0 / np.sqrt(3.0)


def shape(xi):
    """Trilinear shape functions N_a and their derivatives dN_a/dxi at natural point xi."""
    t = 1.0 + _XI * xi[None, :]
    N = t.prod(1) / 8.0
    dN = np.empty((8, 3))
    dN[:, 0] = _XI[:, 0] * t[:, 1] * t[:, 2] / 8.0
    dN[:, 1] = _XI[:, 1] * t[:, 0] * t[:, 2] / 8.0
    dN[:, 2] = _XI[:, 2] * t[:, 0] * t[:, 1] / 8.0
    return N, dN


class _Mesh:
    """What the bar integrator needs from a mesh: nodes X, connectivity conn, and per quadrature
    point its element gp_elem, dN/dX (B), weight x det J0 (wdet); lumped nodal masses."""

    def deformation_gradients(self, u):
        """F = I + sum_a u_a (x) dN_a/dX at every quadrature point, (ngp, 3, 3)."""
        ue = u[self.conn[self.gp_elem]]             # (ngp, nodes per element, 3)
        return np.eye(3)[None] + np.einsum("gai,gaj->gij", ue, self.B)

    def internal_forces(self, P):
        """f_int_a = sum_gp P . dN_a/dX w det J0 (Eq. 12), (nnodes, 3)."""
        fe = np.einsum("gij,gaj->gai", P, self.B) * self.wdet[:, None, None]
        f = np.zeros((self.nnodes, 3))
        np.add.at(f, self.conn[self.gp_elem].ravel(), fe.reshape(-1, 3))
        return f

    def face(self, axis, side):
        lo, hi = self.X[:, axis].min(), self.X[:, axis].max()
        return np.where(np.isclose(self.X[:, axis], hi if side else lo))[0]

    def min_length(self):
        """Smallest element length for the explicit time-step limit: the shortest edge of a brick,
        or the smallest altitude (3 V / largest face area) of a tetrahedron."""
        Xe = self.X[self.conn]                       # (nelem, nodes, 3)
        if self.conn.shape[1] == 8:
            edges = [(0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 7), (7, 4),
                     (0, 4), (1, 5), (2, 6), (3, 7)]
            return float(min(np.linalg.norm(Xe[:, a] - Xe[:, b], axis=1).min() for a, b in edges))
        V = np.abs(np.einsum("ei,ei->e", np.cross(Xe[:, 1] - Xe[:, 0], Xe[:, 2] - Xe[:, 0]),
                             Xe[:, 3] - Xe[:, 0])) / 6.0
        faces = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
        amax = np.max([0.5 * np.linalg.norm(np.cross(Xe[:, b] - Xe[:, a], Xe[:, c] - Xe[:, a]), axis=1)
                       for a, b, c in faces], axis=0)
        return float((3.0 * V / amax).min())


def _grid_nodes(nel, size, imperfection):
    """Nodes of a structured grid of nx x ny x nz bricks on [0, Lx] x [0, Ly] x [0, Lz]; with
    imperfection < 1 the middle cross-section (x = Lx / 2) is scaled laterally about the axis."""
    nx, ny, nz = nel
    Lx, Ly, Lz = size
    xs, ys, zs = np.linspace(0, Lx, nx + 1), np.linspace(0, Ly, ny + 1), np.linspace(0, Lz, nz + 1)
    X = np.array([[x, y, z] for x in xs for y in ys for z in zs])
    if imperfection != 1.0 and nx % 2 == 0:
        mid = np.isclose(X[:, 0], xs[nx // 2])
        X[mid, 1] = Ly / 2 + (X[mid, 1] - Ly / 2) * imperfection
        X[mid, 2] = Lz / 2 + (X[mid, 2] - Lz / 2) * imperfection
    return X, (lambda i, j, k: (i * (ny + 1) + j) * (nz + 1) + k)


class Hex8Bar(_Mesh):
    """Structured nx x ny x nz hex8 mesh of a bar [0, Lx] x [0, Ly] x [0, Lz], 2x2x2 Gauss points.

    imperfection < 1 scales the lateral coordinates of the middle cross-section about the bar axis
    (a seed for necking)."""

    def __init__(self, nel=(8, 2, 2), size=(200.0, 50.0, 50.0), rho0=0.85, imperfection=1.0):
        nx, ny, nz = nel
        self.nel, self.size, self.rho0 = nel, size, rho0
        X, self.node = _grid_nodes(nel, size, imperfection)
        self.X = X
        self.nnodes = len(X)
        conn = []
        for i in range(nx):
            for j in range(ny):
                for k in range(nz):
                    conn.append([self.node(i + a, j + b, k + c) for a, b, c in
                                 ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1))])
        self.conn = np.array(conn)
        # per Gauss point: element, dN/dX (8 x 3), w det J0, N
        gps = [np.array([a, b, c]) * _G for c in (-1, 1) for b in (-1, 1) for a in (-1, 1)]
        elem, B, wdet, Ns = [], [], [], []
        for e, nodes in enumerate(self.conn):
            Xe = X[nodes]
            for xi in gps:
                N, dN = shape(xi)
                J = Xe.T @ dN                       # J_ij = sum_a X_a,i dN_a/dxi_j
                B.append(dN @ np.linalg.inv(J))     # dN_a/dX_j
                wdet.append(np.linalg.det(J))       # Gauss weight 1
                elem.append(e)
                Ns.append(N)
        self.gp_elem = np.array(elem)
        self.B = np.array(B)                        # (ngp, 8, 3)
        self.wdet = np.array(wdet)
        self.ngp = len(self.B)
        self.mass = np.zeros(self.nnodes)
        for g in range(self.ngp):
            np.add.at(self.mass, self.conn[self.gp_elem[g]], rho0 * Ns[g] * self.wdet[g])
        self.volume = self.wdet.sum()



# the four nodes of a linear tetrahedron in natural coordinates: N = (1 - xi - eta - zeta, xi, eta, zeta)
_DN_TET = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


class Tet4Bar(_Mesh):
    """Linear four-node tetrahedra (C3D4) on a structured grid of nx x ny x nz bricks of the bar
    [0, Lx] x [0, Ly] x [0, Lz]: five tetrahedra per brick, one quadrature point per tetrahedron
    (constant strain), lumped mass a quarter of the element mass per node.

    Each brick is split into the tetrahedron spanned by its four corners of even global index
    parity (i + j + k) and the four corner tetrahedra of its odd corners, each with that corner's
    three neighbours along the brick edges.  Every face diagonal then joins the two even corners of
    the face on both sides, so the mesh is conforming.  2 x 2 x 5 bricks give the 100 elements of
    the paper's cubic polymer specimen (Sec. 3.2)."""

    def __init__(self, nel=(5, 2, 2), size=(22.7, 22.7, 22.7), rho0=0.85, imperfection=1.0):
        nx, ny, nz = nel
        self.nel, self.size, self.rho0 = nel, size, rho0
        X, self.node = _grid_nodes(nel, size, imperfection)
        self.X = X
        self.nnodes = len(X)
        corners = [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]
        conn = []
        for i in range(nx):
            for j in range(ny):
                for k in range(nz):
                    gid = {t: self.node(i + t[0], j + t[1], k + t[2]) for t in corners}
                    even = [t for t in corners if (i + t[0] + j + t[1] + k + t[2]) % 2 == 0]
                    odd = [t for t in corners if (i + t[0] + j + t[1] + k + t[2]) % 2 == 1]
                    tets = [even]
                    for t in odd:
                        nb = [u for u in even if sum(abs(u[q] - t[q]) for q in range(3)) == 1]
                        tets.append([t] + nb)
                    for tet in tets:
                        ids = [gid[t] for t in tet]
                        if np.linalg.det((X[ids[1:]] - X[ids[0]]).T) < 0:
                            ids[1], ids[2] = ids[2], ids[1]      # positive orientation
                        conn.append(ids)
        self.conn = np.array(conn)
        self.gp_elem = np.arange(len(self.conn))
        B, wdet = [], []
        for nodes in self.conn:
            J = X[nodes].T @ _DN_TET                 # J_ij = sum_a X_a,i dN_a/dxi_j
            B.append(_DN_TET @ np.linalg.inv(J))
            wdet.append(np.linalg.det(J) / 6.0)      # one point, weight 1/6 of the unit tetrahedron
        self.B = np.array(B)                         # (ngp, 4, 3)
        self.wdet = np.array(wdet)
        self.ngp = len(self.B)
        self.mass = np.zeros(self.nnodes)
        np.add.at(self.mass, self.conn.ravel(), np.repeat(rho0 * self.wdet / 4.0, 4))
        self.volume = self.wdet.sum()


CFL_SAFETY = 0.9


def cfl_limit(mesh, wave_speed):
    """Largest stable time step of the explicit central differences: 0.9 h / c with h the smallest
    element length and c the material's longitudinal wave speed."""
    return CFL_SAFETY * mesh.min_length() / wave_speed


def wave_speed(modulus, rho0):
    """Longitudinal wave speed c = sqrt(M / rho0) for the P-wave modulus M."""
    return float(np.sqrt(modulus / rho0))


def md_wave_speed(params, cells, rho0, md_steps, delta=0.02, warmup_steps=0):
    """Wave speed of an r-cell material as the explicit integrator sees it: the P-wave modulus
    M = d sigma_xx / d eps_xx of the stress the cells return for one load step - the average over
    md_steps MD steps after a step F = diag(1 +- delta, 1, 1) - by central differences over the
    given cells (two batches on the GPU, the same initial states and noise for both signs).  The
    instantaneous affine modulus of a dense repulsive melt is an order of magnitude larger, but it
    relaxes within a fraction of the window, and the FE update only ever sees window averages."""
    from .rcell import RCellBatch
    sxx = []
    for e in (delta, -delta):
        g = RCellBatch(params, cells)
        if warmup_steps:
            g.run(warmup_steps)
        g.get_stress()
        g.set_deformation(np.tile(np.diag([1.0 + e, 1.0, 1.0]), (len(cells), 1, 1)))
        g.run(md_steps)
        sxx.append(float(g.get_stress()[:, 0].mean()))
        g.close()
    return wave_speed((sxx[0] - sxx[1]) / (2.0 * delta), rho0)


class ExplicitBar:
    """Central-difference time stepping of the bar under a constant pull velocity.

    provider(F) -> (P, sigma): first Piola-Kirchhoff stress (ngp, 3, 3) and Cauchy stress (ngp, 6)
    for the deformation gradients F (ngp, 3, 3) of one load step.  With wave_speed given, a time
    step beyond the CFL limit (cfl_limit) is refused with a ValueError."""

    def __init__(self, mesh, provider, dt, pull_velocity, damping=0.0, wave_speed=None):
        if wave_speed is not None:
            lim = cfl_limit(mesh, wave_speed)
            if not dt <= lim:
                raise ValueError(f"FE time step {dt:g} exceeds the CFL limit {CFL_SAFETY} h / c = {lim:g} "
                                 f"(h = {mesh.min_length():g}, c = {wave_speed:g})")
        self.m, self.provider, self.dt, self.vp, self.c = mesh, provider, dt, pull_velocity, damping
        self.u = np.zeros((mesh.nnodes, 3))
        self.v = np.zeros((mesh.nnodes, 3))
        self.left, self.right = mesh.face(0, 0), mesh.face(0, 1)
        corner = self.left[np.argmin(mesh.X[self.left, 1] + mesh.X[self.left, 2])]
        side = self.left[np.argmax(mesh.X[self.left, 1] - mesh.X[self.left, 2])]
        self.pin_yz, self.pin_z = corner, side
        self.v[self.right, 0] = pull_velocity
        self.t = 0.0
        self.u_pull = 0.0                 # prescribed displacement of the pulled face
        self.history = []

    def _apply_bc(self):
        self.v[self.left, 0] = 0.0
        self.u[self.left, 0] = 0.0
        self.v[self.right, 0] = self.vp
        self.u[self.right, 0] = self.u_pull
        self.v[self.pin_yz, 1:] = 0.0
        self.u[self.pin_yz, 1:] = 0.0
        self.v[self.pin_z, 2] = 0.0
        self.u[self.pin_z, 2] = 0.0

    def step(self):
        """One load step: stresses at the current configuration, then v and u advance by dt."""
        F = self.begin_step()
        P, sigma = self.provider(F)
        return self.finish_step(F, P, sigma)

    def begin_step(self):
        """The deformation gradients of the current configuration (the provider's input)."""
        return self.m.deformation_gradients(self.u)

    def finish_step(self, F, P, sigma):
        """Advance v and u by dt under the stresses P of the configuration F (several bars can
        share one batched stress provider between begin_step and finish_step)."""
        f = -self.m.internal_forces(P)
        a = f / self.m.mass[:, None] - self.c * self.v
        self.v += self.dt * a
        self.t += self.dt
        self.u_pull += self.dt * self.vp
        self.u += self.dt * self.v
        self._apply_bc()
        strain = self.u_pull / self.m.size[0]
        self.history.append(dict(strain=strain, F=F, P=P, sigma=sigma,
                                 tensile=tensile_stress(sigma)))
        return F, P, sigma


def tensile_stress(sigma):
    """Largest eigenvalue of sigma_FEM averaged over the Gauss points (the measure of Fig. 6)."""
    s = np.asarray(sigma)
    m = np.array([[s[:, 0], s[:, 3], s[:, 4]], [s[:, 3], s[:, 1], s[:, 5]], [s[:, 4], s[:, 5], s[:, 2]]])
    return float(np.linalg.eigvalsh(m.transpose(2, 0, 1))[:, -1].mean())


def neo_hookean(mu, lam):
    """Compressible neo-Hookean material (for checks of the driver): P = mu (F - F^-T) + lam ln J F^-T."""
    def provider(F):
        J = np.linalg.det(F)
        FiT = np.linalg.inv(F).transpose(0, 2, 1)
        P = mu * (F - FiT) + lam * np.log(J)[:, None, None] * FiT
        sig = np.einsum("gij,gkj->gik", P, F) / J[:, None, None]
        return P, np.stack([sig[:, 0, 0], sig[:, 1, 1], sig[:, 2, 2], sig[:, 0, 1], sig[:, 0, 2], sig[:, 1, 2]], 1)

    def energy(F):
        J = np.linalg.det(F)
        I1 = np.einsum("gij,gij->g", F, F)
        return 0.5 * mu * (I1 - 3) - mu * np.log(J) + 0.5 * lam * np.log(J) ** 2
    provider.energy = energy
    return provider


class MDStress:
    """Stress provider backed by batched MD r-cells: set_deformation (Eqs. 4, 5, 9), md_steps MD
    steps, windowed stress rotated back (Eqs. 7, 8).  cells[g] is the r-cell of Gauss point g."""

    def __init__(self, params, cells, md_steps, stream=None):
        from .rcell import RCellBatch
        self.g = RCellBatch(params, cells, stream=stream)
        self.md_steps = md_steps
        self.last_md = None           # MD-frame stress of the last load step (training targets)

    def __call__(self, F):
        self.g.set_deformation(F)
        self.g.run(self.md_steps)
        s, P, self.last_md = self.g.get_stress_ext()
        return P, s
