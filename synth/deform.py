"""Deformation-gradient inputs: random rotations, uniaxial stretches, symmetric stretches and the
four printed deformation gradients of the paper's Table 1 (row-major, F_ij = dx_i/dX_j)."""
import numpy as np

# Table 1 (Sec. 3.1), cases B(t), B(c), C(t), C(c): deformation gradients as printed, row-major.
TABLE1_F = {
    "B(t)": np.array([[1.0, 0.0, 0.0], [-0.075, 1.075, 0.075], [0.0, 0.0, 1.0]]),
    "B(c)": np.array([[1.0, 0.0, 0.0], [0.075, 0.925, -0.075], [0.0, 0.0, 1.0]]),
    "C(t)": np.array([[1.075, 0.075, 0.075], [0.075, 1.075, 0.075], [0.075, 0.075, 1.075]]),
    "C(c)": np.array([[0.925, -0.075, -0.075], [-0.075, 0.925, -0.075], [-0.075, -0.075, 0.925]]),
}


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a unit quaternion of four iid standard normals."""
    q = rng.standard_normal(4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def uniaxial_isochoric(e: float, axis: int = 0) -> np.ndarray:
    """diag(1+e, (1+e)^-1/2, (1+e)^-1/2) with the stretched direction on `axis`."""
    lam = 1.0 + e
    d = np.full(3, lam ** -0.5)
    d[axis] = lam
    return np.diag(d)


def rotated_uniaxial(e: float, Qg: np.ndarray, axis: int = 2) -> np.ndarray:
    """F = Qg . diag(...1+e on axis...): uniaxial stretch followed by a rigid rotation."""
    d = np.ones(3)
    d[axis] = 1.0 + e
    return Qg @ np.diag(d)


def rotated_stretch(rng: np.random.Generator, lo: float = 0.9, hi: float = 1.1) -> np.ndarray:
    """F = Q . V diag(lambda) V^T with lambda_i ~ U[lo, hi] and Q, V uniform rotations."""
    Q = random_rotation(rng)
    V = random_rotation(rng)
    lam = rng.uniform(lo, hi, 3)
    return Q @ (V @ np.diag(lam) @ V.T)


def stretch_paths(ncells, nsteps, rng, rate_max=0.012, nu=(0.2, 0.5), shear=0.01):
    """Rotation-free deformation paths for surrogate training: per cell, an upper-triangular stretch
    R_k = U_k with axial stretch lambda_k (increments ~ U[0, rate_max] per load step along x),
    lateral stretch lambda_k^-nu (nu ~ U[nu]) and small random-walk upper shears.  (ncells, nsteps, 3, 3)."""
    out = np.zeros((ncells, nsteps, 3, 3))
    for c in range(ncells):
        lam, s = 1.0, np.zeros(3)
        rate = rng.uniform(0.0, rate_max)
        v = rng.uniform(*nu)
        for k in range(nsteps):
            lam *= 1.0 + rate * rng.uniform(0.5, 1.5)
            s = s + rng.normal(0.0, shear / np.sqrt(nsteps), 3)
            lt = lam ** (-v)
            out[c, k] = np.array([[lam, s[0], s[1]], [0.0, lt, s[2]], [0.0, 0.0, lt]])
    return out
