"""Maxwell-Boltzmann initial velocities with the centre-of-mass momentum removed and the
kinetic energy rescaled to exactly (3N-3)/2 kB T."""
import numpy as np


def maxwell_boltzmann(n: int, T: float, mass: float, kB: float, mvv2e: float,
                      rng: np.random.Generator) -> np.ndarray:
    if n == 0:
        return np.zeros((0, 3))
    v = rng.standard_normal((n, 3)) * np.sqrt(kB * T / (mass * mvv2e))
    v -= v.mean(axis=0, keepdims=True)
    dof = 3 * n - 3
    if dof <= 0 or T <= 0.0:
        return np.zeros((n, 3)) if T <= 0.0 else v
    ke = 0.5 * mass * mvv2e * float((v * v).sum())
    v *= np.sqrt(0.5 * dof * kB * T / ke)
    return np.ascontiguousarray(v)
