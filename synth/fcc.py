"""Perfect FCC lattice in a cubic periodic cell (the copper validation cell of Sec. 3.1:
10 x 10 x 10 conventional cells, 4000 atoms, edge 36.15 Angstrom)."""
import numpy as np

_BASIS = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])


def fcc_lattice(ncell: int = 10, a: float = 3.615):
    """Return (x [4*ncell^3, 3], H0 [3,3]) with H0 = ncell*a*I (columns are box edges)."""
    g = np.arange(ncell, dtype=np.float64)
    ijk = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    x = ((ijk[:, None, :] + _BASIS[None, :, :]) * a).reshape(-1, 3)
    H0 = np.eye(3) * (ncell * a)
    return np.ascontiguousarray(x), H0
