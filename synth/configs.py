"""The synthetic r-cell MD workloads, as plain dictionaries of numpy arrays.

Each builder returns {"name", "params", "cells", "F"/"F_path", ...}.  "params" is a dict of the
MD parameters (the same keys for the GPU library and the oracle); "cells" is a list of
{"x", "v", "bonds", "H0"}.  Units: Kremer-Grest in LJ units (epsilon, sigma, m = 1); copper in
eV / Angstrom / amu / fs, where 1 amu*A^2/fs^2 = 103.64269656 eV.

Workloads (their shapes follow the paper's cells; the states are synthetic, not equilibrated):
  kg_single   one 1000-bead KG melt cell (20 x 50), plain FP64, isochoric uniaxial ramp to e=0.2
  cu_element  8 FCC copper cells (4000 atoms each) of one hex8 element, Sutton-Chen EAM, 300 K,
              per-cell uniaxial F to 5 % strain followed by a random rotation
  kg_batched  512 KG cells of 2k-20k beads, chain lengths U{50..200}, F = rotation x stretch
  kg_glassy   100 glassy KG cells (LJ to 2.5 sigma, T = 0.1) of 100 x 100 beads
  fe_bar      256 KG cells x 40 000 beads (400 chains x 100), the r-cells of an 8x2x2 hex8 bar
  fe_tet      KG cells of 100 x 100 beads, one per C3D4 element (the paper's specimen and its
              1000-element scaling system)
"""
import numpy as np

from .deform import rotated_stretch, rotated_uniaxial, random_rotation, uniaxial_isochoric
from .fcc import fcc_lattice
from .kg import kg_melt
from .rng import cell_seed, generator
from .velocities import maxwell_boltzmann

MASTER_SEED = 1902
MVV2E_METAL_FS = 103.64269656   # eV per (amu * Angstrom^2 / fs^2)
KB_EV = 8.617333262e-5          # eV / K
EV_A3_TO_GPA = 160.21766208


def kg_params(**over):
    p = dict(potential="kg", precision="mixed", dt=0.005, temperature=1.0, gamma=0.5, mass=1.0,
             kB=1.0, mvv2e=1.0, rc=2.0 ** (1.0 / 6.0), skin=0.4, lj_eps=1.0, lj_sigma=1.0,
             fene_K=30.0, fene_R0=1.5, sc_eps=0.0, sc_a=0.0, sc_c=0.0, sc_n=0, sc_m=0,
             seed=MASTER_SEED, include_kinetic=1)
    p.update(over)
    return p


def cu_params(**over):
    a = 3.615
    p = dict(potential="sc_eam", precision="mixed", dt=1.0, temperature=300.0, gamma=0.01,
             mass=63.546, kB=KB_EV, mvv2e=MVV2E_METAL_FS, rc=1.95 * a, skin=1.75, lj_eps=0.0,
             lj_sigma=0.0, fene_K=0.0, fene_R0=0.0, sc_eps=1.2382e-2, sc_a=a, sc_c=39.432,
             sc_n=9, sc_m=6, seed=MASTER_SEED, include_kinetic=1)
    p.update(over)
    return p


def kg_glassy_params(**over):
    """Glassy Kremer-Grest: the LJ attraction kept (cut and shifted at 2.5 sigma) at T = 0.1, below
    the glass transition (~0.35); otherwise the standard parameters.  Skin 0.3 sigma: with ~90
    neighbours per bead and little motion at T = 0.1 the pair work, not the rebuilds, sets the cost."""
    p = kg_params(rc=2.5, temperature=0.1, skin=0.3)
    p.update(over)
    return p


def kg_cell(chain_lengths, seed, T=1.0, with_velocities=True):
    x, bonds, H0 = kg_melt(chain_lengths, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5A5A5A5A))
    v = (maxwell_boltzmann(len(x), T, 1.0, 1.0, 1.0, rng) if with_velocities
         else np.zeros_like(x))
    return dict(x=x, v=v, bonds=bonds, H0=H0)


def kg_single(nchains=20, chain_len=50, steps=1000, e_max=0.2, precision="fp64"):
    """One KG cell; F(e_k) = diag(1+e, (1+e)^-1/2, (1+e)^-1/2) with e_k = e_max*k/steps."""
    seed = cell_seed(MASTER_SEED, 0)
    cell = kg_cell([chain_len] * nchains, seed)
    F_path = np.stack([uniaxial_isochoric(e_max * k / steps) for k in range(1, steps + 1)])
    return dict(name="kg_single", params=kg_params(precision=precision), cells=[cell],
                F_path=F_path[:, None, :, :], steps=steps, stress_every=100)


def cu_cell(seed, ncell=10, a=3.615, T=300.0):
    x, H0 = fcc_lattice(ncell, a)
    rng = generator(seed, 1)
    v = maxwell_boltzmann(len(x), T, 63.546, KB_EV, MVV2E_METAL_FS, rng) if T > 0 else np.zeros_like(x)
    return dict(x=x, v=v, bonds=np.zeros((0, 2), np.int32), H0=H0)


def cu_element(ncells=8, ncell=10, load_steps=10, md_per_load=100, eps_max=0.05,
               precision="mixed", T=300.0):
    """8 copper r-cells; F_c(k) = Q_c . diag(1, 1, 1 + eps_max*k/load_steps), k = 1..load_steps."""
    cells, Qs = [], []
    for c in range(ncells):
        s = cell_seed(MASTER_SEED, c)
        cells.append(cu_cell(s, ncell=ncell, T=T))
        Qs.append(random_rotation(generator(s, 2)))
    F_path = np.stack([np.stack([rotated_uniaxial(eps_max * k / load_steps, Qs[c])
                                 for c in range(ncells)]) for k in range(1, load_steps + 1)])
    return dict(name="cu_element", params=cu_params(precision=precision, temperature=T),
                cells=cells, F_path=F_path, steps=load_steps * md_per_load,
                md_per_load=md_per_load, rotations=np.stack(Qs))


def kg_batched_sizes(ncells=512, lo=2000, hi=20000, lmin=50, lmax=200):
    """Per cell: N_target ~ U[lo, hi]; chains of length U{lmin..lmax} appended until sum >= N_target."""
    out = []
    for c in range(ncells):
        rng = generator(MASTER_SEED, c)
        target = int(rng.integers(lo, hi + 1))
        lens, tot = [], 0
        while tot < target:
            l = int(rng.integers(lmin, lmax + 1))
            lens.append(l)
            tot += l
        out.append(lens)
    return out


def kg_batched(ncells=512, lo=2000, hi=20000, precision="mixed", cells_subset=None):
    sizes = kg_batched_sizes(ncells, lo, hi)
    idx = range(ncells) if cells_subset is None else cells_subset
    cells, F = [], []
    for c in idx:
        s = cell_seed(MASTER_SEED, c)
        cells.append(kg_cell(sizes[c], s))
        F.append(rotated_stretch(generator(s, 3)))
    return dict(name="kg_batched", params=kg_params(precision=precision), cells=cells,
                F=np.stack(F), steps=1000)


def kg_glassy(ncells=100, nchains=100, chain_len=100, precision="mixed", cells_subset=None):
    """The size of the paper's production run (100 r-cells of 100 chains x 100 beads, 10^6 beads) with
    the glassy potential; velocities at T = 0.1, each cell under a small isochoric uniaxial stretch."""
    idx = range(ncells) if cells_subset is None else cells_subset
    cells = [kg_cell([chain_len] * nchains, cell_seed(MASTER_SEED + 5, c), T=0.1) for c in idx]
    F = np.stack([uniaxial_isochoric(0.01 * (1 + c % 4), axis=c % 3) for c in idx])
    return dict(name="kg_glassy", params=kg_glassy_params(precision=precision), cells=cells, F=F)


def fe_bar_cells(ncells=256, nchains=400, chain_len=100, precision="mixed", cells_subset=None):
    idx = range(ncells) if cells_subset is None else cells_subset
    cells = [kg_cell([chain_len] * nchains, cell_seed(MASTER_SEED + 4, c)) for c in idx]
    return dict(name="fe_bar", params=kg_params(precision=precision), cells=cells)


def fe_tet_cells(ncells=100, nchains=100, chain_len=100, precision="mixed", cells_subset=None, stream=7):
    """r-cells of the paper's polymer specimen (Sec. 3.2): one per C3D4 element, 100 chains of 100
    beads each (10^4 beads); stream 8 gives the cells of the 1000-element scaling workload."""
    idx = range(ncells) if cells_subset is None else cells_subset
    cells = [kg_cell([chain_len] * nchains, cell_seed(MASTER_SEED + stream, c)) for c in idx]
    return dict(name="fe_tet", params=kg_params(precision=precision), cells=cells)
