/* rcell.h — C ABI of the batched r-cell molecular-dynamics library for MI355X (gfx950).
 *
 * Method: Murashima, Urata & Li, "Coupling finite element method with LAMMPS for hierarchical
 * multiscale simulations", arXiv:1902.09171.  Every finite-element quadrature point owns a
 * periodic MD representative cell (r-cell).  The FE solver hands each cell a deformation
 * gradient F; the cell's box follows only the upper-triangular stretch R of F = Q R (Sec. 2.1,
 * Eqs. 4-6, 9); MD runs in that box; the time-averaged MD stress is rotated back by Q and
 * converted to the first Piola-Kirchhoff stress (Eqs. 7-8).  This library runs many such cells
 * batched on one GPU.
 *
 * Conventions for every call:
 *  - All functions return an int status: RCELL_OK (0) or a negative RCELL_ERR_* code.  No C++
 *    exception crosses the ABI.  rcell_last_error() gives a human-readable message.
 *  - Host pointers are read (or written) during the call only; the library copies every input.
 *    Pointers named *_dev are device pointers owned by the caller, used on the context's stream.
 *  - Matrices are 3x3 row-major doubles.  F_ij = dx_i / dX_j.  A box matrix H has the cell edge
 *    vectors as its columns, so r = H S for scaled coordinates S in [0,1)^3 (Eq. 1).
 *  - 6-component stresses are Voigt-ordered xx, yy, zz, xy, xz, yz, Cauchy, tension positive,
 *    in the potential's native units (LJ: epsilon/sigma^3; metal units: eV/Angstrom^3).
 *  - A context is used from one host thread at a time; several contexts may coexist.
 *  - Work is enqueued on the context's HIP stream.  rcell_run only enqueues; errors raised on the
 *    device during a run are reported by the next call that synchronises (get_* calls).
 */
#ifndef RCELL_H
#define RCELL_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RCELL_OK = 0,
  RCELL_ERR_ARG = -1,        /* invalid argument, null pointer, unknown option */
  RCELL_ERR_BAD_F = -2,      /* F non-finite, det F <= 0, or some R_ii < 1e-12 |F|_F */
  RCELL_ERR_BOX = -3,        /* a perpendicular cell width w satisfies w/2 < rc + skin */
  RCELL_ERR_BOND = -4,       /* a FENE bond reached r >= R0 */
  RCELL_ERR_NONFINITE = -5,  /* a returned stress is not finite */
  RCELL_ERR_OOM = -6,        /* device or host allocation failed, or a neighbour list beyond 2^32 entries */
  RCELL_ERR_DEVICE = -7,     /* a HIP runtime call failed */
  RCELL_ERR_STATE = -8       /* invalid state (bad box in set_state, neighbour capacity exceeded) */
};
enum { RCELL_POT_KG = 1, RCELL_POT_SC_EAM = 2 };
enum { RCELL_PREC_FP64 = 0, RCELL_PREC_MIXED = 1 };

typedef struct {
  int32_t potential;       /* RCELL_POT_KG: Kremer-Grest bead-spring (Sec. 3.2); RCELL_POT_SC_EAM:
                              Sutton-Chen embedded atom (stand-in for the copper EAM of Sec. 3.1) */
  int32_t precision;       /* RCELL_PREC_MIXED: FP32 pair forces, FP64 positions, velocities,
                              integration and stress; RCELL_PREC_FP64: everything in FP64 */
  double dt;               /* time step */
  double temperature;      /* Langevin target temperature */
  double gamma;            /* Langevin friction rate (1/time); 0 gives plain velocity Verlet */
  double mass;             /* particle mass */
  double kB;               /* Boltzmann constant in energy units per temperature unit */
  double mvv2e;            /* energy of mass*velocity^2 (1 in LJ units; 103.64269656 eV per
                              amu*A^2/fs^2 in metal units with fs) */
  double rc;               /* interaction cutoff */
  double skin;             /* neighbour-list skin; the list is rebuilt when an atom of the cell
                              has moved more than skin/2 since the last build */
  double lj_eps, lj_sigma; /* KG: LJ truncated at rc and shifted to zero there (WCA at 2^(1/6)) */
  double fene_K, fene_R0;  /* KG: FENE bonds U = -K R0^2/2 ln(1 - (r/R0)^2) */
  double sc_eps, sc_a, sc_c; /* Sutton-Chen: E = sum_i [1/2 sum_j eps phi(r_ij) - eps c sqrt(rho_i)] */
  int32_t sc_n, sc_m;      /* phi = (a/r)^n - (a/rc)^n, rho_i = sum_j (a/r)^m - (a/rc)^m; 1..31 */
  uint64_t seed;           /* Philox4x32-10 key = (low, high 32 bits of seed) */
  int32_t include_kinetic; /* 1: sigma includes -sum m v (x) v / V (thermal r-cells) */
} rcell_params;

typedef struct {           /* one cell, host arrays copied at create */
  int32_t natoms;          /* >= 1 */
  int32_t nbonds;          /* number of FENE bonds (KG), 0 otherwise */
  const double* H0;        /* 9, upper triangular with positive diagonal: initial box H(0) */
  const double* x;         /* natoms*3 positions (any periodic image; wrapped into the box) */
  const double* v;         /* natoms*3 velocities, or NULL: Maxwell-Boltzmann at the temperature,
                              drawn on the device from the seed (see rcell_create) */
  const int32_t* bonds;    /* nbonds*2 atom indices within the cell, or NULL; at most 4 bonds per atom */
} rcell_cell_init;

typedef struct rcell_ctx rcell_ctx;

/* Create a batch of ncells r-cells on the current HIP device.  hip_stream: a hipStream_t to
 * enqueue on (e.g. torch.cuda.current_stream().cuda_stream), or NULL for a library-owned
 * stream.  Validates the boxes (RCELL_ERR_BOX), bond lengths (RCELL_ERR_BOND) and indices, then
 * computes the initial forces and the instantaneous stress.  Before any rcell_set_deformation
 * the cells have F = Q = R = I.  A cell given v == NULL starts from Maxwell-Boltzmann
 * velocities: atom l of cell c takes the four words of Philox4x32-10 at counter
 * (l, c, 0xFFFFFFFF, 0xFFFFFFFF) (a counter that the Langevin noise, whose third word is the
 * step, never reaches), mapped to (0,1) as (w + 1/2) 2^-32, two Box-Muller pairs give its three
 * Cartesian components (the fourth normal is unused); the cell's mean velocity is removed and the
 * velocities are scaled so that mvv2e sum m v.v = (3 N - 3) kB T exactly.  On failure *out is NULL
 * and everything the call allocated is freed.  For tests of that path, the environment variable
 * RCELL_FAULT_ALLOC = k (k >= 1) makes the k-th device allocation of the call fail as if the device
 * were out of memory (RCELL_ERR_OOM). */
int rcell_create(const rcell_params* params, const rcell_cell_init* cells, int32_t ncells,
                 void* hip_stream, rcell_ctx** out);

/* Eqs. (4), (5), (9) of Sec. 2.1: per cell, F = Q R by Gram-Schmidt with R_ii > 0; the box is
 * updated incrementally by Delta R = R R_prev^-1 (H <- Delta R H, kept within half-tilt bounds by
 * lattice-preserving basis changes) and every position is mapped by Delta R (affine remap,
 * velocities unchanged); then R_prev <- R, forces are recomputed (conservative part only) and
 * the stress window is cleared.  F: ncells*9 host doubles.  Every cell is validated before any
 * state changes: on RCELL_ERR_BAD_F or RCELL_ERR_BOX no cell is modified.  Synchronises. */
int rcell_set_deformation(rcell_ctx* ctx, const double* F);

/* As rcell_set_deformation, with F (ncells*9 doubles) in device memory. */
int rcell_set_deformation_dev(rcell_ctx* ctx, const void* F_dev);

/* Advance every cell by nsteps velocity-Verlet steps with the Langevin thermostat; after each
 * step the MD stress sigma_MD = (W - sum m v (x) v)/V (pair virial W of Eq. 15) is added to the
 * cell's averaging window.  Only enqueues; device-side errors (FENE bond r >= R0, neighbour
 * capacity) set the cell's status and are returned by the next synchronising call. */
int rcell_run(rcell_ctx* ctx, int32_t nsteps);

/* Molecular statics (Sec. 2.1, Eqs. 16-20): relax every cell's atoms in its current box to a
 * minimum of the potential energy, starting from the current positions - after a deformation these
 * are the affine (Cauchy-Born) guess F H(0) S(t-1) of Eq. 17 - so that the next get_stress returns
 * the 0 K stress of the relaxed configuration (Eq. 20 equals J sigma F^-T of its virial stress).
 * Minimiser: FIRE (Bitzek et al., Phys. Rev. Lett. 97, 170201 (2006)); per cell, iterations until
 * max_i |f_i| <= ftol (force units) or max_iter moves.  Afterwards velocities are zero, the stored
 * force is the conservative one, the averaging window is empty and holds the relaxed stress as its
 * last sample, and the MD step counter is unchanged (a later rcell_run continues MD from here).
 * iters: ncells host int32 receiving the moves each cell used (or NULL).  Synchronises; returns
 * RCELL_ERR_ARG for max_iter < 0 or ftol <= 0, else the first per-cell error status. */
int rcell_minimize(rcell_ctx* ctx, int32_t max_iter, double ftol, int32_t* iters);

/* Window average of sigma_MD since the last get_stress / set_deformation (or the instantaneous
 * stress if the window is empty), rotated to the FE frame sigma_FEM = Q sigma Q^T (Eq. 7), and
 * the first Piola-Kirchhoff stress P = J sigma_FEM F^-T (Eq. 8).  sigma: ncells*6 host doubles;
 * P: ncells*9 host doubles or NULL.  Clears the window.  Synchronises; returns the first
 * per-cell error status if any (RCELL_ERR_NONFINITE for a non-finite stress). */
int rcell_get_stress(rcell_ctx* ctx, double* sigma, double* P);

/* As rcell_get_stress, and also the window-averaged stress in the MD frame (before the rotation of
 * Eq. 7) into sigma_md (ncells*6 host doubles, or NULL).  Clears the window once. */
int rcell_get_stress_ext(rcell_ctx* ctx, double* sigma, double* P, double* sigma_md);

/* As rcell_get_stress, writing ncells*6 (and ncells*9, if P_dev is not NULL) doubles to
 * caller-owned device memory, enqueued on the context's stream; does not synchronise. */
int rcell_get_stress_dev(rcell_ctx* ctx, void* sigma_dev, void* P_dev);

/* Free every device and host resource of the context.  Always safe, also on NULL. */
int rcell_destroy(rcell_ctx* ctx);

/* Message of the last error on this context (or of the last failed create when ctx is NULL). */
const char* rcell_last_error(const rcell_ctx* ctx);

/* ---- diagnostics, checkpointing and test hooks (all synchronise) ---- */
/* per-cell status codes (0 or RCELL_ERR_*), ncells int32 */
int rcell_get_status(rcell_ctx* ctx, int32_t* status);
/* total force of the last completed step (or the conservative force after create /
 * set_deformation / set_state), natoms*3 doubles, original atom order */
int rcell_get_forces(rcell_ctx* ctx, int32_t cell, double* f);
/* state of one cell: x, v natoms*3; H 9; Rprev 9; step.  Any pointer may be NULL. */
int rcell_get_state(rcell_ctx* ctx, int32_t cell, double* x, double* v, double* H, double* Rprev,
                    int64_t* step);
/* overwrite the state of one cell (checkpoint restore); recomputes its conservative forces and
 * clears its window.  The Langevin part of the last step's total force is not part of the state,
 * so the first half kick after a restore uses the conservative force alone: two runs restored
 * from the same state agree bit for bit, but not with the run that was never interrupted.
 * H must be upper triangular with w/2 >= rc + skin (else RCELL_ERR_STATE / _BOX). */
int rcell_set_state(rcell_ctx* ctx, int32_t cell, const double* x, const double* v, const double* H,
                    const double* Rprev, int64_t step);
/* potential energy of the last force evaluation and kinetic energy 1/2 sum m v^2, ncells each */
int rcell_get_energy(rcell_ctx* ctx, double* pe, double* ke);
/* box H, rotation Q, stretch R (9 each) and J = det F of one cell; any pointer may be NULL */
int rcell_get_box(rcell_ctx* ctx, int32_t cell, double* H, double* Q, double* R, double* J);
/* neighbour-list rebuilds performed so far, summed over cells */
int rcell_get_rebuilds(rcell_ctx* ctx, int64_t* count);
/* choose the lanes-per-atom of the force kernels: 0 = autotune by timing each variant's MD-step
 * force pass on copies of the current positions, velocities and forces (advances no state; holds a
 * temporary device buffer of 72 bytes per atom during the call, RCELL_ERR_OOM if it cannot be
 * allocated), or 1, 2, 4, 8, 16 */
int rcell_set_lanes(rcell_ctx* ctx, int32_t lanes);
/* How a neighbour rebuild prepares its cells (binning, bin order, reordering the atoms by bin):
 * mode 1 runs all of it in one launch with one block per cell (every cell must have at most 4096
 * atoms, else RCELL_ERR_ARG), mode 2 in six launches over the tiles of the cells that rebuild,
 * mode 0 (the default) picks 1 when every cell is small enough.  Results are identical either way;
 * mode 1 also runs the per-cell reduction of each MD step in the same launch, which makes a step
 * six launches shorter. */
int rcell_set_build_mode(rcell_ctx* ctx, int32_t mode);
int rcell_get_lanes(rcell_ctx* ctx, int32_t* lanes);
/* Width of the neighbour-build bins: at least (rc + skin) / f along every perpendicular box width,
 * with a stencil of +- f bins (f = 1, the default, or 2; else RCELL_ERR_ARG).  Narrower bins give
 * fewer candidates per atom for wider skins, more bins to scan.  Takes effect at each cell's next
 * neighbour build; the list in place stays valid.  The pair set within rc never depends on it. */
int rcell_set_bin_factor(rcell_ctx* ctx, int32_t f);
int rcell_get_bin_factor(rcell_ctx* ctx, int32_t* f);
/* Autotune of the batch engine: the bin factor, by rebuilding every cell at its current positions
 * with each factor (best of three timed rounds), and then the lanes per atom as rcell_set_lanes(0)
 * does.  The per-atom state, the list and the cell table are copied aside before the trials and
 * copied back after them (a temporary device buffer of ~100 bytes per atom plus the list,
 * RCELL_ERR_OOM if it cannot be allocated), so the state and the trajectory that follows are those
 * of rcell_set_lanes / rcell_set_bin_factor called with the chosen values.  use_cache != 0 reuses
 * the choice of an earlier call in this process with the same potential, precision, list width,
 * skin, densest cell and cell / batch size ranges instead of timing again.  lanes and bin_factor
 * (either may be NULL) receive the choice. */
int rcell_autotune(rcell_ctx* ctx, int32_t use_cache, int32_t* lanes, int32_t* bin_factor);
/* MD steps inside a run are replayed from captured HIP graphs of `steps` steps (even; default
 * 10); 0 launches every kernel individually.  Results are identical either way. */
int rcell_set_graph_steps(rcell_ctx* ctx, int32_t steps);
/* kernel timing: while enabled, each launch of the pair-force pass (which = 0: the force kernel
 * with the fused Langevin/Verlet update; which = 1: the EAM density pass) carries the start and
 * stop HIP events of its own dispatch (hipExtLaunchKernel: the kernel's duration, without launch
 * latency), on the context's stream; 8192 events are created when enabling, and graphs are not
 * used meanwhile.  rcell_prof_read synchronises, returns the summed duration in milliseconds and
 * the number of launches since the last read, and resets both. */
int rcell_prof_enable(rcell_ctx* ctx, int32_t on);
int rcell_prof_read(rcell_ctx* ctx, int32_t which, double* total_ms, int64_t* launches);

/* ---- stateless coupling utilities (no context; enqueued on hip_stream, NULL = null stream) ---- */
/* Eq. (4) for n deformation gradients in device memory (n*9 doubles, row-major): Q and R (n*9
 * doubles each, device) by the same Gram-Schmidt as rcell_set_deformation; status_dev (n int32,
 * device, or NULL) receives 0 or RCELL_ERR_BAD_F per F (Q, R zero for a bad F). */
int rcell_qr_dev(const void* F_dev, int32_t n, void* Q_dev, void* R_dev, void* status_dev, void* hip_stream);
/* Eqs. (7), (8) for n MD-frame stresses (n*6 Voigt doubles, device) and their F (n*9, device):
 * sigma_FEM = Q sigma_MD Q^T (n*6) and, if P_dev is not NULL, P = J sigma_FEM F^-T (n*9); NaN
 * for a bad F.  Used by the surrogate path, whose stresses come from the network. */
int rcell_stress_return_dev(const void* F_dev, const void* sigma_md_dev, int32_t n, void* sigma_fem_dev, void* P_dev,
                            void* hip_stream);

/* ---- measured machine peaks (no context) ---- */
/* Times, on hip_stream (NULL = null stream), a device copy of copy_bytes (read + write; two
 * buffers of that size are allocated and freed) and independent FP32 FMA chains on every CU (built
 * without packed FP32, like the MD kernels), each after one warm-up launch.  copy_gbs receives the
 * copy's read + write bandwidth in GB/s, fma_tflops the FP32 FMA rate in TFLOP/s (FMA = 2 FLOP).
 * Synchronises.  RCELL_ERR_ARG for null outputs or copy_bytes < 16, RCELL_ERR_OOM if the buffers
 * cannot be allocated. */
int rcell_probe_peaks(size_t copy_bytes, double* copy_gbs, double* fma_tflops, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
