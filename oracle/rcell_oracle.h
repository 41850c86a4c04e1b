/* FP64 CPU oracle for batched r-cell molecular dynamics.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg may load this library.  It shares no code with the GPU library: it has its own
 * header, its own types and its own implementation of every step, written plainly in double
 * precision from the paper's equations and the readings listed in the oracle's source.
 *
 * Status codes mirror the library's documented values: 0 ok, -1 bad argument, -2 bad F,
 * -3 box too small for the cutoff, -4 FENE bond at or beyond R0, -5 non-finite stress,
 * -6 out of memory, -8 bad state.
 */
#ifndef RCELL_ORACLE_H
#define RCELL_ORACLE_H
#include <stdint.h>

typedef struct {
  int32_t potential;        /* 1 Kremer-Grest (truncated-shifted LJ + FENE), 2 Sutton-Chen EAM */
  int32_t include_kinetic;  /* 1: sigma includes -sum m v (x) v / V */
  double dt, temperature, gamma, mass, kB, mvv2e;
  double rc, skin;
  double lj_eps, lj_sigma, fene_K, fene_R0;
  double sc_eps, sc_a, sc_c;
  int32_t sc_n, sc_m;
  uint64_t seed;
} orc_params;

typedef struct orc_ctx orc_ctx;

/* pure functions */
int  orc_qr(const double F[9], double Q[9], double R[9]);
void orc_lattice_reduce(double H[9]);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int  orc_pairs(const double H[9], int32_t n, const double* x, double rc,
               int64_t cap, int32_t* ij, double* d, int64_t* npairs);
int  orc_stress_to_fem(const double F[9], const double sigma_md[6], double sigma_fem[6], double P[9]);
int  orc_forces(const orc_params* p, const double H[9], int32_t n, const double* x,
                int32_t nbonds, const int32_t* bonds, double* f, double* pe, double vir[9]);

/* batched r-cell context (same semantics as the library's create / set_deformation / run /
 * get_stress calls); v == NULL draws Maxwell-Boltzmann velocities for every cell from the seed */
int  orc_create(const orc_params* p, int32_t ncells, const int32_t* natoms, const int32_t* nbonds,
                const double* H0, const double* x, const double* v, const int32_t* bonds,
                orc_ctx** out);
int  orc_set_deformation(orc_ctx* c, const double* F);
int  orc_set_cell_ids(orc_ctx* c, const int32_t* ids);   /* noise-counter index of each cell */
int  orc_run(orc_ctx* c, int32_t nsteps);
int  orc_minimize(orc_ctx* c, int32_t max_iter, double ftol, int32_t* iters);   /* statics, FIRE */
int  orc_get_stress(orc_ctx* c, double* sigma, double* P);
int  orc_get_status(orc_ctx* c, int32_t* status);
int  orc_get_forces(orc_ctx* c, int32_t cell, double* f);
int  orc_get_state(orc_ctx* c, int32_t cell, double* x, double* v, double* H, double* Rprev,
                   int64_t* step);
int  orc_set_state(orc_ctx* c, int32_t cell, const double* x, const double* v, const double* H,
                   const double* Rprev, int64_t step);
int  orc_get_energy(orc_ctx* c, double* pe, double* ke);
int  orc_get_box(orc_ctx* c, int32_t cell, double* H, double* Q, double* R, double* J);
const char* orc_last_error(const orc_ctx* c);
void orc_destroy(orc_ctx* c);
int  orc_threads(int32_t n);

#endif
