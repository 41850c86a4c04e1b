/* FP64 CPU oracle for batched r-cell MD (Murashima, Urata & Li, arXiv:1902.09171).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the benchmark's CPU
 * baseline leg, never by the GPU library.  Shares no code with it.  Plain double precision,
 * no blocking, no fusion, no neighbour skin: every force evaluation enumerates the exact pair
 * set within the cutoff from scratch.
 *
 * What each part follows:
 *   orc_qr              Eq. (4), Sec. 2.1: F = Q R by Gram-Schmidt (classical, with one
 *                       re-orthogonalisation pass), R with positive diagonal.
 *   orc_lattice_reduce  box bookkeeping that keeps the triangular box of Eq. (5) within half-tilt
 *                       bounds by unimodular changes of basis (the lattice is unchanged).
 *   set_deformation     Eqs. (4), (5), (9): Delta R = R(t) R(t-1)^-1, box and positions mapped by
 *                       Delta R (affine remap), velocities unchanged.
 *   orc_pairs           exact pair set {(i, j, image n): |x_j + H n - x_i| < rc}, Eq. (1) r = H S.
 *   orc_forces          Kremer-Grest (Sec. 3.2): LJ truncated at rc and shifted to zero there
 *                       (WCA at rc = 2^(1/6) sigma) on every pair, FENE on bonds.
 *                       Sutton-Chen EAM (stand-in for the copper EAM of Sec. 3.1): pair term
 *                       eps*phi, embedding -eps*c*sqrt(rho), phi and rho shifted to zero at rc.
 *                       Pair virial W = sum_{pairs} g d (x) d / r with g = dE/dr, Eq. (15).
 *   run                 velocity Verlet with Langevin drag and uniform noise (noise mean removed
 *                       per cell), stress sampled after every completed step.
 *   get_stress          window average, sigma_FEM = Q sigma Q^T (Eq. 7), P = J sigma_FEM F^-T (Eq. 8).
 */
#include "rcell_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OK = 0, E_ARG = -1, E_BAD_F = -2, E_BOX = -3, E_BOND = -4, E_NONFINITE = -5, E_OOM = -6,
       E_STATE = -8 };

/* ---------------------------------------------------------------- small 3x3 helpers (row-major) */
static double det3(const double A[9]) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}
static void inv3(const double A[9], double B[9]) {
  double d = det3(A);
  B[0] = (A[4] * A[8] - A[5] * A[7]) / d;
  B[1] = (A[2] * A[7] - A[1] * A[8]) / d;
  B[2] = (A[1] * A[5] - A[2] * A[4]) / d;
  B[3] = (A[5] * A[6] - A[3] * A[8]) / d;
  B[4] = (A[0] * A[8] - A[2] * A[6]) / d;
  B[5] = (A[2] * A[3] - A[0] * A[5]) / d;
  B[6] = (A[3] * A[7] - A[4] * A[6]) / d;
  B[7] = (A[1] * A[6] - A[0] * A[7]) / d;
  B[8] = (A[0] * A[4] - A[1] * A[3]) / d;
}
static void mul3(const double A[9], const double B[9], double C[9]) {
  double T[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
  memcpy(C, T, sizeof T);
}
static void matvec(const double A[9], const double v[3], double out[3]) {
  double t[3];
  for (int i = 0; i < 3; ++i) t[i] = A[3 * i] * v[0] + A[3 * i + 1] * v[1] + A[3 * i + 2] * v[2];
  out[0] = t[0]; out[1] = t[1]; out[2] = t[2];
}
static void eye3(double A[9]) { memset(A, 0, 9 * sizeof(double)); A[0] = A[4] = A[8] = 1.0; }
/* component a of H k (a lattice vector for integer k) */
static double H_dot(const double H[9], int a, const double k[3]) {
  return H[3 * a] * k[0] + H[3 * a + 1] * k[1] + H[3 * a + 2] * k[2];
}

/* perpendicular widths of the cell spanned by the columns of H: w_k = V / |a_i x a_j| */
static void widths(const double H[9], double w[3]) {
  double c[3][3];
  for (int k = 0; k < 3; ++k) for (int a = 0; a < 3; ++a) c[k][a] = H[3 * a + k];
  double V = fabs(det3(H));
  for (int k = 0; k < 3; ++k) {
    const double* u = c[(k + 1) % 3]; const double* v = c[(k + 2) % 3];
    double x = u[1] * v[2] - u[2] * v[1], y = u[2] * v[0] - u[0] * v[2], z = u[0] * v[1] - u[1] * v[0];
    w[k] = V / sqrt(x * x + y * y + z * z);
  }
}

/* ---------------------------------------------------------------- Eq. (4): QR by Gram-Schmidt */
int orc_qr(const double F[9], double Q[9], double R[9]) {
  double nrm = 0;
  for (int k = 0; k < 9; ++k) { if (!isfinite(F[k])) return E_BAD_F; nrm += F[k] * F[k]; }
  nrm = sqrt(nrm);
  if (!(det3(F) > 0.0)) return E_BAD_F;
  double q[3][3], r[3][3] = {{0}};
  for (int j = 0; j < 3; ++j) {
    double v[3] = {F[j], F[3 + j], F[6 + j]};              /* column j of F */
    for (int pass = 0; pass < 2; ++pass)                      /* classical GS, then one re-orthogonalisation */
      for (int i = 0; i < j; ++i) {
        double s = q[i][0] * v[0] + q[i][1] * v[1] + q[i][2] * v[2];
        r[i][j] += s;
        v[0] -= s * q[i][0]; v[1] -= s * q[i][1]; v[2] -= s * q[i][2];
      }
    r[j][j] = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (!(r[j][j] >= 1e-12 * nrm)) return E_BAD_F;
    for (int a = 0; a < 3; ++a) q[j][a] = v[a] / r[j][j];
  }
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 3; ++j) { Q[3 * a + j] = q[j][a]; R[3 * a + j] = r[a][j]; }
  return OK;
}

/* Keep an upper-triangular box within half-tilt bounds: c -= k b (yz), c -= k a (xz), b -= k a (xy),
 * each applied only when the tilt exceeds half of the edge it is measured against. */
void orc_lattice_reduce(double H[9]) {
  double lx = H[0], ly = H[4];
  if (fabs(H[5]) > 0.5 * ly) {                 /* yz */
    double k = floor(H[5] / ly + 0.5);
    H[2] -= k * H[1]; H[5] -= k * H[4];
  }
  if (fabs(H[2]) > 0.5 * lx) {                 /* xz */
    double k = floor(H[2] / lx + 0.5);
    H[2] -= k * H[0];
  }
  if (fabs(H[1]) > 0.5 * lx) {                 /* xy */
    double k = floor(H[1] / lx + 0.5);
    H[1] -= k * H[0];
  }
}

/* ---------------------------------------------------------------- Philox4x32-10 (Salmon et al., SC'11) */
static inline void mulhilo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32); *lo = (uint32_t)p;
}
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo(0xD2511F53u, c0, &hi0, &lo0);
    mulhilo(0xCD9E8D57u, c2, &hi1, &lo1);
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ---------------------------------------------------------------- exact pair enumeration */
typedef struct { int32_t i, j; double d[3]; double r; } pair_t;
typedef struct { pair_t* p; int64_t n, cap; } pairlist;

static int push_pair(pairlist* L, int32_t i, int32_t j, const double d[3], double r) {
  if (L->n == L->cap) {
    int64_t nc = L->cap ? 2 * L->cap : 1024;
    pair_t* np = (pair_t*)realloc(L->p, (size_t)nc * sizeof(pair_t));
    if (!np) return E_OOM;
    L->p = np; L->cap = nc;
  }
  pair_t* q = &L->p[L->n++];
  q->i = i; q->j = j; q->d[0] = d[0]; q->d[1] = d[1]; q->d[2] = d[2]; q->r = r;
  return OK;
}

/* d = x_j + H n - x_i */
static void image_sep(const double H[9], const double* xi, const double* xj, const double n[3], double d[3]) {
  for (int a = 0; a < 3; ++a)
    d[a] = (xj[a] - xi[a]) + (H[3 * a] * n[0] + H[3 * a + 1] * n[1] + H[3 * a + 2] * n[2]);
}

/* Every (i, j, n) with |x_j + H n - x_i| < rc, each unordered interaction once: i < j with every
 * image n, and i == j with n != 0 taken from one half of the image lattice.  Large cells
 * (every perpendicular width >= 3 rc) use a cell list in scaled coordinates; otherwise all
 * pairs are scanned over every image that can reach rc. */
static int build_pairs(const double H[9], int32_t n, const double* x, double rc, pairlist* L) {
  L->n = 0;
  if (n <= 0) return OK;
  double Hi[9], w[3];
  inv3(H, Hi);
  widths(H, w);
  double rc2 = rc * rc;
  double* S = (double*)malloc((size_t)n * 3 * sizeof(double));
  if (!S) return E_OOM;
  for (int32_t i = 0; i < n; ++i) matvec(Hi, &x[3 * i], &S[3 * i]);
  int rc_status = OK;
  if (w[0] >= 3 * rc && w[1] >= 3 * rc && w[2] >= 3 * rc) {
    int nb[3];
    for (int k = 0; k < 3; ++k) nb[k] = (int)floor(w[k] / rc);
    int64_t nbins = (int64_t)nb[0] * nb[1] * nb[2];
    int32_t* head = (int32_t*)malloc((size_t)nbins * sizeof(int32_t));
    int32_t* next = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* bin = (int32_t*)malloc((size_t)n * 3 * sizeof(int32_t));
    if (!head || !next || !bin) { free(head); free(next); free(bin); free(S); return E_OOM; }
    for (int64_t b = 0; b < nbins; ++b) head[b] = -1;
    for (int32_t i = n - 1; i >= 0; --i) {
      for (int k = 0; k < 3; ++k) {
        double s = S[3 * i + k] - floor(S[3 * i + k]);
        int b = (int)floor(s * nb[k]);
        if (b >= nb[k]) b = nb[k] - 1;
        if (b < 0) b = 0;
        bin[3 * i + k] = b;
      }
      int64_t id = ((int64_t)bin[3 * i] * nb[1] + bin[3 * i + 1]) * nb[2] + bin[3 * i + 2];
      next[i] = head[id]; head[id] = i;
    }
    for (int32_t i = 0; i < n && rc_status == OK; ++i)
      for (int o0 = -1; o0 <= 1; ++o0)
        for (int o1 = -1; o1 <= 1; ++o1)
          for (int o2 = -1; o2 <= 1; ++o2) {
            int b0 = (bin[3 * i] + o0 + nb[0]) % nb[0], b1 = (bin[3 * i + 1] + o1 + nb[1]) % nb[1],
                b2 = (bin[3 * i + 2] + o2 + nb[2]) % nb[2];
            for (int32_t j = head[((int64_t)b0 * nb[1] + b1) * nb[2] + b2]; j >= 0; j = next[j]) {
              if (j <= i) continue;
              double im[3], d[3];
              for (int k = 0; k < 3; ++k) im[k] = -nearbyint(S[3 * j + k] - S[3 * i + k]);
              image_sep(H, &x[3 * i], &x[3 * j], im, d);
              double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
              if (r2 < rc2) rc_status = push_pair(L, i, j, d, sqrt(r2));
            }
          }
    free(head); free(next); free(bin);
  } else {
    int m[3];
    for (int k = 0; k < 3; ++k) m[k] = (int)ceil(rc / w[k]) + 1;
    for (int32_t i = 0; i < n && rc_status == OK; ++i)
      for (int32_t j = i; j < n; ++j) {
        double c[3];
        for (int k = 0; k < 3; ++k) c[k] = -nearbyint(S[3 * j + k] - S[3 * i + k]);
        for (int a = -m[0]; a <= m[0]; ++a)
          for (int b = -m[1]; b <= m[1]; ++b)
            for (int e = -m[2]; e <= m[2]; ++e) {
              double im[3] = {c[0] + a, c[1] + b, c[2] + e};
              if (i == j) {  /* self images: n != 0, first non-zero component positive */
                if (im[0] == 0 && im[1] == 0 && im[2] == 0) continue;
                if (im[0] < 0 || (im[0] == 0 && (im[1] < 0 || (im[1] == 0 && im[2] < 0)))) continue;
              }
              double d[3];
              image_sep(H, &x[3 * i], &x[3 * j], im, d);
              double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
              if (r2 < rc2) rc_status = push_pair(L, i, j, d, sqrt(r2));
            }
      }
  }
  free(S);
  return rc_status;
}

int orc_pairs(const double H[9], int32_t n, const double* x, double rc, int64_t cap, int32_t* ij,
              double* d, int64_t* npairs) {
  pairlist L = {0};
  int st = build_pairs(H, n, x, rc, &L);
  if (st == OK) {
    *npairs = L.n;
    for (int64_t k = 0; k < L.n && k < cap; ++k) {
      ij[2 * k] = L.p[k].i; ij[2 * k + 1] = L.p[k].j;
      d[3 * k] = L.p[k].d[0]; d[3 * k + 1] = L.p[k].d[1]; d[3 * k + 2] = L.p[k].d[2];
    }
  }
  free(L.p);
  return st;
}

/* ---------------------------------------------------------------- potentials */
/* Accumulate pair interaction g = dU/dr along d = x_j - x_i: f_i += g d/r, f_j -= g d/r,
 * W += g d (x) d / r. */
static void add_pair_force(double* f, double W[9], int32_t i, int32_t j, const double d[3], double r, double g) {
  for (int a = 0; a < 3; ++a) {
    f[3 * i + a] += g * d[a] / r;
    f[3 * j + a] -= g * d[a] / r;
    for (int b = 0; b < 3; ++b) W[3 * a + b] += g * d[a] * d[b] / r;
  }
}

/* Conservative forces, potential energy and pair virial for one cell of box H. */
static int eval_forces(const orc_params* p, const double H[9], int32_t n, const double* x,
                       int32_t nb, const int32_t* bonds, double* f, double* pe, double W[9],
                       pairlist* L) {
  memset(f, 0, (size_t)n * 3 * sizeof(double));
  memset(W, 0, 9 * sizeof(double));
  *pe = 0.0;
  int st = build_pairs(H, n, x, p->rc, L);
  if (st != OK) return st;
  if (p->potential == 1) {
    double e = p->lj_eps, s = p->lj_sigma;
    double src6 = pow(s / p->rc, 6.0);
    double shift = 4.0 * e * (src6 * src6 - src6);
    for (int64_t k = 0; k < L->n; ++k) {
      const pair_t* q = &L->p[k];
      double sr6 = pow(s / q->r, 6.0);
      *pe += 4.0 * e * (sr6 * sr6 - sr6) - shift;
      double g = -24.0 * e * (2.0 * sr6 * sr6 - sr6) / q->r;
      add_pair_force(f, W, q->i, q->j, q->d, q->r, g);
    }
    double Hi[9];
    inv3(H, Hi);
    double K = p->fene_K, R0 = p->fene_R0;
    for (int32_t b = 0; b < nb; ++b) {
      int32_t i = bonds[2 * b], j = bonds[2 * b + 1];
      double si[3], sj[3], im[3], d[3];
      matvec(Hi, &x[3 * i], si);
      matvec(Hi, &x[3 * j], sj);
      for (int a = 0; a < 3; ++a) im[a] = -nearbyint(sj[a] - si[a]);
      image_sep(H, &x[3 * i], &x[3 * j], im, d);
      double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double t = (r / R0) * (r / R0);
      if (!(t < 1.0)) return E_BOND;
      *pe += -0.5 * K * R0 * R0 * log(1.0 - t);
      double g = K * r / (1.0 - t);
      add_pair_force(f, W, i, j, d, r, g);
    }
  } else if (p->potential == 2) {
    double e = p->sc_eps, a = p->sc_a, c = p->sc_c, rc = p->rc;
    double phic = pow(a / rc, p->sc_n), rhoc = pow(a / rc, p->sc_m);
    double* rho = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!rho) return E_OOM;
    for (int64_t k = 0; k < L->n; ++k) {            /* pass 1: host electron densities */
      const pair_t* q = &L->p[k];
      double rr = pow(a / q->r, p->sc_m) - rhoc;
      rho[q->i] += rr; rho[q->j] += rr;
      *pe += e * (pow(a / q->r, p->sc_n) - phic);
    }
    for (int32_t i = 0; i < n; ++i) {
      *pe += -e * c * sqrt(rho[i]);
      rho[i] = rho[i] > 0.0 ? -e * c / (2.0 * sqrt(rho[i])) : 0.0;   /* now F'(rho_i) */
    }
    for (int64_t k = 0; k < L->n; ++k) {            /* pass 2: forces */
      const pair_t* q = &L->p[k];
      double dphi = -(p->sc_n / q->r) * pow(a / q->r, p->sc_n);
      double drho = -(p->sc_m / q->r) * pow(a / q->r, p->sc_m);
      double g = e * dphi + (rho[q->i] + rho[q->j]) * drho;
      add_pair_force(f, W, q->i, q->j, q->d, q->r, g);
    }
    free(rho);
  } else {
    return E_ARG;
  }
  return OK;
}

int orc_forces(const orc_params* p, const double H[9], int32_t n, const double* x, int32_t nbonds,
               const int32_t* bonds, double* f, double* pe, double vir[9]) {
  pairlist L = {0};
  int st = eval_forces(p, H, n, x, nbonds, bonds, f, pe, vir, &L);
  free(L.p);
  return st;
}

/* ---------------------------------------------------------------- batched context */
typedef struct {
  int32_t n, nb;
  double *x, *v, *f;
  int32_t* bonds;
  double H[9], Rprev[9], Q[9], R[9], F[9], J;
  int64_t step;
  double wsum[6], last[6], pe;
  int64_t wcount;
  int32_t status;
  int32_t id;          /* the cell's index in the Langevin noise counter (its batch position) */
  pairlist L;
} ocell;

struct orc_ctx {
  orc_params p;
  int32_t ncells;
  ocell* c;
  char err[256];
};

static void set_err(orc_ctx* c, const char* m) { snprintf(c->err, sizeof c->err, "%s", m); }

static int box_ok(const orc_params* p, const double H[9]) {
  double w[3];
  widths(H, w);
  double wmin = fmin(w[0], fmin(w[1], w[2]));
  return p->rc + p->skin <= 0.5 * wmin;
}

/* sigma_MD = (W - sum m v (x) v) / V, Voigt order xx yy zz xy xz yz; tension positive */
static void sample_stress(const orc_params* p, const ocell* c, const double W[9], double s[6]) {
  double K[9] = {0};
  if (p->include_kinetic)
    for (int32_t i = 0; i < c->n; ++i)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) K[3 * a + b] += p->mass * p->mvv2e * c->v[3 * i + a] * c->v[3 * i + b];
  double V = fabs(det3(c->H));
  static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
  for (int k = 0; k < 6; ++k) s[k] = (W[3 * ia[k] + ib[k]] - K[3 * ia[k] + ib[k]]) / V;
}

/* Conservative forces at the current positions; f holds them afterwards (no Langevin term). */
static int prime(const orc_params* p, ocell* c) {
  double W[9];
  int st = eval_forces(p, c->H, c->n, c->x, c->nb, c->bonds, c->f, &c->pe, W, &c->L);
  if (st != OK) return st;
  sample_stress(p, c, W, c->last);
  return OK;
}

static void wrap_positions(ocell* c) {
  double Hi[9];
  inv3(c->H, Hi);
  for (int32_t i = 0; i < c->n; ++i) {
    double s[3], k[3];
    matvec(Hi, &c->x[3 * i], s);
    for (int a = 0; a < 3; ++a) k[a] = floor(s[a]);
    if (k[0] != 0 || k[1] != 0 || k[2] != 0)
      for (int a = 0; a < 3; ++a) c->x[3 * i + a] -= H_dot(c->H, a, k);
  }
}

/* Initial velocities of a cell created without them: Maxwell-Boltzmann at the temperature T.  Each
 * atom draws four uniform deviates u = (w + 1/2) 2^-32 from Philox4x32-10 (key: the seed; counter:
 * atom index, cell index, and an all-ones step, which the Langevin noise never reaches), and the
 * Box-Muller transform turns (u0, u1) into two and (u2, u3) into one standard normal deviate, scaled
 * by sqrt(kB T / m).  Then the centre-of-mass velocity is subtracted, and all velocities are scaled
 * so that sum m v^2 = (3N - 3) kB T (the equipartition value without the removed momentum). */
static void maxwell_boltzmann(const orc_params* p, ocell* c) {
  const uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
  const double kt_m = p->kB * p->temperature / (p->mass * p->mvv2e);
  const double sd = sqrt(kt_m);
  const double two_pi = 6.283185307179586476925286766559;
  double mean[3] = {0.0, 0.0, 0.0};
  for (int32_t i = 0; i < c->n; ++i) {
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)c->id, 0xFFFFFFFFu, 0xFFFFFFFFu}, w[4];
    orc_philox4x32_10(ctr, key, w);
    double u[4];
    for (int q = 0; q < 4; ++q) u[q] = ((double)w[q] + 0.5) / 4294967296.0;
    double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    c->v[3 * i] = sd * r0 * cos(two_pi * u[1]);
    c->v[3 * i + 1] = sd * r0 * sin(two_pi * u[1]);
    c->v[3 * i + 2] = sd * r1 * cos(two_pi * u[3]);
    for (int q = 0; q < 3; ++q) mean[q] += c->v[3 * i + q];
  }
  double sum2 = 0.0;
  for (int q = 0; q < 3; ++q) mean[q] /= (c->n > 0 ? c->n : 1);
  for (int32_t i = 0; i < c->n; ++i)
    for (int q = 0; q < 3; ++q) {
      c->v[3 * i + q] -= mean[q];
      sum2 += c->v[3 * i + q] * c->v[3 * i + q];
    }
  double scale = (c->n > 1 && sum2 > 0.0) ? sqrt(kt_m * (3.0 * c->n - 3.0) / sum2) : 0.0;
  for (int64_t k = 0; k < 3 * (int64_t)c->n; ++k) c->v[k] *= scale;
}

/* v == NULL: every cell starts from Maxwell-Boltzmann velocities (maxwell_boltzmann) */
int orc_create(const orc_params* p, int32_t ncells, const int32_t* natoms, const int32_t* nbonds,
               const double* H0, const double* x, const double* v, const int32_t* bonds,
               orc_ctx** out) {
  if (!p || !out || ncells < 0 || (ncells > 0 && (!natoms || !nbonds || !H0 || !x))) return E_ARG;
  if (p->potential != 1 && p->potential != 2) return E_ARG;
  orc_ctx* C = (orc_ctx*)calloc(1, sizeof(orc_ctx));
  if (!C) return E_OOM;
  C->p = *p;
  C->ncells = ncells;
  C->c = (ocell*)calloc((size_t)(ncells > 0 ? ncells : 1), sizeof(ocell));
  if (!C->c) { free(C); return E_OOM; }
  int64_t off = 0, boff = 0;
  int st = OK;
  for (int32_t k = 0; k < ncells && st == OK; ++k) {
    ocell* c = &C->c[k];
    c->n = natoms[k]; c->nb = nbonds[k];
    c->id = k;
    if (c->n < 0 || c->nb < 0 || (c->nb > 0 && !bonds)) { st = E_ARG; break; }
    size_t bytes = (size_t)(c->n > 0 ? c->n : 1) * 3 * sizeof(double);
    c->x = (double*)malloc(bytes); c->v = (double*)calloc(1, bytes); c->f = (double*)calloc(1, bytes);
    c->bonds = (int32_t*)malloc((size_t)(c->nb > 0 ? c->nb : 1) * 2 * sizeof(int32_t));
    if (!c->x || !c->v || !c->f || !c->bonds) { st = E_OOM; break; }
    memcpy(c->x, x + 3 * off, (size_t)c->n * 3 * sizeof(double));
    if (v) memcpy(c->v, v + 3 * off, (size_t)c->n * 3 * sizeof(double));
    else maxwell_boltzmann(p, c);
    if (c->nb) memcpy(c->bonds, bonds + 2 * boff, (size_t)c->nb * 2 * sizeof(int32_t));
    for (int32_t b = 0; b < 2 * c->nb; ++b)
      if (c->bonds[b] < 0 || c->bonds[b] >= c->n) st = E_ARG;
    memcpy(c->H, H0 + 9 * k, sizeof c->H);
    eye3(c->Rprev); eye3(c->Q); eye3(c->R); eye3(c->F); c->J = 1.0;
    if (st == OK && !(det3(c->H) > 0.0)) st = E_ARG;
    if (st == OK && !box_ok(p, c->H)) st = E_BOX;
    off += c->n; boff += c->nb;
  }
  for (int32_t k = 0; k < ncells && st == OK; ++k) {
    wrap_positions(&C->c[k]);
    st = prime(&C->p, &C->c[k]);
  }
  if (st != OK) { orc_destroy(C); return st; }
  *out = C;
  return OK;
}

int orc_set_deformation(orc_ctx* C, const double* F) {
  if (!C || !F) return E_ARG;
  int32_t nc = C->ncells;
  double* Q = (double*)malloc((size_t)(nc > 0 ? nc : 1) * 9 * 4 * sizeof(double));
  if (!Q) return E_OOM;
  double *R = Q + 9 * nc, *dR = R + 9 * nc, *Hn = dR + 9 * nc;
  for (int32_t k = 0; k < nc; ++k) {          /* validate every cell before touching any state */
    int st = orc_qr(F + 9 * k, Q + 9 * k, R + 9 * k);
    if (st != OK) { free(Q); set_err(C, "set_deformation: bad F"); return st; }
    double Ri[9];
    inv3(C->c[k].Rprev, Ri);
    mul3(R + 9 * k, Ri, dR + 9 * k);                                  /* Eq. (9) */
    mul3(dR + 9 * k, C->c[k].H, Hn + 9 * k);
    Hn[9 * k + 3] = Hn[9 * k + 6] = Hn[9 * k + 7] = 0.0;   /* product of upper-triangular matrices */
    orc_lattice_reduce(Hn + 9 * k);
    if (!box_ok(&C->p, Hn + 9 * k)) { free(Q); set_err(C, "set_deformation: box too small"); return E_BOX; }
  }
  int st_all = OK;
#pragma omp parallel for schedule(dynamic) reduction(min : st_all)
  for (int32_t k = 0; k < nc; ++k) {
    ocell* c = &C->c[k];
    for (int32_t i = 0; i < c->n; ++i) matvec(dR + 9 * k, &c->x[3 * i], &c->x[3 * i]);
    memcpy(c->H, Hn + 9 * k, sizeof c->H);
    memcpy(c->Rprev, R + 9 * k, sizeof c->Rprev);
    memcpy(c->R, R + 9 * k, sizeof c->R);
    memcpy(c->Q, Q + 9 * k, sizeof c->Q);
    memcpy(c->F, F + 9 * k, sizeof c->F);
    c->J = c->R[0] * c->R[4] * c->R[8];
    memset(c->wsum, 0, sizeof c->wsum); c->wcount = 0;
    wrap_positions(c);
    int st = prime(&C->p, c);
    if (st != OK) { c->status = st; st_all = st; }
  }
  free(Q);
  return st_all;
}

/* One velocity-Verlet step with Langevin thermostat for one cell. */
static int step_cell(const orc_params* p, ocell* c, int32_t cell_index) {
  double h = p->dt / (2.0 * p->mass * p->mvv2e);
  for (int64_t k = 0; k < 3 * (int64_t)c->n; ++k) c->v[k] += h * c->f[k];
  for (int64_t k = 0; k < 3 * (int64_t)c->n; ++k) c->x[k] += p->dt * c->v[k];
  wrap_positions(c);
  double W[9];
  int st = eval_forces(p, c->H, c->n, c->x, c->nb, c->bonds, c->f, &c->pe, W, &c->L);
  if (st != OK) return st;
  int64_t s_new = c->step + 1;
  if (p->gamma > 0.0 && c->n > 0) {
    /* noise: u = (w >> 8) 2^-24 per Philox word; k = (w >> 8) - 2^23 is u - 1/2 in units of 2^-24.
     * The per-cell mean is removed exactly: S = sum k in integers, xi = c24 * (k - S/N). */
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    int64_t S[3] = {0, 0, 0};
    int32_t* kk = (int32_t*)malloc((size_t)c->n * 3 * sizeof(int32_t));
    if (!kk) return E_OOM;
    for (int32_t i = 0; i < c->n; ++i) {
      uint32_t ctr[4] = {(uint32_t)i, (uint32_t)cell_index, (uint32_t)s_new, (uint32_t)((uint64_t)s_new >> 32)}, w[4];
      orc_philox4x32_10(ctr, key, w);
      for (int a = 0; a < 3; ++a) { kk[3 * i + a] = (int32_t)(w[a] >> 8) - (1 << 23); S[a] += kk[3 * i + a]; }
    }
    double c24 = sqrt(24.0 * p->gamma * p->mass * p->kB * p->temperature * p->mvv2e / p->dt) * 0x1.0p-24;
    double drag = -(p->gamma * p->mass * p->mvv2e);
    double mean[3];
    for (int a = 0; a < 3; ++a) mean[a] = (double)S[a] / (double)c->n;
    for (int32_t i = 0; i < c->n; ++i)
      for (int a = 0; a < 3; ++a) {
        double xi = c24 * ((double)kk[3 * i + a] - mean[a]);
        c->f[3 * i + a] = (c->f[3 * i + a] + drag * c->v[3 * i + a]) + xi;
      }
    free(kk);
  }
  for (int64_t k = 0; k < 3 * (int64_t)c->n; ++k) c->v[k] += h * c->f[k];
  double s[6];
  sample_stress(p, c, W, s);
  for (int k = 0; k < 6; ++k) { c->wsum[k] += s[k]; c->last[k] = s[k]; }
  c->wcount += 1;
  c->step = s_new;
  return OK;
}

/* Give the cells other noise-counter indices (default: their position in this context), so that
 * a few cells of a large batch, run here alone, draw the noise they draw inside that batch. */
int orc_set_cell_ids(orc_ctx* C, const int32_t* ids) {
  if (!C || !ids) return E_ARG;
  for (int32_t k = 0; k < C->ncells; ++k) C->c[k].id = ids[k];
  return OK;
}

int orc_run(orc_ctx* C, int32_t nsteps) {
  if (!C || nsteps < 0) return E_ARG;
  int st_all = OK;
#pragma omp parallel for schedule(dynamic) reduction(min : st_all)
  for (int32_t k = 0; k < C->ncells; ++k) {
    ocell* c = &C->c[k];
    for (int32_t s = 0; s < nsteps && c->status == OK; ++s) {
      int st = step_cell(&C->p, c, c->id);
      if (st != OK) c->status = st;
    }
    if (c->status != OK) st_all = c->status;
  }
  return st_all;
}

/* Molecular statics (Sec. 2.1, Eqs. 16-20): relax each cell's atoms in its current box to a minimum
 * of the potential energy, starting from the current positions - after a deformation these are the
 * affine guess F H(0) S(t-1) of Eq. 17 - and return the stress of the relaxed configuration
 * (Eq. 20 is J sigma F^-T of its virial stress, which get_stress returns).  The minimiser is FIRE
 * (Bitzek, Koskinen, Gaehler, Moseler, Gumbsch, Phys. Rev. Lett. 97, 170201 (2006)): per iteration,
 * forces at the current positions; stop when max_i |f_i| <= ftol; if the power P = f.v is positive,
 * the velocity is mixed towards the force, v = (1 - alpha) v + alpha |v| f / |f| (norms over the
 * cell), and after more than 5 such iterations in a row dt grows by 1.1 (at most 10 MD time steps)
 * and alpha shrinks by 0.99; otherwise dt halves, alpha returns to 0.1 and v is zeroed; then
 * v += dt f / m and x += dt v.  dt starts at the MD time step.  Afterwards v = 0, f holds the
 * conservative force, the stress window is empty and its last sample is the relaxed stress. */
int orc_minimize(orc_ctx* C, int32_t max_iter, double ftol, int32_t* iters) {
  if (!C || max_iter < 0 || !(ftol > 0)) return E_ARG;
  int st_all = OK;
#pragma omp parallel for schedule(dynamic) reduction(min : st_all)
  for (int32_t k = 0; k < C->ncells; ++k) {
    ocell* c = &C->c[k];
    const orc_params* p = &C->p;
    const int64_t n3 = 3 * (int64_t)c->n;
    const double inv_m = 1.0 / (p->mass * p->mvv2e), dt_max = 10.0 * p->dt;
    double dt = p->dt, alpha = 0.1, W[9];
    int32_t count = 0, it = 0;
    int st = OK;
    memset(c->v, 0, (size_t)n3 * sizeof(double));
    for (;;) {
      wrap_positions(c);
      st = eval_forces(p, c->H, c->n, c->x, c->nb, c->bonds, c->f, &c->pe, W, &c->L);
      if (st != OK) break;
      double fmax2 = 0.0, P = 0.0, F2 = 0.0, V2 = 0.0;
      for (int32_t i = 0; i < c->n; ++i) {
        const double* f = &c->f[3 * i];
        const double* v = &c->v[3 * i];
        const double f2 = f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
        fmax2 = fmax(fmax2, f2);
        F2 += f2;
        V2 += v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        P += f[0] * v[0] + f[1] * v[1] + f[2] * v[2];
      }
      if (fmax2 <= ftol * ftol || it >= max_iter) break;
      if (P > 0.0) {
        if (++count > 5) { dt = fmin(1.1 * dt, dt_max); alpha *= 0.99; }
        const double a = 1.0 - alpha, b = alpha * sqrt(V2 / F2);
        for (int64_t q = 0; q < n3; ++q) c->v[q] = a * c->v[q] + b * c->f[q];
      } else {
        dt *= 0.5;
        alpha = 0.1;
        count = 0;
        memset(c->v, 0, (size_t)n3 * sizeof(double));
      }
      for (int64_t q = 0; q < n3; ++q) c->v[q] += dt * inv_m * c->f[q];
      for (int64_t q = 0; q < n3; ++q) c->x[q] += dt * c->v[q];
      ++it;
    }
    memset(c->v, 0, (size_t)n3 * sizeof(double));
    if (st == OK) sample_stress(p, c, W, c->last);
    for (int q = 0; q < 6; ++q) c->wsum[q] = 0.0;
    c->wcount = 0;
    if (iters) iters[k] = it;
    if (st != OK) { c->status = st; st_all = st; }
  }
  return st_all;
}

/* sigma_FEM = Q sigma_MD Q^T (Eq. 7) and P = J sigma_FEM F^-T (Eq. 8); Voigt in and out. */
static void stress_return(const double Q[9], const double F[9], double J, const double sv[6],
                          double out6[6], double* P9) {
  static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
  double s[9];
  for (int q = 0; q < 6; ++q) { s[3 * ia[q] + ib[q]] = sv[q]; s[3 * ib[q] + ia[q]] = sv[q]; }
  double Qt[9], t[9], sf[9];
  for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) Qt[3 * a + b] = Q[3 * b + a];
  mul3(Q, s, t);
  mul3(t, Qt, sf);
  for (int q = 0; q < 6; ++q) out6[q] = sf[3 * ia[q] + ib[q]];
  if (P9) {
    double Fi[9], FiT[9], pm[9];
    inv3(F, Fi);
    for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) FiT[3 * a + b] = Fi[3 * b + a];
    mul3(sf, FiT, pm);
    for (int q = 0; q < 9; ++q) P9[q] = J * pm[q];
  }
}

int orc_stress_to_fem(const double F[9], const double sigma_md[6], double sigma_fem[6], double P[9]) {
  double Q[9], R[9];
  int st = orc_qr(F, Q, R);
  if (st != OK) return st;
  stress_return(Q, F, R[0] * R[4] * R[8], sigma_md, sigma_fem, P);
  return OK;
}

int orc_get_stress(orc_ctx* C, double* sigma, double* P) {
  if (!C || !sigma) return E_ARG;
  int st = OK;
  for (int32_t k = 0; k < C->ncells; ++k) {
    ocell* c = &C->c[k];
    double sv[6];
    for (int q = 0; q < 6; ++q) sv[q] = c->wcount > 0 ? c->wsum[q] / (double)c->wcount : c->last[q];
    stress_return(c->Q, c->F, c->J, sv, sigma + 6 * k, P ? P + 9 * k : NULL);
    for (int q = 0; q < 6; ++q)
      if (!isfinite(sigma[6 * k + q])) c->status = E_NONFINITE;
    memset(c->wsum, 0, sizeof c->wsum); c->wcount = 0;
    if (c->status != OK && st == OK) st = c->status;
  }
  return st;
}

int orc_get_status(orc_ctx* C, int32_t* status) {
  if (!C || !status) return E_ARG;
  for (int32_t k = 0; k < C->ncells; ++k) status[k] = C->c[k].status;
  return OK;
}

int orc_get_forces(orc_ctx* C, int32_t cell, double* f) {
  if (!C || !f || cell < 0 || cell >= C->ncells) return E_ARG;
  memcpy(f, C->c[cell].f, (size_t)C->c[cell].n * 3 * sizeof(double));
  return OK;
}

int orc_get_state(orc_ctx* C, int32_t cell, double* x, double* v, double* H, double* Rprev, int64_t* step) {
  if (!C || cell < 0 || cell >= C->ncells) return E_ARG;
  ocell* c = &C->c[cell];
  if (x) memcpy(x, c->x, (size_t)c->n * 3 * sizeof(double));
  if (v) memcpy(v, c->v, (size_t)c->n * 3 * sizeof(double));
  if (H) memcpy(H, c->H, sizeof c->H);
  if (Rprev) memcpy(Rprev, c->Rprev, sizeof c->Rprev);
  if (step) *step = c->step;
  return OK;
}

int orc_set_state(orc_ctx* C, int32_t cell, const double* x, const double* v, const double* H,
                  const double* Rprev, int64_t step) {
  if (!C || cell < 0 || cell >= C->ncells || !x || !v || !H || !Rprev) return E_ARG;
  ocell* c = &C->c[cell];
  if (!(det3(H) > 0.0) || H[3] != 0.0 || H[6] != 0.0 || H[7] != 0.0) return E_STATE;
  if (!box_ok(&C->p, H)) return E_BOX;
  memcpy(c->x, x, (size_t)c->n * 3 * sizeof(double));
  memcpy(c->v, v, (size_t)c->n * 3 * sizeof(double));
  memcpy(c->H, H, sizeof c->H);
  memcpy(c->Rprev, Rprev, sizeof c->Rprev);
  c->step = step;
  memset(c->wsum, 0, sizeof c->wsum); c->wcount = 0;
  c->status = OK;
  wrap_positions(c);
  return prime(&C->p, c);
}

int orc_get_energy(orc_ctx* C, double* pe, double* ke) {
  if (!C) return E_ARG;
  for (int32_t k = 0; k < C->ncells; ++k) {
    ocell* c = &C->c[k];
    if (pe) pe[k] = c->pe;
    if (ke) {
      double s = 0;
      for (int64_t q = 0; q < 3 * (int64_t)c->n; ++q) s += c->v[q] * c->v[q];
      ke[k] = 0.5 * C->p.mass * C->p.mvv2e * s;
    }
  }
  return OK;
}

int orc_get_box(orc_ctx* C, int32_t cell, double* H, double* Q, double* R, double* J) {
  if (!C || cell < 0 || cell >= C->ncells) return E_ARG;
  ocell* c = &C->c[cell];
  if (H) memcpy(H, c->H, sizeof c->H);
  if (Q) memcpy(Q, c->Q, sizeof c->Q);
  if (R) memcpy(R, c->R, sizeof c->R);
  if (J) *J = c->J;
  return OK;
}

const char* orc_last_error(const orc_ctx* C) { return C ? C->err : "null context"; }

void orc_destroy(orc_ctx* C) {
  if (!C) return;
  for (int32_t k = 0; k < C->ncells; ++k) {
    free(C->c[k].x); free(C->c[k].v); free(C->c[k].f); free(C->c[k].bonds); free(C->c[k].L.p);
  }
  free(C->c);
  free(C);
}

int orc_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}
