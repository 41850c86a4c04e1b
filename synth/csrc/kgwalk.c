/* Random-walk bead-spring chains in a cubic periodic box, grown bead by bead with a soft
 * excluded-volume rejection so that no two beads start closer than dmin (where possible).
 *
 * Input generator only: it places beads, it computes no potential, force or stress.
 * Every chain starts at a uniform random point; each next bead sits at distance `bond` from the
 * previous one along a uniform random direction.  Up to `ntries` candidates are drawn per bead;
 * the first whose nearest placed bead (minimum image) is at least dmin away is taken, otherwise the
 * candidate with the largest nearest distance.  A uniform grid of side >= dmin finds neighbours.
 * RNG: xoshiro256** (Blackman & Vigna) seeded through SplitMix64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static uint64_t s_[4];

static uint64_t splitmix(uint64_t* st) {
  uint64_t z = (*st += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static uint64_t next_u64(void) {
  uint64_t r = rotl(s_[1] * 5, 7) * 9, t = s_[1] << 17;
  s_[2] ^= s_[0]; s_[3] ^= s_[1]; s_[1] ^= s_[2]; s_[0] ^= s_[3]; s_[2] ^= t; s_[3] = rotl(s_[3], 45);
  return r;
}
static inline double unif(void) { return (double)(next_u64() >> 11) * 0x1.0p-53; }

static double L_, dmin2_;
static int g_;
static int *head_, *next_;
static const double* xs_;

static inline double wrap1(double a) { a = fmod(a, L_); return a < 0 ? a + L_ : (a >= L_ ? 0.0 : a); }
static inline int gidx(double a) { int k = (int)(a / L_ * g_); return k >= g_ ? g_ - 1 : (k < 0 ? 0 : k); }

static double nearest2(const double p[3], int nplaced) {
  double best = 1e300;
  if (g_ < 3) {
    for (int j = 0; j < nplaced; ++j) {
      double d2 = 0;
      for (int k = 0; k < 3; ++k) { double d = xs_[3 * j + k] - p[k]; d -= L_ * nearbyint(d / L_); d2 += d * d; }
      if (d2 < best) best = d2;
    }
    return best;
  }
  int c0 = gidx(p[0]), c1 = gidx(p[1]), c2 = gidx(p[2]);
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b)
      for (int c = -1; c <= 1; ++c) {
        int cell = (((c0 + a + g_) % g_) * g_ + (c1 + b + g_) % g_) * g_ + (c2 + c + g_) % g_;
        for (int j = head_[cell]; j >= 0; j = next_[j]) {
          double d2 = 0;
          for (int k = 0; k < 3; ++k) { double d = xs_[3 * j + k] - p[k]; d -= L_ * nearbyint(d / L_); d2 += d * d; }
          if (d2 < best) best = d2;
        }
      }
  return best;
}

/* Returns 0 on success, -1 on bad arguments or allocation failure. */
int kg_random_walk(double L, int32_t nchains, const int32_t* lens, double bond, double dmin,
                   int32_t ntries, uint64_t seed, double* x_out) {
  if (L <= 0 || nchains < 0 || bond <= 0 || dmin < 0 || ntries < 1) return -1;
  int64_t n = 0;
  for (int c = 0; c < nchains; ++c) { if (lens[c] < 1) return -1; n += lens[c]; }
  uint64_t st = seed;
  for (int k = 0; k < 4; ++k) s_[k] = splitmix(&st);
  L_ = L; dmin2_ = dmin * dmin; xs_ = x_out;
  g_ = dmin > 0 ? (int)floor(L / dmin) : 1;
  if (g_ < 1) g_ = 1;
  if (g_ > 1024) g_ = 1024;
  size_t ncell = (size_t)g_ * g_ * g_;
  head_ = (int*)malloc(ncell * sizeof(int));
  next_ = (int*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
  if (!head_ || !next_) { free(head_); free(next_); return -1; }
  for (size_t i = 0; i < ncell; ++i) head_[i] = -1;
  int64_t placed = 0;
  double prev[3] = {0, 0, 0};
  for (int c = 0; c < nchains; ++c) {
    for (int b = 0; b < lens[c]; ++b) {
      double best[3] = {0, 0, 0}, bestd2 = -1.0;
      for (int t = 0; t < ntries; ++t) {
        double p[3];
        if (b == 0) {
          for (int k = 0; k < 3; ++k) p[k] = unif() * L;
        } else {
          double z = 2.0 * unif() - 1.0, phi = 6.283185307179586 * unif(), s = sqrt(1.0 - z * z);
          p[0] = wrap1(prev[0] + bond * s * cos(phi));
          p[1] = wrap1(prev[1] + bond * s * sin(phi));
          p[2] = wrap1(prev[2] + bond * z);
        }
        double d2 = placed > 0 ? nearest2(p, (int)placed) : 1e300;
        if (d2 > bestd2) { bestd2 = d2; best[0] = p[0]; best[1] = p[1]; best[2] = p[2]; }
        if (d2 >= dmin2_) break;
      }
      for (int k = 0; k < 3; ++k) { x_out[3 * placed + k] = best[k]; prev[k] = best[k]; }
      int cell = (gidx(best[0]) * g_ + gidx(best[1])) * g_ + gidx(best[2]);
      next_[placed] = head_[cell];
      head_[cell] = (int)placed;
      ++placed;
    }
  }
  free(head_); free(next_);
  head_ = next_ = NULL;
  return 0;
}

/* Geometric overlap relaxation (no potential, no forces): repeated Jacobi sweeps that move every
 * non-bonded pair closer than dpush apart by a fraction of the deficit, then pull every bond back
 * towards bond_len.  Stops after `iters` sweeps or when no pair is closer than dpush.
 * x: n*3 positions in [0,L)^3 (updated, rewrapped); bonds: nbonds*2 indices.
 * Returns the smallest non-bonded distance found in the last sweep, or -1 on bad input. */
double kg_relax(double L, int32_t n, double* x, int32_t nbonds, const int32_t* bonds, double dpush,
                double bond_len, int32_t iters) {
  if (L <= 0 || n < 0 || dpush <= 0 || iters < 0) return -1.0;
  int32_t* part = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * 4 * sizeof(int32_t));
  double* dx = (double*)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
  if (!part || !dx) { free(part); free(dx); return -1.0; }
  for (int64_t k = 0; k < 4 * (int64_t)n; ++k) part[k] = -1;
  for (int32_t b = 0; b < nbonds; ++b)
    for (int s = 0; s < 2; ++s) {
      int32_t a = bonds[2 * b + s], o = bonds[2 * b + 1 - s];
      for (int q = 0; q < 4; ++q) if (part[4 * a + q] < 0) { part[4 * a + q] = o; break; }
    }
  L_ = L; g_ = (int)floor(L / dpush); if (g_ < 1) g_ = 1; if (g_ > 1024) g_ = 1024;
  size_t ncell = (size_t)g_ * g_ * g_;
  head_ = (int*)malloc(ncell * sizeof(int));
  next_ = (int*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
  double dmin_seen = 1e300;
  for (int it = 0; it < iters; ++it) {
    for (size_t c = 0; c < ncell; ++c) head_[c] = -1;
    for (int32_t i = n - 1; i >= 0; --i) {
      int cell = (gidx(x[3 * i]) * g_ + gidx(x[3 * i + 1])) * g_ + gidx(x[3 * i + 2]);
      next_[i] = head_[cell]; head_[cell] = i;
    }
    for (int64_t k = 0; k < 3 * (int64_t)n; ++k) dx[k] = 0.0;
    dmin_seen = 1e300;
#pragma omp parallel for schedule(static) reduction(min : dmin_seen)
    for (int32_t i = 0; i < n; ++i) {
      int c0 = gidx(x[3 * i]), c1 = gidx(x[3 * i + 1]), c2 = gidx(x[3 * i + 2]);
      int span = g_ < 3 ? 0 : 1;
      for (int a = -span; a <= span; ++a)
        for (int b = -span; b <= span; ++b)
          for (int c = -span; c <= span; ++c) {
            int cell = g_ < 3 ? -1 : (((c0 + a + g_) % g_) * g_ + (c1 + b + g_) % g_) * g_ + (c2 + c + g_) % g_;
            int j = g_ < 3 ? 0 : head_[cell];
            for (; g_ < 3 ? j < n : j >= 0; j = g_ < 3 ? j + 1 : next_[j]) {
              if (j == i) continue;
              int bonded = 0;
              for (int q = 0; q < 4; ++q) bonded |= part[4 * i + q] == j;
              if (bonded) continue;
              double d[3], r2 = 0;
              for (int k = 0; k < 3; ++k) { d[k] = x[3 * j + k] - x[3 * i + k]; d[k] -= L * nearbyint(d[k] / L); r2 += d[k] * d[k]; }
              double r = sqrt(r2);
              if (r < dmin_seen) dmin_seen = r;
              if (r < dpush && r > 1e-12)
                for (int k = 0; k < 3; ++k) dx[3 * i + k] -= 0.25 * (dpush - r) * d[k] / r;
            }
          }
      for (int q = 0; q < 4; ++q) {
        int32_t j = part[4 * i + q];
        if (j < 0) continue;
        double d[3], r2 = 0;
        for (int k = 0; k < 3; ++k) { d[k] = x[3 * j + k] - x[3 * i + k]; d[k] -= L * nearbyint(d[k] / L); r2 += d[k] * d[k]; }
        double r = sqrt(r2);
        if (r > 1e-12)
          for (int k = 0; k < 3; ++k) dx[3 * i + k] += 0.5 * (r - bond_len) * d[k] / r;
      }
    }
    for (int32_t i = 0; i < n; ++i)
      for (int k = 0; k < 3; ++k) x[3 * i + k] = wrap1(x[3 * i + k] + dx[3 * i + k]);
    if (dmin_seen >= dpush) break;
  }
  free(head_); free(next_); free(part); free(dx);
  head_ = next_ = NULL;
  return dmin_seen;
}
