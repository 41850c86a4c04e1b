// Device side of the batched r-cell MD library (gfx950).
//
// Data layout (one batch = all cells of a context, atoms of cell c at [off_c, off_c + n_c)):
//   x, y, z     FP64 SoA master positions        vx, vy, vz  FP64 SoA velocities
//   fx, fy, fz  FP64 total force of the last completed step (read by the first kick of a run)
//   s[2]        double-buffered fixed-point scaled coordinates: S = frac(H^-1 x) * 2^32 (int32,
//               mixed) or * 2^64 (int64, FP64 mode); .w carries F'(rho) for the EAM force pass (scaled by sc_fscale).
//               Differences of two such integers wrap modulo 2^32 (2^64), which is exactly the
//               per-component minimum image in scaled space: the pair separation needs no
//               image shifts (d = H dS, formed in FP64 and rounded once in mixed precision).
//   sb          s at the last neighbour build, quantised to its top 16 bits per component (8 bytes;
//               the displacement check allows for the quantisation, see qeps)
//   nbr         Verlet list within rc + skin, cell-local j, as 16-bit indices when every cell has
//               at most 65536 atoms (mixed precision), else 32-bit; entries of one atom in blocks
//               of B = 8 (Kremer-Grest) or 16 (Sutton-Chen), the blocks of entries [b B, (b+1) B) of
//               all atoms side by side (list_index), so a lane loads its UNR entries of a trip with
//               one vector load
//   bond        up to four FENE partners per atom (cell-local positions; the atom's own position marks an
//               empty slot), 16-bit slots when the list entries are 16-bit, else 32-bit
//   gid         original cell-local index of the atom stored at each position; pos_of inverts it;
//               bond0 holds the partners by original index.  At every neighbour build a cell's
//               atoms are reordered by (bin, original index), so that neighbours sit close in
//               memory; everything that identifies an atom (noise counter, host API order) uses gid.
// Work is distributed over 64-atom tiles (a tile never straddles two cells); each tile writes
// one partial record and a per-cell kernel reduces them in a fixed order (deterministic).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rcell {

constexpr int TILE = 64;
constexpr int BIN_BITS = 10;     // bins per dimension < 2^BIN_BITS (bin coordinates are packed)
constexpr int BIN_MASK = (1 << BIN_BITS) - 1;
constexpr int UNR = 4;           // neighbour-loop unroll: gathers in flight per lane
constexpr int NBLK_MAX = 16;     // list blocks: 2^lblk consecutive entries of one atom, 8 or 16 (the
                                 // capacity is a multiple of 16)
constexpr double TWO32 = 4294967296.0;
constexpr double TWOM32 = 1.0 / 4294967296.0;

enum Mode : int { MODE_PRIME = 0, MODE_STEP = 1, MODE_LAST = 2, MODE_DRY = 3, MODE_STATIC = 4 };
enum RedMode : int { RED_START = 0, RED_PRIME = 1, RED_STEP = 2, RED_LAST = 3, RED_STATIC = 4, RED_MOVE = 5 };
enum Status : int { ST_OK = 0, ST_BOND = -4, ST_CAP = -8, ST_BOX = -3, ST_BAD_F = -2 };

struct alignas(32) S64 { long long x, y, z, w; };

// Element index of list entry k of atom i (batch position) in a list of npad atoms: blocks of
// B = 2^lb consecutive entries of one atom, the blocks of all atoms for entries [b B, (b+1) B) stored
// together in atom order.  The list holds < 2^32 elements, so 32-bit arithmetic is exact.  Short
// Kremer-Grest lists (~20 entries) take B = 8, so that an atom's last block wastes fewer fetched
// bytes; Sutton-Chen lists take B = 16, so that the 16 entries its lane group reads per trip are one
// contiguous piece.
__host__ __device__ inline unsigned list_index(unsigned k, unsigned npad, unsigned i, int lb) {
  return (((k >> lb) * npad + i) << lb) | (k & ((1u << lb) - 1u));
}

struct CellDev {
  double H[9], Hi[9];             // box (upper triangular) and its inverse
  double Rprev[9], Q[9], R[9], F[9];
  double J, V;
  double xi_mean[3];              // per-cell mean of the integer noise for the next time level
  double wsum[6], last[6];        // stress window sum and last sample (Voigt, tension +)
  double pe;
  double Hd[6];                   // H * 2^-64, upper triangle (FP64 mode)
  double Hm[6];                   // H * 2^-32, upper triangle (mixed mode)
  long long wcount, step, nrebuild;
  int off, n, tile_off, ntile;
  int nb[3], bin_off, bin_cap;
  int rebuild, pending, status, pad;
  double Hb[6];                   // H at the last neighbour build, upper triangle (0 1 2 4 5 8)
  float hs2;                      // squared (measured) displacement that still keeps the list complete
  float dmax2;                    // largest squared measured displacement since the last build, as last reduced
  float qeps;                     // bound on the error of a measured displacement: the 16-bit build reference
  int pad3;
  // molecular statics (FIRE): time step, mixing parameter, the velocity update of this iteration
  // (v = fa v + fb f, or zero when frozen), iterations since the power last turned negative,
  // converged flag and iterations used
  double fdt, falpha, fa, fb;
  int fcount, fdone, ffreeze, fiter;
};

struct Tile { int cell, begin, count, pad; };

// Tile-grid kernels: the grid has ntiles blocks rounded up to a multiple of 8; block w works on
// tile w (w < ntiles).  The pair kernels use block_tile_xcd instead: the GPU hands consecutive
// blocks to its 8 XCDs in turn, so XCD x receives blocks x, x + 8, ..., and this mapping gives it
// the contiguous tile range [x per, (x + 1) per) - whole cells whose positions then stay in that
// XCD's own L2 for the neighbour gathers.
__host__ __device__ inline int tile_grid(int ntiles) { return (ntiles + 7) / 8 * 8; }
__device__ __forceinline__ int block_tile(int ntiles, int block) { return block; }
__device__ __forceinline__ int block_tile_xcd(int ntiles, int block) {
  return (block % 8) * ((ntiles + 7) / 8) + block / 8;
}
// The same placement for block-strided loops over n work items (the rebuild phases): with a grid
// that is a multiple of 8, XCD x runs blocks x, x + 8, ..., and they share out the contiguous item
// range [x per, (x + 1) per), per = ceil(n / 8), so the cells that XCD rebuilds stay in its own L2.
// A block may split its share further over sub workers (its waves): worker w of a block takes the
// items k, k + step, ... below end.
struct XcdLoop {
  int k, end, step;
  __device__ XcdLoop(int n, int sub = 1, int w = 0) {
    const int per = (n + 7) / 8, x = (int)(blockIdx.x & 7u);
    k = x * per + (int)(blockIdx.x >> 3) * sub + w;
    end = min(n, (x + 1) * per);
    step = (int)(gridDim.x >> 3) * sub;
  }
};

struct Part {                     // one tile's contribution
  double V[6];                    // MD: pair virial minus the kinetic term; statics: the FIRE sums
  double pe;
  long long xi[3];
  float maxd2;
  int status;
};

struct Stage {                    // set_deformation staging, one per cell
  double Q[9], R[9], dR[9], Hn[9], F[9];
  double J, wmin;
  int nb[3], nbins, status;
  double density;
};

struct MDArgs {
  double *x, *y, *z, *vx, *vy, *vz;
  void *fx, *fy, *fz;
  void *s_cur, *s_nxt;
  uint2* sb;
  void* bond;                      // 4 partner slots per atom: uint16_t when bond16, else int
  const int4* bond0;
  int bond16;
  int* gid;
  int* pos_of;
  char* pscr;                      // reorder scratch: 6 doubles, one S and two ints per atom (npad rows)
  int* nn;
  void* nbr;                       // LT entries (uint16_t or int), see the kernels' LT parameter
  long long npad;
  int maxnb;
  int lblk;                        // list blocks of 2^lblk entries (list_index)
  CellDev* cells;
  const Tile* tiles;
  Part* parts;
  int ntiles, ncells;
  int* abin; int* bcount; int* bstart; int* bnum; int* bfill; int* binned; int* sort_tmp;
  long long bins_total;
  // work list of the rebuild phases (k_rebuild_work): the cells flagged for a rebuild in cell
  // order, and the exclusive prefix sums of their tiles and of their 64-bin chunks (ncell + 1
  // entries each); work_count[0..2] = cells, tiles, chunks
  int *work_cells, *work_tstart, *work_kstart, *work_count;
  int bin_factor;                  // bins at least (rc + skin) / bin_factor wide; stencil +- bin_factor
  // integrator constants (computed once on the host, documented expressions)
  double dt, h, drag, c24, mmv, half_skin2, rcs2;
  double fire_ftol2;               // statics: converged when max_i |f_i|^2 <= fire_ftol2
  int fire_max_iter;               // statics: at most this many moves per cell
  uint32_t key0, key1;
  int gamma_on, include_kinetic, pot;
  // pair constants
  double rc2, lj_eps, lj_sig2, lj_shift, fene_K, fene_R02, sc_eps, sc_a, sc_c, sc_phic, sc_rhoc;
  int sc_n, sc_m;
};

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror & Shaw (SC'11): 10 rounds of two 32x32->64 multiplies with the published
// multipliers; the key is bumped by the published Weyl increments between rounds.
__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// integer noise units k = (w >> 8) - 2^23 for the three components of atom gid of cell at level step
__device__ __forceinline__ void noise_units(const MDArgs& a, int gid, int cell, long long step, int k[3]) {
  uint32_t w[4];
  philox((uint32_t)gid, (uint32_t)cell, (uint32_t)(unsigned long long)step,
         (uint32_t)((unsigned long long)step >> 32), a.key0, a.key1, w);
  k[0] = (int)(w[0] >> 8) - (1 << 23);
  k[1] = (int)(w[1] >> 8) - (1 << 23);
  k[2] = (int)(w[2] >> 8) - (1 << 23);
}

// ------------------------------------------------------------------ precision policies
struct Mixed {
  using S = int4;
  using R = float;
  using Fst = double;   // stored total force: touched once per run, kept in FP64 so runs split bitwise
  __device__ static S load(const void* p, long long i) { return ((const int4*)p)[i]; }
  // element j of a per-cell base pointer, as a 32-bit unsigned byte offset
  __device__ static S load_rel(const S* base, int j) {
    return *(const S*)((const char*)base + ((unsigned)j << 4));
  }
  __device__ static void store_xyz(void* p, long long i, const S& v) { ((int4*)p)[i] = v; }
  __device__ static void store_w(void* p, long long i, R fp) { ((int4*)p)[i].w = __float_as_int(fp); }
  __device__ static R get_w(const S& v) { return __int_as_float(v.w); }
  // scaled fraction f in [0,1) -> 32-bit fixed point (2^32 wraps to 0)
  __device__ static int fix1(double f) {
    return (int)(unsigned int)(unsigned long long)(long long)rint(f * TWO32);
  }
  __device__ static S make(double f0, double f1, double f2) { return make_int4(fix1(f0), fix1(f1), fix1(f2), 0); }
  // the cell's H * 2^-32 (upper triangular: 0 xx, 1 xy, 2 xz, 3 yy, 4 yz, 5 zz), held in
  // registers across a neighbour loop.  The separation H dS is formed in FP64 (full rate on this
  // GPU, like FP32 without packing) and rounded once to FP32, so no rounding of H acts as a
  // strain of the whole cell.
  struct Geo { double h[6]; };
  __device__ static Geo geo(const CellDev& C) {
    Geo g;
#pragma unroll
    for (int q = 0; q < 6; ++q) g.h[q] = C.Hm[q];
    return g;
  }
  __device__ static void sep(const S& sj, const S& si, const Geo& g, R d[3]) {
    const double a = (double)(int)((unsigned)sj.x - (unsigned)si.x);
    const double b = (double)(int)((unsigned)sj.y - (unsigned)si.y);
    const double c = (double)(int)((unsigned)sj.z - (unsigned)si.z);
    d[0] = (float)fma(g.h[0], a, fma(g.h[1], b, g.h[2] * c));
    d[1] = (float)fma(g.h[3], b, g.h[4] * c);
    d[2] = (float)(g.h[5] * c);
  }
  __device__ static void sep(const S& sj, const S& si, const CellDev& C, R d[3]) { sep(sj, si, geo(C), d); }
  // the same separation, also kept in FP64 before the rounding: the pair virial is accumulated
  // from it in FP64, so neither the rounding of d nor FP32 sums enter the stress
  __device__ static void sep2(const S& sj, const S& si, const Geo& g, R d[3], double dd[3]) {
    const double a = (double)(int)((unsigned)sj.x - (unsigned)si.x);
    const double b = (double)(int)((unsigned)sj.y - (unsigned)si.y);
    const double c = (double)(int)((unsigned)sj.z - (unsigned)si.z);
    dd[0] = fma(g.h[0], a, fma(g.h[1], b, g.h[2] * c));
    dd[1] = fma(g.h[3], b, g.h[4] * c);
    dd[2] = g.h[5] * c;
    d[0] = (float)dd[0]; d[1] = (float)dd[1]; d[2] = (float)dd[2];
  }
  // single hardware instructions (about 1 ulp): ample for FP32 pair forces
  __device__ static R rsq(R x) { return __builtin_amdgcn_rsqf(x); }
  __device__ static R rcp(R x) { return __builtin_amdgcn_rcpf(x); }
  // the build reference: each fixed-point component rounded to its top 16 bits (x | y << 16, z)
  __device__ static uint2 quant(const S& s) {
    const unsigned qx = ((unsigned)s.x + 0x8000u) >> 16, qy = ((unsigned)s.y + 0x8000u) >> 16;
    const unsigned qz = ((unsigned)s.z + 0x8000u) >> 16;
    return make_uint2(qx | (qy << 16), qz);
  }
  // displacement of sn from a quantised reference (minimum image, like sep)
  __device__ static void disp(const S& sn, uint2 q, const Geo& g, R d[3]) {
    const double a = (double)(int)((unsigned)sn.x - ((q.x & 0xffffu) << 16));
    const double b = (double)(int)((unsigned)sn.y - (q.x & 0xffff0000u));
    const double c = (double)(int)((unsigned)sn.z - ((q.y & 0xffffu) << 16));
    d[0] = (float)fma(g.h[0], a, fma(g.h[1], b, g.h[2] * c));
    d[1] = (float)fma(g.h[3], b, g.h[4] * c);
    d[2] = (float)(g.h[5] * c);
  }
};

struct FP64 {
  using S = S64;
  using R = double;
  using Fst = double;
  __device__ static S load(const void* p, long long i) { return ((const S64*)p)[i]; }
  __device__ static S load_rel(const S* base, int j) {
    return *(const S*)((const char*)base + ((unsigned)j << 5));
  }
  __device__ static void store_xyz(void* p, long long i, const S& v) { ((S64*)p)[i] = v; }
  __device__ static void store_w(void* p, long long i, R fp) { ((S64*)p)[i].w = __double_as_longlong(fp); }
  __device__ static R get_w(const S& v) { return __longlong_as_double(v.w); }
  // scaled fraction f in [0,1) -> 64-bit fixed point, rounded to nearest, 2^64 wraps to 0
  __device__ static long long fix1(double f) {
    const double t = f * TWO32;
    const double hi = floor(t);
    const double lo = rint((t - hi) * TWO32);
    const unsigned long long u = ((unsigned long long)(unsigned int)(long long)hi << 32) + (unsigned long long)(long long)lo;
    return (long long)u;
  }
  __device__ static S make(double f0, double f1, double f2) { S s; s.x = fix1(f0); s.y = fix1(f1); s.z = fix1(f2); s.w = 0; return s; }
  __device__ static double cvt(long long v) {       // signed 64-bit integer to double, rounded
    return (double)v;
  }
  struct Geo { double h[6]; };                     // H * 2^-64, upper triangle
  __device__ static Geo geo(const CellDev& C) {
    Geo g;
#pragma unroll
    for (int q = 0; q < 6; ++q) g.h[q] = C.Hd[q];
    return g;
  }
  __device__ static void sep(const S& sj, const S& si, const Geo& g, R d[3]) {
    const double a = cvt((long long)((unsigned long long)sj.x - (unsigned long long)si.x));
    const double b = cvt((long long)((unsigned long long)sj.y - (unsigned long long)si.y));
    const double c = cvt((long long)((unsigned long long)sj.z - (unsigned long long)si.z));
    d[0] = g.h[0] * a + g.h[1] * b + g.h[2] * c;
    d[1] = g.h[3] * b + g.h[4] * c;
    d[2] = g.h[5] * c;
  }
  __device__ static void sep(const S& sj, const S& si, const CellDev& C, R d[3]) { sep(sj, si, geo(C), d); }
  __device__ static void sep2(const S& sj, const S& si, const Geo& g, R d[3], double dd[3]) {
    sep(sj, si, g, d);
    dd[0] = d[0]; dd[1] = d[1]; dd[2] = d[2];
  }
  __device__ static R rsq(R x) { return 1.0 / sqrt(x); }
  __device__ static R rcp(R x) { return 1.0 / x; }
  __device__ static uint2 quant(const S& s) {
    const unsigned long long h = 1ull << 47;
    const unsigned qx = (unsigned)(((unsigned long long)s.x + h) >> 48);
    const unsigned qy = (unsigned)(((unsigned long long)s.y + h) >> 48);
    const unsigned qz = (unsigned)(((unsigned long long)s.z + h) >> 48);
    return make_uint2(qx | (qy << 16), qz);
  }
  __device__ static void disp(const S& sn, uint2 q, const Geo& g, R d[3]) {
    const double a = cvt((long long)((unsigned long long)sn.x - ((unsigned long long)(q.x & 0xffffu) << 48)));
    const double b = cvt((long long)((unsigned long long)sn.y - ((unsigned long long)(q.x >> 16) << 48)));
    const double c = cvt((long long)((unsigned long long)sn.z - ((unsigned long long)(q.y & 0xffffu) << 48)));
    d[0] = g.h[0] * a + g.h[1] * b + g.h[2] * c;
    d[1] = g.h[3] * b + g.h[4] * c;
    d[2] = g.h[5] * c;
  }
};

// S = H^-1 x for upper-triangular H^-1, reduced to its fractional part
// (explicit fused multiply-adds: every caller rounds identically, so the fixed-point coordinates
// that the Kremer-Grest force pass recomputes from x equal the stored ones bit for bit)
__device__ __forceinline__ void scaled_frac(const CellDev& C, double x, double y, double z, double f[3]) {
  const double s0 = fma(C.Hi[0], x, fma(C.Hi[1], y, C.Hi[2] * z));
  const double s1 = fma(C.Hi[4], y, C.Hi[5] * z);
  const double s2 = C.Hi[8] * z;
  f[0] = s0 - floor(s0);
  f[1] = s1 - floor(s1);
  f[2] = s2 - floor(s2);
}

template <class P>
__device__ __forceinline__ typename P::S fixed_pos(const CellDev& C, double x, double y, double z) {
  double f[3];
  scaled_frac(C, x, y, z, f);
  return P::make(f[0], f[1], f[2]);
}

// t^N for a compile-time exponent (binary powering)
template <int N, class T>
__device__ __forceinline__ T powc(T t) {
  if constexpr (N == 0) return (T)1;
  else if constexpr (N == 1) return t;
  else if constexpr (N % 2 == 0) { const T h = powc<N / 2>(t); return h * h; }
  else return powc<N - 1>(t) * t;
}

// t^n for a run-time exponent 0 <= n < 32, branch free (the exponent is uniform over the grid)
template <class T>
__device__ __forceinline__ T powr(T t, int n) {
  T r = (T)1;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    r = ((n >> b) & 1) ? r * t : r;
    t *= t;
  }
  return r;
}

// Sutton-Chen powers tn = t^n and tm = t^m; SN = SM = 0 takes the exponents at run time
template <int SN, int SM, class T>
__device__ __forceinline__ void sc_powers(T t, int n, int m, T& tn, T& tm) {
  if constexpr (SN == 9 && SM == 6) {
    const T t3 = t * t * t;
    tm = t3 * t3;
    tn = tm * t3;
  } else if constexpr (SN > 0) {
    tn = powc<SN>(t);
    tm = powc<SM>(t);
  } else {
    tn = powr(t, n);
    tm = powr(t, m);
  }
}

// ------------------------------------------------------------------ block reductions
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  // fixed-shape tree: deterministic for a given block size
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ long long block_sum_ll(long long v, long long* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const long long r = sh[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ float block_max(float v, float* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmaxf(sh[t], sh[t + s]);
    __syncthreads();
  }
  const float r = sh[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ int block_min_i(int v, int* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = min(sh[t], sh[t + s]);
    __syncthreads();
  }
  const int r = sh[0];
  __syncthreads();
  return r;
}

// reduce a value across the TPA consecutive lanes that share one atom (result in every lane)
template <int TPA, class T>
__device__ __forceinline__ T lane_sum(T v) {
#pragma unroll
  for (int o = TPA / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, TPA);
  return v;
}

// ------------------------------------------------------------------ per-atom integration tail
// Completes the time level of atom i after its conservative force fc is known:
//   Langevin (drag + noise with the per-cell mean removed), second half kick (v_full), the
//   kinetic stress term, and in MODE_STEP the next first half kick and drift with the new
//   fixed-point position, displacement check and the next level's noise sums.
struct TailOut {
  double K[6];
  float maxd2;
  long long xi[3];
};

template <class P>
__device__ __forceinline__ void atom_tail(const MDArgs& a, const CellDev& C, int cell, long long i,
                                          double fcx, double fcy, double fcz, int mode, TailOut& o,
                                          const double* xin = nullptr) {
  double vx = a.vx[i], vy = a.vy[i], vz = a.vz[i];
  const int gid = a.gid[i];
  double f0 = fcx, f1 = fcy, f2 = fcz;
  if (mode == MODE_STATIC) {
    // statics: keep the conservative force and report f.v, |f|^2, |v|^2 and max |f|^2 (FIRE)
    ((typename P::Fst*)a.fx)[i] = (typename P::Fst)f0;
    ((typename P::Fst*)a.fy)[i] = (typename P::Fst)f1;
    ((typename P::Fst*)a.fz)[i] = (typename P::Fst)f2;
    const double ff = f0 * f0 + f1 * f1 + f2 * f2;
    o.K[0] = f0 * vx + f1 * vy + f2 * vz; o.K[1] = ff; o.K[2] = vx * vx + vy * vy + vz * vz;
    o.K[3] = o.K[4] = o.K[5] = 0.0;
    o.maxd2 = (float)ff;
    o.xi[0] = o.xi[1] = o.xi[2] = 0;
    return;
  }
  if (mode == MODE_PRIME) {
    // forces after create / deformation / restore: conservative part only; v is a full-step velocity
    ((typename P::Fst*)a.fx)[i] = (typename P::Fst)f0;
    ((typename P::Fst*)a.fy)[i] = (typename P::Fst)f1;
    ((typename P::Fst*)a.fz)[i] = (typename P::Fst)f2;
  } else {
    if (a.gamma_on) {
      int k[3];
      noise_units(a, gid, cell, C.step + 1, k);
      f0 = (f0 + a.drag * vx) + a.c24 * ((double)k[0] - C.xi_mean[0]);
      f1 = (f1 + a.drag * vy) + a.c24 * ((double)k[1] - C.xi_mean[1]);
      f2 = (f2 + a.drag * vz) + a.c24 * ((double)k[2] - C.xi_mean[2]);
    }
    vx += a.h * f0;  // v(t + dt) from the half-step velocity
    vy += a.h * f1;
    vz += a.h * f2;
  }
  o.K[0] = a.mmv * vx * vx; o.K[1] = a.mmv * vy * vy; o.K[2] = a.mmv * vz * vz;
  o.K[3] = a.mmv * vx * vy; o.K[4] = a.mmv * vx * vz; o.K[5] = a.mmv * vy * vz;
  o.maxd2 = 0.f;
  o.xi[0] = o.xi[1] = o.xi[2] = 0;
  if (mode == MODE_LAST) {
    a.vx[i] = vx; a.vy[i] = vy; a.vz[i] = vz;
    ((typename P::Fst*)a.fx)[i] = (typename P::Fst)f0;
    ((typename P::Fst*)a.fy)[i] = (typename P::Fst)f1;
    ((typename P::Fst*)a.fz)[i] = (typename P::Fst)f2;
  } else if (mode == MODE_STEP) {
    vx += a.h * f0;  // first half kick of the next step
    vy += a.h * f1;
    vz += a.h * f2;
    const double x0 = xin ? xin[0] : a.x[i], y0 = xin ? xin[1] : a.y[i], z0 = xin ? xin[2] : a.z[i];
    const double x = x0 + a.dt * vx, y = y0 + a.dt * vy, z = z0 + a.dt * vz;
    a.vx[i] = vx; a.vy[i] = vy; a.vz[i] = vz;
    a.x[i] = x; a.y[i] = y; a.z[i] = z;
    const typename P::S sn = fixed_pos<P>(C, x, y, z);
    P::store_xyz(a.s_nxt, i, sn);
    typename P::R d[3];
    P::disp(sn, a.sb[i], P::geo(C), d);
    o.maxd2 = (float)(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (a.gamma_on) {
      int k[3];
      noise_units(a, gid, cell, C.step + 2, k);
      o.xi[0] = k[0]; o.xi[1] = k[1]; o.xi[2] = k[2];
    }
  }
}

// sum over the 64 lanes of a wave by xor shuffles (fixed pattern: deterministic)
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

// the same trees over the lanes whose index is a multiple of L only (the other lanes hold zeros):
// lane 0 receives the result
template <int L, class T>
__device__ __forceinline__ T wave_sum_from(T v) {
#pragma unroll
  for (int o = 32; o >= L; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
template <int L>
__device__ __forceinline__ float wave_max_from(float v) {
#pragma unroll
  for (int o = 32; o >= L; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
template <int L>
__device__ __forceinline__ int wave_min_from(int v) {
#pragma unroll
  for (int o = 32; o >= L; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

template <int NW>
struct PartShared {
  double d[NW][7];
  int l[NW][3];
  float f[NW];
  int i[NW];
};

// Reduce one tile's contributions (every thread of the block calls this) and write its Part.  Only
// the first of each atom's TPA lanes holds values, so the shuffle tree of each wave runs over those
// lanes only; a wave's noise sum (at most 64 integers below 2^23 in magnitude) fits 32 bits.  The
// energy is reduced only where it is reported (with_pe, uniform over the block).  Thread 0 then
// adds the NW wave results in order.
template <int NT, int TPA>
__device__ __forceinline__ void write_part(Part* parts, int part, const double V[6], double pe, bool with_pe,
                                           const long long xi[3], float maxd2, int status,
                                           PartShared<NT / 64>& sh) {
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  double r[7];
#pragma unroll
  for (int q = 0; q < 6; ++q) r[q] = wave_sum_from<TPA>(V[q]);
  r[6] = with_pe ? wave_sum_from<TPA>(pe) : 0.0;
  int x[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) x[q] = wave_sum_from<TPA>((int)xi[q]);
  const float m = wave_max_from<TPA>(maxd2);
  const int st = wave_min_from<TPA>(status);
  if (ln == 0) {
#pragma unroll
    for (int q = 0; q < 7; ++q) sh.d[wv][q] = r[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) sh.l[wv][q] = x[q];
    sh.f[wv] = m;
    sh.i[wv] = st;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Part& p = parts[part];
    double acc[7];
    long long la[3] = {0, 0, 0};
    float mm = 0.f;
    int ss = 0;
#pragma unroll
    for (int q = 0; q < 7; ++q) acc[q] = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
#pragma unroll
      for (int q = 0; q < 7; ++q) acc[q] += sh.d[w][q];
#pragma unroll
      for (int q = 0; q < 3; ++q) la[q] += sh.l[w][q];
      mm = fmaxf(mm, sh.f[w]);
      ss = min(ss, sh.i[w]);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) p.V[q] = acc[q];
    p.pe = acc[6];
    p.xi[0] = la[0]; p.xi[1] = la[1]; p.xi[2] = la[2];
    p.maxd2 = mm;
    p.status = ss;
  }
}

// The per-atom stress contribution of the MD modes, W - K (K only where the kinetic term is
// included), or in statics the FIRE sums carried in K
__device__ __forceinline__ void part_values(const MDArgs& a, int mode, const double W[6], const double K[6], double V[6]) {
  const double kin = a.include_kinetic ? 1.0 : 0.0;
#pragma unroll
  for (int q = 0; q < 6; ++q) V[q] = mode == MODE_STATIC ? K[q] : W[q] - kin * K[q];
}

// Twice the pair virial of one listed pair, g d (x) d / r with gr = g / r, accumulated in FP64 from
// the FP64 separation (halved once after the loop, exact in binary).
__device__ __forceinline__ void add_virial(double w[6], double gr, const double dd[3]) {
  const double t0 = gr * dd[0], t1 = gr * dd[1], t2 = gr * dd[2];
  w[0] = fma(t0, dd[0], w[0]); w[1] = fma(t1, dd[1], w[1]); w[2] = fma(t2, dd[2], w[2]);
  w[3] = fma(t0, dd[1], w[3]); w[4] = fma(t0, dd[2], w[4]); w[5] = fma(t1, dd[2], w[5]);
}

// ------------------------------------------------------------------ force kernels
// List entries of one trip: UNR consecutive entries of one list block, as 32-bit words loaded with
// one vector load (the trip's first entry is a multiple of UNR, so they are aligned).
template <class LT>
struct ListVec {
  static constexpr int W = UNR * (int)sizeof(LT) / 4;
  static_assert(W == 1 || W == 2 || W == 4, "one vector load per trip");
  uint32_t w[W];
  __device__ void load(const LT* p) {
    if constexpr (W == 1) {
      w[0] = *(const uint32_t*)p;
    } else if constexpr (W == 2) {
      const uint2 v = *(const uint2*)p;
      w[0] = v.x; w[1] = v.y;
    } else {
      const uint4 v = *(const uint4*)p;
      w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    }
  }
  __device__ int get(int u) const {
    if constexpr (sizeof(LT) == 2) return (int)((w[u >> 1] >> ((u & 1) * 16)) & 0xffffu);
    else return (int)w[u];
  }
};
static_assert(8 % UNR == 0, "a trip's entries must lie in one list block");

// One lane's walk over atom i's list.  Per trip the lane takes UNR consecutive entries (one vector
// load) and the TPA lanes of the atom take consecutive groups of UNR.  The next trip's entries are
// requested right after this trip's gathers are issued, so a trip waits for one memory round trip
// (the gathers), not two.  Entries at or past nn gather the cell's first atom and come back with
// ok = false: the pair loops run straight-line code and mask those slots out.  sc points at the
// cell's first atom.
template <class P, int TPA, class LT>
struct NbrWalk {
  const LT* list;
  unsigned np, ii;
  int nn, k0, lb;
  ListVec<LT> nx;
  __device__ NbrWalk(const MDArgs& a, long long i, int nn_, int lane)
      : list((const LT*)a.nbr), np((unsigned)a.npad), ii((unsigned)i), nn(nn_), k0(lane * UNR), lb(a.lblk), nx{} {
    if (k0 < nn) nx.load(list + list_index((unsigned)k0, np, ii, lb));
  }
  __device__ bool more() const { return k0 < nn; }
  __device__ void next(const typename P::S* sc, typename P::S sj[UNR], bool ok[UNR]) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      ok[u] = k0 + u < nn;
      sj[u] = P::load_rel(sc, ok[u] ? nx.get(u) : 0);
    }
    k0 += UNR * TPA;
    if (k0 < nn) nx.load(list + list_index((unsigned)k0, np, ii, lb));
  }
};

// Kremer-Grest: LJ truncated and shifted at rc on every listed pair + FENE on bonds; then the
// integration tail.  TPA lanes share one atom's neighbour list.
template <class P, int TPA, class LT>
__global__ __launch_bounds__(TILE * TPA) void k_force_kg(MDArgs a, int mode) {
  using R = typename P::R;
  constexpr int NT = TILE * TPA;
  __shared__ PartShared<NT / 64> psh;
  const int tb = block_tile_xcd(a.ntiles, blockIdx.x);
  if (tb >= a.ntiles) return;
  const Tile t = a.tiles[tb];
  const CellDev& C = a.cells[t.cell];
  const int slot = threadIdx.x / TPA, lane = threadIdx.x % TPA;
  const bool skip = (mode == MODE_PRIME && !C.pending) || (mode == MODE_STATIC && C.fdone);
  const bool active = slot < t.count && !skip;
  const long long i = (long long)t.begin + slot;
  R f[3] = {0, 0, 0}, pe = 0;
  double w[6] = {0, 0, 0, 0, 0, 0};
  double xi[3] = {0.0, 0.0, 0.0};
  int status = 0;
  if (active) {
    // the atom's own fixed-point coordinates are recomputed from its position (they are stored only
    // for the neighbours' gathers): the position is read here for the drift anyway
    xi[0] = a.x[i]; xi[1] = a.y[i]; xi[2] = a.z[i];
    const typename P::S si = fixed_pos<P>(C, xi[0], xi[1], xi[2]);
    const int nn = a.nn[i];
    const R rc2 = (R)a.rc2, sig2 = (R)a.lj_sig2, e24 = (R)(24.0 * a.lj_eps), e4 = (R)(4.0 * a.lj_eps), sh = (R)a.lj_shift;
    const typename P::Geo g = P::geo(C);
    const typename P::S* sc = (const typename P::S*)a.s_cur + C.off;
    // the pair energy is summed only where it is reported: not in the middle steps of a run
    auto pairs = [&](auto with_pe) {
      for (NbrWalk<P, TPA, LT> walk(a, i, nn, lane); walk.more();) {
        typename P::S sj[UNR];
        bool ok[UNR];
        walk.next(sc, sj, ok);
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          R d[3];
          double dd[3];
          P::sep2(sj[u], si, g, d, dd);
          const R r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          const bool in = ok[u] && r2 < rc2;
          const R r2i = P::rcp(r2);
          const R s2 = sig2 * r2i;
          const R s6 = s2 * s2 * s2;
          const R gr = in ? -e24 * (s6 * ((R)2 * s6 - (R)1)) * r2i : (R)0;   // (dU/dr) / r
          f[0] += gr * d[0]; f[1] += gr * d[1]; f[2] += gr * d[2];
          add_virial(w, (double)gr, dd);
          if constexpr (decltype(with_pe)::value) pe += in ? (R)0.5 * (e4 * s6 * (s6 - (R)1) - sh) : (R)0;
        }
      }
    };
    if (mode == MODE_STEP || mode == MODE_DRY) pairs(std::false_type{});
    else pairs(std::true_type{});
    if (lane == 0) {
      const int li = (int)(i - C.off);
      int bp[4];
      if constexpr (sizeof(LT) == 2) {
        const uint2 b = ((const uint2*)a.bond)[i];
        bp[0] = (int)(b.x & 0xffffu); bp[1] = (int)(b.x >> 16); bp[2] = (int)(b.y & 0xffffu); bp[3] = (int)(b.y >> 16);
      } else {
        const int4 b = ((const int4*)a.bond)[i];
        bp[0] = b.x; bp[1] = b.y; bp[2] = b.z; bp[3] = b.w;
      }
      const R K = (R)a.fene_K, R02 = (R)a.fene_R02;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (bp[q] == li) continue;               // empty slot
        R d[3];
        double dd[3];
        P::sep2(P::load_rel(sc, bp[q]), si, g, d, dd);
        const R r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const R tt = r2 / R02;
        if (!(tt < (R)1)) { status = ST_BOND; continue; }
        const R gr = K / ((R)1 - tt);
        f[0] += gr * d[0]; f[1] += gr * d[1]; f[2] += gr * d[2];
        add_virial(w, (double)gr, dd);
        pe += (R)(-0.25 * a.fene_K * a.fene_R02) * (R)log((double)((R)1 - tt));
      }
    }
  }
  double W[6], K[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 6; ++q) W[q] = 0.5 * lane_sum<TPA>(w[q]);
  double PE = (double)lane_sum<TPA>(pe);
  const double fc0 = (double)lane_sum<TPA>(f[0]), fc1 = (double)lane_sum<TPA>(f[1]), fc2 = (double)lane_sum<TPA>(f[2]);
  long long nz[3] = {0, 0, 0};
  float maxd2 = 0.f;
  if (lane != 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) W[q] = 0.0;
    PE = 0.0;
  }
  if (active && lane == 0 && mode != MODE_DRY) {
    TailOut o;
    atom_tail<P>(a, C, t.cell, i, fc0, fc1, fc2, mode, o, xi);
#pragma unroll
    for (int q = 0; q < 6; ++q) K[q] = o.K[q];
    nz[0] = o.xi[0]; nz[1] = o.xi[1]; nz[2] = o.xi[2];
    maxd2 = o.maxd2;
  }
  double V[6];
  part_values(a, mode, W, K, V);
  write_part<NT, TPA>(a.parts, tb, V, PE, mode != MODE_STEP, nz, maxd2, status, psh);
}

// Sutton-Chen with n = 9, m = 6 is evaluated in powers of s3 = r^-3: with t = a / r,
// t^6 = a^6 s3^2 and t^9 = a^9 s3^3, and the pair scalar of pass 2 becomes
//   g / r = -r^-2 s3^2 (eps n a^9 s3 + m a^6 (F'_i + F'_j)),
// so pass 1 stores F' scaled by m a^6 (sc_fscale); other exponents store F' itself.
template <int SN, int SM>
__device__ __forceinline__ double sc_fscale(const MDArgs& a) {
  if constexpr (SN == 9 && SM == 6) {
    const double a3 = a.sc_a * a.sc_a * a.sc_a;
    return (double)a.sc_m * a3 * a3;
  } else {
    return 1.0;
  }
}

// Sutton-Chen pass 1: host density rho_i and F'(rho_i) = -eps c / (2 sqrt(rho_i)), stored in s.w
// (times sc_fscale)
template <class P, int TPA, int SN, int SM, class LT>
__global__ __launch_bounds__(TILE * TPA) void k_eam_rho(MDArgs a, int mode) {
  using R = typename P::R;
  const int tb = block_tile_xcd(a.ntiles, blockIdx.x);
  if (tb >= a.ntiles) return;
  const Tile t = a.tiles[tb];
  const CellDev& C = a.cells[t.cell];
  const int slot = threadIdx.x / TPA, lane = threadIdx.x % TPA;
  const bool active = slot < t.count && !(mode == MODE_PRIME && !C.pending) && !(mode == MODE_STATIC && C.fdone);
  const long long i = (long long)t.begin + slot;
  R rho = 0;
  if (active) {
    const typename P::S si = P::load(a.s_cur, i);
    const int nn = a.nn[i];
    const double a3 = a.sc_a * a.sc_a * a.sc_a;
    const R rc2 = (R)a.rc2, sa = (R)a.sc_a, sa6 = (R)(a3 * a3), rhoc = (R)a.sc_rhoc;
    const typename P::Geo g = P::geo(C);
    const typename P::S* sc = (const typename P::S*)a.s_cur + C.off;
    for (NbrWalk<P, TPA, LT> walk(a, i, nn, lane); walk.more();) {
      typename P::S sj[UNR];
      bool ok[UNR];
      walk.next(sc, sj, ok);
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        R d[3];
        P::sep(sj[u], si, g, d);
        const R r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        R tm;
        if constexpr (SN == 9 && SM == 6) {
          const R ri = P::rsq(r2), s3 = ri * ri * ri;
          tm = sa6 * (s3 * s3);
        } else {
          R tn;
          sc_powers<SN, SM>(sa * P::rsq(r2), a.sc_n, a.sc_m, tn, tm);
        }
        rho += (ok[u] && r2 < rc2) ? tm - rhoc : (R)0;
      }
    }
  }
  rho = lane_sum<TPA>(rho);
  if (active && lane == 0) {
    const R fp = rho > (R)0 ? (R)(-0.5 * a.sc_eps * a.sc_c * sc_fscale<SN, SM>(a)) / sqrt(rho) : (R)0;
    P::store_w(a.s_cur, i, fp);
  }
}

// Sutton-Chen pass 2: pair scalar g = eps phi'(r) + (F'_i + F'_j) rho'(r), then the tail
template <class P, int TPA, int SN, int SM, class LT>
__global__ __launch_bounds__(TILE * TPA) void k_force_eam(MDArgs a, int mode) {
  using R = typename P::R;
  constexpr int NT = TILE * TPA;
  __shared__ PartShared<NT / 64> psh;
  const int tb = block_tile_xcd(a.ntiles, blockIdx.x);
  if (tb >= a.ntiles) return;
  const Tile t = a.tiles[tb];
  const CellDev& C = a.cells[t.cell];
  const int slot = threadIdx.x / TPA, lane = threadIdx.x % TPA;
  const bool active = slot < t.count && !(mode == MODE_PRIME && !C.pending) && !(mode == MODE_STATIC && C.fdone);
  const long long i = (long long)t.begin + slot;
  R f[3] = {0, 0, 0}, pe = 0;
  double w[6] = {0, 0, 0, 0, 0, 0};
  R fpi = 0;
  if (active) {
    const typename P::S si = P::load(a.s_cur, i);
    fpi = P::get_w(si);
    const int nn = a.nn[i];
    const double a3 = a.sc_a * a.sc_a * a.sc_a;
    const R rc2 = (R)a.rc2, sa = (R)a.sc_a, en = (R)(a.sc_eps * a.sc_n), m = (R)a.sc_m;
    const R eh = (R)(0.5 * a.sc_eps), phic = (R)a.sc_phic;
    const R en9 = (R)(a.sc_eps * a.sc_n * a3 * a3 * a3), eh9 = (R)(0.5 * a.sc_eps * a3 * a3 * a3);
    const typename P::Geo g = P::geo(C);
    const typename P::S* sc = (const typename P::S*)a.s_cur + C.off;
    // the pair energy is summed only where it is reported: not in the middle steps of a run
    auto pairs = [&](auto with_pe) {
      for (NbrWalk<P, TPA, LT> walk(a, i, nn, lane); walk.more();) {
        typename P::S sj[UNR];
        bool ok[UNR];
        walk.next(sc, sj, ok);
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          R d[3];
          double dd[3];
          P::sep2(sj[u], si, g, d, dd);
          const R r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          const bool in = ok[u] && r2 < rc2;
          const R ri = P::rsq(r2);
          R g0, tn;                                                             // g / r, t^n
          if constexpr (SN == 9 && SM == 6) {
            const R ri2 = ri * ri, s3 = ri2 * ri, s6 = s3 * s3;
            g0 = -(ri2 * s6) * (en9 * s3 + (fpi + P::get_w(sj[u])));
            if constexpr (decltype(with_pe)::value) tn = s6 * s3;             // t^9 / a^9
          } else {
            R tm;
            sc_powers<SN, SM>(sa * ri, a.sc_n, a.sc_m, tn, tm);
            g0 = -(ri * ri) * (en * tn + (fpi + P::get_w(sj[u])) * m * tm);
          }
          const R gr = in ? g0 : (R)0;
          f[0] += gr * d[0]; f[1] += gr * d[1]; f[2] += gr * d[2];
          add_virial(w, (double)gr, dd);
          if constexpr (decltype(with_pe)::value) {
            if constexpr (SN == 9 && SM == 6) pe += in ? eh9 * tn - eh * phic : (R)0;
            else pe += in ? eh * (tn - phic) : (R)0;
          }
        }
      }
    };
    if (mode == MODE_STEP || mode == MODE_DRY) pairs(std::false_type{});
    else pairs(std::true_type{});
  }
  double W[6], K[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 6; ++q) W[q] = 0.5 * lane_sum<TPA>(w[q]);
  double PE = (double)lane_sum<TPA>(pe);
  const double fc0 = (double)lane_sum<TPA>(f[0]), fc1 = (double)lane_sum<TPA>(f[1]), fc2 = (double)lane_sum<TPA>(f[2]);
  long long xi[3] = {0, 0, 0};
  float maxd2 = 0.f;
  if (lane != 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) W[q] = 0.0;
    PE = 0.0;
  } else if (active && mode != MODE_STEP && mode != MODE_DRY) {
    // embedding energy -eps c sqrt(rho) = (eps c)^2 / (2 F'(rho)), zero where rho = 0
    const double ec = a.sc_eps * a.sc_c;
    if (fpi != (R)0) PE += ec * ec * sc_fscale<SN, SM>(a) / (2.0 * (double)fpi);
  }
  if (active && lane == 0 && mode != MODE_DRY) {
    TailOut o;
    atom_tail<P>(a, C, t.cell, i, fc0, fc1, fc2, mode, o);
#pragma unroll
    for (int q = 0; q < 6; ++q) K[q] = o.K[q];
    xi[0] = o.xi[0]; xi[1] = o.xi[1]; xi[2] = o.xi[2];
    maxd2 = o.maxd2;
  }
  double V[6];
  part_values(a, mode, W, K, V);
  write_part<NT, TPA>(a.parts, tb, V, PE, mode != MODE_STEP, xi, maxd2, 0, psh);
}

// First half kick and drift of a run (the remaining ones are fused into the force kernels).
template <class P>
__global__ __launch_bounds__(TILE) void k_start(MDArgs a) {
  __shared__ PartShared<1> psh;
  const int tb = block_tile(a.ntiles, blockIdx.x);
  if (tb >= a.ntiles) return;
  const Tile t = a.tiles[tb];
  const CellDev& C = a.cells[t.cell];
  const long long i = (long long)t.begin + threadIdx.x;
  long long xi[3] = {0, 0, 0};
  float maxd2 = 0.f;
  if ((int)threadIdx.x < t.count) {
    const double f0 = (double)((const typename P::Fst*)a.fx)[i];
    const double f1 = (double)((const typename P::Fst*)a.fy)[i];
    const double f2 = (double)((const typename P::Fst*)a.fz)[i];
    const double vx = a.vx[i] + a.h * f0, vy = a.vy[i] + a.h * f1, vz = a.vz[i] + a.h * f2;
    const double x = a.x[i] + a.dt * vx, y = a.y[i] + a.dt * vy, z = a.z[i] + a.dt * vz;
    a.vx[i] = vx; a.vy[i] = vy; a.vz[i] = vz;
    a.x[i] = x; a.y[i] = y; a.z[i] = z;
    const typename P::S sn = fixed_pos<P>(C, x, y, z);
    P::store_xyz(a.s_cur, i, sn);
    typename P::R d[3];
    P::disp(sn, a.sb[i], P::geo(C), d);
    maxd2 = (float)(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (a.gamma_on) {
      int k[3];
      noise_units(a, a.gid[i], t.cell, C.step + 1, k);
      xi[0] = k[0]; xi[1] = k[1]; xi[2] = k[2];
    }
  }
  const double Z[6] = {0, 0, 0, 0, 0, 0};
  write_part<TILE, 1>(a.parts, tb, Z, 0.0, false, xi, maxd2, 0, psh);
}

// ------------------------------------------------------------------ initial velocities
// Maxwell-Boltzmann velocities for the cells created without them (flag[cell] != 0), one block of
// MB_NT threads per cell, before the first neighbour build (atoms still in their original order):
// three normal variates per atom by the Box-Muller transform of four Philox4x32-10 uniforms
// u = (w + 1/2) 2^-32 (counter: atom, cell, and an all-ones step, a domain the Langevin noise never
// reaches; key: the seed), times sqrt(kB T / m); then the centre-of-mass velocity is removed and the
// velocities are scaled so that sum m v^2 = (3N - 3) kB T exactly.  The two sums run in a fixed tree.
constexpr int MB_NT = 256;
__global__ __launch_bounds__(MB_NT) void k_mb_velocities(MDArgs a, const int* flag, double sd, double dof_kt_m) {
  __shared__ double sh[MB_NT];
  const int c = blockIdx.x;
  if (!flag[c]) return;                           // uniform over the block
  const CellDev& C = a.cells[c];
  const int n = C.n;
  double s[3] = {0.0, 0.0, 0.0};
  for (int l = threadIdx.x; l < n; l += MB_NT) {
    uint32_t w[4];
    philox((uint32_t)l, (uint32_t)c, 0xFFFFFFFFu, 0xFFFFFFFFu, a.key0, a.key1, w);
    double u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = ((double)w[q] + 0.5) * 0x1.0p-32;
    const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    const double t0 = 2.0 * M_PI * u[1], t1 = 2.0 * M_PI * u[3];
    const long long i = (long long)C.off + l;
    a.vx[i] = sd * r0 * cos(t0);
    a.vy[i] = sd * r0 * sin(t0);
    a.vz[i] = sd * r1 * cos(t1);
    s[0] += a.vx[i]; s[1] += a.vy[i]; s[2] += a.vz[i];
  }
  double mean[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) mean[q] = block_sum<MB_NT>(s[q], sh) / (double)n;
  double k2 = 0.0;
  for (int l = threadIdx.x; l < n; l += MB_NT) {
    const long long i = (long long)C.off + l;
    const double vx = a.vx[i] - mean[0], vy = a.vy[i] - mean[1], vz = a.vz[i] - mean[2];
    a.vx[i] = vx; a.vy[i] = vy; a.vz[i] = vz;
    k2 += vx * vx + vy * vy + vz * vz;
  }
  k2 = block_sum<MB_NT>(k2, sh);
  const double scale = (n > 1 && k2 > 0.0) ? sqrt(dof_kt_m * (double)(3 * n - 3) / k2) : 0.0;
  for (int l = threadIdx.x; l < n; l += MB_NT) {
    const long long i = (long long)C.off + l;
    a.vx[i] *= scale; a.vy[i] *= scale; a.vz[i] *= scale;
  }
}

// ------------------------------------------------------------------ molecular statics (FIRE)
// Start of a relaxation: FIRE state of every cell, empty stress window, zero velocities.
__global__ void k_fire_cells(CellDev* cells, int ncells, double dt) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  CellDev& C = cells[c];
  C.fdt = dt; C.falpha = 0.1; C.fa = 1.0; C.fb = 0.0;
  C.fcount = 0; C.fdone = 0; C.ffreeze = 1; C.fiter = 0;
  for (int q = 0; q < 6; ++q) C.wsum[q] = 0.0;
  C.wcount = 0;
}

__global__ __launch_bounds__(TILE) void k_zero_v(MDArgs a) {
  const int tb = block_tile(a.ntiles, blockIdx.x);
  if (tb >= a.ntiles) return;
  const Tile t = a.tiles[tb];
  if ((int)threadIdx.x >= t.count) return;
  const long long i = (long long)t.begin + threadIdx.x;
  a.vx[i] = 0.0; a.vy[i] = 0.0; a.vz[i] = 0.0;
}

// One FIRE move of the atoms of unconverged cells: velocity mixing (or zero), v += dt f / m,
// x += dt v, new fixed-point coordinates and the displacement since the last build.
template <class P>
__global__ __launch_bounds__(TILE) void k_fire_move(MDArgs a) {
  __shared__ PartShared<1> psh;
  const int tb = block_tile(a.ntiles, blockIdx.x);
  if (tb >= a.ntiles) return;
  const Tile t = a.tiles[tb];
  const CellDev& C = a.cells[t.cell];
  const long long i = (long long)t.begin + threadIdx.x;
  float maxd2 = 0.f;
  if ((int)threadIdx.x < t.count && !C.fdone) {
    const double f0 = (double)((const typename P::Fst*)a.fx)[i];
    const double f1 = (double)((const typename P::Fst*)a.fy)[i];
    const double f2 = (double)((const typename P::Fst*)a.fz)[i];
    double vx = 0.0, vy = 0.0, vz = 0.0;
    if (!C.ffreeze) {
      vx = C.fa * a.vx[i] + C.fb * f0;
      vy = C.fa * a.vy[i] + C.fb * f1;
      vz = C.fa * a.vz[i] + C.fb * f2;
    }
    const double k = C.fdt * (2.0 * a.h / a.dt);    // dt / (m mvv2e)
    vx += k * f0; vy += k * f1; vz += k * f2;
    const double x = a.x[i] + C.fdt * vx, y = a.y[i] + C.fdt * vy, z = a.z[i] + C.fdt * vz;
    a.vx[i] = vx; a.vy[i] = vy; a.vz[i] = vz;
    a.x[i] = x; a.y[i] = y; a.z[i] = z;
    const typename P::S sn = fixed_pos<P>(C, x, y, z);
    P::store_xyz(a.s_cur, i, sn);
    typename P::R d[3];
    P::disp(sn, a.sb[i], P::geo(C), d);
    maxd2 = (float)(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  }
  const double Z[6] = {0, 0, 0, 0, 0, 0};
  const long long xi[3] = {0, 0, 0};
  write_part<TILE, 1>(a.parts, tb, Z, 0.0, false, xi, maxd2, 0, psh);
}

__global__ void k_fire_iters(const CellDev* cells, int ncells, int* iters, int* done) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  iters[c] = cells[c].fiter;
  done[c] = cells[c].fdone;
}

// Per-cell reduction of the tile partials: one wave per cell.  Lane t sums every 64th tile in
// order; the 64 lane sums of each of the 10 summed quantities (V, pe, xi) are then added through
// LDS in a fixed two-level order (four groups of 16 lanes, then the four group sums in order), so
// the result is deterministic for a given tile count.  The cell fields that the update reads are
// loaded at the start, beside the partials, so that none of them waits behind the reduction.
// Every thread of the block calls it (it holds two block barriers); threads from RED_NT on only
// take part in the barriers.
constexpr int RED_NT = 64;
constexpr int RED_Q = 10;         // V[6], pe, xi[3]
struct RedShared {
  double col[RED_Q][RED_NT + 1];
  double grp[4][RED_Q];
};
__device__ __forceinline__ void reduce_cell(const MDArgs& a, int cell, int mode, RedShared& sh) {
  CellDev& C = a.cells[cell];
  auto& col = sh.col;
  auto& grp = sh.grp;
  const int t = threadIdx.x;
  const int ntile = C.ntile, tile_off = C.tile_off;
  const int pending = C.pending, fdone = C.fdone;
  const int cstatus = C.status, crebuild = C.rebuild, cn = C.n;
  const float chs2 = C.hs2;
  const double cV = C.V;
  const long long cnreb = C.nrebuild, cwcount = C.wcount, cstep = C.step;
  double cw[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) cw[q] = C.wsum[q];
  double V[6] = {0, 0, 0, 0, 0, 0}, pe = 0;
  long long xi[3] = {0, 0, 0};
  float m = 0.f;
  int st = 0;
  for (int k = t; k < (t < RED_NT ? ntile : 0); k += RED_NT) {
    const Part& p = a.parts[tile_off + k];
#pragma unroll
    for (int q = 0; q < 6; ++q) V[q] += p.V[q];
    pe += p.pe;
    xi[0] += p.xi[0]; xi[1] += p.xi[1]; xi[2] += p.xi[2];
    m = fmaxf(m, p.maxd2);
    st = min(st, p.status);
  }
  if (mode == RED_PRIME && !pending) return;                              // uniform over the block
  if ((mode == RED_STATIC || mode == RED_MOVE) && fdone) return;
  if (t < RED_NT) {
#pragma unroll
    for (int q = 0; q < 6; ++q) col[q][t] = V[q];
    col[6][t] = pe;
#pragma unroll
    for (int q = 0; q < 3; ++q) col[7 + q][t] = __longlong_as_double(xi[q]);
  }
  const float md = wave_max(m);
  st = wave_min(st);
  __syncthreads();
  if (t < RED_NT) {
    const int q = t % 16, g = t / 16;
    const double* c = &col[q < RED_Q ? q : 0][g * 16];
    if (q < 7) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) s += c[k];
      grp[g][q] = s;
    } else if (q < RED_Q) {
      long long s = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) s += __double_as_longlong(c[k]);
      grp[g][q] = __longlong_as_double(s);
    }
  }
  __syncthreads();
  if (t != 0) return;
  double r[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) r[q] = ((grp[0][q] + grp[1][q]) + grp[2][q]) + grp[3][q];
  long long xs[3];
#pragma unroll
  for (int q = 0; q < 3; ++q)
    xs[q] = __double_as_longlong(grp[0][7 + q]) + __double_as_longlong(grp[1][7 + q]) +
            __double_as_longlong(grp[2][7 + q]) + __double_as_longlong(grp[3][7 + q]);
  const long long x0 = xs[0], x1 = xs[1], x2 = xs[2];
  if (st != 0 && cstatus == 0) C.status = st;
  if (mode == RED_MOVE) {                // statics: positions moved; rebuild when they left the skin
    C.rebuild = md > chs2;
    C.dmax2 = md;
    return;
  }
  if (mode == RED_STATIC) {              // statics: one FIRE decision per cell (same order as the oracle)
    C.pe = r[6];
    const double P = r[0], F2 = r[1], V2 = r[2];
    if ((double)md <= a.fire_ftol2 || st != 0 || C.fiter >= a.fire_max_iter) { C.fdone = 1; return; }
    if (P > 0.0) {
      if (++C.fcount > 5) { C.fdt = fmin(1.1 * C.fdt, 10.0 * a.dt); C.falpha *= 0.99; }
      C.fa = 1.0 - C.falpha;
      C.fb = C.falpha * sqrt(V2 / F2);
      C.ffreeze = 0;
    } else {
      C.fdt *= 0.5;
      C.falpha = 0.1;
      C.fcount = 0;
      C.ffreeze = 1;
    }
    C.fiter += 1;
    return;
  }
  if (crebuild) C.nrebuild = cnreb + 1;
  if (mode == RED_START) {
    C.rebuild = md > chs2;
    C.dmax2 = md;
    C.xi_mean[0] = (double)x0 / (double)cn;
    C.xi_mean[1] = (double)x1 / (double)cn;
    C.xi_mean[2] = (double)x2 / (double)cn;
    return;
  }
  double s[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) s[q] = r[q] / cV;
  if (mode != RED_STEP) C.pe = r[6];      // the middle steps of a run do not sum the energy
  if (mode == RED_PRIME) {
#pragma unroll
    for (int q = 0; q < 6; ++q) C.last[q] = s[q];
    C.rebuild = 0;
    C.pending = 0;
    return;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) { C.wsum[q] = cw[q] + s[q]; C.last[q] = s[q]; }
  C.wcount = cwcount + 1;
  C.step = cstep + 1;
  if (mode == RED_STEP) {
    C.rebuild = md > chs2;
    C.dmax2 = md;
    C.xi_mean[0] = (double)x0 / (double)cn;
    C.xi_mean[1] = (double)x1 / (double)cn;
    C.xi_mean[2] = (double)x2 / (double)cn;
  } else {
    C.rebuild = 0;
  }
}

__global__ __launch_bounds__(RED_NT) void k_reduce(MDArgs a, int mode) {
  __shared__ RedShared sh;
  reduce_cell(a, blockIdx.x, mode, sh);
}

// ------------------------------------------------------------------ neighbour build
// Neighbour build of the cells flagged for a rebuild, in four phases (each kernel exits at
// once for cells that are not flagged):
//   k_bin        per atom: wrap into the box, fixed-point S and the build reference, bin index
//                in scaled space, histogram (tiles)
//   k_bin_scan   exclusive scan of the histogram (one block per cell)
//   k_bin_fill   scatter of cell-local indices into their bins (tiles)
//   k_bin_sort   order every bin by atom index (one thread per bin), so that the neighbour lists
//                and the force sums built from them are deterministic
// atomicAdd(ctr + key, 1) for every valid lane of the wave, one atomic per run of equal keys in
// consecutive lanes: the atoms of a tile are stored in bin order from the last build and have
// mostly stayed in their bins, so neighbouring lanes usually share a key.  The run's first lane
// adds the run length and shares the old value; a lane's slot is that value plus its rank in the
// run (distinct slots, as with one atomic per lane).  Every lane of the wave calls this.
__device__ __forceinline__ int wave_run_add(int* ctr, int key, bool valid) {
  const int lane = (int)(threadIdx.x & 63u);
  const int pkey = __shfl_up(key, 1), pvalid = __shfl_up((int)valid, 1);
  const bool brk = !valid || lane == 0 || !pvalid || pkey != key;
  const unsigned long long breaks = __ballot(brk);
  const unsigned long long le = (2ull << lane) - 1ull;           // lanes <= this one (all for 63)
  const int head = 63 - __clzll(breaks & le);
  const unsigned long long gt = breaks & ~le;
  const int end = gt ? __ffsll((long long)gt) - 1 : 64;
  int old = 0;
  if (valid && head == lane) old = atomicAdd(ctr + key, end - lane);
  return __shfl(old, head) + (lane - head);
}

template <class P>
__device__ __forceinline__ int bin_one(const MDArgs& a, const CellDev& C, long long i) {
  double x = a.x[i], y = a.y[i], z = a.z[i];
  const double s0 = C.Hi[0] * x + C.Hi[1] * y + C.Hi[2] * z, s1 = C.Hi[4] * y + C.Hi[5] * z, s2 = C.Hi[8] * z;
  const double k0 = floor(s0), k1 = floor(s1), k2 = floor(s2);
  if (k0 != 0.0 || k1 != 0.0 || k2 != 0.0) {       // x -= H k (a lattice vector), H upper triangular
    x -= C.H[0] * k0 + C.H[1] * k1 + C.H[2] * k2;
    y -= C.H[4] * k1 + C.H[5] * k2;
    z -= C.H[8] * k2;
    a.x[i] = x; a.y[i] = y; a.z[i] = z;
  }
  double f[3];
  scaled_frac(C, x, y, z, f);
  const typename P::S sv = P::make(f[0], f[1], f[2]);
  P::store_xyz(a.s_cur, i, sv);
  a.sb[i] = P::quant(sv);
  int b[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) b[q] = min((int)(f[q] * C.nb[q]), C.nb[q] - 1);
  const int bin = (b[0] * C.nb[1] + b[1]) * C.nb[2] + b[2];
  a.abin[i] = b[0] | (b[1] << BIN_BITS) | (b[2] << (2 * BIN_BITS));   // packed bin coordinates
  return bin;
}

template <class P>
__device__ __forceinline__ void bin_atom(const MDArgs& a, const CellDev& C, long long i, bool valid) {
  int bin = -1;
  if (valid) bin = bin_one<P>(a, C, i);
  (void)wave_run_add(a.bcount + C.bin_off, bin, valid);
}

// Tile phases of a rebuild walk the work list: WORK_WAVES tiles per block, one wave per tile,
// block-strided over the tiles of the rebuilding cells, so a step in which few cells rebuild
// launches a small grid instead of one block per tile of the batch.
constexpr int WORK_WAVES = 4;
// the k with start[k] <= w < start[k + 1] in a strictly increasing prefix array of n + 1 entries
__device__ __forceinline__ int work_find(const int* start, int n, int w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}
// batch tile index of the w-th tile of the rebuild work list
__device__ __forceinline__ int work_tile(const MDArgs& a, int w) {
  const int k = work_find(a.work_tstart, a.work_count[0], w);
  return a.cells[a.work_cells[k]].tile_off + (w - a.work_tstart[k]);
}
template <class Fn>
__device__ __forceinline__ void for_work_tiles(const MDArgs& a, Fn&& fn) {
  const int lane = threadIdx.x & 63;
  const XcdLoop L(a.work_count[1], WORK_WAVES, threadIdx.x >> 6);
  for (int k = L.k; k < L.end; k += L.step) {
    const Tile t = a.tiles[work_tile(a, k)];
    if (lane < t.count) fn(t, (long long)t.begin + lane);
  }
}
// the same walk with every lane of the wave calling fn (valid: the lane holds an atom of the tile)
template <class Fn>
__device__ __forceinline__ void for_work_tiles_wave(const MDArgs& a, Fn&& fn) {
  const int lane = threadIdx.x & 63;
  const XcdLoop L(a.work_count[1], WORK_WAVES, threadIdx.x >> 6);
  for (int k = L.k; k < L.end; k += L.step) {
    const Tile t = a.tiles[work_tile(a, k)];
    const bool valid = lane < t.count;
    fn(t, (long long)t.begin + (valid ? lane : 0), valid);
  }
}

template <class P>
__global__ __launch_bounds__(TILE * WORK_WAVES) void k_bin(MDArgs a) {
  for_work_tiles_wave(a, [&](const Tile& t, long long i, bool valid) { bin_atom<P>(a, a.cells[t.cell], i, valid); });
}

// The displacement threshold for displacements measured against the 16-bit build reference: a
// measured displacement is within qeps of the true one, so the list stays complete while the
// measured one is at most the true bound (squared: hs2) minus qeps.
__device__ __forceinline__ float measured_threshold(double hs2, float qeps) {
  const double h = sqrt(fmax(hs2, 0.0)) - (double)qeps;
  return h > 0.0 ? (float)(h * h) : -1.0f;
}

constexpr int SCAN_NT = 1024;
// Exclusive scan of one value per thread over a block of SCAN_NT threads: an inclusive scan inside
// each wave by shuffles, the 16 wave totals scanned by the first wave through LDS (wsum: 16 ints),
// two barriers.  Returns the exclusive prefix; *total receives the block's sum.
__device__ __forceinline__ int block_exscan(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  if (wv == 0) {
    int w = lane < SCAN_NT / 64 ? wsum[lane] : 0;
#pragma unroll
    for (int o = 1; o < SCAN_NT / 64; o <<= 1) {
      const int y = __shfl_up(w, o);
      if (lane >= o) w += y;
    }
    if (lane < SCAN_NT / 64) wsum[lane] = w;
  }
  __syncthreads();
  const int before = wv > 0 ? wsum[wv - 1] : 0;
  *total = wsum[SCAN_NT / 64 - 1];
  __syncthreads();                 // wsum is reused by the next call
  return before + inc - v;
}

// exclusive scan of one cell's histogram by a block of SCAN_NT threads (sh: at least 16 ints of LDS)
__device__ __forceinline__ void scan_cell(const MDArgs& a, CellDev& C, int* sh) {
  const int nbins = C.nb[0] * C.nb[1] * C.nb[2];
  const int t = threadIdx.x;
  if (t == 0) {                    // the list about to be built holds every pair within rc + skin
    const int up[6] = {0, 1, 2, 4, 5, 8};
    for (int q = 0; q < 6; ++q) C.Hb[q] = C.H[up[q]];
    C.hs2 = measured_threshold(a.half_skin2, C.qeps);
    C.dmax2 = 0.f;
  }
  int carry = 0;
  for (int base = 0; base < nbins; base += SCAN_NT) {   // coalesced chunks of SCAN_NT bins
    const int b = base + t;
    const int c = b < nbins ? a.bcount[C.bin_off + b] : 0;
    int tot;
    const int ex = block_exscan(c, sh, &tot);
    if (b < nbins) {
      a.bstart[C.bin_off + b] = carry + ex;
      a.bnum[C.bin_off + b] = c;
      a.bfill[C.bin_off + b] = 0;
      a.bcount[C.bin_off + b] = 0;                        // ready for the next build
    }
    carry += tot;
  }
  __syncthreads();                 // the starts are read by other threads of a fused caller
}

// one block per rebuilding cell, block-strided over the work list
__global__ __launch_bounds__(SCAN_NT) void k_bin_scan(MDArgs a) {
  __shared__ int sh[SCAN_NT / 64];
  const XcdLoop L(a.work_count[0]);
  for (int k = L.k; k < L.end; k += L.step) scan_cell(a, a.cells[a.work_cells[k]], sh);
}

// The work list of a rebuild: the cells flagged for one, in cell order, with the prefix sums of
// their tiles and of their 64-bin chunks (a cell's bins start at a multiple of 64, so a chunk
// belongs to one cell).  One block of SCAN_NT threads: exclusive scans of the flags and counts.
__global__ __launch_bounds__(SCAN_NT) void k_rebuild_work(MDArgs a) {
  __shared__ int sh[SCAN_NT / 64];
  int bc = 0, bt = 0, bk = 0;
  for (int c0 = 0; c0 < a.ncells; c0 += SCAN_NT) {
    const int c = c0 + threadIdx.x;
    int fl = 0, nt = 0, nk = 0;
    if (c < a.ncells) {
      const CellDev& C = a.cells[c];
      if (C.rebuild) {
        fl = 1;
        nt = C.ntile;
        nk = (C.nb[0] * C.nb[1] * C.nb[2] + 63) / 64;
      }
    }
    int tc, tt, tk;
    const int ec = block_exscan(fl, sh, &tc);
    const int et = block_exscan(nt, sh, &tt);
    const int ek = block_exscan(nk, sh, &tk);
    if (fl) {
      a.work_cells[bc + ec] = c;
      a.work_tstart[bc + ec] = bt + et;
      a.work_kstart[bc + ec] = bk + ek;
    }
    bc += tc; bt += tt; bk += tk;
  }
  if (threadIdx.x == 0) {
    a.work_tstart[bc] = bt;
    a.work_kstart[bc] = bk;
    a.work_count[0] = bc; a.work_count[1] = bt; a.work_count[2] = bk;
  }
}

__device__ __forceinline__ void fill_atom(const MDArgs& a, const CellDev& C, long long i, bool valid) {
  int bin = -1;
  if (valid) {
    const int pk = a.abin[i];
    bin = ((pk & BIN_MASK) * C.nb[1] + ((pk >> BIN_BITS) & BIN_MASK)) * C.nb[2] + (pk >> (2 * BIN_BITS));
  }
  const int slot = wave_run_add(a.bfill + C.bin_off, bin, valid);
  if (valid) a.binned[C.off + a.bstart[C.bin_off + bin] + slot] = (int)(i - C.off);
}

__global__ __launch_bounds__(TILE * WORK_WAVES) void k_bin_fill(MDArgs a) {
  for_work_tiles_wave(a, [&](const Tile& t, long long i, bool valid) { fill_atom(a, a.cells[t.cell], i, valid); });
}

// one lane per bin slot of every cell (grid over the bin capacity), one wave per block.  Each bin
// is ordered by the original index (gid) of its atoms, so that the reorder that follows depends
// only on positions, not on earlier reorders.  When the wave's 64 bins fit in the cap keys of
// dynamic LDS (sized by the host from the expected bin occupancy) their keys are staged there and every lane rank-sorts its own bin (key v goes to position
// #{keys < v}; keys are distinct); otherwise bins of up to SMALL_BIN atoms are insertion-sorted by
// their lane and larger bins are rank-sorted by the whole wave, one after another, through the
// scratch array.  Sorted keys are mapped back to current cell-local indices through pos_of.
constexpr int SMALL_BIN = 24;
constexpr int SORT_LDS_MAX = 16384;  // staged keys per wave at most (64 KB)
__device__ __forceinline__ void sort_chunk(const MDArgs& a, const int* bin_cell, int cap, long long g, int* stage) {
  int big = 0;                       // this lane's bin needs the wave
  int *p = nullptr, n = 0, off = 0;
  {
    const int c = bin_cell[g];
    const CellDev& C = a.cells[c];
    const int b = (int)(g - C.bin_off);
    if (b < C.nb[0] * C.nb[1] * C.nb[2]) {
      p = a.binned + C.off + a.bstart[g];
      n = a.bnum[g];
      off = C.off;
    }
  }
  int incl = n;                      // exclusive offsets of the 64 bins in the staging array
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o);
    if ((int)threadIdx.x >= o) incl += v;
  }
  const int total = __shfl(incl, 63);
  if (total == 0) return;
  if (total <= cap) {
    int* sk = stage + (incl - n);
    for (int e = 0; e < n; ++e) sk[e] = a.gid[off + p[e]];
    __syncthreads();
    for (int e = 0; e < n; ++e) {
      const int v = sk[e];
      int rank = 0;
      for (int q = 0; q < n; ++q) rank += sk[q] < v;
      p[rank] = a.pos_of[off + v];
    }
    return;
  }
  for (int e = 0; e < n; ++e) p[e] = a.gid[off + p[e]];     // sort keys in place
  big = n > SMALL_BIN;
  if (!big)
    for (int u = 1; u < n; ++u) {
      const int v = p[u];
      int q = u - 1;
      while (q >= 0 && p[q] > v) { p[q + 1] = p[q]; --q; }
      p[q + 1] = v;
    }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  // large bins, one after another, by all 64 lanes
  unsigned long long mask = __ballot(big);
  while (mask) {
    const int src = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    int* pb = (int*)__shfl((long long)(size_t)p, src);
    const int m = __shfl(n, src);
    int* tmp = a.sort_tmp + (pb - a.binned);
    for (int e = threadIdx.x; e < m; e += 64) {
      const int v = pb[e];
      int rank = 0;
      for (int q = 0; q < m; ++q) rank += pb[q] < v;
      tmp[rank] = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    for (int e = threadIdx.x; e < m; e += 64) pb[e] = tmp[e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
  }
  for (int e = 0; e < n; ++e) p[e] = a.pos_of[off + p[e]];  // keys back to current indices
}

// one wave per 64-bin chunk of the rebuilding cells, block-strided over the work list
__global__ __launch_bounds__(64) void k_bin_sort(MDArgs a, const int* bin_cell, int cap) {
  extern __shared__ int stage[];
  const XcdLoop L(a.work_count[2]);
  for (int w = L.k; w < L.end; w += L.step) {
    __syncthreads();                 // the previous chunk's keys have been read
    const int k = work_find(a.work_kstart, a.work_count[0], w);
    const long long chunk = a.cells[a.work_cells[k]].bin_off / 64 + (w - a.work_kstart[k]);
    sort_chunk(a, bin_cell, cap, chunk * 64 + threadIdx.x, stage);
  }
}

// Reorder the atoms of every rebuilding cell by (bin, original index): position q of the cell
// receives the atom binned[q].  Phase 1 gathers positions, velocities, the fixed-point coordinates,
// bin coordinates and original indices into the scratch rows and records pos_of; phase 2 copies
// them back (also as the build reference) and rewrites the bond partners from bond0 through pos_of
// (inside the list build, or as the last phase of the one-block-per-cell preparation).
// The stored total force is not moved: the prime or last step of the run writes it afterwards.
template <class P>
struct Reorder {
  double *x, *y, *z, *vx, *vy, *vz;
  typename P::S* s;
  int *abin, *gid;
  __device__ explicit Reorder(const MDArgs& a) {
    const long long np = a.npad;
    x = (double*)a.pscr; y = x + np; z = y + np; vx = z + np; vy = vx + np; vz = vy + np;
    s = (typename P::S*)(vz + np);
    abin = (int*)(s + np); gid = abin + np;
  }
};

// the four partner slots of the atom at position i (cell-local positions, its own for an empty slot)
__device__ __forceinline__ void store_bonds(const MDArgs& a, long long i, int b0, int b1, int b2, int b3) {
  if (a.bond16)
    ((uint2*)a.bond)[i] = make_uint2((unsigned)b0 | ((unsigned)b1 << 16), (unsigned)b2 | ((unsigned)b3 << 16));
  else
    ((int4*)a.bond)[i] = make_int4(b0, b1, b2, b3);
}

template <class P>
__device__ __forceinline__ void reorder_gather_atom(const MDArgs& a, const CellDev& C, long long q) {
  const long long src = C.off + a.binned[q];
  const Reorder<P> r(a);
  r.x[q] = a.x[src]; r.y[q] = a.y[src]; r.z[q] = a.z[src];
  r.vx[q] = a.vx[src]; r.vy[q] = a.vy[src]; r.vz[q] = a.vz[src];
  r.s[q] = P::load(a.s_cur, src);
  r.abin[q] = a.abin[src];
  const int g = a.gid[src];
  r.gid[q] = g;
  a.pos_of[C.off + g] = (int)(q - C.off);
}

template <class P>
__global__ __launch_bounds__(TILE * WORK_WAVES) void k_reorder_gather(MDArgs a) {
  for_work_tiles(a, [&](const Tile& t, long long i) { reorder_gather_atom<P>(a, a.cells[t.cell], i); });
}

template <class P>
__device__ __forceinline__ void reorder_scatter_atom(const MDArgs& a, const CellDev& C, long long q) {
  const Reorder<P> r(a);
  a.x[q] = r.x[q]; a.y[q] = r.y[q]; a.z[q] = r.z[q];
  a.vx[q] = r.vx[q]; a.vy[q] = r.vy[q]; a.vz[q] = r.vz[q];
  const typename P::S sq = r.s[q];
  P::store_xyz(a.s_cur, q, sq);
  a.sb[q] = P::quant(sq);
  a.abin[q] = r.abin[q];
  const int g = r.gid[q];
  a.gid[q] = g;
  const int4 b0 = a.bond0[C.off + g];
  const int self = (int)(q - C.off);
  store_bonds(a, q, b0.x < 0 ? self : a.pos_of[C.off + b0.x], b0.y < 0 ? self : a.pos_of[C.off + b0.y],
              b0.z < 0 ? self : a.pos_of[C.off + b0.z], b0.w < 0 ? self : a.pos_of[C.off + b0.w]);
}


// The six preparation phases of a rebuild (bin, scan, fill, sort, reorder gather and scatter) for
// cells of at most PREP_ATOMS atoms: one block per cell runs them in turn, separated by block
// barriers, so a step in which no cell rebuilds costs one launch instead of six.  Same results as
// the phase kernels: the bins are ordered by original index (keys staged in LDS, each bin
// rank-sorted by one thread; keys are distinct), so the reorder depends only on positions.
constexpr int PREP_ATOMS = 4096;
template <class P>
__device__ __forceinline__ void prep_cell(const MDArgs& a, int cell, int* sh, int* key) {
  CellDev& C = a.cells[cell];
  const int n = C.n, t = threadIdx.x;
  for (int l0 = 0; l0 < n; l0 += SCAN_NT) {     // whole waves: the bin counts aggregate over lanes
    const bool v = l0 + t < n;
    bin_atom<P>(a, C, (long long)C.off + (v ? l0 + t : 0), v);
  }
  __syncthreads();
  scan_cell(a, C, sh);                       // ends with a barrier
  for (int l0 = 0; l0 < n; l0 += SCAN_NT) {
    const bool v = l0 + t < n;
    fill_atom(a, C, (long long)C.off + (v ? l0 + t : 0), v);
  }
  __syncthreads();
  for (int q = t; q < n; q += SCAN_NT) key[q] = a.gid[C.off + a.binned[C.off + q]];
  __syncthreads();
  const int nbins = C.nb[0] * C.nb[1] * C.nb[2];
  for (int b = t; b < nbins; b += SCAN_NT) {
    const int p0 = a.bstart[C.bin_off + b], m = a.bnum[C.bin_off + b];
    for (int e = 0; e < m; ++e) {
      const int v = key[p0 + e];
      int rank = 0;
      for (int q = 0; q < m; ++q) rank += key[p0 + q] < v;
      a.binned[C.off + p0 + rank] = a.pos_of[C.off + v];
    }
  }
  __syncthreads();
  for (int q = t; q < n; q += SCAN_NT) reorder_gather_atom<P>(a, C, (long long)C.off + q);
  __syncthreads();
  for (int q = t; q < n; q += SCAN_NT) reorder_scatter_atom<P>(a, C, (long long)C.off + q);
}

template <class P>
__global__ __launch_bounds__(SCAN_NT) void k_cell_prep(MDArgs a) {
  __shared__ int sh[SCAN_NT];
  __shared__ int key[PREP_ATOMS];
  if (!a.cells[blockIdx.x].rebuild) return;
  prep_cell<P>(a, blockIdx.x, sh, key);
}

// The per-cell reduction of a time step followed, in the same block, by the rebuild preparation
// of a cell that it flags (cells of at most PREP_ATOMS atoms): one launch instead of two per MD
// step.  The flag is read back through the device-coherent path after the barrier.
template <class P>
__global__ __launch_bounds__(SCAN_NT) void k_reduce_prep(MDArgs a, int mode) {
  __shared__ RedShared rsh;
  __shared__ int sh[SCAN_NT];
  __shared__ int key[PREP_ATOMS];
  reduce_cell(a, blockIdx.x, mode, rsh);
  __syncthreads();
  if (!__hip_atomic_load(&a.cells[blockIdx.x].rebuild, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  prep_cell<P>(a, blockIdx.x, sh, key);
}

// Original order for the atoms of cells [first, first + count) (create, set_state): gid and
// pos_of the identity, bonds as given.  Grid over all tiles.
__global__ __launch_bounds__(TILE) void k_reset_order(MDArgs a, int first, int count) {
  const int tb = block_tile(a.ntiles, blockIdx.x);
  if (tb >= a.ntiles) return;
  const Tile t = a.tiles[tb];
  if (t.cell < first || t.cell >= first + count || (int)threadIdx.x >= t.count) return;
  const long long i = (long long)t.begin + threadIdx.x;
  const int li = (int)(i - a.cells[t.cell].off);
  a.gid[i] = li;
  a.pos_of[i] = li;
  const int4 b0 = a.bond0[i];
  store_bonds(a, i, b0.x < 0 ? li : b0.x, b0.y < 0 ? li : b0.y, b0.z < 0 ? li : b0.z, b0.w < 0 ? li : b0.w);
}

// Verlet list of every atom (after the reorder, so positions are in bin order): cell-local j with
// |d| < rc + skin over the neighbour bins b - f ... b + f of every dimension (bins at least
// (rc + skin) / f wide).  Because the atoms are stored in bin order and bins are numbered with z
// fastest, the z-neighbour bins of each (x, y) column of the stencil are one contiguous range of
// positions (two at the periodic edge in z).  One lane per atom walks its ranges in stencil order,
// UNR candidates in flight, and appends every accepted one to its list: the list comes out in
// candidate order (nearly sorted by position, so its gathers hit few cache lines) and is
// deterministic.  A range's bounds come from the bin table while the previous range is walked.  The
// atoms of a wave are 64 consecutive atoms of one cell, mostly of a few neighbouring bins, so at a
// given step their lanes read the same or nearby positions.
constexpr int MAX_BIN_FACTOR = 2;
constexpr int BUILD_WAVES = 4;     // tiles per block of the list build, one per wave
struct BuildGeo {                  // one atom's stencil: bins per dimension and the z ranges
  int lo[3], cnt[3], nb[3];        // first neighbour bin (unwrapped) and count per dimension
  int zr[2][2], nzr;               // z bins [z0, z1] of every column, or two such ranges
  int ncol, nrange;
};
__device__ __forceinline__ void build_geo(const CellDev& C, int pk, int fb, BuildGeo& G) {
  const int bb[3] = {pk & BIN_MASK, (pk >> BIN_BITS) & BIN_MASK, pk >> (2 * BIN_BITS)};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    G.nb[q] = C.nb[q];
    // a pair within rc + skin is at most f bins apart in every dimension; a dimension with fewer
    // than 2 f + 1 bins is scanned whole
    if (G.nb[q] >= 2 * fb + 1) { G.lo[q] = bb[q] - fb; G.cnt[q] = 2 * fb + 1; }
    else { G.lo[q] = 0; G.cnt[q] = G.nb[q]; }
  }
  const int nbz = G.nb[2];
  G.zr[0][0] = 0; G.zr[0][1] = nbz - 1; G.zr[1][0] = 0; G.zr[1][1] = 0; G.nzr = 1;
  if (nbz >= 2 * fb + 1) {
    const int lo = bb[2] - fb, hi = bb[2] + fb;
    if (lo < 0) { G.zr[0][0] = 0; G.zr[0][1] = hi; G.zr[1][0] = lo + nbz; G.zr[1][1] = nbz - 1; G.nzr = 2; }
    else if (hi >= nbz) { G.zr[0][0] = lo; G.zr[0][1] = nbz - 1; G.zr[1][0] = 0; G.zr[1][1] = hi - nbz; G.nzr = 2; }
    else { G.zr[0][0] = lo; G.zr[0][1] = hi; }
  }
  G.ncol = G.cnt[0] * G.cnt[1];
  G.nrange = G.ncol * G.nzr;
}
// range r of the stencil (column-major over x, y, then the z parts): first position and count
__device__ __forceinline__ int2 build_range(const MDArgs& a, const CellDev& C, const BuildGeo& G, int r) {
  const int col = r / G.nzr, part = r - col * G.nzr;
  const int u0 = col / G.cnt[1], u1 = col - u0 * G.cnt[1];
  int x = G.lo[0] + u0, y = G.lo[1] + u1;
  x = x < 0 ? x + G.nb[0] : (x >= G.nb[0] ? x - G.nb[0] : x);
  y = y < 0 ? y + G.nb[1] : (y >= G.nb[1] ? y - G.nb[1] : y);
  const int bc = C.bin_off + (x * G.nb[1] + y) * G.nb[2];
  const int bf = bc + G.zr[part][0], bl = bc + G.zr[part][1];
  const int beg = a.bstart[bf];
  return make_int2(beg, a.bstart[bl] + a.bnum[bl] - beg);
}
// The reorder's second half for this atom happens here (its row copied from the reorder scratch to
// the per-atom arrays, bond partners renumbered), and the candidates are read from the scratch, which
// holds the same reordered coordinates: no other lane reads the arrays being written, and the
// rebuild needs no separate scatter launch.
template <class P, class LT>
__device__ __forceinline__ void build_tile(const MDArgs& a, const Tile& t, int slot) {
  if (slot >= t.count) return;
  const CellDev& C = a.cells[t.cell];
  const long long i = (long long)t.begin + slot;
  const int li = (int)(i - C.off);
  const Reorder<P> ro(a);
  reorder_scatter_atom<P>(a, C, i);
  const typename P::S* sbase = (const typename P::S*)ro.s;
  const typename P::S si = sbase[i];
  BuildGeo G;
  build_geo(C, ro.abin[i], a.bin_factor, G);
  const typename P::R rcs2 = (typename P::R)a.rcs2;
  const typename P::Geo g = P::geo(C);
  const typename P::S* sc = sbase + C.off;
  LT* const list = (LT*)a.nbr;
  const unsigned np = (unsigned)a.npad, ii = (unsigned)i;
  const int cap = a.maxnb;
  int count = 0;
  int2 cur = build_range(a, C, G, 0);
  for (int r = 0; r < G.nrange; ++r) {
    const int2 nxt = r + 1 < G.nrange ? build_range(a, C, G, r + 1) : make_int2(0, 0);
    for (int p = 0; p < cur.y; p += UNR) {
      int pos[UNR];
      typename P::S sj[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        pos[u] = p + u < cur.y ? cur.x + p + u : li;
        sj[u] = P::load_rel(sc, pos[u]);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        typename P::R d[3];
        P::sep(sj[u], si, g, d);
        if (pos[u] != li && d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < rcs2) {
          if (count < cap) list[list_index((unsigned)count, np, ii, a.lblk)] = (LT)pos[u];
          ++count;
        }
      }
    }
    cur = nxt;
  }
  if (count > cap) {
    atomicMin(&a.cells[t.cell].status, (int)ST_CAP);
    count = cap;
  }
  a.nn[i] = count;
}

// The tiles of the rebuild work list, one per wave, block-strided (XcdLoop), with the reorder's
// scatter fused in.  Rebuild sets of fewer than BUILD_SPLIT tiles leave most of the GPU idle with one
// lane per atom; there k_build_list_lanes builds the same lists with BUILD_LPA lanes per atom.
constexpr int BUILD_SPLIT = 4096;
template <class P, class LT>
__global__ __launch_bounds__(TILE * BUILD_WAVES) void k_build_list(MDArgs a) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (a.work_count[1] < BUILD_SPLIT) return;
  const XcdLoop L(a.work_count[1], BUILD_WAVES, wave);
  for (int k = L.k; k < L.end; k += L.step) build_tile<P, LT>(a, a.tiles[work_tile(a, k)], lane);
}

// The same lists for small rebuild sets, BUILD_LPA lanes per atom: the atom's ranges are looked up
// once into LDS, its lanes walk the concatenated candidates interleaved (lane l takes candidates l,
// l + BUILD_LPA, ...), and for each candidate slot a ballot over the atom's lanes gives every
// accepted candidate its index (the running count plus the accepted lanes below), so the list
// comes out in the same candidate order as with one lane per atom.  SCATTER: the reorder's scatter
// is fused in as in k_build_list (the atom's first lane copies its row); without it (after the
// one-block-per-cell preparation, which reorders completely) the candidates come from s_cur.
constexpr int BUILD_LPA = 8;
constexpr int MAX_RANGES = (2 * MAX_BIN_FACTOR + 1) * (2 * MAX_BIN_FACTOR + 1) * 2;
template <class P, class LT, bool SCATTER>
__device__ __forceinline__ void build_tile_lanes(const MDArgs& a, const Tile& t, int2 (*rng)[MAX_RANGES]) {
  const int slot = threadIdx.x / BUILD_LPA, lane = threadIdx.x % BUILD_LPA;
  const bool active = slot < t.count;
  const CellDev& C = a.cells[t.cell];
  const long long i = (long long)t.begin + (active ? slot : 0);
  const int li = (int)(i - C.off);
  const Reorder<P> ro(a);
  if constexpr (SCATTER) {
    if (active && lane == 0) reorder_scatter_atom<P>(a, C, i);
  }
  const typename P::S* sc = (SCATTER ? (const typename P::S*)ro.s : (const typename P::S*)a.s_cur) + C.off;
  const typename P::S si = sc[li];
  BuildGeo G;
  build_geo(C, SCATTER ? ro.abin[i] : a.abin[i], a.bin_factor, G);
  int2* rg = rng[slot];
  for (int r = lane; r < G.nrange; r += BUILD_LPA) rg[r] = build_range(a, C, G, r);
  __syncthreads();
  const typename P::R rcs2 = (typename P::R)a.rcs2;
  const typename P::Geo g = P::geo(C);
  const unsigned np = (unsigned)a.npad, ii = (unsigned)i;
  const unsigned gshift = (threadIdx.x & 63u) & ~(unsigned)(BUILD_LPA - 1), below = (1u << lane) - 1u;
  int count = 0;
  if (active && G.nrange > 0) {
    int r = 0, off = 0;                       // range r holds candidates [off, off + cur.y)
    int2 cur = rg[0];
    for (int c0 = lane;; c0 += UNR * BUILD_LPA) {
      int pos[UNR];
      bool ok[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int c = c0 + u * BUILD_LPA;
        while (r < G.nrange && c >= off + cur.y) {
          off += cur.y;
          if (++r < G.nrange) cur = rg[r];
        }
        ok[u] = r < G.nrange;
        pos[u] = ok[u] ? cur.x + (c - off) : li;
      }
      if (!ok[0]) break;
      typename P::S sj[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) sj[u] = P::load_rel(sc, pos[u]);
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        bool acc = false;
        if (ok[u] && pos[u] != li) {
          typename P::R d[3];
          P::sep(sj[u], si, g, d);
          acc = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < rcs2;
        }
        const unsigned gm = (unsigned)(__ballot(acc) >> gshift) & ((1u << BUILD_LPA) - 1u);
        if (acc) {
          const int k = count + __popc(gm & below);
          if (k < a.maxnb) ((LT*)a.nbr)[list_index((unsigned)k, np, ii, a.lblk)] = (LT)pos[u];
        }
        count += __popc(gm);
      }
      if (!ok[UNR - 1]) break;
    }
  }
  // the atom's total: its lanes stop counting when their own candidates end, so take the largest
  int n = count;
#pragma unroll
  for (int o = 1; o < BUILD_LPA; o <<= 1) n = max(n, __shfl_xor(n, o, BUILD_LPA));
  if (active && lane == 0) {
    if (n > a.maxnb) {
      atomicMin(&a.cells[t.cell].status, (int)ST_CAP);
      n = a.maxnb;
    }
    a.nn[i] = n;
  }
}

// use_work: the work list's tiles, block-strided (XcdLoop), when there are fewer than BUILD_SPLIT;
// else one block per tile of the batch (placed like the force passes), exiting at once for cells
// that do not rebuild
template <class P, class LT>
__global__ __launch_bounds__(TILE * BUILD_LPA) void k_build_list_lanes(MDArgs a, int use_work) {
  __shared__ int2 rng[TILE][MAX_RANGES];      // candidate ranges (first position, count) per atom
  if (use_work) {
    if (a.work_count[1] >= BUILD_SPLIT) return;
    const XcdLoop L(a.work_count[1]);
    for (int k = L.k; k < L.end; k += L.step) {
      __syncthreads();                        // the previous tile's ranges have been read
      build_tile_lanes<P, LT, true>(a, a.tiles[work_tile(a, k)], rng);
    }
  } else {
    const int tb = block_tile_xcd(a.ntiles, blockIdx.x);
    if (tb >= a.ntiles) return;
    const Tile t = a.tiles[tb];
    if (!a.cells[t.cell].rebuild) return;
    build_tile_lanes<P, LT, false>(a, t, rng);
  }
}

// ------------------------------------------------------------------ QR box remap (Eqs. 4, 5, 9)
__device__ inline double det3(const double A[9]) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) + A[2] * (A[3] * A[7] - A[4] * A[6]);
}
__device__ inline void mat3mul(const double A[9], const double B[9], double C[9]) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}
__device__ inline void upper_inv(const double U[9], double Ui[9]) {   // inverse of an upper-triangular matrix
  const double a = U[0], b = U[1], c = U[2], d = U[4], e = U[5], f = U[8];
  Ui[0] = 1.0 / a; Ui[1] = -b / (a * d); Ui[2] = (b * e - c * d) / (a * d * f);
  Ui[3] = 0.0; Ui[4] = 1.0 / d; Ui[5] = -e / (d * f);
  Ui[6] = 0.0; Ui[7] = 0.0; Ui[8] = 1.0 / f;
}
__device__ inline void box_widths(const double H[9], double w[3]) {  // w_k = V / |a_i x a_j| for columns of H
  const double V = fabs(det3(H));
  for (int k = 0; k < 3; ++k) {
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    const double u0 = H[i], u1 = H[3 + i], u2 = H[6 + i], v0 = H[j], v1 = H[3 + j], v2 = H[6 + j];
    const double cx = u1 * v2 - u2 * v1, cy = u2 * v0 - u0 * v2, cz = u0 * v1 - u1 * v0;
    w[k] = V / sqrt(cx * cx + cy * cy + cz * cz);
  }
}

// F = Q R by classical Gram-Schmidt on the columns of F with one re-orthogonalisation pass;
// R_jj = |v_j| > 0.  Returns 0 or ST_BAD_F (non-finite F, det F <= 0, R_jj < 1e-12 |F|_F).
__device__ inline int qr_gs(const double F[9], double Q[9], double R[9]) {
  double fn = 0.0;
  for (int k = 0; k < 9; ++k) {
    if (!isfinite(F[k])) return ST_BAD_F;
    fn += F[k] * F[k];
    R[k] = 0.0;
  }
  fn = sqrt(fn);
  if (!(det3(F) > 0.0)) return ST_BAD_F;
  double q[3][3];
  for (int j = 0; j < 3; ++j) {
    double v0 = F[j], v1 = F[3 + j], v2 = F[6 + j];
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        const double s = q[i][0] * v0 + q[i][1] * v1 + q[i][2] * v2;
        R[3 * i + j] += s;
        v0 -= s * q[i][0]; v1 -= s * q[i][1]; v2 -= s * q[i][2];
      }
    const double nv = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    if (!(nv >= 1e-12 * fn)) return ST_BAD_F;
    R[3 * j + j] = nv;
    q[j][0] = v0 / nv; q[j][1] = v1 / nv; q[j][2] = v2 / nv;
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Q[3 * r + c] = q[c][r];
  return 0;
}

// keep |yz| <= ly/2, |xz| <= lx/2, |xy| <= lx/2 by subtracting integer multiples of box edges
__device__ inline void tilt_reduce(double H[9]) {
  if (fabs(H[5]) > 0.5 * H[4]) { const double k = floor(H[5] / H[4] + 0.5); H[2] -= k * H[1]; H[5] -= k * H[4]; }
  if (fabs(H[2]) > 0.5 * H[0]) { const double k = floor(H[2] / H[0] + 0.5); H[2] -= k * H[0]; }
  if (fabs(H[1]) > 0.5 * H[0]) { const double k = floor(H[1] / H[0] + 0.5); H[1] -= k * H[0]; }
}

// stage everything a deformation needs; no state is modified (bw: the bin width, (rc + skin) / f)
__global__ void k_qr_stage(const double* Fall, const CellDev* cells, Stage* st, int ncells, double rcs, double bw) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  Stage& S = st[c];
  const CellDev& C = cells[c];
  for (int k = 0; k < 9; ++k) S.F[k] = Fall[9 * c + k];
  S.status = qr_gs(S.F, S.Q, S.R);
  if (S.status) return;
  double Ri[9];
  upper_inv(C.Rprev, Ri);
  mat3mul(S.R, Ri, S.dR);                       // Eq. (9)
  S.dR[3] = S.dR[6] = S.dR[7] = 0.0;
  mat3mul(S.dR, C.H, S.Hn);                     // H <- Delta R H
  S.Hn[3] = S.Hn[6] = S.Hn[7] = 0.0;
  tilt_reduce(S.Hn);
  S.J = S.R[0] * S.R[4] * S.R[8];
  double w[3];
  box_widths(S.Hn, w);
  S.wmin = fmin(w[0], fmin(w[1], w[2]));
  if (rcs > 0.5 * S.wmin) { S.status = ST_BOX; return; }
  for (int q = 0; q < 3; ++q) S.nb[q] = min(BIN_MASK, max(1, (int)floor(w[q] / bw)));
  S.nbins = S.nb[0] * S.nb[1] * S.nb[2];
  S.density = (double)C.n / fabs(det3(S.Hn));
}

// fill the derived box fields of a cell from C.H (bw: the bin width)
__device__ inline void set_box_fields(CellDev& C, double bw) {
  upper_inv(C.H, C.Hi);
  C.V = det3(C.H);
  const int up[6] = {0, 1, 2, 4, 5, 8};
  for (int q = 0; q < 6; ++q) {
    const double hs = C.H[up[q]] * TWOM32;
    C.Hm[q] = hs;
    C.Hd[q] = hs * TWOM32;
  }
  // the 16-bit build reference is within 2^-17 of the position in each scaled coordinate, so a
  // measured displacement is within |H|_F sqrt(3) 2^-17 of the true one (with a relative margin for
  // the FP32 arithmetic of the check)
  double hf = 0.0;
  for (int q = 0; q < 6; ++q) hf += C.H[up[q]] * C.H[up[q]];
  C.qeps = (float)(1.001 * sqrt(3.0 * hf) * 0x1.0p-17);
  double w[3];
  box_widths(C.H, w);
  for (int q = 0; q < 3; ++q) C.nb[q] = min(BIN_MASK, max(1, (int)floor(w[q] / bw)));
  // never exceed the bins allocated to this cell: coarser bins are still valid (>= the bin width)
  while (C.nb[0] * C.nb[1] * C.nb[2] > max(C.bin_cap, 1)) {
    int q = 0;
    if (C.nb[1] > C.nb[q]) q = 1;
    if (C.nb[2] > C.nb[q]) q = 2;
    C.nb[q] -= 1;
  }
}

// Whether the neighbour list survives a box change.  With A = H Hb^-1 the affine map since the
// last build and u the largest atom displacement since then (measured in the current box), a pair
// left out of the list (|d_build| >= rc + skin) is now at least sigma_min(A) (rc + skin) - 2 u
// apart, and sigma_min(A) >= 1 - |A - I|_F.  The list therefore still holds every pair within rc
// while u <= ((1 - |A - I|_F)(rc + skin) - rc) / 2; that bound becomes the cell's displacement
// threshold.  A rebuild is forced when it is not positive, or when the displacement the atoms
// already have exceeds it: the remap x <- dR x leaves the scaled offsets since the build unchanged,
// so it stretches the last measured displacement by at most |dR|_2 <= 1 + |dR - I|_F.
__device__ inline float kept_list_threshold(const CellDev& C, double rc, double rcs) {
  const double Hb[9] = {C.Hb[0], C.Hb[1], C.Hb[2], 0.0, C.Hb[3], C.Hb[4], 0.0, 0.0, C.Hb[5]};
  double Hbi[9], A[9];
  upper_inv(Hb, Hbi);
  mat3mul(C.H, Hbi, A);
  double e2 = 0.0;
  for (int k = 0; k < 9; ++k) {
    const double d = A[k] - ((k % 4 == 0) ? 1.0 : 0.0);
    e2 += d * d;
  }
  const double hs = 0.5 * ((1.0 - sqrt(e2)) * rcs - rc);
  return hs > 0.0 ? (float)(hs * hs) : -1.0f;
}

__global__ void k_qr_commit(CellDev* cells, const Stage* st, int ncells, double rc, double rcs, double bw,
                            int force_build) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  CellDev& C = cells[c];
  const Stage& S = st[c];
  for (int k = 0; k < 9; ++k) {
    C.H[k] = S.Hn[k]; C.Q[k] = S.Q[k]; C.R[k] = S.R[k]; C.Rprev[k] = S.R[k]; C.F[k] = S.F[k];
  }
  C.J = S.J;
  const float qeps_old = C.qeps;
  set_box_fields(C, bw);
  for (int q = 0; q < 6; ++q) C.wsum[q] = 0.0;
  C.wcount = 0;
  const float hs2 = kept_list_threshold(C, rc, rcs);
  double e2 = 0.0;
  for (int k = 0; k < 9; ++k) {
    const double d = S.dR[k] - ((k % 4 == 0) ? 1.0 : 0.0);
    e2 += d * d;
  }
  const double grow = 1.0 + sqrt(e2);
  const double u = (sqrt((double)C.dmax2) + (double)qeps_old) * grow;   // bound on the true displacement
  const float hs2m = hs2 > 0.0f ? measured_threshold((double)hs2, C.qeps) : -1.0f;
  const bool moved = !(hs2 > 0.0f) || u * u >= (double)hs2;
  if (force_build || C.rebuild || moved || !(hs2m > 0.0f)) {
    C.rebuild = 1;
  } else {
    C.hs2 = hs2m;
  }
  C.pending = 1;
}

// x <- Delta R x for every atom (affine remap, Eq. 6 applied incrementally), with the fixed-point
// scaled coordinates of the remapped positions in the committed box (they equal the old ones up
// to rounding: the remap leaves S = H^-1 x unchanged)
template <class P>
__global__ __launch_bounds__(TILE) void k_remap(MDArgs a, const Stage* st) {
  const int tb = block_tile(a.ntiles, blockIdx.x);
  if (tb >= a.ntiles) return;
  const Tile t = a.tiles[tb];
  if ((int)threadIdx.x >= t.count) return;
  const double* d = st[t.cell].dR;
  const long long i = (long long)t.begin + threadIdx.x;
  const double x = a.x[i], y = a.y[i], z = a.z[i];
  const double xn = d[0] * x + d[1] * y + d[2] * z, yn = d[4] * y + d[5] * z, zn = d[8] * z;
  a.x[i] = xn; a.y[i] = yn; a.z[i] = zn;
  P::store_xyz(a.s_cur, i, fixed_pos<P>(a.cells[t.cell], xn, yn, zn));
}

// set a cell's box from H (create / set_state) and request a rebuild + prime
__global__ void k_set_box(CellDev* cells, int first, int count, double bw) {
  const int c = first + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= first + count) return;
  CellDev& C = cells[c];
  set_box_fields(C, bw);
  for (int q = 0; q < 6; ++q) C.wsum[q] = 0.0;
  C.wcount = 0;
  C.rebuild = 1;
  C.pending = 1;
}

// ------------------------------------------------------------------ stress return (Eqs. 7, 8)
__global__ void k_stress_out(CellDev* cells, int ncells, double* sig, double* P, double* smd) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  CellDev& C = cells[c];
  double sv[6];
  for (int q = 0; q < 6; ++q) sv[q] = C.wcount > 0 ? C.wsum[q] / (double)C.wcount : C.last[q];
  if (smd)
    for (int q = 0; q < 6; ++q) smd[6 * c + q] = sv[q];
  const double s[9] = {sv[0], sv[3], sv[4], sv[3], sv[1], sv[5], sv[4], sv[5], sv[2]};
  double Qt[9], T[9], Sf[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) Qt[3 * r + k] = C.Q[3 * k + r];
  mat3mul(C.Q, s, T);
  mat3mul(T, Qt, Sf);                              // sigma_FEM = Q sigma_MD Q^T
  const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
  bool finite = true;
  for (int q = 0; q < 6; ++q) {
    sig[6 * c + q] = Sf[3 * ia[q] + ib[q]];
    finite = finite && isfinite(Sf[3 * ia[q] + ib[q]]);
  }
  if (!finite && C.status == 0) C.status = -5;
  if (P) {
    const double* F = C.F;
    const double d = det3(F);
    // F^-T: transpose of the adjugate over det
    double FiT[9];
    FiT[0] = (F[4] * F[8] - F[5] * F[7]) / d; FiT[3] = (F[2] * F[7] - F[1] * F[8]) / d; FiT[6] = (F[1] * F[5] - F[2] * F[4]) / d;
    FiT[1] = (F[5] * F[6] - F[3] * F[8]) / d; FiT[4] = (F[0] * F[8] - F[2] * F[6]) / d; FiT[7] = (F[2] * F[3] - F[0] * F[5]) / d;
    FiT[2] = (F[3] * F[7] - F[4] * F[6]) / d; FiT[5] = (F[1] * F[6] - F[0] * F[7]) / d; FiT[8] = (F[0] * F[4] - F[1] * F[3]) / d;
    double Pm[9];
    mat3mul(Sf, FiT, Pm);                          // P = J sigma_FEM F^-T
    for (int q = 0; q < 9; ++q) P[9 * c + q] = C.J * Pm[q];
  }
  for (int q = 0; q < 6; ++q) C.wsum[q] = 0.0;
  C.wcount = 0;
}

// kinetic energy 1/2 sum m v^2 per cell (one block per cell, fixed order)
__global__ __launch_bounds__(RED_NT) void k_kinetic(MDArgs a, double* ke) {
  const CellDev& C = a.cells[blockIdx.x];
  double s = 0.0;
  for (int k = threadIdx.x; k < C.n; k += RED_NT) {
    const long long i = (long long)C.off + k;
    s += a.vx[i] * a.vx[i] + a.vy[i] * a.vy[i] + a.vz[i] * a.vz[i];
  }
  s = wave_sum(s);
  if (threadIdx.x == 0) ke[blockIdx.x] = 0.5 * a.mmv * s;
}

// Eq. (4) for a batch of deformation gradients (no cell state): Q, R, status per F
__global__ void k_qr_batch(const double* F, int n, double* Q, double* R, int* status) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double f[9], q[9], r[9];
  for (int k = 0; k < 9; ++k) f[k] = F[9 * c + k];
  const int st = qr_gs(f, q, r);
  for (int k = 0; k < 9; ++k) { Q[9 * c + k] = st ? 0.0 : q[k]; R[9 * c + k] = st ? 0.0 : r[k]; }
  if (status) status[c] = st;
}

// Eqs. (7), (8) for a batch: sigma_FEM = Q sigma_MD Q^T and P = J sigma_FEM F^-T, with Q and
// J = prod R_ii from the QR of each F (Voigt in and out; non-finite output for a bad F)
__global__ void k_return_batch(const double* F, const double* smd, int n, double* sfem, double* P) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double f[9], Q[9], R[9];
  for (int k = 0; k < 9; ++k) f[k] = F[9 * c + k];
  const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
  if (qr_gs(f, Q, R)) {
    for (int q = 0; q < 6; ++q) sfem[6 * c + q] = __longlong_as_double(0x7ff8000000000000LL);
    if (P) for (int q = 0; q < 9; ++q) P[9 * c + q] = __longlong_as_double(0x7ff8000000000000LL);
    return;
  }
  const double* sv = smd + 6 * c;
  const double s[9] = {sv[0], sv[3], sv[4], sv[3], sv[1], sv[5], sv[4], sv[5], sv[2]};
  double Qt[9], T[9], Sf[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) Qt[3 * r + k] = Q[3 * k + r];
  mat3mul(Q, s, T);
  mat3mul(T, Qt, Sf);
  for (int q = 0; q < 6; ++q) sfem[6 * c + q] = Sf[3 * ia[q] + ib[q]];
  if (P) {
    const double d = det3(f);
    double FiT[9];
    FiT[0] = (f[4] * f[8] - f[5] * f[7]) / d; FiT[3] = (f[2] * f[7] - f[1] * f[8]) / d; FiT[6] = (f[1] * f[5] - f[2] * f[4]) / d;
    FiT[1] = (f[5] * f[6] - f[3] * f[8]) / d; FiT[4] = (f[0] * f[8] - f[2] * f[6]) / d; FiT[7] = (f[2] * f[3] - f[0] * f[5]) / d;
    FiT[2] = (f[3] * f[7] - f[4] * f[6]) / d; FiT[5] = (f[1] * f[6] - f[0] * f[7]) / d; FiT[8] = (f[0] * f[4] - f[1] * f[3]) / d;
    double Pm[9];
    mat3mul(Sf, FiT, Pm);
    const double J = R[0] * R[4] * R[8];
    for (int q = 0; q < 9; ++q) P[9 * c + q] = J * Pm[q];
  }
}

// a new bin width for every cell: bin counts recomputed from the box; the list stays valid and the
// next build uses the new bins
__global__ void k_set_bin_width(CellDev* cells, int ncells, double bw) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncells) set_box_fields(cells[c], bw);
}

__global__ void k_set_pending(CellDev* cells, int first, int count) {
  const int c = first + blockIdx.x * blockDim.x + threadIdx.x;
  if (c < first + count) { cells[c].rebuild = 1; cells[c].pending = 1; }
}

}  // namespace rcell
