// Host side of the batched r-cell MD C ABI (include/rcell.h): context lifetime, memory layout,
// argument marshalling (AoS <-> SoA), and the launch sequence of every call.  All arithmetic of
// the method runs in the kernels of md_device.h.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rcell.h"
#include "md_device.h"

using namespace rcell;

namespace {

thread_local std::string g_create_error;

// A roctx range over a scope: every API call and every phase it enqueues shows up as a named range
// in a marker trace (rocprofv3 --marker-trace); without a profiler the calls cost a few ns.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePush(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace

struct rcell_ctx {
  rcell_params p{};
  bool fp64 = false;
  int ncells = 0;
  long long N = 0, npad = 0;
  int ntiles = 0;
  int maxnb = 0;
  int lanes = 1;
  int bin_factor = 1;             // bins at least (rc + skin) / bin_factor wide
  int cur = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::vector<int> off, n, tile_off, ntile, bin_off, bin_cap;
  long long bins_total = 0, bins_alloc = 0;
  std::vector<double> occ;        // expected atoms per bin of each cell
  double density_max = 0.0;       // the densest cell at create (atoms per volume)
  double fire_ftol2 = 0.0;        // statics: convergence threshold and move limit of the current call
  int fire_max_iter = 0;
  int sort_cap = 256;             // keys staged in LDS per wave by the bin sort
  // device memory
  double *x = nullptr, *y = nullptr, *z = nullptr, *vx = nullptr, *vy = nullptr, *vz = nullptr;
  void *fx = nullptr, *fy = nullptr, *fz = nullptr;
  void *s[2] = {nullptr, nullptr};
  uint2* sb = nullptr;            // build reference, 16 bits per scaled coordinate
  void* bond = nullptr;           // 4 partner slots per atom, 16-bit when list16 else 32-bit
  int4* bond0 = nullptr;
  int *gid = nullptr, *pos_of = nullptr;
  char* pscr = nullptr;           // reorder scratch rows
  void* nbr = nullptr;
  bool list16 = false;            // 16-bit list entries (every cell has at most 65536 atoms, mixed)
  bool small_cells = false;       // every cell has at most PREP_ATOMS atoms
  bool cell_prep = false;         // rebuild preparation by one block per cell (k_cell_prep)
  int *nn = nullptr, *abin = nullptr, *binned = nullptr, *bin_cell = nullptr, *sort_tmp = nullptr;
  int *bcount = nullptr, *bstart = nullptr, *bnum = nullptr, *bfill = nullptr;
  // rebuild work list (k_rebuild_work): cells, prefix sums of their tiles and chunks, three counts
  int *work_cells = nullptr, *work_tstart = nullptr, *work_kstart = nullptr, *work_count = nullptr;
  CellDev* cells = nullptr;
  Tile* tiles = nullptr;
  Part* parts = nullptr;
  Stage* stage = nullptr;
  double* dscratch = nullptr;     // ncells * 17 doubles: F / sigma + P / kinetic, then pe
  double* dscratch2 = nullptr;    // ncells * 6 doubles: MD-frame stress
  int* iscratch = nullptr;        // ncells ints
  long long* lscratch = nullptr;  // ncells long longs
  std::vector<void*> allocs;
  // fault injection for tests of the error paths: the fault_alloc-th device allocation of this
  // context fails as if the device were out of memory (RCELL_FAULT_ALLOC at create; 0 = off)
  int fault_alloc = 0, n_alloc = 0;
  // captured MD steps: graph[p] holds graph_steps middle steps starting from buffer parity p
  int graph_steps = 10;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  // kernel timing (rcell_prof_*): pending event pairs per pass, and a pool of free events
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[2];
  std::vector<hipEvent_t> ev_pool;
};

namespace {

void drop_graphs(rcell_ctx* c) {
  for (int q = 0; q < 2; ++q)
    if (c->graph[q]) { (void)hipGraphExecDestroy(c->graph[q]); c->graph[q] = nullptr; }
}

// the bin sort stages twice the expected keys of its 64 bins in LDS (a fuller wave falls back to
// the slower paths); a change of that size invalidates the captured graphs
void set_occupancy(rcell_ctx* c, int cell, double atoms_per_bin) {
  c->occ[cell] = atoms_per_bin;
  double m = 0.0;
  for (double o : c->occ) m = std::max(m, o);
  const int cap = (int)std::min<double>(SORT_LDS_MAX, std::max(256.0, 2.0 * 64.0 * std::ceil(m) + 64.0));
  if (cap != c->sort_cap) {
    drop_graphs(c);
    c->sort_cap = cap;
  }
}

int fail(rcell_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail((ctx), RCELL_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
int dalloc(rcell_ctx* c, T** out, size_t count) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  if (c && c->fault_alloc > 0 && ++c->n_alloc == c->fault_alloc)
    return fail(c, RCELL_ERR_OOM, "injected failure of device allocation " + std::to_string(c->n_alloc) +
                                      " (" + std::to_string(bytes) + " bytes)");
  const hipError_t r = hipMalloc(&p, bytes);
  if (r != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, r == hipErrorOutOfMemory || r == hipErrorMemoryAllocation ? RCELL_ERR_OOM : RCELL_ERR_DEVICE,
                "device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(r));
  }
  c->allocs.push_back(p);
  *out = (T*)p;
  return RCELL_OK;
}

void dfree(rcell_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  (void)hipFree(p);
}

double width_min(const double H[9]) {   // host-side validation of a box against rc + skin
  auto col = [&](int k, double v[3]) { v[0] = H[k]; v[1] = H[3 + k]; v[2] = H[6 + k]; };
  double a[3][3];
  for (int k = 0; k < 3; ++k) col(k, a[k]);
  const double V = std::fabs(a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                             a[1][0] * (a[0][1] * a[2][2] - a[0][2] * a[2][1]) +
                             a[2][0] * (a[0][1] * a[1][2] - a[0][2] * a[1][1]));
  double w = 1e300;
  for (int k = 0; k < 3; ++k) {
    const double* u = a[(k + 1) % 3];
    const double* v = a[(k + 2) % 3];
    const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
    w = std::min(w, V / std::sqrt(cx * cx + cy * cy + cz * cz));
  }
  return w;
}

// host twin of the device's bin count: floor of each perpendicular width over rc + skin
int bins_exact(const double H[9], double rcs) {
  auto col = [&](int k, double v[3]) { v[0] = H[k]; v[1] = H[3 + k]; v[2] = H[6 + k]; };
  double a[3][3];
  for (int k = 0; k < 3; ++k) col(k, a[k]);
  const double V = std::fabs(a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                             a[1][0] * (a[0][1] * a[2][2] - a[0][2] * a[2][1]) +
                             a[2][0] * (a[0][1] * a[1][2] - a[0][2] * a[1][1]));
  long long nb = 1;
  for (int k = 0; k < 3; ++k) {
    const double* u = a[(k + 1) % 3];
    const double* v = a[(k + 2) % 3];
    const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
    const double w = V / std::sqrt(cx * cx + cy * cy + cz * cz);
    nb *= std::min(BIN_MASK, std::max(1, (int)std::floor(w / rcs)));
  }
  return (int)std::min<long long>(nb, 1 << 30);
}

int bins_for(const double H[9], double rcs) {
  // an upper bound on floor(w0/rcs) floor(w1/rcs) floor(w2/rcs): V / rcs^3
  const double V = H[0] * H[4] * H[8];
  return std::max(1, (int)std::floor(V / (rcs * rcs * rcs)));
}

double bin_width(const rcell_ctx* c) { return (c->p.rc + c->p.skin) / c->bin_factor; }

int list_capacity(double density, double rcs) {
  const double expect = density * 4.0 / 3.0 * M_PI * rcs * rcs * rcs;
  return (int)std::ceil(1.6 * expect + 24.0);
}

MDArgs make_args(const rcell_ctx* c) {
  MDArgs a{};
  a.x = c->x; a.y = c->y; a.z = c->z; a.vx = c->vx; a.vy = c->vy; a.vz = c->vz;
  a.fx = c->fx; a.fy = c->fy; a.fz = c->fz;
  a.s_cur = c->s[c->cur]; a.s_nxt = c->s[1 - c->cur]; a.sb = c->sb;
  a.bond = c->bond; a.bond0 = c->bond0; a.bond16 = c->list16 ? 1 : 0;
  a.gid = c->gid; a.pos_of = c->pos_of; a.pscr = c->pscr;
  a.nn = c->nn; a.nbr = c->nbr; a.npad = c->npad; a.maxnb = c->maxnb;
  a.lblk = c->p.potential == RCELL_POT_KG ? 3 : 4;   // list blocks of 8 (short KG lists) or 16 entries
  a.cells = c->cells; a.tiles = c->tiles; a.parts = c->parts; a.ntiles = c->ntiles; a.ncells = c->ncells;
  a.abin = c->abin; a.bcount = c->bcount; a.bstart = c->bstart; a.bnum = c->bnum; a.bfill = c->bfill;
  a.binned = c->binned;
  a.sort_tmp = c->sort_tmp;
  a.bins_total = c->bins_total;
  a.work_cells = c->work_cells; a.work_tstart = c->work_tstart; a.work_kstart = c->work_kstart;
  a.work_count = c->work_count;
  a.bin_factor = c->bin_factor;
  const rcell_params& p = c->p;
  // integrator constants: the same expressions, in the same order, as the method's definition
  a.dt = p.dt;
  a.fire_ftol2 = c->fire_ftol2;
  a.fire_max_iter = c->fire_max_iter;
  a.h = p.dt / (2.0 * p.mass * p.mvv2e);
  a.drag = -(p.gamma * p.mass * p.mvv2e);
  a.c24 = std::sqrt(24.0 * p.gamma * p.mass * p.kB * p.temperature * p.mvv2e / p.dt) * 0x1.0p-24;
  a.mmv = p.mass * p.mvv2e;
  a.half_skin2 = 0.25 * p.skin * p.skin;
  a.rcs2 = (p.rc + p.skin) * (p.rc + p.skin);
  a.key0 = (uint32_t)p.seed;
  a.key1 = (uint32_t)(p.seed >> 32);
  a.gamma_on = p.gamma > 0.0;
  a.include_kinetic = p.include_kinetic;
  a.pot = p.potential;
  a.rc2 = p.rc * p.rc;
  a.lj_eps = p.lj_eps;
  a.lj_sig2 = p.lj_sigma * p.lj_sigma;
  {
    const double sr6 = std::pow(p.lj_sigma / p.rc, 6.0);
    a.lj_shift = 4.0 * p.lj_eps * (sr6 * sr6 - sr6);
  }
  a.fene_K = p.fene_K;
  a.fene_R02 = p.fene_R0 * p.fene_R0;
  a.sc_eps = p.sc_eps; a.sc_a = p.sc_a; a.sc_c = p.sc_c;
  a.sc_n = p.sc_n; a.sc_m = p.sc_m;
  a.sc_phic = p.potential == RCELL_POT_SC_EAM ? std::pow(p.sc_a / p.rc, p.sc_n) : 0.0;
  a.sc_rhoc = p.potential == RCELL_POT_SC_EAM ? std::pow(p.sc_a / p.rc, p.sc_m) : 0.0;
  return a;
}

// ---------------------------------------------------------------- launch helpers
hipEvent_t prof_event(rcell_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Timing of the pair passes (rcell_prof_*): the start and stop events are those of the kernel
// dispatch itself (hipExtLaunchKernel), so a pair holds the kernel's own duration, without the
// queue and launch latency that events recorded around the launch would add.
bool prof_pair(rcell_ctx* c, hipEvent_t* e0, hipEvent_t* e1) {
  if (!c->prof || !(*e0 = prof_event(c))) return false;
  if (!(*e1 = prof_event(c))) {
    c->ev_pool.push_back(*e0);
    return false;
  }
  return true;
}

#define LAUNCH_PASS(c, which, kernel, grid, block, ...)                                      \
  do {                                                                                       \
    hipEvent_t e0_ = nullptr, e1_ = nullptr;                                                 \
    if (prof_pair(c, &e0_, &e1_)) {                                                          \
      hipExtLaunchKernelGGL(kernel, grid, block, 0, (c)->stream, e0_, e1_, 0, __VA_ARGS__);  \
      (c)->prof_ev[which].push_back({e0_, e1_});                                             \
    } else {                                                                                 \
      hipLaunchKernelGGL(kernel, grid, block, 0, (c)->stream, __VA_ARGS__);                  \
    }                                                                                        \
  } while (0)

template <class P, int TPA, int SN, int SM, class LT>
void force_eam_t(rcell_ctx* c, const MDArgs& a, int mode) {
  const dim3 grid(tile_grid(c->ntiles)), block(TILE * TPA);
  LAUNCH_PASS(c, 1, (k_eam_rho<P, TPA, SN, SM, LT>), grid, block, a, mode);
  LAUNCH_PASS(c, 0, (k_force_eam<P, TPA, SN, SM, LT>), grid, block, a, mode);
}

template <class P, int TPA, class LT>
void force_t(rcell_ctx* c, const MDArgs& a, int mode) {
  if (c->p.potential == RCELL_POT_KG) {
    LAUNCH_PASS(c, 0, (k_force_kg<P, TPA, LT>), dim3(tile_grid(c->ntiles)), dim3(TILE * TPA), a, mode);
  } else if (a.sc_n == 9 && a.sc_m == 6) {      // copper, nickel: exponents fixed at compile time
    force_eam_t<P, TPA, 9, 6, LT>(c, a, mode);
  } else {
    force_eam_t<P, TPA, 0, 0, LT>(c, a, mode);
  }
}

template <class P, class LT>
void force_p(rcell_ctx* c, const MDArgs& a, int mode, int lanes) {
  switch (lanes) {
    case 2: force_t<P, 2, LT>(c, a, mode); break;
    case 4: force_t<P, 4, LT>(c, a, mode); break;
    case 8: force_t<P, 8, LT>(c, a, mode); break;
    case 16: force_t<P, 16, LT>(c, a, mode); break;
    default: force_t<P, 1, LT>(c, a, mode); break;
  }
}

void launch_force_args(rcell_ctx* c, const MDArgs& a, int mode, int l) {
  if (c->fp64) force_p<FP64, int>(c, a, mode, l);
  else if (c->list16) force_p<Mixed, uint16_t>(c, a, mode, l);
  else force_p<Mixed, int>(c, a, mode, l);
}

void launch_force(rcell_ctx* c, int mode, int lanes = -1) {
  TraceRange tr(mode == MODE_STEP ? "rcell: force pass + integration" : "rcell: force pass");
  launch_force_args(c, make_args(c), mode, lanes > 0 ? lanes : c->lanes);
}

void launch_reduce(rcell_ctx* c, int mode) {
  const MDArgs a = make_args(c);
  hipLaunchKernelGGL(k_reduce, dim3(c->ncells), dim3(RED_NT), 0, c->stream, a, mode);
}

// blocks of the block-strided rebuild phases: enough to fill the GPU when many cells rebuild,
// few enough that a step without rebuilds costs little
constexpr int WORK_BLOCKS = 2048;
unsigned round8(int blocks) { return (unsigned)((std::max(1, blocks) + 7) / 8 * 8); }

// reduce_mode >= 0: the per-cell reduction of that mode runs first, fused into the preparation
// launch when the cells are small enough for it
void launch_build(rcell_ctx* c, int reduce_mode = -1) {
  TraceRange tr("rcell: reduce + neighbour rebuild");
  const MDArgs a = make_args(c);
  const dim3 gt(tile_grid(c->ntiles)), bt(TILE), gc(c->ncells), bc(SCAN_NT);
  if (c->cell_prep) {              // small cells: the six preparation phases in one launch
    if (reduce_mode >= 0) {
      if (c->fp64) hipLaunchKernelGGL(k_reduce_prep<FP64>, gc, bc, 0, c->stream, a, reduce_mode);
      else hipLaunchKernelGGL(k_reduce_prep<Mixed>, gc, bc, 0, c->stream, a, reduce_mode);
    } else {
      if (c->fp64) hipLaunchKernelGGL(k_cell_prep<FP64>, gc, bc, 0, c->stream, a);
      else hipLaunchKernelGGL(k_cell_prep<Mixed>, gc, bc, 0, c->stream, a);
    }
  } else {
    // the phases walk the work list of the cells that rebuild: small grids, block-strided
    if (reduce_mode >= 0) launch_reduce(c, reduce_mode);
    hipLaunchKernelGGL(k_rebuild_work, dim3(1), dim3(SCAN_NT), 0, c->stream, a);
    // grids of whole multiples of 8 blocks: the loops share the work out per XCD (XcdLoop)
    const dim3 gw(round8(std::min(WORK_BLOCKS, (c->ntiles + WORK_WAVES - 1) / WORK_WAVES))), bw(TILE * WORK_WAVES);
    const dim3 gs(round8(std::min(c->ncells, WORK_BLOCKS / 8)));
    const dim3 gk(round8((int)std::min<long long>(4 * WORK_BLOCKS, c->bins_total / 64)));
    if (c->fp64) hipLaunchKernelGGL(k_bin<FP64>, gw, bw, 0, c->stream, a);
    else hipLaunchKernelGGL(k_bin<Mixed>, gw, bw, 0, c->stream, a);
    hipLaunchKernelGGL(k_bin_scan, gs, bc, 0, c->stream, a);
    hipLaunchKernelGGL(k_bin_fill, gw, bw, 0, c->stream, a);
    hipLaunchKernelGGL(k_bin_sort, gk, dim3(64), sizeof(int) * c->sort_cap, c->stream, a,
                       (const int*)c->bin_cell, c->sort_cap);
    // the reorder's scatter runs inside the list build (build_tile)
    if (c->fp64) hipLaunchKernelGGL(k_reorder_gather<FP64>, gw, bw, 0, c->stream, a);
    else hipLaunchKernelGGL(k_reorder_gather<Mixed>, gw, bw, 0, c->stream, a);
  }
  const int use_work = c->cell_prep ? 0 : 1;
  if (use_work) {                  // large rebuild sets: one lane per atom
    const dim3 gl(round8(std::min(WORK_BLOCKS, (c->ntiles + BUILD_WAVES - 1) / BUILD_WAVES))), bl(TILE * BUILD_WAVES);
    if (c->fp64) hipLaunchKernelGGL((k_build_list<FP64, int>), gl, bl, 0, c->stream, a);
    else if (c->list16) hipLaunchKernelGGL((k_build_list<Mixed, uint16_t>), gl, bl, 0, c->stream, a);
    else hipLaunchKernelGGL((k_build_list<Mixed, int>), gl, bl, 0, c->stream, a);
  }
  // small rebuild sets, and every build after the one-block-per-cell preparation: the same lists
  // with several lanes per atom
  const dim3 gs2(use_work ? round8(std::min(WORK_BLOCKS, c->ntiles)) : (unsigned)tile_grid(c->ntiles)),
      bs2(TILE * BUILD_LPA);
  if (c->fp64) hipLaunchKernelGGL((k_build_list_lanes<FP64, int>), gs2, bs2, 0, c->stream, a, use_work);
  else if (c->list16) hipLaunchKernelGGL((k_build_list_lanes<Mixed, uint16_t>), gs2, bs2, 0, c->stream, a, use_work);
  else hipLaunchKernelGGL((k_build_list_lanes<Mixed, int>), gs2, bs2, 0, c->stream, a, use_work);
}

void launch_start(rcell_ctx* c) {
  const MDArgs a = make_args(c);
  if (c->fp64) hipLaunchKernelGGL(k_start<FP64>, dim3(tile_grid(c->ntiles)), dim3(TILE), 0, c->stream, a);
  else hipLaunchKernelGGL(k_start<Mixed>, dim3(tile_grid(c->ntiles)), dim3(TILE), 0, c->stream, a);
}

// neighbour build + conservative forces for every cell flagged pending
int prime(rcell_ctx* c) {
  launch_build(c);
  launch_force(c, MODE_PRIME);
  launch_reduce(c, RED_PRIME);
  HIPCHK(c, hipGetLastError());
  return RCELL_OK;
}

struct Gathered {
  std::vector<int> status;
  std::vector<double> pe;
  std::vector<long long> nreb, step;
};

__global__ void k_gather(const CellDev* cells, int ncells, int* st, double* pe, long long* nreb, long long* step) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  st[c] = cells[c].status;
  pe[c] = cells[c].pe;
  nreb[c] = cells[c].nrebuild;
  step[c] = cells[c].step;
}

__global__ void k_set_bins(CellDev* cells, int ncells, const int* off, const int* cap) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  cells[c].bin_off = off[c];
  cells[c].bin_cap = cap[c];
}

int gather(rcell_ctx* c, Gathered& g) {
  const int nc = c->ncells;
  double* pe = c->dscratch + 16 * nc;
  long long* nreb = c->lscratch;
  long long* step = c->lscratch + nc;
  hipLaunchKernelGGL(k_gather, dim3((nc + 127) / 128), dim3(128), 0, c->stream, c->cells, nc, c->iscratch, pe, nreb, step);
  g.status.resize(nc); g.pe.resize(nc); g.nreb.resize(nc); g.step.resize(nc);
  HIPCHK(c, hipMemcpyAsync(g.status.data(), c->iscratch, sizeof(int) * nc, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(g.pe.data(), pe, sizeof(double) * nc, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(g.nreb.data(), nreb, sizeof(long long) * nc, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(g.step.data(), step, sizeof(long long) * nc, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RCELL_OK;
}

int first_error(rcell_ctx* c, const std::vector<int>& st) {
  for (size_t k = 0; k < st.size(); ++k)
    if (st[k] != 0) {
      const char* what = st[k] == RCELL_ERR_BOND ? "FENE bond reached R0" :
                         st[k] == RCELL_ERR_STATE ? "neighbour capacity exceeded" :
                         st[k] == RCELL_ERR_NONFINITE ? "non-finite stress" : "cell error";
      return fail(c, st[k], std::string(what) + " in cell " + std::to_string(k));
    }
  return RCELL_OK;
}

// the host's bin layout (offsets, capacities) into the device cell table
int push_bin_layout(rcell_ctx* c) {
  int *doff = c->iscratch, *dcap = c->iscratch + c->ncells;
  HIPCHK(c, hipMemcpyAsync(doff, c->bin_off.data(), sizeof(int) * c->ncells, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(dcap, c->bin_cap.data(), sizeof(int) * c->ncells, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_set_bins, dim3((c->ncells + 127) / 128), dim3(128), 0, c->stream, c->cells, c->ncells, doff, dcap);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RCELL_OK;
}

// lay out bins with capacity caps (>= need), update the device cell table
int layout_bins(rcell_ctx* c, const std::vector<int>& need) {
  drop_graphs(c);
  long long total = 0;
  std::vector<int> off(c->ncells), cap(c->ncells);
  for (int k = 0; k < c->ncells; ++k) {
    // whole 64-bin chunks per cell: the bin sort works on chunks of one cell each
    cap[k] = (std::max(need[k], c->bin_cap.empty() ? 0 : c->bin_cap[k]) + 63) / 64 * 64;
    off[k] = (int)total;
    total += cap[k];
  }
  if (total > (1ll << 31) - 1) return fail(c, RCELL_ERR_OOM, "too many neighbour bins");
  if (total > c->bins_alloc) {
    dfree(c, c->bcount); dfree(c, c->bstart); dfree(c, c->bnum); dfree(c, c->bfill); dfree(c, c->bin_cell);
    c->bcount = c->bstart = c->bnum = c->bfill = c->bin_cell = nullptr;
    int st;
    if ((st = dalloc(c, &c->bcount, total)) || (st = dalloc(c, &c->bstart, total)) ||
        (st = dalloc(c, &c->bnum, total)) || (st = dalloc(c, &c->bfill, total)) ||
        (st = dalloc(c, &c->bin_cell, total)))
      return st;
    HIPCHK(c, hipMemsetAsync(c->bcount, 0, sizeof(int) * total, c->stream));
    c->bins_alloc = total;
  }
  c->bins_total = total;
  std::vector<int> owner(total);
  for (int k = 0; k < c->ncells; ++k)
    for (int b = 0; b < cap[k]; ++b) owner[off[k] + b] = k;
  HIPCHK(c, hipMemcpyAsync(c->bin_cell, owner.data(), sizeof(int) * total, hipMemcpyHostToDevice, c->stream));
  c->bin_off = off;
  c->bin_cap = cap;
  return push_bin_layout(c);
}

int ensure_list_capacity(rcell_ctx* c, int need) {
  need = (need + NBLK_MAX - 1) / NBLK_MAX * NBLK_MAX;   // whole list blocks of either length
  if (need <= c->maxnb) return RCELL_OK;
  // the pair loops address the list with 32-bit element indices
  if ((unsigned long long)need * (unsigned long long)c->npad >= (1ull << 32))
    return fail(c, RCELL_ERR_OOM, "neighbour list would exceed 2^32 entries (16 GiB); split the batch");
  drop_graphs(c);
  // the new list is allocated before the old one is freed: on failure the context keeps its list
  // and its capacity
  char* q = nullptr;
  const int st = dalloc(c, &q, (size_t)need * c->npad * (c->list16 ? sizeof(uint16_t) : sizeof(int)));
  if (st) return st;
  dfree(c, c->nbr);
  c->nbr = q;
  c->maxnb = need;
  return RCELL_OK;
}

void destroy_all(rcell_ctx* c) {
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  for (int w = 0; w < 2; ++w)
    for (auto& pr : c->prof_ev[w]) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  c->prof_ev[0].clear(); c->prof_ev[1].clear(); c->ev_pool.clear();
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  c->stream = nullptr;
}

int deformation_common(rcell_ctx* c, const double* F_dev) {
  TraceRange tr("rcell_set_deformation");
  const int nc = c->ncells;
  const double rcs = c->p.rc + c->p.skin;
  hipLaunchKernelGGL(k_qr_stage, dim3((nc + 63) / 64), dim3(64), 0, c->stream, F_dev, c->cells, c->stage, nc, rcs,
                     bin_width(c));
  std::vector<Stage> st(nc);
  HIPCHK(c, hipMemcpyAsync(st.data(), c->stage, sizeof(Stage) * nc, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < nc; ++k)
    if (st[k].status != 0)
      return fail(c, st[k].status, (st[k].status == RCELL_ERR_BOX ? std::string("box too small for rc + skin")
                                                                   : std::string("bad deformation gradient")) +
                                       " in cell " + std::to_string(k));
  std::vector<int> need(nc);
  double dens = 0.0;
  bool grow = false;
  for (int k = 0; k < nc; ++k) {
    need[k] = st[k].nbins;
    set_occupancy(c, k, (double)c->n[k] / std::max(1, st[k].nbins));
    grow = grow || need[k] > c->bin_cap[k];
    dens = std::max(dens, st[k].density);
  }
  int e;
  if (grow && (e = layout_bins(c, need))) return e;
  const int cap = list_capacity(dens, rcs);
  const int relist = cap > c->maxnb;               // a reallocated list must be rebuilt everywhere
  if ((e = ensure_list_capacity(c, cap))) return e;
  hipLaunchKernelGGL(k_qr_commit, dim3((nc + 63) / 64), dim3(64), 0, c->stream, c->cells, c->stage, nc, c->p.rc,
                     rcs, bin_width(c), relist);
  const MDArgs a = make_args(c);
  if (c->fp64) hipLaunchKernelGGL(k_remap<FP64>, dim3(tile_grid(c->ntiles)), dim3(TILE), 0, c->stream, a, c->stage);
  else hipLaunchKernelGGL(k_remap<Mixed>, dim3(tile_grid(c->ntiles)), dim3(TILE), 0, c->stream, a, c->stage);
  return prime(c);
}

// Bins of every cell at the width (rc + skin) / f for its current box: the layout grows when a
// cell needs more bins; the list stays valid and the next build uses the new bins.
int apply_bin_factor(rcell_ctx* c, int f) {
  const int nc = c->ncells;
  std::vector<CellDev> hc(nc);
  HIPCHK(c, hipMemcpyAsync(hc.data(), c->cells, sizeof(CellDev) * nc, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double bw = (c->p.rc + c->p.skin) / f;
  std::vector<int> need(nc);
  bool grow = false;
  for (int k = 0; k < nc; ++k) {
    need[k] = bins_for(hc[k].H, bw);
    set_occupancy(c, k, (double)c->n[k] / bins_exact(hc[k].H, bw));
    grow = grow || need[k] > c->bin_cap[k];
  }
  drop_graphs(c);                                  // the captured steps carry the bin factor
  c->bin_factor = f;
  int e;
  if (grow && (e = layout_bins(c, need))) return e;
  hipLaunchKernelGGL(k_set_bin_width, dim3((nc + 63) / 64), dim3(64), 0, c->stream, c->cells, nc, bw);
  HIPCHK(c, hipGetLastError());
  return RCELL_OK;
}

// choices of rcell_autotune, per process, keyed by what decides them: potential, precision, list
// entry width, skin, the densest cell and the size ranges of the cells and of the batch
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, long, long, int, int>, std::pair<int, int>> g_tune_cache;

std::tuple<int, int, int, long, long, int, int> tune_key(const rcell_ctx* c) {
  double dens = 0.0;
  for (int k = 0; k < c->ncells; ++k) dens = std::max(dens, (double)c->n[k]);
  const int nmax = (int)std::floor(std::log2(std::max(1.0, dens)));
  return std::make_tuple(c->p.potential, c->p.precision, c->list16 ? 1 : 0, std::lround(c->p.skin * 1000.0),
                         std::lround(c->density_max * 100.0), nmax,
                         (int)std::floor(std::log2(std::max(1.0, (double)c->N))));
}

}  // namespace

// ================================================================= C ABI
extern "C" {

int rcell_create(const rcell_params* params, const rcell_cell_init* cells, int32_t ncells, void* hip_stream,
                 rcell_ctx** out) {
  TraceRange tr("rcell_create");
  if (!out) return fail(nullptr, RCELL_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!params || !cells || ncells < 1) return fail(nullptr, RCELL_ERR_ARG, "params, cells and ncells >= 1 are required");
  const rcell_params& p = *params;
  if (p.potential != RCELL_POT_KG && p.potential != RCELL_POT_SC_EAM)
    return fail(nullptr, RCELL_ERR_ARG, "unknown potential");
  if (p.precision != RCELL_PREC_FP64 && p.precision != RCELL_PREC_MIXED)
    return fail(nullptr, RCELL_ERR_ARG, "unknown precision");
  if (!(p.dt > 0) || !(p.mass > 0) || !(p.mvv2e > 0) || !(p.rc > 0) || !(p.skin >= 0) || !(p.gamma >= 0) ||
      !(p.temperature >= 0) || !(p.kB >= 0))
    return fail(nullptr, RCELL_ERR_ARG, "dt, mass, mvv2e, rc must be > 0; skin, gamma, temperature, kB >= 0");
  if (p.potential == RCELL_POT_KG && (!(p.lj_sigma > 0) || !(p.fene_R0 > 0)))
    return fail(nullptr, RCELL_ERR_ARG, "KG needs lj_sigma > 0 and fene_R0 > 0");
  if (p.potential == RCELL_POT_SC_EAM && (!(p.sc_a > 0) || p.sc_n < 1 || p.sc_m < 1 || p.sc_n > 31 || p.sc_m > 31))
    return fail(nullptr, RCELL_ERR_ARG, "Sutton-Chen needs sc_a > 0 and 1 <= n, m <= 31");
  const double rcs = p.rc + p.skin;

  rcell_ctx* c = new (std::nothrow) rcell_ctx();
  if (!c) return fail(nullptr, RCELL_ERR_OOM, "host allocation failed");
  if (const char* fa = std::getenv("RCELL_FAULT_ALLOC")) c->fault_alloc = std::atoi(fa);
  c->p = p;
  c->fp64 = p.precision == RCELL_PREC_FP64;
  c->ncells = ncells;
  c->lanes = p.potential == RCELL_POT_SC_EAM ? 8 : 1;
  auto bail = [&](int code) {
    g_create_error = c->err.empty() ? g_create_error : c->err;
    destroy_all(c);
    delete c;
    return code;
  };
  // ---- host validation and layout
  long long N = 0;
  int ntiles = 0;
  double dens = 0.0;
  std::vector<int> need_bins(ncells);
  for (int k = 0; k < ncells; ++k) {
    const rcell_cell_init& ci = cells[k];
    if (ci.natoms < 1 || !ci.H0 || !ci.x || ci.nbonds < 0 || (ci.nbonds > 0 && !ci.bonds))
      return bail(fail(c, RCELL_ERR_ARG, "cell " + std::to_string(k) + ": natoms >= 1, H0 and x are required"));
    const double* H = ci.H0;
    if (!(H[0] > 0 && H[4] > 0 && H[8] > 0) || H[3] != 0 || H[6] != 0 || H[7] != 0)
      return bail(fail(c, RCELL_ERR_ARG, "cell " + std::to_string(k) + ": H0 must be upper triangular with positive diagonal"));
    if (0.5 * width_min(H) < rcs)
      return bail(fail(c, RCELL_ERR_BOX, "cell " + std::to_string(k) + ": box too small for rc + skin"));
    c->off.push_back((int)N);
    c->n.push_back(ci.natoms);
    c->tile_off.push_back(ntiles);
    const int nt = (ci.natoms + TILE - 1) / TILE;
    c->ntile.push_back(nt);
    ntiles += nt;
    N += ci.natoms;
    need_bins[k] = bins_for(H, rcs / c->bin_factor);
    dens = std::max(dens, ci.natoms / (H[0] * H[4] * H[8]));
  }
  if (N > (1ll << 31) - 1) return bail(fail(c, RCELL_ERR_ARG, "too many atoms"));
  c->N = N;
  c->density_max = dens;
  c->npad = (N + 63) / 64 * 64;
  c->list16 = !c->fp64 && *std::max_element(c->n.begin(), c->n.end()) <= 65536;
  c->small_cells = *std::max_element(c->n.begin(), c->n.end()) <= PREP_ATOMS;
  c->cell_prep = c->small_cells;
  c->ntiles = ntiles;
  c->occ.assign(ncells, 0.0);
  for (int k = 0; k < ncells; ++k)
    set_occupancy(c, k, (double)cells[k].natoms / bins_exact(cells[k].H0, rcs / c->bin_factor));

  // ---- stream and memory
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    const hipError_t r = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (r != hipSuccess) {
      c->stream = nullptr;
      return bail(fail(c, RCELL_ERR_DEVICE, std::string("hipStreamCreate failed: ") + hipGetErrorString(r)));
    }
    c->own_stream = true;
  }
  const size_t fsz = sizeof(double);
  const size_t ssz = c->fp64 ? sizeof(S64) : sizeof(int4);
  int e;
  char *f0, *s0, *s1, *bondp;
  if ((e = dalloc(c, &c->x, N)) || (e = dalloc(c, &c->y, N)) || (e = dalloc(c, &c->z, N)) ||
      (e = dalloc(c, &c->vx, N)) || (e = dalloc(c, &c->vy, N)) || (e = dalloc(c, &c->vz, N)) ||
      (e = dalloc(c, &f0, 3 * fsz * N)) || (e = dalloc(c, &s0, ssz * N)) || (e = dalloc(c, &s1, ssz * N)) ||
      (e = dalloc(c, &c->sb, N)) || (e = dalloc(c, &bondp, (c->list16 ? 8 : 16) * (size_t)N)) ||
      (e = dalloc(c, &c->bond0, N)) ||
      (e = dalloc(c, &c->gid, N)) || (e = dalloc(c, &c->pos_of, N)) ||
      (e = dalloc(c, &c->pscr, (6 * sizeof(double) + ssz + 2 * sizeof(int)) * (size_t)c->npad)) ||
      (e = dalloc(c, &c->nn, N)) ||
      (e = dalloc(c, &c->abin, N)) || (e = dalloc(c, &c->binned, N)) || (e = dalloc(c, &c->sort_tmp, N)) ||
      (e = dalloc(c, &c->cells, ncells)) || (e = dalloc(c, &c->tiles, ntiles)) || (e = dalloc(c, &c->parts, ntiles)) ||
      (e = dalloc(c, &c->stage, ncells)) || (e = dalloc(c, &c->dscratch, (size_t)17 * ncells)) || (e = dalloc(c, &c->dscratch2, (size_t)6 * ncells)) ||
      (e = dalloc(c, &c->iscratch, (size_t)2 * ncells)) || (e = dalloc(c, &c->lscratch, (size_t)2 * ncells)) ||
      (e = dalloc(c, &c->work_cells, ncells)) || (e = dalloc(c, &c->work_tstart, ncells + 1)) ||
      (e = dalloc(c, &c->work_kstart, ncells + 1)) || (e = dalloc(c, &c->work_count, 4)))
    return bail(e);
  c->fx = f0; c->fy = f0 + fsz * N; c->fz = f0 + 2 * fsz * N;
  c->s[0] = s0; c->s[1] = s1; c->bond = bondp;
  if ((e = ensure_list_capacity(c, list_capacity(dens, rcs)))) return bail(e);

  // ---- marshal the initial state (AoS -> SoA), bonds -> per-atom partner slots
  std::vector<double> hx(N), hy(N), hz(N), hvx(N, 0.0), hvy(N, 0.0), hvz(N, 0.0);
  std::vector<int> mb(ncells, 0);                  // cells whose velocities are drawn on the device
  std::vector<int4> hb(N, make_int4(-1, -1, -1, -1));
  std::vector<Tile> tl;
  tl.reserve(ntiles);
  for (int k = 0; k < ncells; ++k) {
    const rcell_cell_init& ci = cells[k];
    const long long o = c->off[k];
    for (int i = 0; i < ci.natoms; ++i) {
      hx[o + i] = ci.x[3 * i]; hy[o + i] = ci.x[3 * i + 1]; hz[o + i] = ci.x[3 * i + 2];
      if (!std::isfinite(hx[o + i]) || !std::isfinite(hy[o + i]) || !std::isfinite(hz[o + i]))
        return bail(fail(c, RCELL_ERR_ARG, "non-finite position in cell " + std::to_string(k)));
      if (ci.v) { hvx[o + i] = ci.v[3 * i]; hvy[o + i] = ci.v[3 * i + 1]; hvz[o + i] = ci.v[3 * i + 2]; }
    }
    mb[k] = ci.v ? 0 : 1;
    for (int b = 0; b < ci.nbonds; ++b) {
      const int i = ci.bonds[2 * b], j = ci.bonds[2 * b + 1];
      if (i < 0 || j < 0 || i >= ci.natoms || j >= ci.natoms || i == j)
        return bail(fail(c, RCELL_ERR_ARG, "bad bond index in cell " + std::to_string(k)));
      for (int side = 0; side < 2; ++side) {
        const int a = side ? j : i, partner = side ? i : j;
        int* slot = &hb[o + a].x;
        int q = 0;
        while (q < 4 && slot[q] >= 0) ++q;
        if (q == 4) return bail(fail(c, RCELL_ERR_ARG, "more than 4 bonds on one atom in cell " + std::to_string(k)));
        slot[q] = partner;
      }
    }
    for (int t = 0; t < c->ntile[k]; ++t)
      tl.push_back(Tile{k, (int)(o + t * TILE), std::min(TILE, ci.natoms - t * TILE), 0});
  }
  std::vector<CellDev> hc(ncells);
  for (int k = 0; k < ncells; ++k) {
    CellDev& C = hc[k];
    std::memset(&C, 0, sizeof(C));
    std::memcpy(C.H, cells[k].H0, sizeof(C.H));
    for (int q = 0; q < 9; ++q) C.Rprev[q] = C.Q[q] = C.R[q] = C.F[q] = (q % 4 == 0) ? 1.0 : 0.0;
    C.J = 1.0;
    C.off = c->off[k]; C.n = c->n[k]; C.tile_off = c->tile_off[k]; C.ntile = c->ntile[k];
  }
  const size_t nb = sizeof(double) * N;
  if (hipMemcpyAsync(c->x, hx.data(), nb, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->y, hy.data(), nb, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->z, hz.data(), nb, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->vx, hvx.data(), nb, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->vy, hvy.data(), nb, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->vz, hvz.data(), nb, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->bond0, hb.data(), sizeof(int4) * N, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->tiles, tl.data(), sizeof(Tile) * ntiles, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->cells, hc.data(), sizeof(CellDev) * ncells, hipMemcpyHostToDevice, c->stream) ||
      hipMemsetAsync(f0, 0, 3 * fsz * N, c->stream) || hipMemsetAsync(s0, 0, ssz * N, c->stream) ||
      hipMemsetAsync(s1, 0, ssz * N, c->stream) || hipStreamSynchronize(c->stream))
    return bail(fail(c, RCELL_ERR_DEVICE, "initial upload failed"));
  if ((e = layout_bins(c, need_bins))) return bail(e);
  hipLaunchKernelGGL(k_reset_order, dim3(tile_grid(c->ntiles)), dim3(TILE), 0, c->stream, make_args(c), 0, ncells);
  if (std::any_of(mb.begin(), mb.end(), [](int f) { return f != 0; })) {   // Maxwell-Boltzmann from the seed
    int* dflag = c->iscratch;
    if (hipMemcpyAsync(dflag, mb.data(), sizeof(int) * ncells, hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return bail(fail(c, RCELL_ERR_DEVICE, "velocity flags upload failed"));
    const double sd = std::sqrt(p.kB * p.temperature / (p.mass * p.mvv2e));
    hipLaunchKernelGGL(k_mb_velocities, dim3(ncells), dim3(MB_NT), 0, c->stream, make_args(c), (const int*)dflag, sd,
                       p.kB * p.temperature / (p.mass * p.mvv2e));
  }
  hipLaunchKernelGGL(k_set_box, dim3((ncells + 63) / 64), dim3(64), 0, c->stream, c->cells, 0, ncells, bin_width(c));
  if ((e = prime(c))) return bail(e);
  Gathered g;
  if ((e = gather(c, g))) return bail(e);
  if ((e = first_error(c, g.status))) return bail(e);
  *out = c;
  return RCELL_OK;
}

int rcell_set_deformation(rcell_ctx* c, const double* F) {
  if (!c || !F) return c ? fail(c, RCELL_ERR_ARG, "F is NULL") : RCELL_ERR_ARG;
  for (int k = 0; k < 9 * c->ncells; ++k)
    if (!std::isfinite(F[k])) return fail(c, RCELL_ERR_BAD_F, "non-finite F in cell " + std::to_string(k / 9));
  double* Fd = c->dscratch;
  HIPCHK(c, hipMemcpyAsync(Fd, F, sizeof(double) * 9 * c->ncells, hipMemcpyHostToDevice, c->stream));
  return deformation_common(c, Fd);
}

int rcell_set_deformation_dev(rcell_ctx* c, const void* F_dev) {
  if (!c || !F_dev) return c ? fail(c, RCELL_ERR_ARG, "F_dev is NULL") : RCELL_ERR_ARG;
  return deformation_common(c, (const double*)F_dev);
}

// one MD step that is not the last of a run: forces at the current positions fused with the
// update to the next positions, buffer swap, per-cell reduction and conditional neighbour build
// (the reduction reads only the tile partials and the cell table, not the swapped buffers)
static void middle_step(rcell_ctx* c) {
  launch_force(c, MODE_STEP);
  c->cur = 1 - c->cur;
  launch_build(c, RED_STEP);
}

// capture graph_steps (even) middle steps starting at the current buffer parity
static int capture_graph(rcell_ctx* c) {
  const int par = c->cur;
  hipGraph_t g = nullptr;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
  for (int k = 0; k < c->graph_steps; ++k) middle_step(c);
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  c->cur = par;                                    // capture does not execute anything
  if (e != hipSuccess) return fail(c, RCELL_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  const hipError_t ei = hipGraphInstantiate(&c->graph[par], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    c->graph[par] = nullptr;
    return fail(c, RCELL_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
  }
  return RCELL_OK;
}

int rcell_run(rcell_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return c ? fail(c, RCELL_ERR_ARG, "nsteps < 0") : RCELL_ERR_ARG;
  if (nsteps == 0) return RCELL_OK;
  TraceRange tr("rcell_run");
  launch_start(c);
  launch_build(c, RED_START);
  int left = nsteps - 1;                           // middle steps; the last step ends the run
  const bool graphs = c->graph_steps > 0 && !c->prof;
  while (graphs && left >= c->graph_steps) {
    if (!c->graph[c->cur]) {
      const int e = capture_graph(c);
      if (e) return e;
    }
    {
      TraceRange tg("rcell: graph replay of middle steps");
      HIPCHK(c, hipGraphLaunch(c->graph[c->cur], c->stream));
    }
    left -= c->graph_steps;                        // an even number of swaps: parity unchanged
  }
  for (; left > 0; --left) middle_step(c);
  launch_force(c, MODE_LAST);
  launch_reduce(c, RED_LAST);
  HIPCHK(c, hipGetLastError());
  return RCELL_OK;
}

static int stress_out(rcell_ctx* c, void* sigma_dev, void* P_dev, void* smd_dev) {
  TraceRange tr("rcell: stress return");
  hipLaunchKernelGGL(k_stress_out, dim3((c->ncells + 63) / 64), dim3(64), 0, c->stream, c->cells, c->ncells,
                     (double*)sigma_dev, (double*)P_dev, (double*)smd_dev);
  HIPCHK(c, hipGetLastError());
  return RCELL_OK;
}

int rcell_get_stress_dev(rcell_ctx* c, void* sigma_dev, void* P_dev) {
  if (!c || !sigma_dev) return c ? fail(c, RCELL_ERR_ARG, "sigma_dev is NULL") : RCELL_ERR_ARG;
  return stress_out(c, sigma_dev, P_dev, nullptr);
}

int rcell_get_stress_ext(rcell_ctx* c, double* sigma, double* P, double* sigma_md) {
  if (!c || !sigma) return c ? fail(c, RCELL_ERR_ARG, "sigma is NULL") : RCELL_ERR_ARG;
  const int nc = c->ncells;
  double* sd = c->dscratch;
  double* pd = c->dscratch + 6 * nc;
  int e = stress_out(c, sd, P ? pd : nullptr, sigma_md ? c->dscratch2 : nullptr);
  if (e) return e;
  HIPCHK(c, hipMemcpyAsync(sigma, sd, sizeof(double) * 6 * nc, hipMemcpyDeviceToHost, c->stream));
  if (P) HIPCHK(c, hipMemcpyAsync(P, pd, sizeof(double) * 9 * nc, hipMemcpyDeviceToHost, c->stream));
  if (sigma_md) HIPCHK(c, hipMemcpyAsync(sigma_md, c->dscratch2, sizeof(double) * 6 * nc, hipMemcpyDeviceToHost, c->stream));
  Gathered g;
  if ((e = gather(c, g))) return e;
  return first_error(c, g.status);
}

int rcell_get_stress(rcell_ctx* c, double* sigma, double* P) {
  if (!c || !sigma) return c ? fail(c, RCELL_ERR_ARG, "sigma is NULL") : RCELL_ERR_ARG;
  const int nc = c->ncells;
  double* sd = c->dscratch;
  double* pd = c->dscratch + 6 * nc;
  int e = rcell_get_stress_dev(c, sd, P ? pd : nullptr);
  if (e) return e;
  HIPCHK(c, hipMemcpyAsync(sigma, sd, sizeof(double) * 6 * nc, hipMemcpyDeviceToHost, c->stream));
  if (P) HIPCHK(c, hipMemcpyAsync(P, pd, sizeof(double) * 9 * nc, hipMemcpyDeviceToHost, c->stream));
  Gathered g;
  if ((e = gather(c, g))) return e;
  return first_error(c, g.status);
}

int rcell_destroy(rcell_ctx* c) {
  if (!c) return RCELL_OK;
  destroy_all(c);
  delete c;
  return RCELL_OK;
}

const char* rcell_last_error(const rcell_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int rcell_minimize(rcell_ctx* c, int32_t max_iter, double ftol, int32_t* iters) {
  TraceRange tr("rcell_minimize");
  if (!c) return RCELL_ERR_ARG;
  if (max_iter < 0 || !(ftol > 0) || !std::isfinite(ftol)) return fail(c, RCELL_ERR_ARG, "max_iter >= 0 and ftol > 0");
  const int nc = c->ncells;
  c->fire_ftol2 = ftol * ftol;
  c->fire_max_iter = max_iter;
  const MDArgs a0 = make_args(c);
  hipLaunchKernelGGL(k_fire_cells, dim3((nc + 63) / 64), dim3(64), 0, c->stream, c->cells, nc, c->p.dt);
  hipLaunchKernelGGL(k_zero_v, dim3(tile_grid(c->ntiles)), dim3(TILE), 0, c->stream, a0);
  int* d_it = c->iscratch;
  int* d_done = c->iscratch + nc;
  std::vector<int> done(nc);
  for (long long it = 0; it <= max_iter; ++it) {
    launch_force(c, MODE_STATIC);
    launch_reduce(c, RED_STATIC);
    const MDArgs a = make_args(c);
    if (c->fp64) hipLaunchKernelGGL(k_fire_move<FP64>, dim3(tile_grid(c->ntiles)), dim3(TILE), 0, c->stream, a);
    else hipLaunchKernelGGL(k_fire_move<Mixed>, dim3(tile_grid(c->ntiles)), dim3(TILE), 0, c->stream, a);
    launch_reduce(c, RED_MOVE);
    launch_build(c);
    if (it % 16 == 15 || it == max_iter) {
      hipLaunchKernelGGL(k_fire_iters, dim3((nc + 63) / 64), dim3(64), 0, c->stream, c->cells, nc, d_it, d_done);
      HIPCHK(c, hipMemcpyAsync(done.data(), d_done, sizeof(int) * nc, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      if (std::all_of(done.begin(), done.end(), [](int d) { return d != 0; })) break;
    }
  }
  // relaxed state: zero velocities, conservative forces and the relaxed stress as the last sample
  hipLaunchKernelGGL(k_zero_v, dim3(tile_grid(c->ntiles)), dim3(TILE), 0, c->stream, a0);
  hipLaunchKernelGGL(k_set_pending, dim3((nc + 63) / 64), dim3(64), 0, c->stream, c->cells, 0, nc);
  int e = prime(c);
  if (e) return e;
  hipLaunchKernelGGL(k_fire_iters, dim3((nc + 63) / 64), dim3(64), 0, c->stream, c->cells, nc, d_it, d_done);
  std::vector<int> hit(nc);
  HIPCHK(c, hipMemcpyAsync(hit.data(), d_it, sizeof(int) * nc, hipMemcpyDeviceToHost, c->stream));
  Gathered g;
  if ((e = gather(c, g))) return e;
  if (iters) std::copy(hit.begin(), hit.end(), iters);
  return first_error(c, g.status);
}

int rcell_get_status(rcell_ctx* c, int32_t* status) {
  if (!c || !status) return c ? fail(c, RCELL_ERR_ARG, "status is NULL") : RCELL_ERR_ARG;
  Gathered g;
  int e = gather(c, g);
  if (e) return e;
  std::copy(g.status.begin(), g.status.end(), status);
  return RCELL_OK;
}

int rcell_get_forces(rcell_ctx* c, int32_t cell, double* f) {
  if (!c || !f || cell < 0 || cell >= c->ncells) return c ? fail(c, RCELL_ERR_ARG, "bad cell or f") : RCELL_ERR_ARG;
  const long long o = c->off[cell], n = c->n[cell];
  const size_t fsz = sizeof(double);
  std::vector<char> buf(3 * fsz * n);
  std::vector<int> ids(n);
  void* src[3] = {c->fx, c->fy, c->fz};
  for (int q = 0; q < 3; ++q)
    HIPCHK(c, hipMemcpyAsync(buf.data() + q * fsz * n, (char*)src[q] + fsz * o, fsz * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(ids.data(), c->gid + o, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int q = 0; q < 3; ++q)
    for (long long i = 0; i < n; ++i)                // position i holds original atom ids[i]
      f[3 * (long long)ids[i] + q] = ((const double*)buf.data())[q * n + i];
  return RCELL_OK;
}

int rcell_get_state(rcell_ctx* c, int32_t cell, double* x, double* v, double* H, double* Rprev, int64_t* step) {
  if (!c || cell < 0 || cell >= c->ncells) return c ? fail(c, RCELL_ERR_ARG, "bad cell") : RCELL_ERR_ARG;
  const long long o = c->off[cell], n = c->n[cell];
  std::vector<double> buf(6 * n);
  double* src[6] = {c->x, c->y, c->z, c->vx, c->vy, c->vz};
  std::vector<int> ids(n);
  for (int q = 0; q < 6; ++q)
    HIPCHK(c, hipMemcpyAsync(buf.data() + q * n, src[q] + o, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(ids.data(), c->gid + o, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream));
  CellDev C;
  HIPCHK(c, hipMemcpyAsync(&C, c->cells + cell, sizeof(CellDev), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (long long i = 0; i < n; ++i)                  // position i holds original atom ids[i]
    for (int q = 0; q < 3; ++q) {
      if (x) x[3 * (long long)ids[i] + q] = buf[q * n + i];
      if (v) v[3 * (long long)ids[i] + q] = buf[(3 + q) * n + i];
    }
  if (H) std::memcpy(H, C.H, sizeof(C.H));
  if (Rprev) std::memcpy(Rprev, C.Rprev, sizeof(C.Rprev));
  if (step) *step = C.step;
  return RCELL_OK;
}

int rcell_set_state(rcell_ctx* c, int32_t cell, const double* x, const double* v, const double* H,
                    const double* Rprev, int64_t step) {
  if (!c || cell < 0 || cell >= c->ncells || !x || !v || !H || !Rprev)
    return c ? fail(c, RCELL_ERR_ARG, "bad cell or NULL argument") : RCELL_ERR_ARG;
  if (!(H[0] > 0 && H[4] > 0 && H[8] > 0) || H[3] != 0 || H[6] != 0 || H[7] != 0)
    return fail(c, RCELL_ERR_STATE, "H must be upper triangular with positive diagonal");
  const double rcs = c->p.rc + c->p.skin;
  if (0.5 * width_min(H) < rcs) return fail(c, RCELL_ERR_BOX, "box too small for rc + skin");
  const long long o = c->off[cell], n = c->n[cell];
  std::vector<int> need(c->bin_cap);
  need[cell] = std::max(need[cell], bins_for(H, bin_width(c)));
  set_occupancy(c, cell, (double)n / bins_exact(H, bin_width(c)));
  int e;
  if (need[cell] > c->bin_cap[cell] && (e = layout_bins(c, need))) return e;
  if ((e = ensure_list_capacity(c, list_capacity(n / (H[0] * H[4] * H[8]), rcs)))) return e;
  std::vector<double> buf(6 * n);
  for (long long i = 0; i < n; ++i)
    for (int q = 0; q < 3; ++q) { buf[q * n + i] = x[3 * i + q]; buf[(3 + q) * n + i] = v[3 * i + q]; }
  double* dst[6] = {c->x, c->y, c->z, c->vx, c->vy, c->vz};
  for (int q = 0; q < 6; ++q)
    HIPCHK(c, hipMemcpyAsync(dst[q] + o, buf.data() + q * n, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  CellDev C;
  HIPCHK(c, hipMemcpyAsync(&C, c->cells + cell, sizeof(CellDev), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::memcpy(C.H, H, sizeof(C.H));
  std::memcpy(C.Rprev, Rprev, sizeof(C.Rprev));
  C.step = step;
  C.status = 0;
  HIPCHK(c, hipMemcpyAsync(c->cells + cell, &C, sizeof(CellDev), hipMemcpyHostToDevice, c->stream));
  // the state arrives in original order: identity order, then the rebuild reorders the cell
  hipLaunchKernelGGL(k_reset_order, dim3(tile_grid(c->ntiles)), dim3(TILE), 0, c->stream, make_args(c), cell, 1);
  hipLaunchKernelGGL(k_set_box, dim3(1), dim3(64), 0, c->stream, c->cells, cell, 1, bin_width(c));
  if ((e = prime(c))) return e;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RCELL_OK;
}

int rcell_get_energy(rcell_ctx* c, double* pe, double* ke) {
  if (!c) return RCELL_ERR_ARG;
  Gathered g;
  int e = gather(c, g);
  if (e) return e;
  if (pe) std::copy(g.pe.begin(), g.pe.end(), pe);
  if (ke) {
    const MDArgs a = make_args(c);
    double* kd = c->dscratch;
    hipLaunchKernelGGL(k_kinetic, dim3(c->ncells), dim3(RED_NT), 0, c->stream, a, kd);
    HIPCHK(c, hipMemcpyAsync(ke, kd, sizeof(double) * c->ncells, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return RCELL_OK;
}

int rcell_get_box(rcell_ctx* c, int32_t cell, double* H, double* Q, double* R, double* J) {
  if (!c || cell < 0 || cell >= c->ncells) return c ? fail(c, RCELL_ERR_ARG, "bad cell") : RCELL_ERR_ARG;
  CellDev C;
  HIPCHK(c, hipMemcpyAsync(&C, c->cells + cell, sizeof(CellDev), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (H) std::memcpy(H, C.H, sizeof(C.H));
  if (Q) std::memcpy(Q, C.Q, sizeof(C.Q));
  if (R) std::memcpy(R, C.R, sizeof(C.R));
  if (J) *J = C.J;
  return RCELL_OK;
}

int rcell_get_rebuilds(rcell_ctx* c, int64_t* count) {
  if (!c || !count) return RCELL_ERR_ARG;
  Gathered g;
  int e = gather(c, g);
  if (e) return e;
  long long s = 0;
  for (long long v : g.nreb) s += v;
  *count = s;
  return RCELL_OK;
}

int rcell_set_graph_steps(rcell_ctx* c, int32_t steps) {
  if (!c || steps < 0 || (steps & 1)) return c ? fail(c, RCELL_ERR_ARG, "graph steps must be even and >= 0") : RCELL_ERR_ARG;
  drop_graphs(c);
  c->graph_steps = steps;
  return RCELL_OK;
}

int rcell_set_build_mode(rcell_ctx* c, int32_t mode) {
  if (!c || mode < 0 || mode > 2) return c ? fail(c, RCELL_ERR_ARG, "build mode must be 0, 1 or 2") : RCELL_ERR_ARG;
  if (mode == 1 && !c->small_cells)
    return fail(c, RCELL_ERR_ARG, "one block per cell needs every cell to have at most " +
                                      std::to_string(PREP_ATOMS) + " atoms");
  drop_graphs(c);
  c->cell_prep = mode == 0 ? c->small_cells : mode == 1;
  return RCELL_OK;
}

int rcell_set_lanes(rcell_ctx* c, int32_t lanes) {
  if (!c) return RCELL_ERR_ARG;
  drop_graphs(c);
  if (lanes == 1 || lanes == 2 || lanes == 4 || lanes == 8 || lanes == 16) {
    c->lanes = lanes;
    return RCELL_OK;
  }
  if (lanes != 0) return fail(c, RCELL_ERR_ARG, "lanes must be 0, 1, 2, 4, 8 or 16");
  // autotune: time the MD step's force pass (the pair loops and the integration tail) for each
  // variant and keep the fastest; each variant's time is its best of three rounds, taken in turn, so
  // one slow sample decides nothing.  The pass writes positions, velocities and forces, so those
  // point at copies; the other fixed-point buffer, the tile partials and the EAM F' that it also
  // writes are rewritten before they are next read.
  const size_t nb = sizeof(double) * (size_t)c->N;
  char* tmp = nullptr;
  if (hipMalloc(&tmp, 9 * nb) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, RCELL_ERR_OOM, "autotune scratch of " + std::to_string(9 * nb) + " bytes");
  }
  MDArgs a = make_args(c);
  double* d[9];
  for (int k = 0; k < 9; ++k) d[k] = (double*)(tmp + k * nb);
  const void* src[9] = {c->x, c->y, c->z, c->vx, c->vy, c->vz, c->fx, c->fy, c->fz};
  constexpr int NV = 5;
  const int var[NV] = {1, 2, 4, 8, 16};
  float t[NV];
  for (int v = 0; v < NV; ++v) t[v] = 1e30f;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e = hipSuccess;
  for (int k = 0; k < 9 && e == hipSuccess; ++k) e = hipMemcpyAsync(d[k], src[k], nb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  a.x = d[0]; a.y = d[1]; a.z = d[2]; a.vx = d[3]; a.vy = d[4]; a.vz = d[5];
  a.fx = d[6]; a.fy = d[7]; a.fz = d[8];
  for (int round = 0; round < 3 && e == hipSuccess; ++round)
    for (int v = 0; v < NV && e == hipSuccess; ++v) {
      launch_force_args(c, a, MODE_STEP, var[v]);
      e = hipEventRecord(t0, c->stream);
      for (int r = 0; r < 5 && e == hipSuccess; ++r) launch_force_args(c, a, MODE_STEP, var[v]);
      if (e == hipSuccess) e = hipEventRecord(t1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      t[v] = std::min(t[v], ms);
    }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(c, RCELL_ERR_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
  int best = 0;
  for (int v = 1; v < NV; ++v)
    if (t[v] < t[best]) best = v;
  c->lanes = var[best];
  return RCELL_OK;
}

int rcell_set_bin_factor(rcell_ctx* c, int32_t f) {
  if (!c) return RCELL_ERR_ARG;
  if (f < 1 || f > MAX_BIN_FACTOR) return fail(c, RCELL_ERR_ARG, "bin factor must be 1 or 2");
  if (f == c->bin_factor) return RCELL_OK;
  return apply_bin_factor(c, f);
}

int rcell_get_bin_factor(rcell_ctx* c, int32_t* f) {
  if (!c || !f) return RCELL_ERR_ARG;
  *f = c->bin_factor;
  return RCELL_OK;
}

int rcell_autotune(rcell_ctx* c, int32_t use_cache, int32_t* lanes, int32_t* bin_factor) {
  TraceRange tr("rcell_autotune");
  if (!c) return RCELL_ERR_ARG;
  const auto key = tune_key(c);
  int e;
  if (use_cache) {
    std::pair<int, int> hit{0, 0};
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) hit = it->second;
    }
    if (hit.first) {
      if ((e = rcell_set_lanes(c, hit.first)) || (e = rcell_set_bin_factor(c, hit.second))) return e;
      if (lanes) *lanes = c->lanes;
      if (bin_factor) *bin_factor = c->bin_factor;
      return RCELL_OK;
    }
  }
  // The bin factor: every cell rebuilt at the current positions with each factor, best of three
  // rounds taken in turn.  The build reorders atoms and rewrites the fixed-point coordinates, the
  // build references, the partner slots, the list and the cell table, so those are copied aside
  // first and copied back before every trial and at the end: the state is left exactly as found,
  // with only the bins of the next build changed, as rcell_set_bin_factor leaves it.
  const long long N = c->N;
  const size_t ssz = c->fp64 ? sizeof(S64) : sizeof(int4);
  const size_t lsz = (size_t)c->maxnb * (size_t)c->npad * (c->list16 ? sizeof(uint16_t) : sizeof(int));
  struct Piece { void* dev; size_t bytes; };
  const Piece pieces[] = {
      {c->x, 8 * (size_t)N}, {c->y, 8 * (size_t)N}, {c->z, 8 * (size_t)N},
      {c->vx, 8 * (size_t)N}, {c->vy, 8 * (size_t)N}, {c->vz, 8 * (size_t)N},
      {c->s[c->cur], ssz * N}, {c->sb, sizeof(uint2) * N}, {c->gid, 4 * (size_t)N}, {c->pos_of, 4 * (size_t)N},
      {c->bond, (c->list16 ? 8 : 16) * (size_t)N}, {c->nn, 4 * (size_t)N}, {c->nbr, lsz},
      {c->cells, sizeof(CellDev) * (size_t)c->ncells}};
  size_t total = 0;
  for (const Piece& pc : pieces) total += (pc.bytes + 255) / 256 * 256;
  char* keep = nullptr;
  if (hipMalloc(&keep, total) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, RCELL_ERR_OOM, "autotune snapshot of " + std::to_string(total) + " bytes");
  }
  auto copy = [&](bool save) {
    size_t o = 0;
    for (const Piece& pc : pieces) {
      const hipError_t r = save ? hipMemcpyAsync(keep + o, pc.dev, pc.bytes, hipMemcpyDeviceToDevice, c->stream)
                                : hipMemcpyAsync(pc.dev, keep + o, pc.bytes, hipMemcpyDeviceToDevice, c->stream);
      if (r != hipSuccess) return r;
      o += (pc.bytes + 255) / 256 * 256;
    }
    return hipSuccess;
  };
  const int f0 = c->bin_factor;
  float best_t[MAX_BIN_FACTOR + 1];
  for (int f = 0; f <= MAX_BIN_FACTOR; ++f) best_t[f] = 1e30f;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t he = copy(true);
  if (he == hipSuccess) he = hipEventCreate(&t0);
  if (he == hipSuccess) he = hipEventCreate(&t1);
  e = RCELL_OK;
  for (int round = 0; round < 3 && he == hipSuccess && !e; ++round)
    for (int f = 1; f <= MAX_BIN_FACTOR && he == hipSuccess && !e; ++f) {
      if ((he = copy(false)) != hipSuccess) break;
      // the restored cell table holds the bin offsets of the snapshot: the current layout again
      if ((e = push_bin_layout(c)) || (e = apply_bin_factor(c, f))) break;
      hipLaunchKernelGGL(k_set_pending, dim3((c->ncells + 63) / 64), dim3(64), 0, c->stream, c->cells, 0, c->ncells);
      if ((he = hipEventRecord(t0, c->stream)) != hipSuccess) break;
      launch_build(c);
      if ((he = hipEventRecord(t1, c->stream)) != hipSuccess) break;
      if ((he = hipEventSynchronize(t1)) != hipSuccess) break;
      float ms = 0.f;
      if ((he = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
      best_t[f] = std::min(best_t[f], ms);
    }
  int best = f0;
  if (he == hipSuccess && !e) {
    best = 1;
    for (int f = 2; f <= MAX_BIN_FACTOR; ++f)
      if (best_t[f] < best_t[best]) best = f;
    he = copy(false);                               // the state as found, then its bin layout
  }
  if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)hipFree(keep);
  if (he != hipSuccess) return fail(c, RCELL_ERR_DEVICE, std::string("autotune: ") + hipGetErrorString(he));
  if (e) return e;
  if ((e = push_bin_layout(c)) || (e = apply_bin_factor(c, best))) return e;
  // lanes per atom, timed on the MD step's own force pass (on copies; advances no state)
  if ((e = rcell_set_lanes(c, 0))) return e;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = std::make_pair(c->lanes, c->bin_factor);
  }
  if (lanes) *lanes = c->lanes;
  if (bin_factor) *bin_factor = c->bin_factor;
  return RCELL_OK;
}

int rcell_get_lanes(rcell_ctx* c, int32_t* lanes) {
  if (!c || !lanes) return RCELL_ERR_ARG;
  *lanes = c->lanes;
  return RCELL_OK;
}

int rcell_qr_dev(const void* F_dev, int32_t n, void* Q_dev, void* R_dev, void* status_dev, void* hip_stream) {
  if (!F_dev || !Q_dev || !R_dev || n < 0) return RCELL_ERR_ARG;
  if (n == 0) return RCELL_OK;
  hipLaunchKernelGGL(k_qr_batch, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)hip_stream, (const double*)F_dev, n,
                     (double*)Q_dev, (double*)R_dev, (int*)status_dev);
  return hipGetLastError() == hipSuccess ? RCELL_OK : RCELL_ERR_DEVICE;
}

int rcell_stress_return_dev(const void* F_dev, const void* sigma_md_dev, int32_t n, void* sigma_fem_dev, void* P_dev,
                            void* hip_stream) {
  if (!F_dev || !sigma_md_dev || !sigma_fem_dev || n < 0) return RCELL_ERR_ARG;
  if (n == 0) return RCELL_OK;
  hipLaunchKernelGGL(k_return_batch, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)hip_stream, (const double*)F_dev,
                     (const double*)sigma_md_dev, n, (double*)sigma_fem_dev, (double*)P_dev);
  return hipGetLastError() == hipSuccess ? RCELL_OK : RCELL_ERR_DEVICE;
}

int rcell_prof_enable(rcell_ctx* c, int32_t on) {
  if (!c) return RCELL_ERR_ARG;
  c->prof = on != 0;
  // create the events up front so that recording never waits on the host
  while (c->prof && c->ev_pool.size() < 8192) {
    hipEvent_t e = nullptr;
    HIPCHK(c, hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  return RCELL_OK;
}

int rcell_prof_read(rcell_ctx* c, int32_t which, double* total_ms, int64_t* launches) {
  if (!c || which < 0 || which > 1 || !total_ms || !launches) return c ? fail(c, RCELL_ERR_ARG, "bad prof_read arguments") : RCELL_ERR_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double ms = 0.0;
  for (auto& pr : c->prof_ev[which]) {
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, pr.first, pr.second));
    ms += t;
    c->ev_pool.push_back(pr.first);
    c->ev_pool.push_back(pr.second);
  }
  *total_ms = ms;
  *launches = (int64_t)c->prof_ev[which].size();
  c->prof_ev[which].clear();
  return RCELL_OK;
}

}  // extern "C"
