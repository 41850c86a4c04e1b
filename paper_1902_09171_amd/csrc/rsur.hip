// Host side of the stress-surrogate C ABI (include/rsur.h): memory layout, marshalling of the
// flat parameter layout to the padded device layout, and the launch sequence of inference and
// of one training step.  The arithmetic runs in the kernels of rsur_device.h.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rcell.h"
#include "../../include/rsur.h"
#include "rsur_device.h"

using namespace rsur;

namespace {
thread_local std::string g_rsur_create_error;

// A roctx range over a scope (rocprofv3 --marker-trace names each call; a few ns without a profiler)
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePush(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};
}

// Scratch of rsur_forward_static: every member's output for the rows of one call (K x pad64(B) x
// padded dout floats).  One copy per device, holding the last call's outputs until the process
// ends.  Host code never uses this name as an address: the device address of each device's copy
// comes from hipGetSymbolAddress (static_scratch_ptr).
constexpr long long RSUR_STATIC_FLOATS = 1LL << 21;   // 8 MiB
static __device__ __align__(256) float scratch[RSUR_STATIC_FLOATS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {};

// device address of the current device's scratch, looked up once per device (no allocation)
int static_scratch_ptr(float** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    (void)hipGetLastError();
    return RCELL_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* q = nullptr;
    if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) {
      (void)hipGetLastError();
      return RCELL_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = (float*)q;
  }
  *out = g_scratch_ptr[dev];
  return RCELL_OK;
}
}  // namespace

struct rsur_ctx {
  int din = 0, width = 0, depth = 0, dout = 0, K = 0, maxB = 0, Mp = 0, L = 0;
  std::vector<int> dims, dp;                 // logical and padded layer widths (L + 1)
  std::vector<long long> woff, boff;         // offsets of W_l, b_l inside one member's padded block
  long long P = 0, Pflat = 0;                // padded and flat parameter counts per member
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;   // K x P
  bf16* pb = nullptr;                                               // K x P (weights used)
  bf16* pbt = nullptr;                                              // K x P, weights transposed
  bool pbt_stale = true;                                            // pbt behind pb
  std::vector<bf16*> act;                    // act[l]: K x Mp x dp[l] (act[0] shared: Mp x dp[0])
  std::vector<float*> Z;                     // Z[l]: K x Mp x dp[l + 1], hidden layers
  float* out = nullptr;                      // K x Mp x dp[L]
  bf16 *dza = nullptr, *dzb = nullptr;       // K x Mp x max(dp)
  float *xmu = nullptr, *xsd = nullptr, *ymu = nullptr, *ysd = nullptr, *loss = nullptr;
  float *c1 = nullptr, *c2 = nullptr;        // Adam bias corrections per member
  float* split = nullptr;                    // partial sums of the split gradient reductions
  float* lpart = nullptr;                    // K x LOSS_CHUNKS partial losses
  std::vector<long long> t;                  // Adam steps per member
  std::vector<void*> allocs;
};

namespace {

int rfail(rsur_ctx* c, int code, const std::string& m) {
  if (c) c->err = m; else g_rsur_create_error = m;
  return code;
}

#define RCHK(ctx, call)                                                                         \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return rfail((ctx), RCELL_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
int ralloc(rsur_ctx* c, T** out, size_t count) {
  void* q = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  if (hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return rfail(c, RCELL_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  c->allocs.push_back(q);
  *out = (T*)q;
  return RCELL_OK;
}

int pad64(int v) { return (v + 63) / 64 * 64; }

// The gradient reductions over the batch (weight gradients, bias column sums) are split into S
// ranges of at least 256 rows (S a power of two up to MAX_SPLIT dividing Mp / 64) so that enough
// blocks work at once; S partial results are then added in order (deterministic).
constexpr int MAX_SPLIT = 8;
int batch_splits(int Mp) {
  int S = 1;
  while (S < MAX_SPLIT && (Mp / 64) % (2 * S) == 0 && Mp / (2 * S) >= 256) S *= 2;
  return S;
}

template <bool AT, bool BT, int EPI>
void gemm(rsur_ctx* c, const GemmArgs& a) {
  GemmArgs b = a;
  b.nmem = c->K;
  if (b.ksplit < 1) b.ksplit = 1;
  hipLaunchKernelGGL((k_gemm<AT, BT, EPI>), dim3(b.N / TN, b.M / TM, c->K * b.ksplit), dim3(256), 0, c->stream, b);
}

// forward of every member for Mp rows already normalised in act[0]; keeps Z and activations
void forward_layers(rsur_ctx* c, int Mp) {
  for (int l = 0; l < c->L; ++l) {
    GemmArgs a{};
    a.A = c->act[l];
    a.lda = c->dp[l];
    a.sA = l == 0 ? 0 : (long long)c->Mp * c->dp[l];
    a.B = c->pb + c->woff[l];
    a.ldb = c->dp[l + 1];
    a.sB = c->P;
    a.M = Mp; a.N = c->dp[l + 1]; a.K = c->dp[l];
    a.bias = c->p + c->boff[l];
    a.sBias = c->P;
    if (l < c->L - 1) {
      a.Z = c->Z[l]; a.ldz = c->dp[l + 1]; a.sZ = (long long)c->Mp * c->dp[l + 1];
      a.O = c->act[l + 1]; a.ldo = c->dp[l + 1]; a.sO = (long long)c->Mp * c->dp[l + 1];
      gemm<false, false, EPI_FWD_HIDDEN>(c, a);
    } else {
      a.Z = c->out; a.ldz = c->dp[l + 1]; a.sZ = (long long)c->Mp * c->dp[l + 1];
      gemm<false, false, EPI_FWD_OUT>(c, a);
    }
  }
}

int check_batch(rsur_ctx* c, int B) {
  if (B < 1 || B > c->maxB) return rfail(c, RCELL_ERR_ARG, "batch size must be in [1, max_batch]");
  return RCELL_OK;
}

void normalise_inputs(rsur_ctx* c, const float* X, int B, int Mp) {
  const long long n = (long long)Mp * c->dp[0];
  hipLaunchKernelGGL(k_norm_in, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, X, B, c->din, Mp,
                     c->dp[0], c->xmu, c->xsd, c->act[0]);
}

void destroy_all(rsur_ctx* c) {
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (void* q : c->allocs) (void)hipFree(q);
  c->allocs.clear();
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  c->stream = nullptr;
}

}  // namespace

extern "C" {

int rsur_create(int32_t din, int32_t width, int32_t depth, int32_t dout, int32_t ensemble, int32_t max_batch,
                void* hip_stream, rsur_ctx** out) {
  if (!out) return rfail(nullptr, RCELL_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (din < 1 || dout < 1 || depth < 0 || (depth > 0 && width < 1) || ensemble < 1 || max_batch < 1)
    return rfail(nullptr, RCELL_ERR_ARG, "din, dout, ensemble, max_batch >= 1; depth >= 0; width >= 1 with hidden layers");
  rsur_ctx* c = new (std::nothrow) rsur_ctx();
  if (!c) return rfail(nullptr, RCELL_ERR_OOM, "host allocation failed");
  auto bail = [&](int code) {
    g_rsur_create_error = c->err.empty() ? g_rsur_create_error : c->err;
    destroy_all(c);
    delete c;
    return code;
  };
  c->err.reserve(256);             // short error messages are then assigned without allocating
  {
    float* sp = nullptr;             // the static scratch's address on this device, once per device
    if (static_scratch_ptr(&sp) != RCELL_OK)
      return bail(rfail(c, RCELL_ERR_DEVICE, "no usable HIP device (current device, or the static scratch address)"));
  }
  c->din = din; c->width = width; c->depth = depth; c->dout = dout; c->K = ensemble; c->maxB = max_batch;
  c->Mp = pad64(max_batch);
  c->dims.push_back(din);
  for (int k = 0; k < depth; ++k) c->dims.push_back(width);
  c->dims.push_back(dout);
  c->L = (int)c->dims.size() - 1;
  for (int d : c->dims) c->dp.push_back(pad64(d));
  long long o = 0, of = 0;
  for (int l = 0; l < c->L; ++l) {
    c->woff.push_back(o); o += (long long)c->dp[l] * c->dp[l + 1];
    c->boff.push_back(o); o += c->dp[l + 1];
    of += (long long)c->dims[l] * c->dims[l + 1] + c->dims[l + 1];
  }
  c->P = (o + 63) / 64 * 64;
  c->Pflat = of;
  c->t.assign(ensemble, 0);
  if (hip_stream) c->stream = (hipStream_t)hip_stream;
  else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(rfail(c, RCELL_ERR_DEVICE, "hipStreamCreate failed"));
    c->own_stream = true;
  }
  const long long KP = (long long)c->K * c->P;
  int e;
  if ((e = ralloc(c, &c->p, KP)) || (e = ralloc(c, &c->g, KP)) || (e = ralloc(c, &c->m1, KP)) ||
      (e = ralloc(c, &c->m2, KP)) || (e = ralloc(c, &c->pb, KP)) || (e = ralloc(c, &c->pbt, KP)))
    return bail(e);
  c->act.resize(c->L);
  c->Z.resize(std::max(c->L - 1, 0));
  for (int l = 0; l < c->L; ++l)
    if ((e = ralloc(c, &c->act[l], (size_t)(l == 0 ? 1 : c->K) * c->Mp * c->dp[l]))) return bail(e);
  for (int l = 0; l < c->L - 1; ++l)
    if ((e = ralloc(c, &c->Z[l], (size_t)c->K * c->Mp * c->dp[l + 1]))) return bail(e);
  const int dmax = *std::max_element(c->dp.begin(), c->dp.end());
  {
    size_t mn = (size_t)dmax;
    for (int l = 0; l < c->L; ++l) mn = std::max(mn, (size_t)c->dp[l] * c->dp[l + 1]);
    if ((e = ralloc(c, &c->split, (size_t)MAX_SPLIT * c->K * mn))) return bail(e);
  }
  if ((e = ralloc(c, &c->out, (size_t)c->K * c->Mp * c->dp[c->L])) ||
      (e = ralloc(c, &c->dza, (size_t)c->K * c->Mp * dmax)) || (e = ralloc(c, &c->dzb, (size_t)c->K * c->Mp * dmax)) ||
      (e = ralloc(c, &c->xmu, din)) || (e = ralloc(c, &c->xsd, din)) || (e = ralloc(c, &c->ymu, dout)) ||
      (e = ralloc(c, &c->ysd, dout)) || (e = ralloc(c, &c->loss, ensemble)) || (e = ralloc(c, &c->c1, ensemble)) ||
      (e = ralloc(c, &c->c2, ensemble)) || (e = ralloc(c, &c->lpart, (size_t)ensemble * LOSS_CHUNKS)))
    return bail(e);
  std::vector<float> zeros(std::max(din, dout), 0.0f), ones(std::max(din, dout), 1.0f);
  if (hipMemsetAsync(c->p, 0, sizeof(float) * KP, c->stream) || hipMemsetAsync(c->g, 0, sizeof(float) * KP, c->stream) ||
      hipMemsetAsync(c->m1, 0, sizeof(float) * KP, c->stream) || hipMemsetAsync(c->m2, 0, sizeof(float) * KP, c->stream) ||
      hipMemsetAsync(c->pb, 0, sizeof(bf16) * KP, c->stream) ||
      hipMemcpyAsync(c->xmu, zeros.data(), sizeof(float) * din, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->xsd, ones.data(), sizeof(float) * din, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->ymu, zeros.data(), sizeof(float) * dout, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->ysd, ones.data(), sizeof(float) * dout, hipMemcpyHostToDevice, c->stream) ||
      hipStreamSynchronize(c->stream))
    return bail(rfail(c, RCELL_ERR_DEVICE, "initialisation failed"));
  *out = c;
  return RCELL_OK;
}

int rsur_destroy(rsur_ctx* c) {
  if (!c) return RCELL_OK;
  destroy_all(c);
  delete c;
  return RCELL_OK;
}

const char* rsur_last_error(const rsur_ctx* c) { return c ? c->err.c_str() : g_rsur_create_error.c_str(); }

int rsur_num_params(rsur_ctx* c, int64_t* n) {
  if (!c || !n) return RCELL_ERR_ARG;
  *n = c->Pflat;
  return RCELL_OK;
}

int rsur_set_params(rsur_ctx* c, int32_t member, const float* w) {
  if (!c || !w || member < 0 || member >= c->K) return c ? rfail(c, RCELL_ERR_ARG, "bad member or NULL") : RCELL_ERR_ARG;
  std::vector<float> h(c->P, 0.0f);
  long long o = 0;
  for (int l = 0; l < c->L; ++l) {
    for (int i = 0; i < c->dims[l]; ++i)
      for (int j = 0; j < c->dims[l + 1]; ++j) h[c->woff[l] + (long long)i * c->dp[l + 1] + j] = w[o++];
    for (int j = 0; j < c->dims[l + 1]; ++j) h[c->boff[l] + j] = w[o++];
  }
  for (float v : h)
    if (!std::isfinite(v)) return rfail(c, RCELL_ERR_ARG, "non-finite parameter");
  const long long off = (long long)member * c->P;
  RCHK(c, hipMemcpyAsync(c->p + off, h.data(), sizeof(float) * c->P, hipMemcpyHostToDevice, c->stream));
  RCHK(c, hipMemsetAsync(c->m1 + off, 0, sizeof(float) * c->P, c->stream));
  RCHK(c, hipMemsetAsync(c->m2 + off, 0, sizeof(float) * c->P, c->stream));
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((c->P + 255) / 256)), dim3(256), 0, c->stream, c->p + off,
                     c->pb + off, c->P);
  RCHK(c, hipStreamSynchronize(c->stream));
  c->t[member] = 0;
  c->pbt_stale = true;
  return RCELL_OK;
}

static int get_flat(rsur_ctx* c, const float* src_dev, int32_t member, float* w) {
  if (!c || !w || member < 0 || member >= c->K) return c ? rfail(c, RCELL_ERR_ARG, "bad member or NULL") : RCELL_ERR_ARG;
  std::vector<float> h(c->P);
  RCHK(c, hipMemcpyAsync(h.data(), src_dev + (long long)member * c->P, sizeof(float) * c->P, hipMemcpyDeviceToHost,
                         c->stream));
  RCHK(c, hipStreamSynchronize(c->stream));
  long long o = 0;
  for (int l = 0; l < c->L; ++l) {
    for (int i = 0; i < c->dims[l]; ++i)
      for (int j = 0; j < c->dims[l + 1]; ++j) w[o++] = h[c->woff[l] + (long long)i * c->dp[l + 1] + j];
    for (int j = 0; j < c->dims[l + 1]; ++j) w[o++] = h[c->boff[l] + j];
  }
  return RCELL_OK;
}

int rsur_get_params(rsur_ctx* c, int32_t member, float* w) { return c ? get_flat(c, c->p, member, w) : RCELL_ERR_ARG; }
int rsur_get_grads(rsur_ctx* c, int32_t member, float* g) { return c ? get_flat(c, c->g, member, g) : RCELL_ERR_ARG; }

int rsur_set_norm(rsur_ctx* c, const float* x_mu, const float* x_sd, const float* y_mu, const float* y_sd) {
  if (!c || !x_mu || !x_sd || !y_mu || !y_sd) return c ? rfail(c, RCELL_ERR_ARG, "NULL statistics") : RCELL_ERR_ARG;
  for (int k = 0; k < c->din; ++k)
    if (!(x_sd[k] > 0) || !std::isfinite(x_mu[k])) return rfail(c, RCELL_ERR_ARG, "x_sd must be > 0");
  for (int k = 0; k < c->dout; ++k)
    if (!(y_sd[k] > 0) || !std::isfinite(y_mu[k])) return rfail(c, RCELL_ERR_ARG, "y_sd must be > 0");
  RCHK(c, hipMemcpyAsync(c->xmu, x_mu, sizeof(float) * c->din, hipMemcpyHostToDevice, c->stream));
  RCHK(c, hipMemcpyAsync(c->xsd, x_sd, sizeof(float) * c->din, hipMemcpyHostToDevice, c->stream));
  RCHK(c, hipMemcpyAsync(c->ymu, y_mu, sizeof(float) * c->dout, hipMemcpyHostToDevice, c->stream));
  RCHK(c, hipMemcpyAsync(c->ysd, y_sd, sizeof(float) * c->dout, hipMemcpyHostToDevice, c->stream));
  RCHK(c, hipStreamSynchronize(c->stream));
  return RCELL_OK;
}

int rsur_fit_norm(rsur_ctx* c, const void* X_dev, const void* Y_dev, int32_t n) {
  if (!c || !X_dev || !Y_dev || n < 1) return c ? rfail(c, RCELL_ERR_ARG, "bad fit_norm arguments") : RCELL_ERR_ARG;
  hipLaunchKernelGGL(k_fit_norm, dim3(c->din), dim3(FIT_NT), 0, c->stream, (const float*)X_dev, n, c->din, c->xmu, c->xsd);
  hipLaunchKernelGGL(k_fit_norm, dim3(c->dout), dim3(FIT_NT), 0, c->stream, (const float*)Y_dev, n, c->dout, c->ymu,
                     c->ysd);
  RCHK(c, hipGetLastError());
  return RCELL_OK;
}

// inference: every layer in one fused kernel when the padded widths allow it and the batch gives
// enough (row block, member) pairs to fill the GPU; small batches run layer by layer, whose
// per-layer grids spread the same work over more blocks
constexpr int FUSED_MIN_BLOCKS = 512;
static bool fused_shape(const rsur_ctx* c) {
  return *std::max_element(c->dp.begin(), c->dp.end()) <= FW && c->L <= MAXL;
}

// the fused forward of every member for Mp rows into out (K x Mp x dp[L], member stride sOut)
static void forward_fused(rsur_ctx* c, const float* X, int B, int Mp, float* out, long long sOut) {
  if (c->pbt_stale) {
    for (int l = 0; l < c->L; ++l) {
      const long long n = (long long)c->dp[l] * c->dp[l + 1];
      hipLaunchKernelGGL(k_transpose_w, dim3((unsigned)((n + 255) / 256), c->K), dim3(256), 0, c->stream, c->pb,
                         c->pbt, c->P, c->woff[l], c->dp[l], c->dp[l + 1]);
    }
    c->pbt_stale = false;
  }
  MlpArgs g{};
  g.X = X; g.B = B; g.din = c->din; g.xmu = c->xmu; g.xsd = c->xsd;
  g.wt = c->pbt; g.sW = c->P; g.p = c->p; g.sP = c->P;
  g.L = c->L;
  for (int l = 0; l <= c->L; ++l) g.dp[l] = c->dp[l];
  for (int l = 0; l < c->L; ++l) { g.woff[l] = c->woff[l]; g.boff[l] = c->boff[l]; }
  g.out = out; g.sOut = sOut; g.ldo = c->dp[c->L];
  hipLaunchKernelGGL(k_mlp_forward, dim3(Mp / 64, c->K), dim3(256), 0, c->stream, g);
}

static void forward_infer(rsur_ctx* c, const float* X, int B, int Mp) {
  if (!fused_shape(c) || (long long)(Mp / 64) * c->K < FUSED_MIN_BLOCKS) {
    normalise_inputs(c, X, B, Mp);
    forward_layers(c, Mp);
    return;
  }
  forward_fused(c, X, B, Mp, c->out, (long long)c->Mp * c->dp[c->L]);
}

static int forward_common(rsur_ctx* c, const void* X_dev, int32_t B, float* mean, float* var, float* members) {
  int e = check_batch(c, B);
  if (e) return e;
  const int Mp = pad64(B);
  forward_infer(c, (const float*)X_dev, B, Mp);
  const long long n = (long long)B * c->dout;
  hipLaunchKernelGGL(k_ensemble, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->out,
                     (long long)c->Mp * c->dp[c->L], c->dp[c->L], c->K, B, c->dout, c->ymu, c->ysd, mean, var, members);
  RCHK(c, hipGetLastError());
  return RCELL_OK;
}

int rsur_forward(rsur_ctx* c, const void* X_dev, int32_t B, void* mean_dev, void* var_dev) {
  TraceRange tr("rsur_forward");
  if (!c || !X_dev || !mean_dev) return c ? rfail(c, RCELL_ERR_ARG, "NULL pointer") : RCELL_ERR_ARG;
  return forward_common(c, X_dev, B, (float*)mean_dev, (float*)var_dev, nullptr);
}

int rsur_forward_static(rsur_ctx* c, const void* X_dev, int32_t B, void* mean_dev, void* var_dev) {
  TraceRange tr("rsur_forward_static");
  if (!c || !X_dev || !mean_dev) return c ? rfail(c, RCELL_ERR_ARG, "NULL pointer") : RCELL_ERR_ARG;
  if (!fused_shape(c)) return rfail(c, RCELL_ERR_ARG, "static forward: padded widths <= 256, <= 8 layers");
  if (B < 1 || (long long)c->K * pad64(B) * c->dp[c->L] > RSUR_STATIC_FLOATS)
    return rfail(c, RCELL_ERR_ARG, "static forward: B must be >= 1 and K * pad64(B) * pad64(dout) <= 2^21");
  float* out = nullptr;
  if (static_scratch_ptr(&out) != RCELL_OK) return rfail(c, RCELL_ERR_DEVICE, "static scratch address");
  const int Mp = pad64(B);
  const long long sOut = (long long)Mp * c->dp[c->L];
  forward_fused(c, (const float*)X_dev, B, Mp, out, sOut);
  const long long n = (long long)B * c->dout;
  hipLaunchKernelGGL(k_ensemble, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, out, sOut,
                     c->dp[c->L], c->K, B, c->dout, c->ymu, c->ysd, (float*)mean_dev, (float*)var_dev, (float*)nullptr);
  if (hipGetLastError() != hipSuccess) return rfail(c, RCELL_ERR_DEVICE, "static forward: launch failed");
  return RCELL_OK;
}

int rsur_forward_members(rsur_ctx* c, const void* X_dev, int32_t B, void* out_dev) {
  if (!c || !X_dev || !out_dev) return c ? rfail(c, RCELL_ERR_ARG, "NULL pointer") : RCELL_ERR_ARG;
  return forward_common(c, X_dev, B, nullptr, nullptr, (float*)out_dev);
}

int rsur_train_step(rsur_ctx* c, const void* X_dev, const void* Y_dev, int32_t B, float lr, float* loss) {
  TraceRange tr("rsur_train_step");
  if (!c || !X_dev || !Y_dev || !(lr > 0)) return c ? rfail(c, RCELL_ERR_ARG, "bad train_step arguments") : RCELL_ERR_ARG;
  int e = check_batch(c, B);
  if (e) return e;
  const int Mp = pad64(B), L = c->L;
  normalise_inputs(c, (const float*)X_dev, B, Mp);
  forward_layers(c, Mp);
  // loss and dLoss/dOutput of every member
  const long long sOut = (long long)c->Mp * c->dp[L];
  const int dmax = *std::max_element(c->dp.begin(), c->dp.end());
  const long long sdz = (long long)c->Mp * dmax;
  hipLaunchKernelGGL(k_loss, dim3(LOSS_CHUNKS, c->K), dim3(LOSS_NT), 0, c->stream, c->out, sOut, c->dp[L],
                     (const float*)Y_dev, B, c->dout, c->ymu, c->ysd, c->dza, sdz, Mp, c->lpart);
  hipLaunchKernelGGL(k_loss_total, dim3((c->K + 63) / 64), dim3(64), 0, c->stream, c->lpart, c->K, 1.0f / ((float)B * (float)c->dout),
                     c->loss);
  const int S = batch_splits(Mp);
  bf16 *dz = c->dza, *dzn = c->dzb;
  for (int l = L - 1; l >= 0; --l) {
    GemmArgs w{};                                    // dW_l = act_l^T dZ_l
    w.A = c->act[l]; w.lda = c->dp[l]; w.sA = l == 0 ? 0 : (long long)c->Mp * c->dp[l];
    w.B = dz; w.ldb = c->dp[l + 1]; w.sB = sdz;
    w.M = c->dp[l]; w.N = c->dp[l + 1]; w.K = Mp;
    w.Z = c->g + c->woff[l]; w.ldz = c->dp[l + 1]; w.sZ = c->P;
    w.ksplit = S; w.Zs = c->split;
    gemm<true, false, EPI_BWD_DW>(c, w);
    const long long nw = (long long)c->K * w.M * w.N, nb = (long long)c->K * c->dp[l + 1];
    if (S > 1)
      hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, c->stream, c->split, S, c->K,
                         w.M, w.N, c->g + c->woff[l], (long long)w.N, c->P);
    hipLaunchKernelGGL(k_colsum, dim3((c->dp[l + 1] + 63) / 64, c->K, S), dim3(64 * COLSUM_RG), 0, c->stream, dz, sdz,
                       Mp, c->dp[l + 1], c->g + c->boff[l], c->P, S, c->split);
    if (S > 1)
      hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, c->stream, c->split, S, c->K,
                         1, c->dp[l + 1], c->g + c->boff[l], (long long)c->dp[l + 1], c->P);
    if (l > 0) {                                     // dZ_{l-1} = (dZ_l W_l^T) * SiLU'(Z_{l-1})
      GemmArgs d{};
      d.A = dz; d.lda = c->dp[l + 1]; d.sA = sdz;
      d.B = c->pb + c->woff[l]; d.ldb = c->dp[l + 1]; d.sB = c->P;
      d.M = Mp; d.N = c->dp[l]; d.K = c->dp[l + 1];
      d.Zp = c->Z[l - 1]; d.ldzp = c->dp[l]; d.sZp = (long long)c->Mp * c->dp[l];
      d.O = dzn; d.ldo = c->dp[l]; d.sO = sdz;
      gemm<false, true, EPI_BWD_DA>(c, d);
      std::swap(dz, dzn);
    }
  }
  // Adam with per-member bias corrections
  std::vector<float> h1(c->K), h2(c->K);
  for (int k = 0; k < c->K; ++k) {
    c->t[k] += 1;
    h1[k] = (float)(1.0 - std::pow(0.9, (double)c->t[k]));
    h2[k] = (float)(1.0 - std::pow(0.999, (double)c->t[k]));
  }
  RCHK(c, hipMemcpyAsync(c->c1, h1.data(), sizeof(float) * c->K, hipMemcpyHostToDevice, c->stream));
  RCHK(c, hipMemcpyAsync(c->c2, h2.data(), sizeof(float) * c->K, hipMemcpyHostToDevice, c->stream));
  const long long n = (long long)c->K * c->P;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->p, c->g, c->m1, c->m2,
                     c->pb, c->P, c->K, c->c1, c->c2, lr, 0.9f, 0.999f, 1e-8f);
  c->pbt_stale = true;
  RCHK(c, hipGetLastError());
  if (loss) {
    RCHK(c, hipMemcpyAsync(loss, c->loss, sizeof(float) * c->K, hipMemcpyDeviceToHost, c->stream));
    RCHK(c, hipStreamSynchronize(c->stream));
  }
  return RCELL_OK;
}

}  // extern "C"
