// Measured machine peaks: a device copy (HBM read + write bandwidth) and independent FP32 FMA
// chains (vector ALU rate), so that the kernels' roofline fractions can be read against what
// this GPU delivers as well as against its published peaks.  The library is built without packed
// FP32 instructions, so the FMA probe measures the non-packed rate that the MD kernels can reach.
#include <hip/hip_runtime.h>

#include <cstddef>

#include "../../include/rcell.h"

namespace {

constexpr int COPY_NT = 256;
constexpr int FMA_NT = 256;
constexpr int FMA_CHAINS = 8;

// grid-stride copy of n float4 elements
__global__ __launch_bounds__(COPY_NT) void k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                         size_t n) {
  const size_t stride = (size_t)gridDim.x * COPY_NT;
  for (size_t i = (size_t)blockIdx.x * COPY_NT + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// FMA_CHAINS independent chains a <- a b + c per thread, iters times; one result per thread is
// stored so that nothing is eliminated
__global__ __launch_bounds__(FMA_NT) void k_probe_fma(float* out, int iters, float b, float c) {
  float a[FMA_CHAINS];
#pragma unroll
  for (int q = 0; q < FMA_CHAINS; ++q) a[q] = (float)(threadIdx.x + q) * 1e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < FMA_CHAINS; ++q) a[q] = fmaf(a[q], b, c);
  }
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < FMA_CHAINS; ++q) s += a[q];
  out[(size_t)blockIdx.x * FMA_NT + threadIdx.x] = s;
}

struct Events {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Events() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

}  // namespace

extern "C" int rcell_probe_peaks(size_t copy_bytes, double* copy_gbs, double* fma_tflops, void* hip_stream) {
  if (!copy_gbs || !fma_tflops || copy_bytes < 16) return RCELL_ERR_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t n = copy_bytes / sizeof(float4);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return RCELL_ERR_DEVICE;
  const int fma_blocks = cus * 32;                  // 8 waves per SIMD
  const int iters = 4096;
  float4 *src = nullptr, *dst = nullptr;
  float* out = nullptr;
  if (hipMalloc(&src, n * sizeof(float4)) != hipSuccess) return RCELL_ERR_OOM;
  if (hipMalloc(&dst, n * sizeof(float4)) != hipSuccess) {
    (void)hipFree(src);
    return RCELL_ERR_OOM;
  }
  if (hipMalloc(&out, (size_t)fma_blocks * FMA_NT * sizeof(float)) != hipSuccess) {
    (void)hipFree(src);
    (void)hipFree(dst);
    return RCELL_ERR_OOM;
  }
  int rc = RCELL_OK;
  {
    Events ev;
    float ms_copy = 0.f, ms_fma = 0.f;
    const int copy_blocks = cus * 16;
    if (hipEventCreate(&ev.e0) != hipSuccess || hipEventCreate(&ev.e1) != hipSuccess ||
        hipMemsetAsync(src, 0, n * sizeof(float4), st) != hipSuccess) {
      rc = RCELL_ERR_DEVICE;
    } else {
      // one warm-up launch of each, then the timed ones
      hipLaunchKernelGGL(k_probe_copy, dim3(copy_blocks), dim3(COPY_NT), 0, st, src, dst, n);
      (void)hipEventRecord(ev.e0, st);
      hipLaunchKernelGGL(k_probe_copy, dim3(copy_blocks), dim3(COPY_NT), 0, st, src, dst, n);
      (void)hipEventRecord(ev.e1, st);
      if (hipEventSynchronize(ev.e1) != hipSuccess || hipEventElapsedTime(&ms_copy, ev.e0, ev.e1) != hipSuccess)
        rc = RCELL_ERR_DEVICE;
      hipLaunchKernelGGL(k_probe_fma, dim3(fma_blocks), dim3(FMA_NT), 0, st, out, iters, 0.999f, 0.001f);
      (void)hipEventRecord(ev.e0, st);
      hipLaunchKernelGGL(k_probe_fma, dim3(fma_blocks), dim3(FMA_NT), 0, st, out, iters, 0.999f, 0.001f);
      (void)hipEventRecord(ev.e1, st);
      if (hipEventSynchronize(ev.e1) != hipSuccess || hipEventElapsedTime(&ms_fma, ev.e0, ev.e1) != hipSuccess ||
          hipGetLastError() != hipSuccess)
        rc = RCELL_ERR_DEVICE;
      if (rc == RCELL_OK) {
        *copy_gbs = 2.0 * (double)(n * sizeof(float4)) / (ms_copy * 1e-3) / 1e9;
        *fma_tflops = 2.0 * FMA_CHAINS * (double)iters * fma_blocks * FMA_NT / (ms_fma * 1e-3) / 1e12;
      }
    }
  }
  (void)hipFree(src);
  (void)hipFree(dst);
  (void)hipFree(out);
  return rc;
}
