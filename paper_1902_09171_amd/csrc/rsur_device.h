// Device side of the stress surrogate (gfx950): one LDS-staged BF16 matrix-core GEMM with fused
// epilogues, and the small kernels around it (normalisation, loss, bias gradients, Adam,
// ensemble statistics).  All padded dimensions are multiples of 64; padded rows and columns
// carry zeros (inputs, weights, output gradients), so they never contribute.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsur {

typedef __bf16 bf16;
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

enum Epi : int { EPI_FWD_HIDDEN = 0, EPI_FWD_OUT = 1, EPI_BWD_DA = 2, EPI_BWD_DW = 3 };

struct GemmArgs {
  const bf16* A; long long lda, sA;        // operand A, row stride, member stride
  const bf16* B; long long ldb, sB;
  int M, N, K;                             // C is M x N, reduction over K (multiples of 64/64/32)
  const float* bias; long long sBias;
  float* Z; long long ldz, sZ;             // FP32 result (pre-activation, output or gradient)
  bf16* O; long long ldo, sO;              // BF16 result (activation or backpropagated gradient)
  const float* Zp; long long ldzp, sZp;    // pre-activation whose SiLU derivative scales the result
  int nmem, ksplit;                        // members; reduction ranges (weight gradient only, else 1)
  float* Zs;                               // ksplit > 1: partial results [range][member][M][N]
};

constexpr int TM = 64, TN = 64, TK = 32, LDK = 40;   // tile sizes; LDS row stride padded to 40

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// C(m, n) = sum_k A(m, k) B(k, n) for member blockIdx.z, with A(m, k) = A[m lda + k] (or
// A[k lda + m] when AT) and B(k, n) = B[k ldb + n] (or B[n ldb + k] when BT).  A 256-thread block
// computes a 64 x 64 tile: four waves of 32 x 32, each accumulating v_mfma_f32_32x32x16_bf16
// products over K in steps of 32 staged through LDS as [m][k] and [n][k] rows.
template <bool AT, bool BT, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) bf16 sa[TM * LDK];
  __shared__ __attribute__((aligned(16))) bf16 sb[TN * LDK];
  // blockIdx.z = member + nmem * range: the weight gradient's reduction over the batch is split
  // into ksplit consecutive ranges of K / ksplit (a multiple of TK), each block taking one
  const int mem = blockIdx.z % g.nmem, ks = blockIdx.z / g.nmem;
  const int kc = g.K / g.ksplit;
  const bf16* A = g.A + mem * g.sA;
  const bf16* B = g.B + mem * g.sB;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  v16f acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int k0 = ks * kc; k0 < (ks + 1) * kc; k0 += TK) {
    if (!AT) {                                   // 64 rows of 32 contiguous k
      const int r = t >> 2, c = (t & 3) * 8;
      *(v8bf*)&sa[r * LDK + c] = *(const v8bf*)&A[(long long)(m0 + r) * g.lda + k0 + c];
    } else {                                     // 32 k-rows of 64 contiguous m, transposed into LDS
      const int r = t >> 3, c = (t & 7) * 8;
      const v8bf v = *(const v8bf*)&A[(long long)(k0 + r) * g.lda + m0 + c];
#pragma unroll
      for (int q = 0; q < 8; ++q) sa[(c + q) * LDK + r] = v[q];
    }
    if (BT) {                                    // 64 n-rows of 32 contiguous k
      const int r = t >> 2, c = (t & 3) * 8;
      *(v8bf*)&sb[r * LDK + c] = *(const v8bf*)&B[(long long)(n0 + r) * g.ldb + k0 + c];
    } else {                                     // 32 k-rows of 64 contiguous n, transposed into LDS
      const int r = t >> 3, c = (t & 7) * 8;
      const v8bf v = *(const v8bf*)&B[(long long)(k0 + r) * g.ldb + n0 + c];
#pragma unroll
      for (int q = 0; q < 8; ++q) sb[(c + q) * LDK + r] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < TK; s += 16) {
      const v8bf a = *(const v8bf*)&sa[(wm + (l & 31)) * LDK + s + 8 * (l >> 5)];
      const v8bf b = *(const v8bf*)&sb[(wn + (l & 31)) * LDK + s + 8 * (l >> 5)];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator element r of lane l holds C(row, col) with the row below
  const int col = n0 + wn + (l & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const long long row = m0 + wm + (r >> 2) * 8 + (l >> 5) * 4 + (r & 3);
    const float v = acc[r];
    if (EPI == EPI_FWD_HIDDEN) {
      const float z = v + g.bias[mem * g.sBias + col];
      g.Z[mem * g.sZ + row * g.ldz + col] = z;
      g.O[mem * g.sO + row * g.ldo + col] = (bf16)silu(z);
    } else if (EPI == EPI_FWD_OUT) {
      g.Z[mem * g.sZ + row * g.ldz + col] = v + g.bias[mem * g.sBias + col];
    } else if (EPI == EPI_BWD_DA) {
      g.O[mem * g.sO + row * g.ldo + col] = (bf16)(v * silu_grad(g.Zp[mem * g.sZp + row * g.ldzp + col]));
    } else if (g.ksplit > 1) {
      g.Zs[(((long long)ks * g.nmem + mem) * g.M + row) * g.N + col] = v;
    } else {
      g.Z[mem * g.sZ + row * g.ldz + col] = v;
    }
  }
}

// ------------------------------------------------------------------ fused inference
// Every layer of one member for 64 rows in one block: the activations stay in LDS (one buffer,
// overwritten in place between two barriers per layer), the weights are read from L2 in a
// transposed copy (WT[n][k], so a lane's 8 consecutive k are one 16-byte load) straight into the
// matrix-core B operand, and the first layer normalises the raw inputs itself.  Wave w computes
// output columns [64 w, 64 w + 64) of a layer as 2 x 2 tiles of v_mfma_f32_32x32x16_bf16 over k
// in steps of 16 - the operand layout and k order of k_gemm, so the outputs equal the layer-wise
// forward bit for bit.  Padded widths up to FW.
constexpr int FW = 256, FLD = FW + 8, MAXL = 8;

struct MlpArgs {
  const float* X; int B, din;
  const float *xmu, *xsd;
  const bf16* wt; long long sW;              // transposed BF16 weights, member stride
  const float* p; long long sP;              // FP32 parameters (biases), member stride
  int L;
  int dp[MAXL + 1];
  long long woff[MAXL], boff[MAXL];
  float* out; long long sOut; int ldo;       // K x Mp x dp[L]
};

__global__ __launch_bounds__(256, 2) void k_mlp_forward(MlpArgs g) {
  __shared__ __attribute__((aligned(16))) bf16 act[64 * FLD];
  const int mem = blockIdx.y;
  const int m0 = blockIdx.x * 64;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int d0 = g.dp[0];
  for (int e = t; e < 64 * d0; e += 256) {
    const int r = e / d0, k = e % d0, m = m0 + r;
    act[r * FLD + k] = (m < g.B && k < g.din) ? (bf16)((g.X[(long long)m * g.din + k] - g.xmu[k]) / g.xsd[k])
                                              : (bf16)0.0f;
  }
  __syncthreads();
  const bf16* Wm = g.wt + mem * g.sW;
  const float* Pm = g.p + mem * g.sP;
  const int ka = 8 * (l >> 5), ra = l & 31;
  for (int L = 0; L < g.L; ++L) {
    const int K = g.dp[L], N = g.dp[L + 1];
    const int nc = 64 * w;
    const bool on = nc < N;
    v16f acc[2][2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[q][c][r] = 0.0f;
    if (on) {
      const bf16* WT0 = Wm + g.woff[L] + (long long)(nc + ra) * K + ka;
      const bf16* WT1 = WT0 + 32LL * K;
#pragma unroll 2
      for (int k0 = 0; k0 < K; k0 += 16) {
        const v8bf b0 = *(const v8bf*)(WT0 + k0);
        const v8bf b1 = *(const v8bf*)(WT1 + k0);
        const v8bf a0 = *(const v8bf*)&act[ra * FLD + k0 + ka];
        const v8bf a1 = *(const v8bf*)&act[(32 + ra) * FLD + k0 + ka];
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
    __syncthreads();                             // every wave has read this layer's input
    if (on) {
      const bool last = L == g.L - 1;
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int col = nc + 32 * c + (l & 31);
          const float bias = Pm[g.boff[L] + col];
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = 32 * q + (r >> 2) * 8 + (l >> 5) * 4 + (r & 3);
            const float z = acc[q][c][r] + bias;
            if (!last) act[row * FLD + col] = (bf16)silu(z);
            else g.out[mem * g.sOut + (long long)(m0 + row) * g.ldo + col] = z;
          }
        }
    }
    __syncthreads();
  }
}

// transposed BF16 copy of one layer's weights for every member: WT[n][k] = W[k][n]
__global__ void k_transpose_w(const bf16* pb, bf16* pbt, long long P, long long off, int Kd, int Nd) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int mem = blockIdx.y;
  if (e >= (long long)Kd * Nd) return;
  const int n = (int)(e / Kd), k = (int)(e % Kd);
  pbt[mem * P + off + e] = pb[mem * P + off + (long long)k * Nd + n];
}

// raw inputs (B x din, FP32) -> normalised BF16 rows of width dp0, zero padding
__global__ void k_norm_in(const float* X, int B, int din, int Mp, int dp0, const float* mu, const float* sd, bf16* out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)Mp * dp0) return;
  const int m = (int)(e / dp0), k = (int)(e % dp0);
  out[e] = (m < B && k < din) ? (bf16)((X[(long long)m * din + k] - mu[k]) / sd[k]) : (bf16)0.0f;
}

// MSE on normalised outputs per member (one block per member, fixed order) and dLoss/dOutput
// Loss and its output gradient: block (chunk, member) takes rows [chunk Mp / LOSS_CHUNKS, ...) of
// one member and writes its squared-error sum to part[member][chunk] (a fixed tree over the block);
// k_loss_total adds the chunks in order.  Element indices are 64-bit (Mp * ldo may exceed 2^31).
constexpr int LOSS_NT = 256, LOSS_CHUNKS = 16;
__global__ __launch_bounds__(LOSS_NT) void k_loss(const float* out, long long sOut, int ldo, const float* Y, int B,
                                                  int dout, const float* ymu, const float* ysd, bf16* dY,
                                                  long long sdY, int Mp, float* part) {
  __shared__ float sh[LOSS_NT];
  const int chunk = blockIdx.x, mem = blockIdx.y;
  const float inv = 1.0f / ((float)B * (float)dout);
  const long long rows = Mp / LOSS_CHUNKS, e0 = chunk * rows * ldo, e1 = e0 + rows * ldo;
  float acc = 0.0f;
  for (long long e = e0 + (long long)threadIdx.x; e < e1; e += LOSS_NT) {
    const long long m = e / ldo;
    const int n = (int)(e - m * ldo);
    float gr = 0.0f;
    if (m < B && n < dout) {
      const float yn = (Y[(long long)m * dout + n] - ymu[n]) / ysd[n];
      const float d = out[mem * sOut + e] - yn;
      acc += d * d;
      gr = 2.0f * d * inv;
    }
    dY[mem * sdY + e] = (bf16)gr;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = LOSS_NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[mem * LOSS_CHUNKS + chunk] = sh[0];
}

__global__ void k_loss_total(const float* part, int K, float inv, float* loss) {
  const int mem = blockIdx.x * blockDim.x + threadIdx.x;
  if (mem >= K) return;
  float t = 0.0f;
  for (int c = 0; c < LOSS_CHUNKS; ++c) t += part[mem * LOSS_CHUNKS + c];
  loss[mem] = t * inv;
}

// out[member][r][c] = the sum, over the S partial results in order, of part[s][member][r][c]
// (R x C values per member): the second stage of the split reductions
__global__ void k_sum_splits(const float* part, int S, int nmem, int R, int C, float* out, long long ldo,
                             long long sOut) {
  const long long per = (long long)R * C;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per * nmem) return;
  const int mem = (int)(e / per);
  const long long rc = e - mem * per;
  const int r = (int)(rc / C), c = (int)(rc - (long long)r * C);
  float t = 0.0f;
  for (int s = 0; s < S; ++s) t += part[((long long)s * nmem + mem) * per + rc];
  out[mem * sOut + (long long)r * ldo + c] = t;
}

// bias gradient: column sums of the BF16 output gradient.  Block (x, member, range) takes 64
// columns of one member over rows [range Mp / S, (range + 1) Mp / S) with COLSUM_RG row groups
// (group g sums every COLSUM_RG-th row; a wave reads 64 consecutive columns of a row); the group
// sums meet in LDS and are added in group order, and the S range sums go to part[range][member][n]
// for k_sum_splits (S = 1: straight to gb).  Deterministic.
constexpr int COLSUM_RG = 16;
__global__ __launch_bounds__(64 * COLSUM_RG) void k_colsum(const bf16* dZ, long long sdZ, int Mp, int ld,
                                                           float* gb, long long sgb, int S, float* part) {
  __shared__ float sum[COLSUM_RG][64];
  const int mem = blockIdx.y, range = blockIdx.z;
  const int c = threadIdx.x % 64, grp = threadIdx.x / 64;
  const int n = blockIdx.x * 64 + c;
  const int rows = Mp / S, m0 = range * rows;
  float s = 0.0f;
  if (n < ld)
    for (int m = m0 + grp; m < m0 + rows; m += COLSUM_RG) s += (float)dZ[mem * sdZ + (long long)m * ld + n];
  sum[grp][c] = s;
  __syncthreads();
  if (grp == 0 && n < ld) {
    float t = 0.0f;
    for (int g = 0; g < COLSUM_RG; ++g) t += sum[g][c];
    if (S == 1) gb[mem * sgb + n] = t;
    else part[((long long)range * gridDim.y + mem) * ld + n] = t;
  }
}

// Adam on every padded parameter of every member; refreshes the BF16 copy of the weights
__global__ void k_adam(float* p, const float* gr, float* m1, float* m2, bf16* pb, long long P, int K,
                       const float* c1, const float* c2, float lr, float b1, float b2, float eps) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P * K) return;
  const int mem = (int)(e / P);
  const float g = gr[e];
  const float a = b1 * m1[e] + (1.0f - b1) * g;
  const float b = b2 * m2[e] + (1.0f - b2) * g * g;
  m1[e] = a;
  m2[e] = b;
  const float mh = a / c1[mem], vh = b / c2[mem];
  const float q = p[e] - lr * mh / (sqrtf(vh) + eps);
  p[e] = q;
  pb[e] = (bf16)q;
}

__global__ void k_to_bf16(const float* p, bf16* pb, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) pb[e] = (bf16)p[e];
}

// ensemble mean and population variance of the de-normalised outputs (and per-member outputs)
__global__ void k_ensemble(const float* out, long long sOut, int ldo, int K, int B, int dout, const float* ymu,
                           const float* ysd, float* mean, float* var, float* members) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)B * dout) return;
  const int m = (int)(e / dout), n = (int)(e % dout);
  float s = 0.0f;
  for (int k = 0; k < K; ++k) {
    const float y = out[k * sOut + (long long)m * ldo + n] * ysd[n] + ymu[n];
    if (members) members[(long long)k * B * dout + e] = y;
    s += y;
  }
  const float mu = s / (float)K;
  if (mean) mean[e] = mu;
  if (var) {
    float q = 0.0f;
    for (int k = 0; k < K; ++k) {
      const float d = out[k * sOut + (long long)m * ldo + n] * ysd[n] + ymu[n] - mu;
      q += d * d;
    }
    var[e] = q / (float)K;
  }
}

// per-column mean and population standard deviation of n rows (one block per column)
constexpr int FIT_NT = 256;
__global__ __launch_bounds__(FIT_NT) void k_fit_norm(const float* X, int n, int d, float* mu, float* sd) {
  __shared__ double sh[FIT_NT];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int r = threadIdx.x; r < n; r += FIT_NT) s += X[(long long)r * d + c];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = FIT_NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double m = sh[0] / n;
  __syncthreads();
  s = 0.0;
  for (int r = threadIdx.x; r < n; r += FIT_NT) {
    const double q = X[(long long)r * d + c] - m;
    s += q * q;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = FIT_NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mu[c] = (float)m;
    sd[c] = (float)fmax(sqrt(sh[0] / n), 1e-6);
  }
}

}  // namespace rsur
