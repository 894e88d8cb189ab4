// fn_mlp.hip -- the learned T-window surrogate: a 4-layer MLP
// 28 -> 256 -> 256 -> 256 -> 2 (SiLU after the first three layers) mapping an
// edge's two boundary states to (standardised log T*, feasibility logit).
// BF16 weights and activations, FP32 accumulation on the MFMA units
// (v_mfma_f32_16x16x32_bf16), FP32 master weights and Adam moments.
//
// Rounding points (the arithmetic this surrogate is defined with):
//   inputs, weights and hidden activations are rounded to BF16 before every
//   product; pre-activations Z, outputs Y, the loss gradient dY and the
//   back-propagated dZ are FP32, and dY / dZ are rounded to BF16 before the
//   weight- and input-gradient products; bias gradients sum the FP32 dZ.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fn_ctx.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace fn {

constexpr int W = 256;         // hidden width
constexpr int NIN = 28;        // raw inputs
constexpr int NIN_P = 32;      // padded inputs
constexpr int NOUT = 2;
constexpr int NOUT_P = 64;     // padded outputs (one GEMM tile)
// padded parameter layout (FP32 master, gradients, Adam moments)
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + W * NIN_P;
constexpr int OFF_W2 = OFF_B1 + W, OFF_B2 = OFF_W2 + W * W;
constexpr int OFF_W3 = OFF_B2 + W, OFF_B3 = OFF_W3 + W * W;
constexpr int OFF_W4 = OFF_B3 + W, OFF_B4 = OFF_W4 + NOUT_P * W;
constexpr int NP_PAD = OFF_B4 + NOUT_P;
// logical layout (W1[256][28], b1, W2, b2, W3, b3, W4[2][256], b4[2])
constexpr int NP_LOG = W * NIN + W + W * W + W + W * W + W + NOUT * W + NOUT;
constexpr int MAX_SPLIT = 16;

// ---------------------------------------------------------------------------
// Tiled GEMM: C[M][N] = sum_k A(m, k) B(k, n), BF16 operands, FP32
// accumulation.  A(m, k) = A[m*lda + k] (or A[k*lda + m] when TA), B(k, n) =
// B[k*ldb + n] (or B[n*ldb + k] when TB).  64x64 tile per workgroup, four
// wavefronts of 32x32, K step 32 = one 16x16x32 MFMA per 16x16 sub-tile.
// blockIdx.z splits K (partial sums to Cf + z * split_stride).
// M, N and K must be multiples of 8.
// ---------------------------------------------------------------------------
enum { EPI_F32 = 0, EPI_BIAS_SILU = 1, EPI_BIAS_F32 = 2, EPI_DSILU = 3 };
constexpr int BM = 64, BN = 64, BK = 32, LDSR = BK + 8;

// Logistic function with the hardware exponential and reciprocal (1 ulp
// each): an IEEE division here made the activations the largest part of the
// fused inference kernel's instructions.
__device__ __forceinline__ float sigmoidf_(float z) {
  return __builtin_amdgcn_rcpf(1.f + __expf(-z));
}

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void gemm_bf16(const bf16* __restrict__ A, int lda,
                                                 const bf16* __restrict__ B, int ldb, int M,
                                                 int N, int K, int k_per_split,
                                                 float* __restrict__ Cf, bf16* __restrict__ Cb,
                                                 int ldc, int64_t split_stride,
                                                 const float* __restrict__ bias,
                                                 const float* __restrict__ Zaux) {
  __shared__ bf16 As[BM][LDSR];
  __shared__ bf16 Bs[BN][LDSR];
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kb = blockIdx.z * k_per_split, ke = min(K, kb + k_per_split);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero8 = {};
  for (int k0 = kb; k0 < ke; k0 += BK) {
    if (!TA) {
      const int r = tid >> 2, g = (tid & 3) * 8, m = m0 + r, k = k0 + g;
      bf16x8 v = zero8;
      if (m < M && k < ke) v = *reinterpret_cast<const bf16x8*>(A + (size_t)m * lda + k);
      *reinterpret_cast<bf16x8*>(&As[r][g]) = v;
    } else {
      const int kr = tid >> 3, g = (tid & 7) * 8, k = k0 + kr, m = m0 + g;
      bf16x8 v = zero8;
      if (k < ke && m < M) v = *reinterpret_cast<const bf16x8*>(A + (size_t)k * lda + m);
#pragma unroll
      for (int i = 0; i < 8; ++i) As[g + i][kr] = v[i];
    }
    if (TB) {
      const int r = tid >> 2, g = (tid & 3) * 8, n = n0 + r, k = k0 + g;
      bf16x8 v = zero8;
      if (n < N && k < ke) v = *reinterpret_cast<const bf16x8*>(B + (size_t)n * ldb + k);
      *reinterpret_cast<bf16x8*>(&Bs[r][g]) = v;
    } else {
      const int kr = tid >> 3, g = (tid & 7) * 8, k = k0 + kr, n = n0 + g;
      bf16x8 v = zero8;
      if (k < ke && n < N) v = *reinterpret_cast<const bf16x8*>(B + (size_t)k * ldb + n);
#pragma unroll
      for (int i = 0; i < 8; ++i) Bs[g + i][kr] = v[i];
    }
    __syncthreads();
    // operand fragments: lane l holds row (l & 15), k = 8 (l >> 4) .. + 7
    const int row = lane & 15, kg = (lane >> 4) * 8;
    const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(&As[wm + row][kg]);
    const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(&As[wm + 16 + row][kg]);
    const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(&Bs[wn + row][kg]);
    const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 + row][kg]);
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
    __syncthreads();
  }
  // result fragment: lane l holds rows 4 (l >> 4) .. + 3 of column (l & 15)
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = m0 + wm + ti * 16 + (lane >> 4) * 4 + i;
        const int n = n0 + wn + tj * 16 + (lane & 15);
        if (m >= M || n >= N) continue;
        const float v = acc[ti][tj][i];
        const size_t o = (size_t)m * ldc + n;
        if (EPI == EPI_F32) {
          Cf[(size_t)blockIdx.z * split_stride + o] = v;
        } else if (EPI == EPI_BIAS_F32) {
          Cf[o] = v + bias[n];
        } else if (EPI == EPI_BIAS_SILU) {
          const float z = v + bias[n];
          if (Cf) Cf[o] = z;
          Cb[o] = (bf16)(z * sigmoidf_(z));
        } else {
          const float z = Zaux[o];
          const float s = sigmoidf_(z);
          const float dz = v * s * (1.f + z * (1.f - s));
          Cf[o] = dz;
          Cb[o] = (bf16)dz;
        }
      }
}

template <bool TA, bool TB, int EPI>
static void gemm(hipStream_t s, const bf16* A, int lda, const bf16* B, int ldb, int M, int N,
                 int K, float* Cf, bf16* Cb, int ldc, const float* bias = nullptr,
                 const float* Zaux = nullptr, int splits = 1, int64_t split_stride = 0) {
  int kps = (K + splits - 1) / splits;
  kps = (kps + BK - 1) / BK * BK;
  splits = (K + kps - 1) / kps;
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, splits);
  hipLaunchKernelGGL((gemm_bf16<TA, TB, EPI>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K,
                     kps, Cf, Cb, ldc, split_stride, bias, Zaux);
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
struct Norm {
  float shift[NIN], scale[NIN];  // x_norm = (x - shift) * scale
};

// rows r of the batch: source row perm(base + r) of X (raw [N][28]);
// normalise, pad to 32, round to BF16; targets from the slot index.
__global__ void mlp_gather(const float* __restrict__ X, const int16_t* __restrict__ yj, int64_t N,
                           int64_t base, uint64_t pa, uint64_t pc, int rows, Norm nm,
                           const float* __restrict__ grid, int n_t, bf16* __restrict__ Xb,
                           float* __restrict__ tgt, float* __restrict__ feas, int* __restrict__ nf) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const uint64_t i = (uint64_t)(base + r) % (uint64_t)N;
  const int64_t src = (int64_t)((pa * i + pc) % (uint64_t)N);
#pragma unroll 4
  for (int c = 0; c < NIN_P; ++c)
    Xb[(size_t)r * NIN_P + c] =
        (bf16)(c < NIN ? (X[src * NIN + c] - nm.shift[c]) * nm.scale[c] : 0.f);
  if (yj) {
    const int j = yj[src];
    const float l0 = logf(grid[0]), l1 = logf(grid[n_t - 1]);
    const float mu = 0.5f * (l0 + l1), sg = 0.5f * (l1 - l0);
    const bool f = j >= 0 && j < n_t;
    tgt[r] = f ? (logf(grid[j]) - mu) / sg : 0.f;
    feas[r] = f ? 1.f : 0.f;
    if (f) atomicAdd(nf, 1);
  }
}

// loss and dL/dY for one batch (a single workgroup; fixed reduction order)
__global__ __launch_bounds__(1024) void mlp_loss(const float* __restrict__ Y,
                                                 const float* __restrict__ tgt,
                                                 const float* __restrict__ feas,
                                                 const int* __restrict__ nf_p, int rows,
                                                 float* __restrict__ dYf, bf16* __restrict__ dYb,
                                                 float* __restrict__ acc3, float scale) {
  __shared__ float sm[1024], sb[1024];
  const float nf = fmaxf(1.f, (float)*nf_p);
  float lm = 0.f, lb = 0.f;
  for (int r = threadIdx.x; r < rows; r += blockDim.x) {
    const float y0 = Y[(size_t)r * NOUT_P], y1 = Y[(size_t)r * NOUT_P + 1];
    const float f = feas[r];
    const float d = (y0 - tgt[r]) * f;
    lm += d * d;
    lb += fmaxf(y1, 0.f) - y1 * f + log1pf(__expf(-fabsf(y1)));
    const float g0 = 2.f * d / nf, g1 = (sigmoidf_(y1) - f) / (float)rows;
    // columns 2.. of dY stay zero (cleared when the network is created)
    dYf[(size_t)r * NOUT_P] = g0;
    dYf[(size_t)r * NOUT_P + 1] = g1;
    dYb[(size_t)r * NOUT_P] = (bf16)g0;
    dYb[(size_t)r * NOUT_P + 1] = (bf16)g1;
  }
  sm[threadIdx.x] = lm;
  sb[threadIdx.x] = lb;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sm[threadIdx.x] += sm[threadIdx.x + o];
      sb[threadIdx.x] += sb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && acc3) {
    const float m = sm[0] / nf * scale, b = sb[0] / (float)rows * scale;
    acc3[0] += m + b;
    acc3[1] += m;
    acc3[2] += b;
  }
}

// column sums of a [rows][ncol] FP32 matrix (bias gradients), two passes
// with a fixed order: row chunks of COLSUM_ROWS give partial sums, then the
// partials are added in chunk order
constexpr int COLSUM_ROWS = 32;
__global__ void mlp_colsum_part(const float* __restrict__ D, int rows, int ncol, int ld,
                                float* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.y * COLSUM_ROWS;
  if (c >= ncol) return;
  float v[COLSUM_ROWS];
#pragma unroll
  for (int r = 0; r < COLSUM_ROWS; ++r) v[r] = r0 + r < rows ? D[(size_t)(r0 + r) * ld + c] : 0.f;
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < COLSUM_ROWS; ++r) s += v[r];
  part[(size_t)blockIdx.y * ncol + c] = s;
}
__global__ void mlp_colsum_final(const float* __restrict__ part, int chunks, int ncol,
                                 float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  float s = 0.f;
#pragma unroll 16
  for (int z = 0; z < chunks; ++z) s += part[(size_t)z * ncol + c];
  out[c] = s;
}

// sum of split-K partial tiles, in split order
__global__ void mlp_reduce_splits(const float* __restrict__ part, int splits, int64_t stride,
                                  int n, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += part[(size_t)z * stride + i];
  out[i] = s;
}

__device__ __forceinline__ bool is_weight(int i) {
  return i < OFF_B1 || (i >= OFF_W2 && i < OFF_B2) || (i >= OFF_W3 && i < OFF_B3) ||
         (i >= OFF_W4 && i < OFF_B4);
}

// one Adam step with bias correction and a cosine learning-rate decay
__global__ void mlp_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                         const float* __restrict__ g, bf16* __restrict__ wb, int64_t step,
                         int64_t total, float lr0, float b1, float b2, float eps, int cosine) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NP_PAD) return;
  const double t = (double)step;  // 1-based
  const float lr = cosine ? (float)(0.5 * lr0 * (1.0 + cos(M_PI * (t - 1.0) / (double)total))) : lr0;
  const float c1 = (float)(1.0 - pow((double)b1, t)), c2 = (float)(1.0 - pow((double)b2, t));
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (is_weight(i)) wb[i] = (bf16)pi;
}

__global__ void mlp_to_bf16(const float* __restrict__ p, bf16* __restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NP_PAD) wb[i] = (bf16)p[i];
}

// Inference weights packed in the matrix cores' operand order: for a layer
// of N outputs and K inputs, the B operand of output tile nt (16 outputs)
// and K step ks (32 inputs) is one contiguous 1 KiB block at
// ((nt * K/32) + ks) * 512 elements, lane l's 8 values at l * 8 (outputs
// 16 nt + (l & 15), inputs 32 ks + 8 (l >> 4) + e).  A wavefront's operand
// read is then one contiguous KiB instead of 16 half-used cache lines.
constexpr int SW1 = 0, SW2 = SW1 + W * NIN_P, SW3 = SW2 + W * W, SW4 = SW3 + W * W;
constexpr int NSW = SW4 + 16 * W;

__device__ __forceinline__ int64_t packed_src(int64_t i) {
  int off, K;
  int64_t j;
  if (i < SW2) { off = OFF_W1; K = NIN_P; j = i - SW1; }
  else if (i < SW3) { off = OFF_W2; K = W; j = i - SW2; }
  else if (i < SW4) { off = OFF_W3; K = W; j = i - SW3; }
  else { off = OFF_W4; K = W; j = i - SW4; }
  const int64_t block = j / 512, within = j % 512;
  const int l = (int)(within / 8), e = (int)(within % 8);
  const int64_t nt = block / (K / BK), ks = block % (K / BK);
  return off + (16 * nt + (l & 15)) * K + BK * ks + 8 * (l >> 4) + e;
}

__global__ void mlp_pack(const bf16* __restrict__ wb, bf16* __restrict__ wsw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NSW) wsw[i] = wb[packed_src(i)];
}

// padded <-> logical parameter layouts
__device__ __forceinline__ int64_t log_to_pad(int64_t i) {
  int64_t o = 0;
  if (i < W * NIN) return OFF_W1 + (i / NIN) * NIN_P + i % NIN;
  o = W * NIN;
  if (i < o + W) return OFF_B1 + (i - o);
  o += W;
  if (i < o + W * W) return OFF_W2 + (i - o);
  o += W * W;
  if (i < o + W) return OFF_B2 + (i - o);
  o += W;
  if (i < o + W * W) return OFF_W3 + (i - o);
  o += W * W;
  if (i < o + W) return OFF_B3 + (i - o);
  o += W;
  if (i < o + NOUT * W) return OFF_W4 + (i - o);
  o += NOUT * W;
  return OFF_B4 + (i - o);
}
__global__ void mlp_gather_params(const float* __restrict__ pad, float* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < NP_LOG) out[i] = pad[log_to_pad(i)];
}
__global__ void mlp_scatter_params(const float* __restrict__ in, float* __restrict__ pad) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < NP_LOG) pad[log_to_pad(i)] = in[i];
}

// outputs and windows: out[n] = (y0, y1); win_lo = nearest slot to the
// predicted log T minus half, or n_t when the logit is below logit_min
__global__ void mlp_window(const float* __restrict__ Y, int rows, const float* __restrict__ grid,
                           int n_t, int half, float logit_min, float* __restrict__ out,
                           int16_t* __restrict__ win) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const float y0 = Y[(size_t)r * NOUT_P], y1 = Y[(size_t)r * NOUT_P + 1];
  if (out) {
    out[2 * r] = y0;
    out[2 * r + 1] = y1;
  }
  if (!win) return;
  if (!(y1 >= logit_min)) {
    win[r] = (int16_t)n_t;
    return;
  }
  const float l0 = logf(grid[0]), l1 = logf(grid[n_t - 1]);
  const float lt = 0.5f * (l0 + l1) + 0.5f * (l1 - l0) * y0;
  // nearest grid slot in log T (binary search, grid increasing)
  int lo = 0, hi = n_t - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (logf(grid[mid]) <= lt) lo = mid;
    else hi = mid;
  }
  const int j = (lt - logf(grid[lo]) <= logf(grid[hi]) - lt) ? lo : hi;
  win[r] = (int16_t)max(0, j - half);
}

// ---------------------------------------------------------------------------
// Fused inference: all four layers of FR rows (32 or 64) in one workgroup.
// The row tile's activations stay in LDS (one BF16 buffer, row stride HLD);
// wave w computes output columns [64 w, 64 w + 64) of a 256-wide layer for
// all FR rows (FR/16 x 4 tiles of 16 x 16, FP32 accumulators), with the
// weights read
// from L2 straight into the MFMA B operands.  Every wave holds its whole
// output tile in registers until the layer's reads are done, so one barrier
// later the tile overwrites the layer's input in place.  The MFMA
// instruction, operand layout and K order are those of gemm_bf16, so the
// outputs equal the layer-by-layer path bit for bit.
// ---------------------------------------------------------------------------
constexpr int HLD = W + 8;    // LDS row stride of the activation tile (BF16)

// One 256-wide layer, K inputs (a multiple of 32) from Hs, SiLU(z + bias)
// rounded to BF16 back into Hs.
template <int K, int RT>
__device__ __forceinline__ void fused_layer(bf16 (*Hs)[HLD], const bf16* __restrict__ Wp,
                                            const float* __restrict__ bias, int wave, int lane) {
  // rows [64 (wave / 4), + 16 RT), output columns [64 (wave % 4), + 64)
  Hs += 64 * (wave >> 2);
  wave &= 3;
  f32x4 acc[RT][4];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int row = lane & 15, kg = (lane >> 4) * 8, n0 = wave * 64;
  // Weight operands travel PD K steps ahead of the products (a ring of PD
  // register sets): one step's 16 products take far less than an L2 read,
  // so a shallower pipeline leaves the matrix cores waiting.  The
  // scheduling barriers keep the compiler from sinking the reads back.
  constexpr int KS = K / BK, PD = KS < 4 ? KS : 4;
  float bn[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) bn[j] = bias[n0 + 16 * j + row];
  bf16x8 b[PD][4];
#pragma unroll
  for (int ks = 0; ks < PD; ++ks)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      b[ks][j] = *reinterpret_cast<const bf16x8*>(Wp + ((size_t)(4 * wave + j) * KS + ks) * 512 +
                                                  lane * 8);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    bf16x8 a[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(&Hs[16 * i + row][ks * BK + kg]);
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[ks % PD][j], acc[i][j], 0, 0, 0);
    if (ks + PD < KS) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[ks % PD][j] = *reinterpret_cast<const bf16x8*>(
            Wp + ((size_t)(4 * wave + j) * KS + ks + PD) * 512 + lane * 8);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();  // every wave has read the layer's input
  // result fragment: lane l holds rows 4 (l >> 4) .. + 3 of column (l & 15)
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + 16 * j + row;
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float z = acc[i][j][t] + bn[j];
        Hs[16 * i + (lane >> 4) * 4 + t][n] = (bf16)(z * sigmoidf_(z));
      }
  }
  __syncthreads();
}

// Where the input rows come from: a feature matrix X [N][28], or (GATHER)
// the edges themselves -- row e is the state of tree node nbr[e] followed by
// that of candidate e / k, zeros for a padded or out-of-range parent (the
// rows edge_features writes).
struct RowSrc {
  const float* X;
  const float* tree;
  int64_t ld;
  int n_nodes;
  const float* cand;
  const int32_t* nbr;
  int k;
};

template <bool GATHER>
__device__ __forceinline__ float input_of(const RowSrc& src, int64_t row, int c) {
  if constexpr (!GATHER) {
    return src.X[row * NIN + c];
  } else {
    const int p = src.nbr[row];
    if (p < 0 || p >= src.n_nodes) return 0.f;
    return c < FN_STATE ? src.tree[(size_t)c * src.ld + p]
                        : src.cand[(row / src.k) * FN_STATE + c - FN_STATE];
  }
}

// FR rows per workgroup: one group of four wavefronts per 64 rows (FR = 32:
// one group on 32 rows); every group reads the layer weights for its rows
// through the L1, so more groups per workgroup share them.
template <int FR>
constexpr int infer_threads() { return FR <= 64 ? 256 : 256 * (FR / 64); }

template <bool GATHER, int FR>
__global__ __launch_bounds__(infer_threads<FR>()) void mlp_infer_fused(RowSrc src, int64_t N, Norm nm,
                                                       const bf16* __restrict__ wsw,
                                                       const float* __restrict__ p,
                                                       const float* __restrict__ grid, int n_t,
                                                       int half, float logit_min,
                                                       float* __restrict__ out,
                                                       int16_t* __restrict__ win) {
  __shared__ bf16 Hs[FR][HLD];
  __shared__ float s_y[FR][NOUT];
  __shared__ float s_lg[FN_MAX_NT];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t r0 = (int64_t)blockIdx.x * FR;
  constexpr int NT = infer_threads<FR>();
  // normalised inputs, padded to 32 columns, rounded to BF16 (rows past N: 0)
  for (int t = tid; t < FR * NIN_P; t += NT) {
    const int r = t / NIN_P, c = t % NIN_P;
    const int64_t row = r0 + r;
    Hs[r][c] = (bf16)(c < NIN && row < N ? (input_of<GATHER>(src, row, c) - nm.shift[c]) * nm.scale[c]
                                         : 0.f);
  }
  if (win)
    for (int t = tid; t < n_t; t += NT) s_lg[t] = logf(grid[t]);
  __syncthreads();
  constexpr int RT = (FR < 64 ? FR : 64) / 16;
  fused_layer<NIN_P, RT>(Hs, wsw + SW1, p + OFF_B1, wave, lane);
  fused_layer<W, RT>(Hs, wsw + SW2, p + OFF_B2, wave, lane);
  fused_layer<W, RT>(Hs, wsw + SW3, p + OFF_B3, wave, lane);
  for (int rt = wave; rt < FR / 16; rt += NT / 64) {
    // output layer: wave w takes the row tiles rt = w, w + waves, ...,
    // output columns 0..15 (W4 is padded with zero rows; columns 0 and 1 are
    // the outputs)
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    const int row = lane & 15, kg = (lane >> 4) * 8;
    const bf16* W4 = wsw + SW4;
#pragma unroll
    for (int k0 = 0; k0 < W; k0 += BK) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&Hs[16 * rt + row][k0 + kg]);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(W4 + (size_t)(k0 / BK) * 512 + lane * 8);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    if (row < NOUT) {
      const float bn = p[OFF_B4 + row];
#pragma unroll
      for (int t = 0; t < 4; ++t) s_y[16 * rt + (lane >> 4) * 4 + t][row] = acc[t] + bn;
    }
  }
  __syncthreads();
  if (tid >= FR) return;
  const int64_t r = r0 + tid;
  if (r >= N) return;
  const float y0 = s_y[tid][0], y1 = s_y[tid][1];
  if (out) {
    out[2 * r] = y0;
    out[2 * r + 1] = y1;
  }
  if (!win) return;
  if (!(y1 >= logit_min)) {
    win[r] = (int16_t)n_t;
    return;
  }
  const float l0 = s_lg[0], l1 = s_lg[n_t - 1];
  const float lt = 0.5f * (l0 + l1) + 0.5f * (l1 - l0) * y0;
  // nearest grid slot in log T (binary search, grid increasing)
  int lo = 0, hi = n_t - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s_lg[mid] <= lt) lo = mid;
    else hi = mid;
  }
  const int j = (lt - s_lg[lo] <= s_lg[hi] - lt) ? lo : hi;
  win[r] = (int16_t)max(0, j - half);
}

// edge features: row e = (state of tree node nbr[e], state of candidate e / k)
__global__ void edge_features_kernel(const float* __restrict__ tree, int64_t ld, int n_nodes,
                                     const float* __restrict__ cand, const int32_t* __restrict__ nbr,
                                     int k, int64_t E, float* __restrict__ X) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int p = nbr[e];
  const int64_t b = e / k;
  const bool ok = p >= 0 && p < n_nodes;
#pragma unroll
  for (int c = 0; c < FN_STATE; ++c) {
    X[e * 28 + c] = ok ? tree[(size_t)c * ld + p] : 0.f;
    X[e * 28 + FN_STATE + c] = ok ? cand[b * FN_STATE + c] : 0.f;
  }
}

}  // namespace fn

using namespace fn;

struct fn_mlp {
  fn_ctx* ctx;
  Norm norm;
  float *p, *m, *v, *g;   // padded FP32 params, moments, gradient
  bf16* wb;               // BF16 weights (padded layout)
  bf16* wsw;              // BF16 weights packed for the fused inference (mlp_pack)
  int64_t ver, wsw_ver;   // weight version, version wsw was packed from
  int64_t step;
  int rows;               // workspace rows
  bf16 *Xb, *H1, *H2, *H3, *dYb, *dZb0, *dZb1;
  float *Z1, *Z2, *Z3, *Y, *dYf, *dZf0, *dZf1, *tgt, *feas, *part, *acc3, *colpart;
  int* nf;
};

static constexpr int MLP_ROWS = 8192;

static int mlp_alloc(fn_mlp* n) {
  const size_t R = n->rows;
  hipError_t e = hipSuccess;
#define A(ptr, bytes)                                  \
  if (e == hipSuccess) e = hipMalloc((void**)&(ptr), (bytes));
  A(n->p, NP_PAD * 4) A(n->m, NP_PAD * 4) A(n->v, NP_PAD * 4) A(n->g, NP_PAD * 4)
  A(n->wb, NP_PAD * 2) A(n->wsw, NSW * 2) A(n->Xb, R * NIN_P * 2) A(n->H1, R * W * 2) A(n->H2, R * W * 2)
  A(n->H3, R * W * 2) A(n->dYb, R * NOUT_P * 2) A(n->dZb0, R * W * 2) A(n->dZb1, R * W * 2)
  A(n->Z1, R * W * 4) A(n->Z2, R * W * 4) A(n->Z3, R * W * 4) A(n->Y, R * NOUT_P * 4)
  A(n->dYf, R * NOUT_P * 4) A(n->dZf0, R * W * 4) A(n->dZf1, R * W * 4) A(n->tgt, R * 4)
  A(n->feas, R * 4) A(n->part, (size_t)MAX_SPLIT * W * W * 4) A(n->acc3, 64 * 4) A(n->nf, 64 * 4)
  A(n->colpart, ((R + COLSUM_ROWS - 1) / COLSUM_ROWS) * W * 4)
#undef A
  return e == hipSuccess ? FN_OK : fail(FN_E_NOMEM, "fn_mlp: hipMalloc: %s", hipGetErrorString(e));
}

extern "C" void fn_mlp_destroy(fn_mlp* n) {
  if (!n) return;
  (void)hipDeviceSynchronize();
  void* ps[] = {n->p, n->m, n->v, n->g, n->wb, n->wsw, n->Xb, n->H1, n->H2, n->H3, n->dYb, n->dZb0,
                n->dZb1, n->Z1, n->Z2, n->Z3, n->Y, n->dYf, n->dZf0, n->dZf1, n->tgt, n->feas,
                n->part, n->acc3, n->nf, n->colpart};
  for (void* q : ps)
    if (q) (void)hipFree(q);
  delete n;
}

// SplitMix64 (Steele, Lea and Flood, 2014), the default weight initialiser
static uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static int mlp_upload_logical(fn_mlp* n, const float* host) {
  float* d = nullptr;
  hipError_t e = hipMalloc((void**)&d, NP_LOG * 4);
  if (e != hipSuccess) return fail(FN_E_NOMEM, "fn_mlp: %s", hipGetErrorString(e));
  e = hipMemcpy(d, host, NP_LOG * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(n->p, 0, NP_PAD * 4);
  if (e == hipSuccess) e = hipMemset(n->m, 0, NP_PAD * 4);
  if (e == hipSuccess) e = hipMemset(n->v, 0, NP_PAD * 4);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(mlp_scatter_params, dim3((NP_LOG + 255) / 256), dim3(256), 0, 0, d, n->p);
    hipLaunchKernelGGL(mlp_to_bf16, dim3((NP_PAD + 255) / 256), dim3(256), 0, 0, n->p, n->wb);
    e = hipDeviceSynchronize();
  }
  (void)hipFree(d);
  ++n->ver;
  n->step = 0;
  return e == hipSuccess ? FN_OK : hip_fail(e, "fn_mlp: upload");
}

extern "C" int fn_mlp_set_params(fn_mlp* n, const float* host, int64_t count) {
  if (!n || !host) return fail(FN_E_ARG, "fn_mlp_set_params: NULL argument");
  if (count != NP_LOG) return fail(FN_E_SHAPE, "fn_mlp_set_params: %lld values (need %d)", (long long)count, NP_LOG);
  return mlp_upload_logical(n, host);
}

extern "C" int fn_mlp_get_params(const fn_mlp* n, float* host, int64_t count) {
  if (!n || !host) return fail(FN_E_ARG, "fn_mlp_get_params: NULL argument");
  if (count != NP_LOG) return fail(FN_E_SHAPE, "fn_mlp_get_params: %lld values (need %d)", (long long)count, NP_LOG);
  float* d = nullptr;
  hipError_t e = hipMalloc((void**)&d, NP_LOG * 4);
  if (e != hipSuccess) return fail(FN_E_NOMEM, "fn_mlp_get_params: %s", hipGetErrorString(e));
  hipLaunchKernelGGL(mlp_gather_params, dim3((NP_LOG + 255) / 256), dim3(256), 0, 0, n->p, d);
  e = hipMemcpy(host, d, NP_LOG * 4, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  return e == hipSuccess ? FN_OK : hip_fail(e, "fn_mlp_get_params");
}

extern "C" int fn_mlp_param_count(void) { return NP_LOG; }

extern "C" int fn_mlp_create(fn_ctx* ctx, uint64_t seed, fn_mlp** out) {
  if (!ctx || !out) return fail(FN_E_ARG, "fn_mlp_create: NULL argument");
  *out = nullptr;
  fn_mlp* n = new fn_mlp();
  std::memset(n, 0, sizeof(*n));
  n->ctx = ctx;
  n->rows = MLP_ROWS;
  // input normalisation from the arm's limits
  for (int i = 0; i < NJ; ++i) {
    const double cen = 0.5 * (ctx->desc.qmax[i] + ctx->desc.qmin[i]);
    const double half = 0.5 * (ctx->desc.qmax[i] - ctx->desc.qmin[i]);
    n->norm.shift[i] = (float)cen;
    n->norm.scale[i] = (float)(1.0 / half);
    n->norm.shift[NJ + i] = 0.f;
    n->norm.scale[NJ + i] = (float)(1.0 / ctx->desc.qdmax[i]);
    n->norm.shift[FN_STATE + i] = n->norm.shift[i];
    n->norm.scale[FN_STATE + i] = n->norm.scale[i];
    n->norm.shift[FN_STATE + NJ + i] = 0.f;
    n->norm.scale[FN_STATE + NJ + i] = n->norm.scale[NJ + i];
  }
  int rc = mlp_alloc(n);
  if (rc) {
    fn_mlp_destroy(n);
    return rc;
  }
  if (hipMemset(n->dYf, 0, (size_t)n->rows * NOUT_P * 4) != hipSuccess ||
      hipMemset(n->dYb, 0, (size_t)n->rows * NOUT_P * 2) != hipSuccess) {
    fn_mlp_destroy(n);
    return fail(FN_E_HIP, "fn_mlp_create: clear");
  }
  // U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from SplitMix64
  std::vector<float> h(NP_LOG);
  uint64_t s = seed;
  int64_t o = 0;
  const int fan[8] = {NIN, NIN, W, W, W, W, W, W};
  const int cnt[8] = {W * NIN, W, W * W, W, W * W, W, NOUT * W, NOUT};
  for (int t = 0; t < 8; ++t) {
    const double a = 1.0 / std::sqrt((double)fan[t]);
    for (int i = 0; i < cnt[t]; ++i) {
      const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
      h[o++] = (float)((2.0 * u - 1.0) * a);
    }
  }
  rc = mlp_upload_logical(n, h.data());
  if (rc) {
    fn_mlp_destroy(n);
    return rc;
  }
  *out = n;
  return FN_OK;
}

// Forward pass of `rows` prepared rows (n->Xb); keeps Z for the backward.
static void mlp_forward(fn_mlp* n, int rows, bool keep_z, hipStream_t s) {
  gemm<false, true, EPI_BIAS_SILU>(s, n->Xb, NIN_P, n->wb + OFF_W1, NIN_P, rows, W, NIN_P,
                                   keep_z ? n->Z1 : nullptr, n->H1, W, n->p + OFF_B1);
  gemm<false, true, EPI_BIAS_SILU>(s, n->H1, W, n->wb + OFF_W2, W, rows, W, W,
                                   keep_z ? n->Z2 : nullptr, n->H2, W, n->p + OFF_B2);
  gemm<false, true, EPI_BIAS_SILU>(s, n->H2, W, n->wb + OFF_W3, W, rows, W, W,
                                   keep_z ? n->Z3 : nullptr, n->H3, W, n->p + OFF_B3);
  gemm<false, true, EPI_BIAS_F32>(s, n->H3, W, n->wb + OFF_W4, W, rows, NOUT_P, W, n->Y, nullptr,
                                  NOUT_P, n->p + OFF_B4);
}

// dW = dZ^T H (split over rows, summed in split order) and db = column sums of dZ
static void mlp_wgrad(fn_mlp* n, const bf16* dZb, const float* dZf, int ldz, const bf16* Hin,
                      int ldh, int nout, int nin, int rows, float* gW, float* gb, hipStream_t s) {
  const int splits = min(MAX_SPLIT, max(1, rows / 256));
  const int64_t stride = (int64_t)nout * nin;
  int kps = (rows + splits - 1) / splits;
  kps = (kps + BK - 1) / BK * BK;
  const int used = (rows + kps - 1) / kps;
  gemm<true, false, EPI_F32>(s, dZb, ldz, Hin, ldh, nout, nin, rows, n->part, nullptr, nin,
                             nullptr, nullptr, splits, stride);
  hipLaunchKernelGGL(mlp_reduce_splits, dim3((stride + 255) / 256), dim3(256), 0, s, n->part, used,
                     stride, (int)stride, gW);
  const int chunks = (rows + COLSUM_ROWS - 1) / COLSUM_ROWS;
  hipLaunchKernelGGL(mlp_colsum_part, dim3((nout + 63) / 64, chunks), dim3(64), 0, s, dZf, rows,
                     nout, ldz, n->colpart);
  hipLaunchKernelGGL(mlp_colsum_final, dim3((nout + 255) / 256), dim3(256), 0, s, n->colpart, chunks,
                     nout, gb);
}

// Backward pass of the prepared batch (n->dY*): fills n->g.
static void mlp_backward(fn_mlp* n, int rows, hipStream_t s) {
  // layer 4
  mlp_wgrad(n, n->dYb, n->dYf, NOUT_P, n->H3, W, NOUT_P, W, rows, n->g + OFF_W4, n->g + OFF_B4, s);
  gemm<false, false, EPI_DSILU>(s, n->dYb, NOUT_P, n->wb + OFF_W4, W, rows, W, NOUT_P, n->dZf0,
                                n->dZb0, W, nullptr, n->Z3);
  // layer 3
  mlp_wgrad(n, n->dZb0, n->dZf0, W, n->H2, W, W, W, rows, n->g + OFF_W3, n->g + OFF_B3, s);
  gemm<false, false, EPI_DSILU>(s, n->dZb0, W, n->wb + OFF_W3, W, rows, W, W, n->dZf1, n->dZb1, W,
                                nullptr, n->Z2);
  // layer 2
  mlp_wgrad(n, n->dZb1, n->dZf1, W, n->H1, W, W, W, rows, n->g + OFF_W2, n->g + OFF_B2, s);
  gemm<false, false, EPI_DSILU>(s, n->dZb1, W, n->wb + OFF_W2, W, rows, W, W, n->dZf0, n->dZb0, W,
                                nullptr, n->Z1);
  // layer 1
  mlp_wgrad(n, n->dZb0, n->dZf0, W, n->Xb, NIN_P, W, NIN_P, rows, n->g + OFF_W1, n->g + OFF_B1, s);
}

static void perm_params(uint64_t seed, int epoch, int64_t N, uint64_t& a, uint64_t& c) {
  // permutation i -> (a i + c) mod N with gcd(a, N) = 1
  uint64_t st = seed * 0x9E3779B97F4A7C15ull + (uint64_t)epoch * 0xD1B54A32D192ED03ull + 1;
  a = (splitmix64(st) % (uint64_t)N) | 1ull;
  c = splitmix64(st) % (uint64_t)N;
  auto gcd = [](uint64_t x, uint64_t y) {
    while (y) {
      uint64_t t = x % y;
      x = y;
      y = t;
    }
    return x;
  };
  if (N == 1) {
    a = 1;
    c = 0;
    return;
  }
  while (gcd(a % (uint64_t)N, (uint64_t)N) != 1) a += 2;
  a %= (uint64_t)N;
}

extern "C" int edge_features(fn_ctx* c, const float* tree, int64_t ld, int32_t n_nodes,
                             const float* cand, int32_t B, const int32_t* nbr, int32_t k, float* X,
                             void* stream) {
  if (!c) return fail(FN_E_ARG, "edge_features: NULL context");
  if (B < 0 || k < 1 || n_nodes < 0) return fail(FN_E_SHAPE, "edge_features: B = %d, k = %d", B, k);
  const int64_t E = (int64_t)B * k;
  if (E == 0) return FN_OK;
  if (!cand || !nbr || !X || (n_nodes > 0 && !tree)) return fail(FN_E_ARG, "edge_features: NULL array");
  if (ld < n_nodes) return fail(FN_E_ARG, "edge_features: ld < n_nodes");
  hipLaunchKernelGGL(edge_features_kernel, dim3((unsigned)((E + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, tree, ld, n_nodes, cand, nbr, k, E, X);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "edge_features launch");
}

extern "C" int surrogate_grad(fn_ctx* c, fn_mlp* n, const float* X, const int16_t* y_j, int32_t N,
                              const float* grid, int32_t n_t, float* out_grad, float* out_loss3,
                              void* stream) {
  if (!c || !n || !X || !y_j || !grid || !out_grad) return fail(FN_E_ARG, "surrogate_grad: NULL argument");
  if (N < 1 || N > n->rows || (N % 8) != 0) return fail(FN_E_SHAPE, "surrogate_grad: N = %d (1..%d, multiple of 8)", N, n->rows);
  if (n_t < 2 || n_t > FN_MAX_NT) return fail(FN_E_SHAPE, "surrogate_grad: n_t = %d", n_t);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, n->nf, 1);
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, (int32_t*)n->acc3, 3);
  hipLaunchKernelGGL(mlp_gather, dim3((N + 255) / 256), dim3(256), 0, s, X, y_j, (int64_t)N, (int64_t)0,
                     (uint64_t)1, (uint64_t)0, N, n->norm, grid, n_t, n->Xb, n->tgt, n->feas, n->nf);
  mlp_forward(n, N, true, s);
  hipLaunchKernelGGL(mlp_loss, dim3(1), dim3(1024), 0, s, n->Y, n->tgt, n->feas, n->nf, N, n->dYf,
                     n->dYb, n->acc3, 1.f);
  mlp_backward(n, N, s);
  hipLaunchKernelGGL(mlp_gather_params, dim3((NP_LOG + 255) / 256), dim3(256), 0, s, n->g, out_grad);
  if (out_loss3) (void)hipMemcpyAsync(out_loss3, n->acc3, 12, hipMemcpyDeviceToDevice, s);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "surrogate_grad launch");
}

extern "C" int surrogate_train(fn_ctx* c, fn_mlp* n, const float* X, const int16_t* y_j, int64_t N,
                               const fn_train_cfg* cfg, float* out_epoch_loss, void* stream) {
  if (!c || !n || !X || !y_j || !cfg || !cfg->grid) return fail(FN_E_ARG, "surrogate_train: NULL argument");
  const int bs = cfg->batch;
  if (bs < 8 || bs > n->rows || (bs % 8) != 0) return fail(FN_E_SHAPE, "surrogate_train: batch = %d (8..%d, multiple of 8)", bs, n->rows);
  if (N < bs) return fail(FN_E_SHAPE, "surrogate_train: N = %lld < batch", (long long)N);
  if (cfg->epochs < 1 || cfg->n_t < 2 || cfg->n_t > FN_MAX_NT) return fail(FN_E_SHAPE, "surrogate_train: epochs/n_t");
  if (!(cfg->lr > 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) || !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f))
    return fail(FN_E_ARG, "surrogate_train: lr / betas");
  hipStream_t s = (hipStream_t)stream;
  const int64_t per_epoch = N / bs;
  const int64_t total = per_epoch * cfg->epochs;
  for (int ep = 0; ep < cfg->epochs; ++ep) {
    uint64_t pa, pc;
    perm_params(cfg->seed, ep, N, pa, pc);
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, (int32_t*)n->acc3, 3);
    for (int64_t it = 0; it < per_epoch; ++it) {
      hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, n->nf, 1);
      hipLaunchKernelGGL(mlp_gather, dim3((bs + 255) / 256), dim3(256), 0, s, X, y_j, N,
                         it * bs, pa, pc, bs, n->norm, cfg->grid, cfg->n_t, n->Xb, n->tgt,
                         n->feas, n->nf);
      mlp_forward(n, bs, true, s);
      hipLaunchKernelGGL(mlp_loss, dim3(1), dim3(1024), 0, s, n->Y, n->tgt, n->feas, n->nf, bs,
                         n->dYf, n->dYb, n->acc3, 1.f / (float)per_epoch);
      mlp_backward(n, bs, s);
      n->step += 1;
      ++n->ver;
      hipLaunchKernelGGL(mlp_adam, dim3((NP_PAD + 255) / 256), dim3(256), 0, s, n->p, n->m, n->v,
                         n->g, n->wb, n->step, total, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps,
                         cfg->cosine);
    }
    if (out_epoch_loss)
      (void)hipMemcpyAsync(out_epoch_loss + 3 * ep, n->acc3, 12, hipMemcpyDeviceToDevice, s);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "surrogate_train launch");
}

// 32 rows per workgroup while that still leaves fewer than four workgroups
// per compute unit at 64 (more wavefronts to hide the weight loads), else 64
// (half the weight reads per row).
template <bool GATHER>
static void launch_infer(fn_ctx* c, fn_mlp* n, const RowSrc& src, int64_t N, const float* grid,
                         int n_t, int half, float logit_min, float* out, int16_t* win,
                         hipStream_t s) {
  if (n->wsw_ver != n->ver) {
    // weights changed since they were last packed (stream-ordered after the
    // update that changed them)
    hipLaunchKernelGGL(mlp_pack, dim3((NSW + 255) / 256), dim3(256), 0, s, n->wb, n->wsw);
    n->wsw_ver = n->ver;
  }
  const int fr = c->tune.mlp_rows > 0 ? c->tune.mlp_rows : 64;
#define FN_INFER(FRR)                                                                            \
  hipLaunchKernelGGL((mlp_infer_fused<GATHER, FRR>), dim3((unsigned)((N + FRR - 1) / FRR)),       \
                     dim3(infer_threads<FRR>()), 0, s, src, N, n->norm, n->wsw, n->p, grid, n_t, \
                     half, logit_min, out, win)
  if (fr == 32) FN_INFER(32);
  else if (fr == 128) FN_INFER(128);
  else if (fr == 256) FN_INFER(256);
  else FN_INFER(64);
#undef FN_INFER
}

extern "C" int surrogate_infer(fn_ctx* c, const fn_mlp* nc, const float* X, int64_t N,
                               const float* grid, int32_t n_t, int32_t half, float logit_min,
                               float* out, int16_t* out_win_lo, void* stream) {
  fn_mlp* n = const_cast<fn_mlp*>(nc);
  if (!c || !n) return fail(FN_E_ARG, "surrogate_infer: NULL argument");
  if (N < 0 || n_t < 2 || n_t > FN_MAX_NT || half < 0) return fail(FN_E_SHAPE, "surrogate_infer: N / n_t / half");
  if (N == 0) return FN_OK;  // nothing to read or write: the arrays may be NULL
  if (!X || !grid) return fail(FN_E_ARG, "surrogate_infer: NULL argument");
  if ((N + 31) / 32 > 0x7fffffff) return fail(FN_E_SHAPE, "surrogate_infer: N = %lld", (long long)N);
  hipStream_t s = (hipStream_t)stream;
  const RowSrc src{X, nullptr, 0, 0, nullptr, nullptr, 1};
  launch_infer<false>(c, n, src, N, grid, n_t, half, logit_min, out, out_win_lo, s);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "surrogate_infer launch");
}

extern "C" int surrogate_window(fn_ctx* c, const fn_mlp* nc, const float* tree, int64_t ld,
                                int32_t n_nodes, const float* cand, int32_t B,
                                const int32_t* nbr, int32_t k, const float* grid, int32_t n_t,
                                int32_t half, float logit_min, float* out, int16_t* out_win_lo,
                                void* stream) {
  fn_mlp* n = const_cast<fn_mlp*>(nc);
  if (!c || !n) return fail(FN_E_ARG, "surrogate_window: NULL argument");
  if (B < 0 || k < 1 || k > FN_MAX_K || n_nodes < 0 || ld < n_nodes || n_t < 2 ||
      n_t > FN_MAX_NT || half < 0)
    return fail(FN_E_SHAPE, "surrogate_window: B = %d, k = %d, n_nodes = %d, n_t = %d, half = %d",
                B, k, n_nodes, n_t, half);
  const int64_t N = (int64_t)B * k;
  if (N == 0) return FN_OK;  // nothing to read or write: the arrays may be NULL
  if (!cand || !nbr || !grid || (n_nodes > 0 && !tree))
    return fail(FN_E_ARG, "surrogate_window: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const RowSrc src{nullptr, tree, ld, n_nodes, cand, nbr, k};
  launch_infer<true>(c, n, src, N, grid, n_t, half, logit_min, out, out_win_lo, s);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "surrogate_window launch");
}

extern "C" int fn_mlp_save(const fn_mlp* n, const char* path) {
  if (!n || !path) return fail(FN_E_ARG, "fn_mlp_save: NULL argument");
  std::vector<float> buf(3 * (size_t)NP_PAD);
  hipError_t e = hipMemcpy(buf.data(), n->p, NP_PAD * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(buf.data() + NP_PAD, n->m, NP_PAD * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(buf.data() + 2 * NP_PAD, n->v, NP_PAD * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "fn_mlp_save");
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(FN_E_ARG, "fn_mlp_save: cannot open %s", path);
  const char magic[8] = {'F', 'N', 'M', 'L', 'P', '0', '0', '1'};
  const int32_t np = NP_PAD;
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&np, 4, 1, f) == 1 &&
            std::fwrite(&n->step, 8, 1, f) == 1 &&
            std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? FN_OK : fail(FN_E_ARG, "fn_mlp_save: write failed");
}

extern "C" int fn_mlp_load(fn_ctx* ctx, const char* path, fn_mlp** out) {
  if (!ctx || !path || !out) return fail(FN_E_ARG, "fn_mlp_load: NULL argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(FN_E_ARG, "fn_mlp_load: cannot open %s", path);
  char magic[8];
  int32_t np = 0;
  int64_t step = 0;
  std::vector<float> buf(3 * (size_t)NP_PAD);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "FNMLP001", 8) == 0 &&
            std::fread(&np, 4, 1, f) == 1 && np == NP_PAD && std::fread(&step, 8, 1, f) == 1 &&
            std::fread(buf.data(), 4, buf.size(), f) == buf.size();
  std::fclose(f);
  if (!ok) return fail(FN_E_ARG, "fn_mlp_load: %s is not a surrogate file of this library version", path);
  fn_mlp* n = nullptr;
  int rc = fn_mlp_create(ctx, 0, &n);
  if (rc) return rc;
  hipError_t e = hipMemcpy(n->p, buf.data(), NP_PAD * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(n->m, buf.data() + NP_PAD, NP_PAD * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(n->v, buf.data() + 2 * NP_PAD, NP_PAD * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(mlp_to_bf16, dim3((NP_PAD + 255) / 256), dim3(256), 0, 0, n->p, n->wb);
    e = hipDeviceSynchronize();
  }
  if (e != hipSuccess) {
    fn_mlp_destroy(n);
    return hip_fail(e, "fn_mlp_load");
  }
  ++n->ver;
  n->step = step;
  *out = n;
  return FN_OK;
}
