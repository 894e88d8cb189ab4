// fn_knn.hip -- Parents(T, x, M) of Algorithm 1: brute-force k nearest tree
// nodes by Euclidean distance in the 14-D state space (Sec. IV-E).
//
// Stage 1 (knn_scan): one wavefront per (64 queries, node chunk).  Each lane
// holds one query in VGPRs; the chunk's nodes are wave-uniform and arrive
// through the scalar cache as float4 rows of the SoA tree, so every
// distance costs 14 subtractions and 14 FMAs with SGPR operands.  Each lane
// keeps its chunk's k+1 smallest FP32 keys (d^2, index).
// Stage 2 (knn_merge): one wavefront per query merges the chunk lists.  The
// FP32 k-th key bounds a band that provably holds the exact top-k; every
// candidate in the band is re-ranked with the FP64 distance summed in the
// reference order (c = 0..13, separately rounded products and sums).  When
// a chunk's (k+1)-th entry also falls in the band (near ties that the FP32
// lists may have cut), the query is rescanned exactly in FP64.
#include <hip/hip_runtime.h>

#include "fn_ctx.h"

namespace fn {

constexpr int KNN_TARGET_WAVES = 4096;
constexpr float KNN_BAND = 1e-5f;  // >> FP32 relative error of a 14-term sum of squares

__device__ __forceinline__ bool key_less(float d, int i, float d2, int i2) {
  return d < d2 || (d == d2 && (unsigned)i < (unsigned)i2);
}

template <int K1>
__global__ __launch_bounds__(256) void knn_scan(const float* __restrict__ tree, int64_t ld,
                                                int n_nodes, const float* __restrict__ qs, int B,
                                                int n_qtiles, int n_split, int chunk,
                                                float* __restrict__ out_d,
                                                int32_t* __restrict__ out_i) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int pair = blockIdx.x * 4 + wave;
  if (pair >= n_qtiles * n_split) return;
  const int qt = pair / n_split, ch = pair - qt * n_split;
  const int lane = threadIdx.x & 63;
  const int b = qt * 64 + lane;
  const int bq = b < B ? b : B - 1;
  float x[FN_STATE];
#pragma unroll
  for (int c = 0; c < FN_STATE; ++c) x[c] = qs[(size_t)bq * FN_STATE + c];
  float ld_d[K1];
  int ld_i[K1];
#pragma unroll
  for (int r = 0; r < K1; ++r) {
    ld_d[r] = INFINITY;
    ld_i[r] = -1;
  }
  const int n_pad = (n_nodes + 3) & ~3;
  const int n0 = ch * chunk;
  const int n1 = min(n0 + chunk, n_pad);
  for (int n = n0; n < n1; n += 4) {
    float d[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < FN_STATE; ++c) {
      const float4 y = *reinterpret_cast<const float4*>(tree + (size_t)c * ld + n);
      float t;
      t = x[c] - y.x; d[0] = fmaf(t, t, d[0]);
      t = x[c] - y.y; d[1] = fmaf(t, t, d[1]);
      t = x[c] - y.z; d[2] = fmaf(t, t, d[2]);
      t = x[c] - y.w; d[3] = fmaf(t, t, d[3]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = n + u;
      const float dd = d[u];
      if (idx < n_nodes && key_less(dd, idx, ld_d[K1 - 1], ld_i[K1 - 1])) {
        // insert into the sorted list (entries shift up from the back)
#pragma unroll
        for (int r = K1 - 1; r >= 1; --r) {
          const bool shift = key_less(dd, idx, ld_d[r - 1], ld_i[r - 1]);
          const bool here = key_less(dd, idx, ld_d[r], ld_i[r]);
          ld_d[r] = shift ? ld_d[r - 1] : (here ? dd : ld_d[r]);
          ld_i[r] = shift ? ld_i[r - 1] : (here ? idx : ld_i[r]);
        }
        if (key_less(dd, idx, ld_d[0], ld_i[0])) {
          ld_d[0] = dd;
          ld_i[0] = idx;
        }
      }
    }
  }
  if (b < B) {
    const size_t base = ((size_t)b * n_split + ch) * K1;
#pragma unroll
    for (int r = 0; r < K1; ++r) {
      out_d[base + r] = ld_d[r];
      out_i[base + r] = ld_i[r];
    }
  }
}

// FP64 squared distance, summed in the reference order with separately
// rounded operations.
__device__ __forceinline__ double exact_d2(const float* __restrict__ tree, int64_t ld, int node,
                                           const double* x) {
  double d = 0.0;
#pragma unroll
  for (int c = 0; c < FN_STATE; ++c) {
    const double t = __dsub_rn(x[c], (double)tree[(size_t)c * ld + node]);
    d = __dadd_rn(d, __dmul_rn(t, t));
  }
  return d;
}

__device__ __forceinline__ unsigned long long dkey(double d) {
  return (unsigned long long)__double_as_longlong(d);
}

// wave-wide argmin over (d64, idx) keys held one per lane; returns the
// winning lane's (d, idx) in every lane.
__device__ __forceinline__ void wave_argmin(double d, int idx, double& wd, int& wi) {
  unsigned long long k = dkey(d);
  unsigned long long m = k;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long v = __shfl_xor(m, o);
    m = v < m ? v : m;
  }
  unsigned mi = (k == m) ? (unsigned)idx : 0xffffffffu;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned v = __shfl_xor(mi, o);
    mi = v < mi ? v : mi;
  }
  wd = __longlong_as_double((long long)m);
  wi = (int)mi;
}

template <int K1>
__global__ __launch_bounds__(64) void knn_merge(const float* __restrict__ tree, int64_t ld,
                                                int n_nodes, const float* __restrict__ qs,
                                                int k, int n_split,
                                                const float* __restrict__ in_d,
                                                const int32_t* __restrict__ in_i,
                                                int32_t* __restrict__ out_idx,
                                                float* __restrict__ out_d2) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  double x[FN_STATE];
#pragma unroll
  for (int c = 0; c < FN_STATE; ++c) x[c] = (double)qs[(size_t)b * FN_STATE + c];
  const int total = n_split * K1;
  const float* D = in_d + (size_t)b * total;
  const int32_t* I = in_i + (size_t)b * total;

  // (a) FP32 k-th smallest key among every chunk's first k entries
  float th_d = -1.f;
  int th_i = -1;
  for (int r = 0; r < k; ++r) {
    float bd = INFINITY;
    int bi = -1;
    for (int e = lane; e < total; e += 64) {
      if (e % K1 >= k) continue;
      const float d = D[e];
      const int i = I[e];
      if (i < 0) continue;
      const bool after = th_i < 0 ? true : key_less(th_d, th_i, d, i);
      if (after && key_less(d, i, bd, bi)) {
        bd = d;
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const float od = __shfl_xor(bd, o);
      const int oi = __shfl_xor(bi, o);
      if (key_less(od, oi, bd, bi)) {
        bd = od;
        bi = oi;
      }
    }
    if (bi < 0) break;  // fewer than k nodes in total
    th_d = bd;
    th_i = bi;
  }
  const float band = th_d < 0.f ? INFINITY : th_d * (1.0f + KNN_BAND) + 1e-30f;

  // (b) a chunk whose (k+1)-th entry is inside the band may have cut near ties
  int over = 0;
  for (int e = lane; e < total; e += 64)
    if (e % K1 == k && I[e] >= 0 && D[e] <= band) over = 1;
  over = __any(over);

  if (!over) {
    // (c) FP64 re-rank of the band (computed once into LDS), then k rounds
    // of wave argmin over (d64, index)
    __shared__ double s_d[KNN_MAX_SPLIT * (FN_MAX_K + 1)];
    for (int e = lane; e < total; e += 64) {
      const int i = I[e];
      const bool in = (e % K1 < k) && i >= 0 && D[e] <= band;
      s_d[e] = in ? exact_d2(tree, ld, i, x) : INFINITY;
    }
    __syncthreads();
    double prev_d = -1.0;
    int prev_i = -1;
    for (int r = 0; r < k; ++r) {
      double bd = INFINITY;
      int bi = 0x7fffffff;
      for (int e = lane; e < total; e += 64) {
        const double d = s_d[e];
        if (!(d < INFINITY)) continue;
        const int i = I[e];
        const bool after = prev_i < 0 || d > prev_d || (d == prev_d && i > prev_i);
        if (after && (d < bd || (d == bd && i < bi))) {
          bd = d;
          bi = i;
        }
      }
      double wd;
      int wi;
      wave_argmin(bd, bi, wd, wi);
      if (wi == 0x7fffffff) {
        wd = INFINITY;
        wi = -1;
      } else {
        prev_d = wd;
        prev_i = wi;
      }
      if (lane == 0) {
        out_idx[(size_t)b * k + r] = wi;
        if (out_d2) out_d2[(size_t)b * k + r] = (float)wd;
      }
    }
  } else {
    // (d) exact FP64 rescan of the whole tree for this query: each lane keeps
    // a sorted list of its k best, then k rounds of wave argmin over heads
    double ld_d[FN_MAX_K];
    int ld_i[FN_MAX_K];
    for (int r = 0; r < k; ++r) {
      ld_d[r] = INFINITY;
      ld_i[r] = 0x7fffffff;
    }
    for (int n = lane; n < n_nodes; n += 64) {
      const double d = exact_d2(tree, ld, n, x);
      if (d < ld_d[k - 1]) {  // a lane's nodes come in increasing index
        int r = k - 1;
        while (r > 0 && d < ld_d[r - 1]) {
          ld_d[r] = ld_d[r - 1];
          ld_i[r] = ld_i[r - 1];
          --r;
        }
        ld_d[r] = d;
        ld_i[r] = n;
      }
    }
    int head = 0;
    for (int r = 0; r < k; ++r) {
      const double hd = head < k ? ld_d[head] : INFINITY;
      const int hi = head < k ? ld_i[head] : 0x7fffffff;
      double wd;
      int wi;
      wave_argmin(hd, hi, wd, wi);
      if (wi != 0x7fffffff && wi == hi) ++head;
      if (wi == 0x7fffffff) {
        wd = INFINITY;
        wi = -1;
      }
      if (lane == 0) {
        out_idx[(size_t)b * k + r] = wi;
        if (out_d2) out_d2[(size_t)b * k + r] = (float)wd;
      }
    }
  }
}

template <int K1>
static void launch_knn(fn_ctx* c, const float* tree, int64_t ld, int n_nodes, const float* qs,
                       int B, int k, int32_t* out_idx, float* out_d2, hipStream_t s) {
  const int n_qtiles = (B + 63) / 64;
  const int n_pad = (n_nodes + 3) & ~3;
  int n_split = (KNN_TARGET_WAVES + n_qtiles - 1) / n_qtiles;
  n_split = min(n_split, KNN_MAX_SPLIT);
  n_split = max(1, min(n_split, (n_pad + 63) / 64));
  int chunk = (n_pad + n_split - 1) / n_split;
  chunk = max(4, (chunk + 3) & ~3);  // an empty tree still gets one (empty) chunk
  n_split = max(1, (n_pad + chunk - 1) / chunk);
  const int pairs = n_qtiles * n_split;
  hipLaunchKernelGGL(knn_scan<K1>, dim3((pairs + 3) / 4), dim3(256), 0, s, tree, ld, n_nodes, qs,
                     B, n_qtiles, n_split, chunk, c->knn_d, c->knn_i);
  hipLaunchKernelGGL(knn_merge<K1>, dim3(B), dim3(64), 0, s, tree, ld, n_nodes, qs, k, n_split,
                     c->knn_d, c->knn_i, out_idx, out_d2);
}

size_t knn_scratch_entries(int max_batch, int max_k) {
  const size_t qt = (size_t)(max_batch + 63) / 64;
  return (size_t)64 * (KNN_TARGET_WAVES + qt) * knn_k1(max_k);
}

}  // namespace fn

using namespace fn;

extern "C" int plan_knn(fn_ctx* c, const float* tree, int64_t ld, int32_t n_nodes,
                        const float* queries, int32_t B, int32_t k, int32_t* out_idx,
                        float* out_d2, void* stream) {
  if (!c) return fail(FN_E_ARG, "plan_knn: NULL context");
  if (B < 0 || B > c->caps.max_batch) return fail(FN_E_SHAPE, "plan_knn: B = %d (cap %d)", B, c->caps.max_batch);
  if (k < 1 || k > c->caps.max_k) return fail(FN_E_SHAPE, "plan_knn: k = %d (cap %d)", k, c->caps.max_k);
  if (n_nodes < 0 || n_nodes > c->caps.max_nodes)
    return fail(FN_E_SHAPE, "plan_knn: n_nodes = %d (cap %d)", n_nodes, c->caps.max_nodes);
  if (B == 0) return FN_OK;
  if (!queries || !out_idx || (n_nodes > 0 && !tree)) return fail(FN_E_ARG, "plan_knn: NULL array");
  const int n_pad = (n_nodes + 3) & ~3;
  if ((ld & 3) != 0 || ld < n_pad) return fail(FN_E_ARG, "plan_knn: ld = %lld (need a multiple of 4 >= %d)", (long long)ld, n_pad);
  if (((uintptr_t)tree & 15) != 0) return fail(FN_E_ARG, "plan_knn: tree not 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  switch (k + 1) {
#define FN_K(KK) case KK: launch_knn<KK>(c, tree, ld, n_nodes, queries, B, k, out_idx, out_d2, s); break;
    FN_K(2) FN_K(3) FN_K(4) FN_K(5) FN_K(6) FN_K(7) FN_K(8) FN_K(9) FN_K(10) FN_K(11) FN_K(12)
    FN_K(13) FN_K(14) FN_K(15) FN_K(16) FN_K(17)
#undef FN_K
    default:
      if (k + 1 <= 33) launch_knn<33>(c, tree, ld, n_nodes, queries, B, k, out_idx, out_d2, s);
      else return fail(FN_E_SHAPE, "plan_knn: k = %d", k);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "plan_knn launch");
}
