// fn_knn.hip -- single-problem kNN kernels and the plan_knn entry point
// (device functions in fn_knn.h).
#include <hip/hip_runtime.h>

#include "fn_knn.h"

namespace fn {

template <int K1, int QG>
__global__ __launch_bounds__(256) void knn_scan(const float* __restrict__ tree, int64_t ld,
                                                int n_nodes, const float* __restrict__ qs, int B,
                                                int n_groups, int n_split, int chunk,
                                                float* __restrict__ out_d,
                                                int32_t* __restrict__ out_i,
                                                float* __restrict__ out_y2) {
  __shared__ KnnBuf<QG> s_buf[4];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int pair = blockIdx.x * 4 + wave;
  if (pair >= n_groups * n_split) return;
  // the wavefronts of a block share a node chunk (L1 reuse), each with its
  // own query group
  const int ch = pair / n_groups, grp = pair - ch * n_groups;
  knn_scan_item<K1, QG>(tree, ld, n_nodes, qs, B, grp, ch, n_split, chunk, out_d, out_i, out_y2,
                        &s_buf[wave]);
}

// Tiled form: workgroup = (chunk, 4 query groups); the 4 wavefronts share
// each 256-node tile of the chunk through LDS (one global load per node
// instead of four, |y|^2 once per node).
template <int K1, int QG>
__global__ __launch_bounds__(256) void knn_scan_tiled(const float* __restrict__ tree, int64_t ld,
                                                      int n_nodes, const float* __restrict__ qs,
                                                      int B, int n_groups, int n_split, int chunk,
                                                      float* __restrict__ out_d,
                                                      int32_t* __restrict__ out_i,
                                                      float* __restrict__ out_y2) {
  __shared__ KnnBuf<QG> s_buf[4];
  __shared__ float s_tile[KNN_TILE * KNN_TILE_LD];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n_gq = (n_groups + 3) / 4;
  const int ch = blockIdx.x / n_gq, gq = blockIdx.x - ch * n_gq;
  const int grp = gq * 4 + wave;
  knn_scan_item<K1, QG, true>(tree, ld, n_nodes, qs, B, grp, ch, n_split, chunk, out_d, out_i,
                              out_y2, &s_buf[wave], grp < n_groups, s_tile);
}

// Matrix-core form: one wavefront per (16 queries, node chunk), keys by
// v_mfma_f32_16x16x4_f32; the wavefronts of a block share a node chunk.
template <int K1>
__global__ __launch_bounds__(256) void knn_scan_mfma(const float* __restrict__ tree, int64_t ld,
                                                     int n_nodes, const float* __restrict__ qs,
                                                     int B, int n_groups, int n_split, int chunk,
                                                     float* __restrict__ out_d,
                                                     int32_t* __restrict__ out_i,
                                                     float* __restrict__ out_y2) {
  __shared__ KnnBuf<KNN_QB> s_buf[4];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int pair = blockIdx.x * 4 + wave;
  if (pair >= n_groups * n_split) return;
  const int ch = pair / n_groups, grp = pair - ch * n_groups;
  knn_scan_mfma_item<K1>(tree, ld, n_nodes, qs, B, grp, ch, n_split, chunk, out_d, out_i, out_y2,
                         &s_buf[wave]);
}

template <int K1>
__global__ __launch_bounds__(64) void knn_merge(const float* __restrict__ tree, int64_t ld,
                                                int n_nodes, const float* __restrict__ qs,
                                                int k, int n_split,
                                                const float* __restrict__ in_d,
                                                const int32_t* __restrict__ in_i,
                                                const float* __restrict__ in_y2,
                                                int32_t* __restrict__ out_idx,
                                                float* __restrict__ out_d2) {
  knn_merge_query<K1>(tree, ld, n_nodes, qs, blockIdx.x, k, n_split, in_d, in_i, in_y2, out_idx,
                      out_d2);
}

// chunk lists of at most 128 entries per query: sort-based merge, no LDS
template <int K1>
__global__ __launch_bounds__(64) void knn_merge_small_kernel(
    const float* __restrict__ tree, int64_t ld, int n_nodes, const float* __restrict__ qs, int k,
    int n_split, const float* __restrict__ in_d, const int32_t* __restrict__ in_i,
    const float* __restrict__ in_y2, int32_t* __restrict__ out_idx, float* __restrict__ out_d2) {
  knn_merge_small<K1>(tree, ld, n_nodes, qs, blockIdx.x, k, n_split, in_d, in_i, in_y2, out_idx,
                      out_d2);
}

template <int K1>
static void launch_knn(fn_ctx* c, const float* tree, int64_t ld, int n_nodes, const float* qs,
                       int B, int k, int32_t* out_idx, float* out_d2, hipStream_t s) {
  const int form = c->tune.knn_form > 0 ? c->tune.knn_form : (n_nodes > FN_KNN_LARGE_TREE ? 3 : 1);
  const int qpw = form == 3 ? KNN_QB : KNN_QG;  // queries per scan wavefront
  const int n_groups = (B + qpw - 1) / qpw;
  // enough wavefronts to fill the chip, chunks of at least 512 nodes; the
  // matrix-core form (4x the queries per wavefront) takes a quarter of the
  // wavefront target at most, so its chunk lists fit the same scratch
  int target = min(KNN_TARGET_MAX, c->tune.knn_target_waves > 0 ? c->tune.knn_target_waves : KNN_TARGET_WAVES);
  if (form == 3) target = min(target, KNN_TARGET_MAX * KNN_QG / KNN_QB);
  const int minchunk = c->tune.knn_min_chunk > 0 ? c->tune.knn_min_chunk : 512;
  int n_split = (target + n_groups - 1) / n_groups;
  n_split = min(n_split, KNN_MAX_SPLIT);
  n_split = max(1, min(n_split, n_nodes / minchunk));
  int chunk = (n_nodes + n_split - 1) / n_split;
  chunk = max(WAVE, (chunk + WAVE - 1) / WAVE * WAVE);
  n_split = max(1, (n_nodes + chunk - 1) / chunk);
  if (form == 2) {
    const int n_gq = (n_groups + 3) / 4;
    hipLaunchKernelGGL((knn_scan_tiled<K1, KNN_QG>), dim3(n_gq * n_split), dim3(256), 0, s, tree,
                       ld, n_nodes, qs, B, n_groups, n_split, chunk, c->knn_d, c->knn_i, c->knn_y);
  } else if (form == 3) {
    const int pairs = n_groups * n_split;
    hipLaunchKernelGGL((knn_scan_mfma<K1>), dim3((pairs + 3) / 4), dim3(256), 0, s, tree, ld,
                       n_nodes, qs, B, n_groups, n_split, chunk, c->knn_d, c->knn_i, c->knn_y);
  } else {
    const int pairs = n_groups * n_split;
    hipLaunchKernelGGL((knn_scan<K1, KNN_QG>), dim3((pairs + 3) / 4), dim3(256), 0, s, tree, ld,
                       n_nodes, qs, B, n_groups, n_split, chunk, c->knn_d, c->knn_i, c->knn_y);
  }
  if (n_split * K1 <= 2 * WAVE)
    hipLaunchKernelGGL(knn_merge_small_kernel<K1>, dim3(B), dim3(64), 0, s, tree, ld, n_nodes, qs,
                       k, n_split, c->knn_d, c->knn_i, c->knn_y, out_idx, out_d2);
  else
    hipLaunchKernelGGL(knn_merge<K1>, dim3(B), dim3(64), 0, s, tree, ld, n_nodes, qs, k, n_split,
                       c->knn_d, c->knn_i, c->knn_y, out_idx, out_d2);
}

size_t knn_scratch_entries(int max_batch, int max_k, int max_problems) {
  // one problem: B * n_split <= QG * n_groups * ceil(TARGET / n_groups)
  // <= QG * (TARGET + n_groups); P problems of a batch, each with a share of
  // the target and its own rounding: <= QG * (TARGET + sum n_groups) and
  // sum n_groups <= n_groups(sum B) + P.  The matrix-core form (16 queries
  // per wavefront, a quarter of the target): 16 * (TARGET / 4 + n_groups16
  // + P).
  const size_t np = max_problems > 0 ? (size_t)max_problems : 0;
  const size_t g4 = (size_t)(max_batch + KNN_QG - 1) / KNN_QG;
  const size_t g16 = (size_t)(max_batch + KNN_QB - 1) / KNN_QB;
  const size_t e4 = (size_t)KNN_QG * (KNN_TARGET_MAX + g4 + np);
  const size_t e16 = (size_t)KNN_QB * (KNN_TARGET_MAX * KNN_QG / KNN_QB + g16 + np);
  return (e4 > e16 ? e4 : e16) * (max_k > 0 ? knn_k1(max_k) : 1);
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
  if (ld > KNN_MAX_LD) return fail(FN_E_SHAPE, "plan_knn: ld = %lld (max %lld)", (long long)ld, (long long)KNN_MAX_LD);
  if (((uintptr_t)tree & 15) != 0) return fail(FN_E_ARG, "plan_knn: tree not 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  switch (knn_k1(k)) {
#define FN_K(KK) case KK: launch_knn<KK>(c, tree, ld, n_nodes, queries, B, k, out_idx, out_d2, s); break;
    FN_K(5) FN_K(6) FN_K(7) FN_K(8) FN_K(9) FN_K(10) FN_K(11) FN_K(12) FN_K(13) FN_K(14) FN_K(15)
    FN_K(16) FN_K(20) FN_K(24) FN_K(33)
#undef FN_K
    default: return fail(FN_E_SHAPE, "plan_knn: k = %d", k);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "plan_knn launch");
}
