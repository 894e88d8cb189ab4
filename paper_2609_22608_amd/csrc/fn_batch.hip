// fn_batch.hip -- one round of Algorithm 1 for many planning problems at once.
//
// Every stage runs as one launch over all problems: the work item of a
// wavefront (a kNN query group and node chunk, a query to merge, an edge)
// is decoded by binary search over per-problem prefix offsets held on the
// device, so problems of very different sizes share one grid without host
// round trips.  Sizes are fixed at prepare time (node capacity, batch
// sizes); node counts are read on the device at every launch, so the whole
// round can be captured once as a HIP graph and replayed while the trees
// grow.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "fn_edge.h"
#include "fn_knn.h"
#include "fn_reach.h"
#include "fn_risk.h"

namespace fn {

struct KnnProb {
  const float* tree;
  int64_t ld;
  const int32_t* n_nodes;
  const float* qs;
  int B, n_groups, n_split, chunk;
  int64_t part_off;  // entries into the partial-list scratch
  int64_t y_off;     // entries into the per-chunk |y|^2 scratch
  int32_t* nbr;
};

struct InsProb {
  float* tree;
  int64_t ld;
  int32_t* n_nodes;
  float* t_node;
  int32_t* parent;
  float* nu;
  const float* cand;
  const int32_t* kind;
  const float* v_rel;
  const float* vz0;
  const float* t_fall;
  int B;
  const int32_t* nbr;
  const int16_t* j;
  const uint16_t* status;
  const float* rho4;
  const float* T;
  int32_t* out_node;
  float* out_J;
  float* out_best;
  float* inc;  // incumbent J*, node, t_best, rounds (Algorithm 1), or NULL
};

// index p with off[p] <= x < off[p + 1] (n problems)
__device__ __forceinline__ int bsearch_off(const int64_t* __restrict__ off, int n, int64_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Per-wavefront form: one wavefront per (problem, query group, node chunk)
// (pair offsets per problem in pair_off).
template <int K1>
__global__ __launch_bounds__(256) void batch_knn_scan(const KnnProb* __restrict__ P, int n,
                                                      const int64_t* __restrict__ pair_off,
                                                      float* __restrict__ part_d,
                                                      int32_t* __restrict__ part_i,
                                                      float* __restrict__ part_y) {
  __shared__ KnnBuf<KNN_QG> s_buf[4];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t pair = (int64_t)blockIdx.x * 4 + wave;
  if (pair >= pair_off[n]) return;
  const int p = bsearch_off(pair_off, n, pair);
  const KnnProb& q = P[p];
  const int local = (int)(pair - pair_off[p]);
  const int ch = local / q.n_groups, grp = local - ch * q.n_groups;
  knn_scan_item<K1, KNN_QG>(q.tree, q.ld, *q.n_nodes, q.qs, q.B, grp, ch, q.n_split, q.chunk,
                            part_d + q.part_off, part_i + q.part_off, part_y + q.y_off,
                            &s_buf[wave]);
}

// Tiled form: one workgroup per (problem, node chunk, 4 query groups), its
// 4 wavefronts sharing the chunk's node tiles in LDS (workgroup offsets per
// problem in blk_off).
template <int K1>
__global__ __launch_bounds__(256) void batch_knn_scan_tiled(const KnnProb* __restrict__ P, int n,
                                                      const int64_t* __restrict__ blk_off,
                                                      float* __restrict__ part_d,
                                                      int32_t* __restrict__ part_i,
                                                      float* __restrict__ part_y) {
  __shared__ KnnBuf<KNN_QG> s_buf[4];
  __shared__ float s_tile[KNN_TILE * KNN_TILE_LD];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t blk = blockIdx.x;
  if (blk >= blk_off[n]) return;
  const int p = bsearch_off(blk_off, n, blk);
  const KnnProb& q = P[p];
  const int local = (int)(blk - blk_off[p]);
  const int n_gq = (q.n_groups + 3) / 4;
  const int ch = local / n_gq, grp = (local - ch * n_gq) * 4 + wave;
  knn_scan_item<K1, KNN_QG, true>(q.tree, q.ld, *q.n_nodes, q.qs, q.B, grp, ch, q.n_split,
                                  q.chunk, part_d + q.part_off, part_i + q.part_off,
                                  part_y + q.y_off, &s_buf[wave], grp < q.n_groups, s_tile);
}

// Matrix-core form: one wavefront per (problem, 16-query group, node chunk).
template <int K1>
__global__ __launch_bounds__(256) void batch_knn_scan_mfma(const KnnProb* __restrict__ P, int n,
                                                           const int64_t* __restrict__ pair_off,
                                                           float* __restrict__ part_d,
                                                           int32_t* __restrict__ part_i,
                                                           float* __restrict__ part_y) {
  __shared__ KnnBuf<KNN_QB> s_buf[4];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t pair = (int64_t)blockIdx.x * 4 + wave;
  if (pair >= pair_off[n]) return;
  const int p = bsearch_off(pair_off, n, pair);
  const KnnProb& q = P[p];
  const int local = (int)(pair - pair_off[p]);
  const int ch = local / q.n_groups, grp = local - ch * q.n_groups;
  knn_scan_mfma_item<K1>(q.tree, q.ld, *q.n_nodes, q.qs, q.B, grp, ch, q.n_split, q.chunk,
                         part_d + q.part_off, part_i + q.part_off, part_y + q.y_off, &s_buf[wave]);
}

template <int K1>
__global__ __launch_bounds__(64) void batch_knn_merge(const KnnProb* __restrict__ P, int n,
                                                      const int64_t* __restrict__ query_off,
                                                      const float* __restrict__ part_d,
                                                      const int32_t* __restrict__ part_i,
                                                      const float* __restrict__ part_y, int k,
                                                      int32_t* __restrict__ q_count) {
  // the FP64-stage queue of the round's search starts empty (cleared here,
  // one launch before the search, instead of by a launch of its own)
  if (blockIdx.x == 0 && threadIdx.x == 0) *q_count = 0;
  const int64_t qg = blockIdx.x;
  if (qg >= query_off[n]) return;
  const int p = bsearch_off(query_off, n, qg);
  const KnnProb& q = P[p];
  if (q.n_split * K1 <= 2 * WAVE)
    knn_merge_small<K1>(q.tree, q.ld, *q.n_nodes, q.qs, (int)(qg - query_off[p]), k, q.n_split,
                        part_d + q.part_off, part_i + q.part_off, part_y + q.y_off, q.nbr, nullptr);
  else
    knn_merge_query<K1>(q.tree, q.ld, *q.n_nodes, q.qs, (int)(qg - query_off[p]), k, q.n_split,
                        part_d + q.part_off, part_i + q.part_off, part_y + q.y_off, q.nbr, nullptr);
}

// EDGE_WAVES edges per workgroup (see edge_time_kernel).
template <int PAT, int MODE>
__global__ __launch_bounds__(64 * EDGE_WAVES) __attribute__((amdgpu_waves_per_eu(4))) void
batch_edge_kernel(ProbTable pt, const float* __restrict__ grid, int n_t,
                  const ArmConst<float>* __restrict__ Ap, int max_obs) {
  __shared__ float s_end_all[EDGE_WAVES][FN_MAX_NT];
  __shared__ float s_T[FN_MAX_NT];
  __shared__ float s_fix[EDGE_WAVES][4];
  __shared__ float s_mod[EDGE_WAVES][SCREEN_FLOATS];
  __shared__ GeoLDS<float> s_geo[EDGE_WAVES];
  extern __shared__ float s_tab[];  // EDGE_WAVES * nsph * max_obs floats
  for (int t = threadIdx.x; t < n_t; t += blockDim.x) s_T[t] = grid[t];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // global candidate order: problem p's candidates follow problem p - 1's and
  // every problem has the same k, so global edge = global candidate k + i
  const int64_t eg = xcd_edge(blockIdx.x, pt.args[0].k, pt.edge_off[pt.n] / pt.args[0].k);
  if (eg < 0) return;
  if (eg >= pt.edge_off[pt.n]) return;
  const int p = problem_of(pt, eg);
  search_edge<PAT, MODE, true>(pt.args[p], eg - pt.edge_off[p], eg, *Ap, s_end_all[wave], s_T,
                               s_fix[wave], s_mod[wave], &s_geo[wave],
                               s_tab + wave * Ap->nsph * max_obs);
}

// Ordered two-phase search over every problem's edges (edge_form 3), phase
// 1: the triage of each free edge (as for one problem, into the global
// open-slot counts: each problem's tri_items points at its range); a goal
// candidate's edge is only marked open (count 1), the search checks it once
// at its fixed duration.  Four wavefronts (edges) per workgroup.
template <int PAT, int MODE>
__global__ __launch_bounds__(256) void batch_triage_kernel(ProbTable pt,
                                                           const float* __restrict__ grid, int n_t,
                                                           const ArmConst<float>* __restrict__ Ap) {
  __shared__ float s_T[FN_MAX_NT];
  __shared__ float s_mod[4][SCREEN_FLOATS];
  __shared__ float s_x[4][2 * FN_STATE];
  for (int t = threadIdx.x; t < n_t; t += blockDim.x) s_T[t] = grid[t];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t eg = (int64_t)blockIdx.x * 4 + wave;
  if (eg >= pt.edge_off[pt.n]) return;
  const int p = problem_of(pt, eg);
  const EdgeArgs& a = pt.args[p];
  const int64_t e = eg - pt.edge_off[p];
  // a goal candidate's edges (whatever their parent: the search reports an
  // invalid one) go to the search as they are
  if (a.kind && a.kind[e / a.k] == 1) {
    if (lane_id() == 0) a.tri_items[e] = 1;
    return;
  }
  triage_edge<PAT, MODE>(a, e, *Ap, s_T, s_mod[wave], s_x[wave]);
}

// Phase 2: workgroup w takes the w-th edge of the sorted order (global edge
// ids, heaviest open-slot count first); one wavefront per workgroup.
template <int PAT, int MODE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void
batch_edge_open_kernel(ProbTable pt, const float* __restrict__ grid, int n_t,
                       const ArmConst<float>* __restrict__ Ap, const int32_t* __restrict__ order,
                       const int32_t* __restrict__ n_open) {
  __shared__ float s_end[FN_MAX_NT];
  __shared__ float s_T[FN_MAX_NT];
  __shared__ float s_fix[4];
  __shared__ float s_mod[SCREEN_FLOATS];
  __shared__ GeoLDS<float> s_geo;
  extern __shared__ float s_tab[];  // nsph * max_obs floats
  if ((int64_t)blockIdx.x >= __builtin_amdgcn_readfirstlane(*n_open)) return;
  const int64_t eg = __builtin_amdgcn_readfirstlane(order[blockIdx.x]);
  for (int t = threadIdx.x; t < n_t; t += blockDim.x) s_T[t] = grid[t];
  __syncthreads();
  const int p = problem_of(pt, eg);
  search_edge<PAT, MODE, true>(pt.args[p], eg - pt.edge_off[p], eg, *Ap, s_end, s_T, s_fix, s_mod,
                               &s_geo, s_tab);
}

// Endpoint models of every problem's states: 8 lanes per state, first the
// parents of all edges (global edge order), then all candidates.
template <int PAT>
__global__ __launch_bounds__(256) void batch_model_kernel(ProbTable pt,
                                                          const int64_t* __restrict__ cand_off,
                                                          const ArmConst<float>* __restrict__ Ap) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t st = t >> 3;
  const int role = (int)(t & 7);
  const int64_t ne = pt.edge_off[pt.n];
  if (st < ne) {
    const int p = problem_of(pt, st);
    model_state<PAT>(pt.args[p], st - pt.edge_off[p], role, *Ap);
  } else if (st < ne + cand_off[pt.n]) {
    const int64_t cb = st - ne;
    const int p = bsearch_off(cand_off, pt.n, cb);
    const EdgeArgs& a = pt.args[p];
    model_state<PAT>(a, a.E + (cb - cand_off[p]), role, *Ap);
  }
}

constexpr int INS_THREADS = 256;

// Per-chunk results of the attachment kernel and the count of a problem's
// chunks that have finished (reset by the last one, so every launch starts
// from zero).
struct InsScratch {
  int32_t* cnt;   // attached candidates of the chunk
  float* bj;      // the chunk's best goal node: J, node, time-to-come
  int32_t* bn;
  float* bt;
  int32_t* done;  // per problem
};

// Attachment and scoring, one workgroup per (problem, chunk of INS_THREADS
// candidates): candidate b picks the valid parent with the smallest
// t(parent) + T (ties: lower kNN rank; a candidate with a valid edge always
// attaches); the attached candidates are appended in candidate order -- a
// chunk counts the attached candidates of the chunks before it (a candidate
// attaches exactly when one of its edges is valid, so this needs no parent
// times), then ranks its own by ballot -- and every attached goal node is
// scored.  The last chunk of a problem to finish (a counter per problem)
// reduces the chunks' best goal nodes in chunk order, moves the node count
// and updates the incumbent.
__global__ __launch_bounds__(INS_THREADS) void batch_insert_kernel(const InsProb* __restrict__ P,
                                                                   int n,
                                                                   const int64_t* __restrict__ chunk_off,
                                                                   InsScratch sc, int k, fn_risk w) {
  __shared__ int s_cnt[INS_THREADS / 64];
  __shared__ float s_bj[INS_THREADS];
  __shared__ int s_bn[INS_THREADS];
  __shared__ float s_bt[INS_THREADS];
  __shared__ int s_last;
  const int64_t blk = blockIdx.x;
  if (blk >= chunk_off[n]) return;
  const int p = bsearch_off(chunk_off, n, blk);
  const int64_t c0 = chunk_off[p];
  const int c = (int)(blk - c0), nch = (int)(chunk_off[p + 1] - c0);
  const InsProb q = P[p];  // by value: the stores below cannot alias it
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = INS_THREADS / 64;
  const uint16_t fail = FN_S_NONE | FN_S_VEL | FN_S_POS | FN_S_COLL | FN_S_BAD_INPUT | FN_S_NO_PARENT;
  const int n0 = *q.n_nodes;
  // attached candidates of the chunks before this one (four candidates per
  // thread and eight edges of each per step, loads issued together)
  const int lim = c * INS_THREADS;
  int prev = 0;
  for (int b0 = tid; b0 < lim; b0 += 4 * INS_THREADS) {
    bool any[4] = {false, false, false, false};
    for (int i0 = 0; i0 < k; i0 += 8) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int b = b0 + s4 * INS_THREADS;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (b < lim && i0 + u < k) {
            const int64_t e = (int64_t)b * k + i0 + u;
            any[s4] |= (q.j[e] >= 0) & ((q.status[e] & fail) == 0);
          }
        }
      }
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) prev += any[s4] ? 1 : 0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) prev += __shfl_xor(prev, o);
  if (lane == 0) s_cnt[wave] = prev;
  __syncthreads();
  int before = 0;
#pragma unroll
  for (int v = 0; v < NW; ++v) before += s_cnt[v];
  __syncthreads();
  // this chunk: the pick of candidate b (eight edges at a time: their loads,
  // then the parents' times, then the comparisons in rank order)
  const int b = lim + tid;
  int pick = -1;
  float cost = INFINITY;
  if (b < q.B) {
    for (int i0 = 0; i0 < k; i0 += 8) {
      bool ok[8];
      int par[8];
      float Tv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t e = (int64_t)b * k + i0 + u;
        ok[u] = i0 + u < k && q.j[e] >= 0 && !(q.status[e] & fail);
        par[u] = ok[u] ? q.nbr[e] : 0;
        Tv[u] = ok[u] ? q.T[e] : 0.f;
      }
      float tn[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) tn[u] = ok[u] ? q.t_node[par[u]] : 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float cu = tn[u] + Tv[u];
        if (ok[u] && (pick < 0 || cu < cost)) {
          cost = cu;
          pick = i0 + u;
        }
      }
    }
  }
  // rank among the chunk's attached candidates: ballot within a wavefront,
  // counts of the wavefronts before through LDS
  const uint64_t m = __ballot(pick >= 0);
  int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
  if (lane == 0) s_cnt[wave] = (int)__popcll(m);
  __syncthreads();
  int own = 0;
#pragma unroll
  for (int v = 0; v < NW; ++v) {
    rank += v < wave ? s_cnt[v] : 0;
    own += s_cnt[v];
  }
  float best_j = -INFINITY, best_t = 0.f;
  int best_n = -1;
  if (b < q.B) {
    const int64_t pos = (int64_t)n0 + before + rank;
    float J = -INFINITY;
    int node = -1;
    if (pick >= 0 && pos < q.ld) {
      node = (int)pos;
      const int64_t e = (int64_t)b * k + pick;
      const int par = q.nbr[e];
      for (int cc = 0; cc < FN_STATE; ++cc) q.tree[(size_t)cc * q.ld + pos] = q.cand[(size_t)b * FN_STATE + cc];
      q.t_node[pos] = cost;
      q.parent[pos] = par;
      const float nu = fmaxf(q.nu[par], q.rho4[4 * e + 1]);
      q.nu[pos] = nu;
      if (q.kind[b] == 1) {
        J = (float)risk_eval(w, cost, q.v_rel[b], nu, q.vz0[b], q.t_fall[b]);
        best_j = J;
        best_n = node;
        best_t = cost;
      }
    }
    q.out_node[b] = node;
    q.out_J[b] = J;
  }
  // best goal node of the chunk (fixed-order tree reduction)
  s_bj[tid] = best_j;
  s_bn[tid] = best_n;
  s_bt[tid] = best_t;
  __syncthreads();
  for (int o = INS_THREADS / 2; o > 0; o >>= 1) {
    if (tid < o) {
      const float a = s_bj[tid], cj = s_bj[tid + o];
      const int an = s_bn[tid], cn = s_bn[tid + o];
      if (cj > a || (cj == a && cn >= 0 && (an < 0 || cn < an))) {
        s_bj[tid] = cj;
        s_bn[tid] = cn;
        s_bt[tid] = s_bt[tid + o];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    sc.cnt[blk] = own;
    sc.bj[blk] = s_bj[0];
    sc.bn[blk] = s_bn[0];
    sc.bt[blk] = s_bt[0];
    __threadfence();
    s_last = atomicAdd(&sc.done[p], 1) == nch - 1;
  }
  __syncthreads();
  if (!s_last || tid != 0) return;
  // the problem's last chunk: every chunk's results are visible
  __threadfence();
  int total = 0, bn = -1;
  float bj = -INFINITY, btm = 0.f;
  for (int i = 0; i < nch; ++i) {
    const int64_t ci = c0 + i;
    total += __hip_atomic_load(&sc.cnt[ci], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const float cj = __hip_atomic_load(&sc.bj[ci], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int cn = __hip_atomic_load(&sc.bn[ci], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cj > bj || (cj == bj && cn >= 0 && (bn < 0 || cn < bn))) {
      bj = cj;
      bn = cn;
      btm = __hip_atomic_load(&sc.bt[ci], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  sc.done[p] = 0;
  *q.n_nodes = (int)min<int64_t>(q.ld, (int64_t)n0 + total);
  q.out_best[0] = bj;
  q.out_best[1] = (float)bn;
  // incumbent: the rendezvous node of largest J in the tree (earlier nodes
  // win ties) and t_best = its time-to-come
  if (q.inc) {
    if (bn >= 0 && bj > q.inc[0]) {
      q.inc[0] = bj;
      q.inc[1] = (float)bn;
      q.inc[2] = btm;
    }
    q.inc[3] += 1.f;
  }
}

// ---------------------------------------------------------------------------
// Prune (Algorithm 1, end of an anytime iteration) with the arrival-time rule
// of Eq. (8): node n stays when its earliest reach time T_n exists and is at
// most t_best; node 0 (the measured state), the incumbent and every ancestor
// of a kept node stay too.  Kept nodes are compacted in their order and
// parents renumbered.  Grid: (node blocks of 256, problems); node counts are
// read on the device.  Five launches: marks (reach time, keep rule, ancestor
// walks), block counts, new indices (each block sums the counts before it),
// gather into scratch rows, commit (which also clears the ancestor marks for
// the next Prune).
// ---------------------------------------------------------------------------
constexpr int PRUNE_THREADS = 256;
constexpr int PRUNE_COLS = FN_STATE + 3;  // state, t, nu, parent (as bits)

struct PruneProb {
  float* tree;
  int64_t ld;
  int32_t* n_nodes;
  float* t_node;
  int32_t* parent;
  float* nu;
  float* inc;
  const float* flight;
  float* out_reach;  // T_n of every node, or NULL
  int64_t off;       // node offset into keep0 / walked / map; rows at PRUNE_COLS * off
  int64_t blk_off;   // offset into the per-block counts
};

struct PruneScratch {
  int32_t* keep0;
  int32_t* walked;
  int32_t* map;
  int32_t* blk;
  int32_t* meta;  // [problem][2]: node count before, after
  float* rows;
};

// The blade point of node n: forward kinematics of its configuration.
template <typename R, int PAT>
__device__ __forceinline__ void blade_point(const ArmConst<R>& A, const float* tree, int64_t ld,
                                            int64_t n, const float* blade, R p[3]) {
  R sn[NJ], cs[NJ];
#pragma unroll
  for (int i = 0; i < NJ; ++i) sincos_r(R(tree[(size_t)i * ld + n]), sn[i], cs[i]);
  last_link_point<R, PAT>(A, sn, cs, R(blade[0]), R(blade[1]), R(blade[2]), p[0], p[1], p[2]);
}

// T_n of node n: FP32, and FP64 when the FP32 outcome is close to changing
// (reach_ambiguous, with the bound t_best or NaN).  *T64 receives the value
// that decides (the FP64 one where it was computed).
template <int PAT>
__device__ float node_reach(const ArmConst<float>& A, const ArmConst<double>& D,
                            const float* tree, int64_t ld, int64_t n, float tn,
                            const float* fl, const fn_prune& pr, float t_best, double* T64) {
  float p[3], gmin, slope;
  blade_point<float, PAT>(A, tree, ld, n, pr.blade, p);
  const float T = reach_time_dev<float>(p, tn, fl, pr.v_tip, gmin, slope);
  float scale = pr.v_tip * pr.v_tip * fl[10] * fl[10];
#pragma unroll
  for (int i = 0; i < 3; ++i) scale += (p[i] - fl[i]) * (p[i] - fl[i]);
  if (!reach_ambiguous(T, gmin, slope, t_best, scale)) {
    *T64 = T;
    return T;
  }
  double pd[3], gm, sl;
  blade_point<double, PAT>(D, tree, ld, n, pr.blade, pd);
  *T64 = reach_time_dev<double>(pd, (double)tn, fl, (double)pr.v_tip, gm, sl);
  return (float)*T64;
}

template <int PAT>
__global__ __launch_bounds__(256) void reach_kernel(const float* __restrict__ tree, int64_t ld,
                                                    int n, const float* __restrict__ t_node,
                                                    const float* __restrict__ flight, fn_prune pr,
                                                    const ArmConst<float>* __restrict__ Ap,
                                                    const ArmConst<double>* __restrict__ Dp,
                                                    float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double T64;
  out[i] = node_reach<PAT>(*Ap, *Dp, tree, ld, i, t_node[i], flight, pr, __builtin_nanf(""), &T64);
}


// keep0 of every node; a kept node then marks its ancestors: the first
// walker to claim a node (atomic exchange) goes on above it, every other one
// stops there, so each ancestor chain is walked once.
template <int PAT>
__global__ __launch_bounds__(PRUNE_THREADS) void prune_mark(const PruneProb* __restrict__ P,
                                                            PruneScratch sc, fn_prune pr,
                                                            const ArmConst<float>* __restrict__ Ap,
                                                            const ArmConst<double>* __restrict__ Dp) {
  const PruneProb q = P[blockIdx.y];
  const int64_t n = (int64_t)blockIdx.x * PRUNE_THREADS + threadIdx.x;
  const int N = *q.n_nodes;
  if (n >= N) return;
  const float tb = q.inc[2];
  double T64;
  const float T = node_reach<PAT>(*Ap, *Dp, q.tree, q.ld, n, q.t_node[n], q.flight, pr, tb, &T64);
  if (q.out_reach) q.out_reach[n] = T;
  const bool k0 = n == 0 || T64 <= (double)tb || n == (int64_t)q.inc[1];
  sc.keep0[q.off + n] = k0 ? 1 : 0;
  if (!k0) return;
  int64_t v = n;
  for (;;) {
    const int par = q.parent[v];
    if (par < 0 || par >= N) break;
    if (atomicExch(&sc.walked[q.off + par], 1)) break;
    v = par;
  }
}

__device__ __forceinline__ bool prune_kept(const PruneProb& q, const PruneScratch& sc, int64_t n,
                                           int N) {
  return n < N && (sc.keep0[q.off + n] | sc.walked[q.off + n]);
}

// Wave-ballot rank of a flag within its 256-thread block; total in *count.
__device__ __forceinline__ int block_rank(bool f, int* s_w, int* count) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long m = __ballot(f);
  if (lane == 0) s_w[w] = __popcll(m);
  __syncthreads();
  int base = 0;
  for (int i = 0; i < w; ++i) base += s_w[i];
  *count = s_w[0] + s_w[1] + s_w[2] + s_w[3];
  return base + __popcll(m & ((1ull << lane) - 1ull));
}

__global__ __launch_bounds__(PRUNE_THREADS) void prune_count(const PruneProb* __restrict__ P,
                                                             PruneScratch sc) {
  __shared__ int s_w[PRUNE_THREADS / 64];
  const PruneProb q = P[blockIdx.y];
  if ((int64_t)blockIdx.x * PRUNE_THREADS >= q.ld) return;  // whole block: uniform exit
  const int64_t n = (int64_t)blockIdx.x * PRUNE_THREADS + threadIdx.x;
  int count;
  block_rank(prune_kept(q, sc, n, *q.n_nodes), s_w, &count);
  if (threadIdx.x == 0) sc.blk[q.blk_off + blockIdx.x] = count;
}

// Sum of v over the workgroup (every thread gets it).
__device__ __forceinline__ int block_sum(int v, int* s_w) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if (lane == 0) s_w[w] = v;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int i = 0; i < PRUNE_THREADS / 64; ++i) t += s_w[i];
  return t;
}

// Kept node n -> its new index: the kept nodes of the blocks before this
// one (summed here from the block counts, a few hundred at most) plus its
// rank in the block.  Block 0 records the node count before and after.
__global__ __launch_bounds__(PRUNE_THREADS) void prune_map(const PruneProb* __restrict__ P,
                                                           PruneScratch sc) {
  __shared__ int s_w[PRUNE_THREADS / 64];
  const PruneProb q = P[blockIdx.y];
  if ((int64_t)blockIdx.x * PRUNE_THREADS >= q.ld) return;
  const int tid = threadIdx.x;
  const int nb = (int)((q.ld + PRUNE_THREADS - 1) / PRUNE_THREADS);
  const int N0 = *q.n_nodes;
  int part = 0;
  for (int i = tid; i < (int)blockIdx.x; i += PRUNE_THREADS) part += sc.blk[q.blk_off + i];
  const int before = block_sum(part, s_w);
  if (blockIdx.x == 0) {
    int tot = 0;
    for (int i = tid; i < nb; i += PRUNE_THREADS) tot += sc.blk[q.blk_off + i];
    tot = block_sum(tot, s_w);
    if (tid == 0) {
      sc.meta[2 * blockIdx.y] = N0;
      sc.meta[2 * blockIdx.y + 1] = tot;
    }
  }
  const int64_t n = (int64_t)blockIdx.x * PRUNE_THREADS + tid;
  const bool k = prune_kept(q, sc, n, N0);
  __syncthreads();
  int count;
  const int r = block_rank(k, s_w, &count);
  if (n < q.ld) sc.map[q.off + n] = k ? before + r : -1;
}

// Kept node n -> its new row in the scratch columns (parent renumbered).
__global__ __launch_bounds__(PRUNE_THREADS) void prune_gather(const PruneProb* __restrict__ P,
                                                              PruneScratch sc) {
  const PruneProb q = P[blockIdx.y];
  const int64_t n = (int64_t)blockIdx.x * PRUNE_THREADS + threadIdx.x;
  const int N = sc.meta[2 * blockIdx.y];
  if (n >= N) return;
  const int m = sc.map[q.off + n];
  if (m < 0) return;
  float* rows = sc.rows + (size_t)PRUNE_COLS * q.off;
  for (int c = 0; c < FN_STATE; ++c) rows[(size_t)c * q.ld + m] = q.tree[(size_t)c * q.ld + n];
  rows[(size_t)FN_STATE * q.ld + m] = q.t_node[n];
  rows[(size_t)(FN_STATE + 1) * q.ld + m] = q.nu[n];
  const int par = q.parent[n];
  const int np = par >= 0 && par < N ? sc.map[q.off + par] : -1;
  rows[(size_t)(FN_STATE + 2) * q.ld + m] = __int_as_float(np);
}

// Scratch rows back into the tree; parents of the freed rows cleared; node
// count and the incumbent's index updated.
__global__ __launch_bounds__(PRUNE_THREADS) void prune_commit(const PruneProb* __restrict__ P,
                                                              PruneScratch sc) {
  const PruneProb q = P[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * PRUNE_THREADS + threadIdx.x;
  const int N = sc.meta[2 * blockIdx.y], M = sc.meta[2 * blockIdx.y + 1];
  const float* rows = sc.rows + (size_t)PRUNE_COLS * q.off;
  if (i < M) {
    for (int c = 0; c < FN_STATE; ++c) q.tree[(size_t)c * q.ld + i] = rows[(size_t)c * q.ld + i];
    q.t_node[i] = rows[(size_t)FN_STATE * q.ld + i];
    q.nu[i] = rows[(size_t)(FN_STATE + 1) * q.ld + i];
    q.parent[i] = __float_as_int(rows[(size_t)(FN_STATE + 2) * q.ld + i]);
  } else if (i < N) {
    q.parent[i] = -1;
  }
  // the ancestor marks start the next Prune cleared
  if (i < q.ld) sc.walked[q.off + i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *q.n_nodes = M;
    const int in = (int)q.inc[1];
    q.inc[1] = (float)(in >= 0 && in < N ? sc.map[q.off + in] : -1);
  }
}

}  // namespace fn

using namespace fn;

// Host-side batch state (part of the context).
struct fn_batch {
  int n = 0;
  int K1 = 0, k = 0, n_t = 0, pattern = 0, mode = 0;
  const float* grid = nullptr;
  fn_risk risk{};
  int64_t pairs = 0, queries = 0, edges = 0;  // pairs: kNN scan work items
  int form = 1;                                // kNN scan form (fn_tuning)
  int edge_form = 1;  // screened search: 1 one kernel, 3 ordered two-phase (fn_tuning)
  int max_obs = 0;  // most obstacles (spheres + capsules) of a problem (clearance table LDS)
  int rounds = 1;   // candidate rounds held by every problem (tables per round)
  int64_t tab_cap = 0;  // entries of knn / ins / args
  // device tables, round r at offset r * n
  KnnProb* knn = nullptr;
  InsProb* ins = nullptr;
  EdgeArgs* args = nullptr;
  // anytime loop: every problem has an incumbent and a flight
  bool loop = false;
  PruneProb* prune = nullptr;
  PruneScratch psc{};
  int64_t prune_nodes = 0, prune_blocks = 0;  // scratch capacity
  int64_t max_blocks = 0;                     // node blocks of the largest tree
  int64_t *pair_off = nullptr, *query_off = nullptr, *edge_off = nullptr;  // pair_off: scan work items
  // attachment: chunks of INS_THREADS candidates per problem (prefix offsets)
  // and their per-chunk results; capacity ins_cap chunks
  int64_t* chunk_off = nullptr;
  int64_t chunks = 0, ins_cap = 0;
  InsScratch isc{};
  EdgeArgs a0{};  // queue pointers for the FP64 stage
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int batch_alloc(fn_ctx* c) {
  const int np = c->caps.max_problems;
  if (np <= 0) return FN_OK;
  fn_batch* b = new fn_batch();
  c->batch = b;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMalloc((void**)&b->knn, sizeof(KnnProb) * np);
  if (e == hipSuccess) e = hipMalloc((void**)&b->ins, sizeof(InsProb) * np);
  if (e == hipSuccess) e = hipMalloc((void**)&b->args, sizeof(EdgeArgs) * np);
  if (e == hipSuccess) e = hipMalloc((void**)&b->pair_off, sizeof(int64_t) * (np + 1));
  if (e == hipSuccess) e = hipMalloc((void**)&b->query_off, sizeof(int64_t) * (np + 1));
  if (e == hipSuccess) e = hipMalloc((void**)&b->edge_off, sizeof(int64_t) * (np + 1));
  if (e == hipSuccess) e = hipMalloc((void**)&b->prune, sizeof(PruneProb) * np);
  if (e == hipSuccess) e = hipMalloc((void**)&b->psc.meta, sizeof(int32_t) * 2 * np);
  // every problem's candidates in chunks of INS_THREADS: at most
  // max_batch / INS_THREADS + max_problems chunks in all
  b->ins_cap = (int64_t)c->caps.max_batch / INS_THREADS + np;
  if (e == hipSuccess) e = hipMalloc((void**)&b->chunk_off, sizeof(int64_t) * (np + 1));
  if (e == hipSuccess) e = hipMalloc((void**)&b->isc.cnt, sizeof(int32_t) * b->ins_cap);
  if (e == hipSuccess) e = hipMalloc((void**)&b->isc.bj, sizeof(float) * b->ins_cap);
  if (e == hipSuccess) e = hipMalloc((void**)&b->isc.bn, sizeof(int32_t) * b->ins_cap);
  if (e == hipSuccess) e = hipMalloc((void**)&b->isc.bt, sizeof(float) * b->ins_cap);
  if (e == hipSuccess) e = hipMalloc((void**)&b->isc.done, sizeof(int32_t) * np);
  if (e == hipSuccess) e = hipMemset(b->isc.done, 0, sizeof(int32_t) * np);
  b->tab_cap = np;
  return e == hipSuccess ? FN_OK : fail(FN_E_NOMEM, "fn_create: batch tables: %s", hipGetErrorString(e));
}

void batch_free(fn_ctx* c) {
  fn_batch* b = c->batch;
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  void* ps[] = {b->knn, b->ins, b->args, b->pair_off, b->query_off, b->edge_off, b->prune,
                b->psc.keep0, b->psc.walked, b->psc.map, b->psc.blk, b->psc.meta, b->psc.rows,
                b->chunk_off, b->isc.cnt, b->isc.bj, b->isc.bn, b->isc.bt, b->isc.done};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  delete b;
  c->batch = nullptr;
}

extern "C" int fn_batch_prepare(fn_ctx* c, const fn_problem_set* ps) {
  if (!c || !ps || (ps->n_problems > 0 && !ps->problems)) return fail(FN_E_ARG, "fn_batch_prepare: NULL argument");
  fn_batch* bt = c->batch;
  if (!bt) return fail(FN_E_STATE, "fn_batch_prepare: context created with max_problems = 0");
  const int n = ps->n_problems;
  if (n < 1 || n > c->caps.max_problems) return fail(FN_E_SHAPE, "fn_batch_prepare: %d problems (cap %d)", n, c->caps.max_problems);
  if (ps->k < 1 || ps->k > c->caps.max_k) return fail(FN_E_SHAPE, "fn_batch_prepare: k = %d", ps->k);
  if (ps->n_t < 1 || ps->n_t > FN_MAX_NT || !ps->grid) return fail(FN_E_SHAPE, "fn_batch_prepare: n_t = %d", ps->n_t);
  if (ps->samples < 2 || ps->samples > FN_MAX_SAMPLES) return fail(FN_E_SHAPE, "fn_batch_prepare: S = %d", ps->samples);
  if (ps->mode != FN_SEARCH_PLAIN && ps->mode != FN_SEARCH_SCREEN) return fail(FN_E_ARG, "fn_batch_prepare: mode must be PLAIN or SCREEN");
  if (!(ps->margin >= 0.f)) return fail(FN_E_ARG, "fn_batch_prepare: margin");
  const int K1 = knn_k1(ps->k);
  const int64_t cap_part = (int64_t)knn_scratch_entries(c->caps.max_batch, c->caps.max_k, c->caps.max_problems);
  const int64_t cap_y = (int64_t)knn_scratch_entries(c->caps.max_batch, 0, c->caps.max_problems);
  std::vector<KnnProb> kp(n);
  std::vector<InsProb> ip(n);
  std::vector<EdgeArgs> ea(n);
  std::vector<int64_t> po(n + 1), qo(n + 1), eo(n + 1);
  int64_t part = 0, ys = 0, sumB = 0;
  int max_obs = 0;
  po[0] = qo[0] = eo[0] = 0;
  int Sw = 1;
  while (Sw < ps->samples) Sw <<= 1;
  int target = std::min(KNN_TARGET_MAX, c->tune.knn_target_waves > 0 ? c->tune.knn_target_waves : 4096);
  const int minchunk = c->tune.knn_min_chunk > 0 ? c->tune.knn_min_chunk : 512;
  // scan form: tuned, else the matrix-core form once the largest tree
  // capacity outgrows the L2
  int64_t max_ld = 0;
  for (int p = 0; p < n; ++p) max_ld = std::max(max_ld, ps->problems[p].ld);
  // candidate rounds and the anytime-loop state: the same for every problem
  const int rounds = std::max(1, ps->problems[0].n_rounds);
  const bool loop = ps->problems[0].incumbent != nullptr;
  for (int p = 0; p < n; ++p) {
    const fn_problem& q = ps->problems[p];
    if (std::max(1, q.n_rounds) != rounds || q.n_rounds < 0 || rounds > FN_MAX_ROUNDS)
      return fail(FN_E_SHAPE, "fn_batch_prepare: problem %d: %d rounds (problem 0: %d, at most %d)",
                  p, q.n_rounds, rounds, FN_MAX_ROUNDS);
    if ((q.incumbent != nullptr) != loop || (loop && !q.flight))
      return fail(FN_E_ARG, "fn_batch_prepare: problem %d: incumbent and flight must be given for every problem or for none", p);
  }
  const int form = c->tune.knn_form > 0 ? c->tune.knn_form : (max_ld > FN_KNN_LARGE_TREE ? 3 : 1);
  const int qpw = form == 3 ? KNN_QB : KNN_QG;  // queries per scan wavefront
  if (form == 3) target = std::min(target, KNN_TARGET_MAX * KNN_QG / KNN_QB);
  for (int p = 0; p < n; ++p) {
    const fn_problem& q = ps->problems[p];
    if (!q.tree || !q.n_nodes || !q.t_node || !q.parent || !q.nu || !q.cand || !q.kind || !q.t_req ||
        !q.v_rel || !q.vz0 || !q.t_fall || !q.nbr || !q.out_j || !q.out_status || !q.out_margin ||
        !q.out_rho4 || !q.out_T || !q.out_node || !q.out_J || !q.out_best)
      return fail(FN_E_ARG, "fn_batch_prepare: problem %d has a NULL array", p);
    if (q.B < 1 || q.ld < 4 || (q.ld & 3) != 0 || q.ld > KNN_MAX_LD)
      return fail(FN_E_SHAPE, "fn_batch_prepare: problem %d: B = %d, ld = %lld", p, q.B, (long long)q.ld);
    if (q.n_obs < 0 || q.n_obs > FN_MAX_OBS || (q.n_obs > 0 && !q.obs) || q.n_caps < 0 ||
        q.n_caps > FN_MAX_CAPS || q.n_obs + q.n_caps > FN_MAX_OBS || (q.n_caps > 0 && !q.caps))
      return fail(FN_E_SHAPE, "fn_batch_prepare: problem %d: %d obstacle spheres, %d capsules", p,
                  q.n_obs, q.n_caps);
    // kNN geometry from the node capacity (node counts change on the device)
    const int groups = (q.B + qpw - 1) / qpw;
    int split = (int)((target / n + groups - 1) / groups);
    split = std::max(1, std::min(split, std::min(KNN_MAX_SPLIT, (int)(q.ld / minchunk))));
    int chunk = (int)((q.ld + split - 1) / split);
    chunk = std::max(WAVE, (chunk + WAVE - 1) / WAVE * WAVE);
    split = std::max(1, (int)((q.ld + chunk - 1) / chunk));
    kp[p] = KnnProb{q.tree, q.ld, q.n_nodes, q.cand, q.B, groups, split, chunk, part, ys, q.nbr};
    part += (int64_t)q.B * split * K1;
    ys += (int64_t)q.B * split;
    // scan work items: wavefronts (per-wavefront and matrix-core forms) or
    // workgroups (tiled)
    po[p + 1] = po[p] + (form == 2 ? (int64_t)(groups + 3) / 4 : (int64_t)groups) * split;
    qo[p + 1] = qo[p] + q.B;
    eo[p + 1] = eo[p] + (int64_t)q.B * ps->k;
    sumB += q.B;
    EdgeArgs& a = ea[p];
    std::memset(&a, 0, sizeof(a));
    a.tree = q.tree; a.ld = q.ld; a.n_nodes = 0; a.n_nodes_dev = q.n_nodes;
    a.cand = q.cand; a.nbr = q.nbr; a.k = ps->k; a.E = (int64_t)q.B * ps->k;
    a.grid = ps->grid; a.n_t = ps->n_t; a.S = ps->samples; a.Sw = Sw; a.mode = ps->mode;
    a.win_half = 0; a.j_max = nullptr; a.win_lo = nullptr;
    a.obs = q.obs; a.n_obs = q.n_obs; a.margin_c = ps->margin;
    a.caps = q.caps; a.n_caps = q.n_caps;
    max_obs = max_obs > q.n_obs + q.n_caps ? max_obs : q.n_obs + q.n_caps;
    a.out_j = q.out_j; a.out_st = q.out_status; a.out_m = q.out_margin; a.out_rho = q.out_rho4;
    a.out_work = nullptr; a.out_scr = nullptr; a.q_count = c->q_count; a.queue = c->queue;
    a.model_e = c->model_e + eo[p] * MODEL_FLOATS;
    a.model_c = c->model_c + qo[p] * MODEL_FLOATS;
    a.tri_items = c->tri_items + eo[p];  // the problem's edges in the global range
    a.kind = q.kind; a.t_req = q.t_req; a.t_node = q.t_node; a.out_T = q.out_T;
    a.t_best = loop ? q.incumbent + 2 : nullptr;
    ip[p] = InsProb{q.tree, q.ld, q.n_nodes, q.t_node, q.parent, q.nu, q.cand, q.kind, q.v_rel,
                    q.vz0, q.t_fall, q.B, q.nbr, q.out_j, q.out_status, q.out_rho4, q.out_T,
                    q.out_node, q.out_J, q.out_best, q.incumbent};
  }
  if (eo[n] > c->caps.max_edges) return fail(FN_E_SHAPE, "fn_batch_prepare: %lld edges (cap %lld)", (long long)eo[n], (long long)c->caps.max_edges);
  std::vector<int64_t> co(n + 1);
  co[0] = 0;
  for (int p = 0; p < n; ++p)
    co[p + 1] = co[p] + (ps->problems[p].B + INS_THREADS - 1) / INS_THREADS;
  if (co[n] > bt->ins_cap)
    return fail(FN_E_SHAPE, "fn_batch_prepare: %lld candidate chunks (cap %lld)", (long long)co[n], (long long)bt->ins_cap);
  if (sumB > c->caps.max_batch || part > cap_part || ys > cap_y)
    return fail(FN_E_SHAPE, "fn_batch_prepare: %lld candidates in total (cap %d)", (long long)sumB, c->caps.max_batch);
  // round r's tables: the same problems with candidate arrays advanced by r
  // rounds of B
  std::vector<KnnProb> kr(kp.begin(), kp.end());
  std::vector<InsProb> ir(ip.begin(), ip.end());
  std::vector<EdgeArgs> er(ea.begin(), ea.end());
  kr.resize((size_t)n * rounds);
  ir.resize((size_t)n * rounds);
  er.resize((size_t)n * rounds);
  for (int r = 1; r < rounds; ++r)
    for (int p = 0; p < n; ++p) {
      const int64_t B = ps->problems[p].B, o = (int64_t)r * B;
      KnnProb& kq = kr[(size_t)r * n + p];
      InsProb& iq = ir[(size_t)r * n + p];
      EdgeArgs& eq = er[(size_t)r * n + p];
      kq = kp[p];
      iq = ip[p];
      eq = ea[p];
      kq.qs += o * FN_STATE;
      iq.cand += o * FN_STATE; iq.kind += o; iq.v_rel += o; iq.vz0 += o; iq.t_fall += o;
      eq.cand += o * FN_STATE; eq.kind += o; eq.t_req += o;
    }
  hipError_t e = hipSuccess;
  if ((int64_t)n * rounds > bt->tab_cap) {
    // larger tables: a captured graph refers to the old ones
    if (bt->exec) { (void)hipGraphExecDestroy(bt->exec); bt->exec = nullptr; }
    if (bt->graph) { (void)hipGraphDestroy(bt->graph); bt->graph = nullptr; }
    (void)hipFree(bt->knn); (void)hipFree(bt->ins); (void)hipFree(bt->args);
    bt->knn = nullptr; bt->ins = nullptr; bt->args = nullptr; bt->tab_cap = 0;
    const size_t m = (size_t)n * rounds;
    e = hipMalloc((void**)&bt->knn, sizeof(KnnProb) * m);
    if (e == hipSuccess) e = hipMalloc((void**)&bt->ins, sizeof(InsProb) * m);
    if (e == hipSuccess) e = hipMalloc((void**)&bt->args, sizeof(EdgeArgs) * m);
    if (e != hipSuccess) return fail(FN_E_NOMEM, "fn_batch_prepare: round tables: %s", hipGetErrorString(e));
    bt->tab_cap = (int64_t)m;
  }
  // prune tables and scratch (anytime loop only)
  std::vector<PruneProb> pp(n);
  int64_t nodes = 0, blocks = 0;
  for (int p = 0; p < n; ++p) {
    const fn_problem& q = ps->problems[p];
    pp[p] = PruneProb{q.tree, q.ld, q.n_nodes, q.t_node, q.parent, q.nu, q.incumbent, q.flight,
                      q.out_reach, nodes, blocks};
    nodes += q.ld;
    blocks += (q.ld + PRUNE_THREADS - 1) / PRUNE_THREADS;
  }
  if (loop && (nodes > bt->prune_nodes || blocks > bt->prune_blocks)) {
    if (bt->exec) { (void)hipGraphExecDestroy(bt->exec); bt->exec = nullptr; }
    if (bt->graph) { (void)hipGraphDestroy(bt->graph); bt->graph = nullptr; }
    PruneScratch& sc = bt->psc;
    void* old[] = {sc.keep0, sc.walked, sc.map, sc.blk, sc.rows};
    for (void* o : old) (void)hipFree(o);
    sc.keep0 = sc.walked = sc.map = sc.blk = nullptr;
    sc.rows = nullptr;
    bt->prune_nodes = bt->prune_blocks = 0;
    e = hipMalloc((void**)&sc.keep0, sizeof(int32_t) * nodes);
    if (e == hipSuccess) e = hipMalloc((void**)&sc.walked, sizeof(int32_t) * nodes);
    if (e == hipSuccess) e = hipMalloc((void**)&sc.map, sizeof(int32_t) * nodes);
    if (e == hipSuccess) e = hipMalloc((void**)&sc.blk, sizeof(int32_t) * blocks);
    if (e == hipSuccess) e = hipMalloc((void**)&sc.rows, sizeof(float) * PRUNE_COLS * nodes);
    if (e != hipSuccess) return fail(FN_E_NOMEM, "fn_batch_prepare: prune scratch: %s", hipGetErrorString(e));
    bt->prune_nodes = nodes;
    bt->prune_blocks = blocks;
  }
  e = hipMemcpy(bt->knn, kr.data(), sizeof(KnnProb) * kr.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(bt->ins, ir.data(), sizeof(InsProb) * ir.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(bt->args, er.data(), sizeof(EdgeArgs) * er.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(bt->prune, pp.data(), sizeof(PruneProb) * n, hipMemcpyHostToDevice);
  // Prune's ancestor marks start cleared; every Prune's commit clears them again
  if (e == hipSuccess && loop) e = hipMemset(bt->psc.walked, 0, sizeof(int32_t) * nodes);
  if (e == hipSuccess) e = hipMemcpy(bt->pair_off, po.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(bt->query_off, qo.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(bt->edge_off, eo.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(bt->chunk_off, co.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "fn_batch_prepare: upload");
  bt->chunks = co[n];
  // a graph captured before holds the previous launch geometry
  if (bt->exec) { (void)hipGraphExecDestroy(bt->exec); bt->exec = nullptr; }
  if (bt->graph) { (void)hipGraphDestroy(bt->graph); bt->graph = nullptr; }
  bt->n = n;
  bt->K1 = K1;
  bt->k = ps->k;
  bt->n_t = ps->n_t;
  bt->grid = ps->grid;
  bt->risk = ps->risk;
  bt->pattern = c->pattern;
  bt->mode = ps->mode;
  bt->pairs = po[n];
  bt->form = form;
  // the ordered two-phase search only when asked for: a small round pays
  // three more launches for it
  bt->edge_form = c->tune.edge_form == 3 && eo[n] <= INT32_MAX ? 3 : 1;
  bt->queries = qo[n];
  bt->edges = eo[n];
  bt->max_obs = max_obs;
  bt->a0 = ea[0];
  bt->rounds = rounds;
  bt->loop = loop;
  bt->max_blocks = (max_ld + PRUNE_THREADS - 1) / PRUNE_THREADS;
  return FN_OK;
}

template <int K1>
static void launch_batch_knn(fn_ctx* c, fn_batch* bt, const KnnProb* tab, hipStream_t s) {
  if (bt->form == 2)
    hipLaunchKernelGGL(batch_knn_scan_tiled<K1>, dim3((unsigned)bt->pairs), dim3(256), 0, s,
                       tab, bt->n, bt->pair_off, c->knn_d, c->knn_i, c->knn_y);
  else if (bt->form == 3)
    hipLaunchKernelGGL(batch_knn_scan_mfma<K1>, dim3((unsigned)((bt->pairs + 3) / 4)), dim3(256), 0,
                       s, tab, bt->n, bt->pair_off, c->knn_d, c->knn_i, c->knn_y);
  else
    hipLaunchKernelGGL(batch_knn_scan<K1>, dim3((unsigned)((bt->pairs + 3) / 4)), dim3(256), 0, s,
                       tab, bt->n, bt->pair_off, c->knn_d, c->knn_i, c->knn_y);
  hipLaunchKernelGGL(batch_knn_merge<K1>, dim3((unsigned)bt->queries), dim3(64), 0, s, tab,
                     bt->n, bt->query_off, c->knn_d, c->knn_i, c->knn_y, bt->k, c->q_count);
}

// model kernel (screening), search, FP64 stage over all problems
template <int PAT, int MODE>
static void launch_batch_search(fn_ctx* c, fn_batch* bt, const EdgeArgs* et, hipStream_t s) {
  const ProbTable pt{bt->n, bt->edge_off, et};
  if (MODE != FN_SEARCH_PLAIN)
    hipLaunchKernelGGL(batch_model_kernel<PAT>, dim3((unsigned)(((bt->edges + bt->queries) * 8 + 255) / 256)),
                       dim3(256), 0, s, pt, bt->query_off, c->arm32);
  if (MODE != FN_SEARCH_PLAIN && bt->edge_form == 3) {
    // triage, counting sort of the open edges (heaviest first), search in
    // that order; the sort's scratch is laid out as for one problem
    const int64_t E = bt->edges;
    int32_t* order = c->tri_items + c->caps.max_edges;
    int32_t* hist = c->tri_items + 2 * c->caps.max_edges;
    int32_t* n_open = hist + TRI_MAX_BLOCKS * TRI_BINS;
    const int64_t chunk = std::max(TRI_MIN_CHUNK, (E + TRI_MAX_BLOCKS - 1) / TRI_MAX_BLOCKS);
    const int nblk = (int)((E + chunk - 1) / chunk);
    hipLaunchKernelGGL((batch_triage_kernel<PAT, MODE>), dim3((unsigned)((E + 3) / 4)), dim3(256), 0,
                       s, pt, bt->grid, bt->n_t, c->arm32);
    hipLaunchKernelGGL(tri_hist_kernel, dim3(nblk), dim3(256), 0, s, c->tri_items, E, chunk,
                       bt->n_t, hist);
    hipLaunchKernelGGL(tri_scatter_kernel, dim3(nblk), dim3(256), 0, s, c->tri_items, E, chunk,
                       bt->n_t, hist, nblk, order, n_open);
    hipLaunchKernelGGL((batch_edge_open_kernel<PAT, MODE>), dim3((unsigned)E), dim3(64),
                       (size_t)c->desc.n_spheres * bt->max_obs * sizeof(float), s, pt, bt->grid,
                       bt->n_t, c->arm32, order, n_open);
  } else {
    const size_t tab = (size_t)EDGE_WAVES * c->desc.n_spheres * bt->max_obs * sizeof(float);
    hipLaunchKernelGGL((batch_edge_kernel<PAT, MODE>), dim3((unsigned)xcd_grid(bt->queries, bt->k)),
                       dim3(64 * EDGE_WAVES), tab, s, pt, bt->grid, bt->n_t, c->arm32, bt->max_obs);
  }
  const unsigned rw = (unsigned)(bt->edges < RECHECK_WAVES ? bt->edges : RECHECK_WAVES);
  hipLaunchKernelGGL(edge_recheck_kernel<PAT>, dim3(rw), dim3(64),
                     (size_t)c->desc.n_spheres * bt->max_obs * sizeof(double), s, bt->a0, pt,
                     c->arm64);
}

// One round (Algorithm 1's inner loop body) on candidate round r.
static int launch_round(fn_ctx* c, fn_batch* bt, int r, hipStream_t s) {
  const KnnProb* kt = bt->knn + (size_t)r * bt->n;
  const EdgeArgs* et = bt->args + (size_t)r * bt->n;
  const InsProb* it = bt->ins + (size_t)r * bt->n;
  switch (bt->K1) {
#define FN_K(KK) case KK: launch_batch_knn<KK>(c, bt, kt, s); break;
    FN_K(5) FN_K(6) FN_K(7) FN_K(8) FN_K(9) FN_K(10) FN_K(11) FN_K(12) FN_K(13) FN_K(14) FN_K(15)
    FN_K(16) FN_K(20) FN_K(24) FN_K(33)
#undef FN_K
    default: return fail(FN_E_SHAPE, "fn_batch_round: k");
  }
  // (the kNN merge has cleared the FP64-stage queue)
  if (bt->pattern == PAT_FR3) {
    if (bt->mode == FN_SEARCH_PLAIN) launch_batch_search<PAT_FR3, FN_SEARCH_PLAIN>(c, bt, et, s);
    else launch_batch_search<PAT_FR3, FN_SEARCH_SCREEN>(c, bt, et, s);
  } else {
    if (bt->mode == FN_SEARCH_PLAIN) launch_batch_search<PAT_GENERIC, FN_SEARCH_PLAIN>(c, bt, et, s);
    else launch_batch_search<PAT_GENERIC, FN_SEARCH_SCREEN>(c, bt, et, s);
  }
  hipLaunchKernelGGL(batch_insert_kernel, dim3((unsigned)bt->chunks), dim3(INS_THREADS), 0, s, it,
                     bt->n, bt->chunk_off, bt->isc, bt->k, bt->risk);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "fn_batch_round");
}

static bool prune_args_ok(const fn_prune* pr) {
  return pr && std::isfinite(pr->v_tip) && pr->v_tip > 0.f && std::isfinite(pr->blade[0]) &&
         std::isfinite(pr->blade[1]) && std::isfinite(pr->blade[2]);
}

static int launch_prune(fn_ctx* c, fn_batch* bt, const fn_prune& pr, hipStream_t s) {
  const dim3 g((unsigned)bt->max_blocks, (unsigned)bt->n);
  // (the ancestor marks were cleared by the last Prune's commit, or at prepare)
  if (c->pattern == PAT_FR3)
    hipLaunchKernelGGL(prune_mark<PAT_FR3>, g, dim3(PRUNE_THREADS), 0, s, bt->prune, bt->psc, pr, c->arm32, c->arm64);
  else
    hipLaunchKernelGGL(prune_mark<PAT_GENERIC>, g, dim3(PRUNE_THREADS), 0, s, bt->prune, bt->psc, pr, c->arm32, c->arm64);
  hipLaunchKernelGGL(prune_count, g, dim3(PRUNE_THREADS), 0, s, bt->prune, bt->psc);
  hipLaunchKernelGGL(prune_map, g, dim3(PRUNE_THREADS), 0, s, bt->prune, bt->psc);
  hipLaunchKernelGGL(prune_gather, g, dim3(PRUNE_THREADS), 0, s, bt->prune, bt->psc);
  hipLaunchKernelGGL(prune_commit, g, dim3(PRUNE_THREADS), 0, s, bt->prune, bt->psc);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "fn_batch_prune");
}

// n_iter anytime iterations of n_round rounds, Prune after each iteration.
static int launch_cycle(fn_ctx* c, fn_batch* bt, int n_iter, int n_round, const fn_prune& pr,
                        hipStream_t s) {
  for (int a = 0; a < n_iter; ++a) {
    for (int r = 0; r < n_round; ++r) {
      const int rc = launch_round(c, bt, a * n_round + r, s);
      if (rc != FN_OK) return rc;
    }
    const int rc = launch_prune(c, bt, pr, s);
    if (rc != FN_OK) return rc;
  }
  return FN_OK;
}

static int cycle_args(fn_ctx* c, const char* who, int n_iter, int n_round, const fn_prune* pr) {
  fn_batch* bt = c->batch;
  if (!bt || bt->n == 0) return fail(FN_E_STATE, "%s: no prepared problem set", who);
  if (!bt->loop) return fail(FN_E_STATE, "%s: the problems have no incumbent and flight", who);
  if (!prune_args_ok(pr)) return fail(FN_E_ARG, "%s: V_tip must be finite and positive, the blade point finite", who);
  if (n_iter < 1 || n_round < 1 || (int64_t)n_iter * n_round > bt->rounds)
    return fail(FN_E_SHAPE, "%s: %d x %d rounds, %d prepared", who, n_iter, n_round, bt->rounds);
  return FN_OK;
}

extern "C" int fn_batch_round(fn_ctx* c, int32_t round, void* stream) {
  if (!c) return fail(FN_E_ARG, "fn_batch_round: NULL context");
  fn_batch* bt = c->batch;
  if (!bt || bt->n == 0) return fail(FN_E_STATE, "fn_batch_round: no prepared problem set");
  if (round < 0 || round >= bt->rounds)
    return fail(FN_E_SHAPE, "fn_batch_round: round %d of %d", round, bt->rounds);
  return launch_round(c, bt, round, (hipStream_t)stream);
}

extern "C" int fn_batch_launch(fn_ctx* c, void* stream) { return fn_batch_round(c, 0, stream); }

extern "C" int fn_batch_prune(fn_ctx* c, const fn_prune* pr, void* stream) {
  if (!c) return fail(FN_E_ARG, "fn_batch_prune: NULL context");
  const int rc = cycle_args(c, "fn_batch_prune", 1, 1, pr);
  if (rc != FN_OK) return rc;
  return launch_prune(c, c->batch, *pr, (hipStream_t)stream);
}

extern "C" int fn_cycle(fn_ctx* c, int32_t n_iter, int32_t n_round, const fn_prune* pr,
                        void* stream) {
  if (!c) return fail(FN_E_ARG, "fn_cycle: NULL context");
  const int rc = cycle_args(c, "fn_cycle", n_iter, n_round, pr);
  if (rc != FN_OK) return rc;
  return launch_cycle(c, c->batch, n_iter, n_round, *pr, (hipStream_t)stream);
}

extern "C" int fn_reach_time(fn_ctx* c, const float* tree, int64_t ld, int32_t n,
                             const float* t_node, const float* flight, const fn_prune* pr,
                             float* out_T, void* stream) {
  if (!c || !tree || !t_node || !flight || !out_T) return fail(FN_E_ARG, "fn_reach_time: NULL argument");
  if (!prune_args_ok(pr)) return fail(FN_E_ARG, "fn_reach_time: V_tip must be finite and positive, the blade point finite");
  if (n < 0 || ld < n || ld < 1) return fail(FN_E_SHAPE, "fn_reach_time: n = %d, ld = %lld", n, (long long)ld);
  if (n == 0) return FN_OK;
  hipStream_t s = (hipStream_t)stream;
  const unsigned g = (unsigned)((n + 255) / 256);
  if (c->pattern == PAT_FR3)
    hipLaunchKernelGGL(reach_kernel<PAT_FR3>, dim3(g), dim3(256), 0, s, tree, ld, n, t_node, flight, *pr, c->arm32, c->arm64, out_T);
  else
    hipLaunchKernelGGL(reach_kernel<PAT_GENERIC>, dim3(g), dim3(256), 0, s, tree, ld, n, t_node, flight, *pr, c->arm32, c->arm64, out_T);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "fn_reach_time");
}

// Captures what `body` enqueues on `stream` into the context's HIP graph
// (replacing a previous one).
template <typename F>
static int capture_into(fn_ctx* c, void* stream, const char* who, F&& body) {
  fn_batch* bt = c->batch;
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(FN_E_ARG, "%s: capture needs a non-default stream", who);
  if (bt->exec) {
    (void)hipGraphExecDestroy(bt->exec);
    bt->exec = nullptr;
  }
  if (bt->graph) {
    (void)hipGraphDestroy(bt->graph);
    bt->graph = nullptr;
  }
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, who);
  const int rc = body(s);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  if (rc != FN_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, who);
  e = hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, who);
  }
  bt->graph = g;
  return FN_OK;
}

extern "C" int fn_graph_capture(fn_ctx* c, void* stream) {
  if (!c || !c->batch || c->batch->n == 0) return fail(FN_E_STATE, "fn_graph_capture: no prepared problem set");
  return capture_into(c, stream, "fn_graph_capture",
                      [&](hipStream_t s) { return launch_round(c, c->batch, 0, s); });
}

extern "C" int fn_graph_capture_cycle(fn_ctx* c, int32_t n_iter, int32_t n_round,
                                      const fn_prune* pr, void* stream) {
  if (!c) return fail(FN_E_ARG, "fn_graph_capture_cycle: NULL context");
  const int rc = cycle_args(c, "fn_graph_capture_cycle", n_iter, n_round, pr);
  if (rc != FN_OK) return rc;
  const fn_prune p = *pr;
  return capture_into(c, stream, "fn_graph_capture_cycle", [&](hipStream_t s) {
    return launch_cycle(c, c->batch, n_iter, n_round, p, s);
  });
}

extern "C" int fn_graph_launch(fn_ctx* c, void* stream) {
  if (!c || !c->batch || !c->batch->exec) return fail(FN_E_STATE, "fn_graph_launch: nothing captured");
  hipError_t e = hipGraphLaunch(c->batch->exec, (hipStream_t)stream);
  return e == hipSuccess ? FN_OK : hip_fail(e, "fn_graph_launch");
}

extern "C" int fn_set_tuning(fn_ctx* c, const fn_tuning* t) {
  if (!c || !t) return fail(FN_E_ARG, "fn_set_tuning: NULL argument");
  if (t->knn_target_waves < 0 || t->knn_target_waves > KNN_TARGET_MAX || t->knn_min_chunk < 0 ||
      (t->knn_min_chunk & 63) != 0 || t->knn_form < 0 || t->knn_form > 3 || t->edge_form < 0 ||
      t->edge_form > 3 || (t->mlp_rows != 0 && t->mlp_rows != 32 && t->mlp_rows != 64 &&
                              t->mlp_rows != 128 && t->mlp_rows != 256))
    return fail(FN_E_ARG, "fn_set_tuning: target waves in [0, %d], min chunk >= 0 and a multiple of 64, kNN form 0..3, edge form 0..2, MLP rows 0, 32, 64, 128 or 256", KNN_TARGET_MAX);
  c->tune = *t;
  return FN_OK;
}
