// fn_edge.hip -- single-problem kernels and C entry points of the edge search
// (edge_time_batch) and of the fixed-duration check (edge_check).
//
// One wavefront per edge.  The 64 lanes are mapped over (slot, sample)
// pairs: a pass evaluates G = 64 / Sw slots at once (Sw = S rounded up to a
// power of two), every lane one point of Eq. (4) along the cubic of Eq. (6).
// A slot's ratio is the max over its lane group (xor shuffles); slots are
// decided in ascending order, so the first feasible slot of the grid is the
// result whatever order the work is done in.  See fn_edge.h.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fn_edge.h"

namespace fn {

// Endpoint models of every screened state: 8 lanes per state (the E
// parents, then the B candidates).
template <int PAT>
__global__ __launch_bounds__(256) void edge_model_kernel(EdgeArgs a,
                                                         const ArmConst<float>* __restrict__ Ap) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t == 0) *a.q_count = 0;  // the FP64-stage queue of the search that follows
  const int64_t st = t >> 3;
  if (st >= a.E + a.E / a.k) return;
  model_state<PAT>(a, st, (int)(t & 7), *Ap);
}

// EDGE_WAVES wavefronts (edges) per workgroup.  Edges take very different
// times (some stop after the screen, some run several full passes and the
// post-checks); a one-wave workgroup hands its slot to the next edge as
// soon as it ends instead of holding it until the slowest of its group
// ends.  Four waves per SIMD: measured faster than three (no spills, 154
// VGPRs) despite a few spilled registers, and than five.
template <int PAT, int MODE>
__global__ __launch_bounds__(64 * EDGE_WAVES) __attribute__((amdgpu_waves_per_eu(4))) void
edge_time_kernel(EdgeArgs a, const ArmConst<float>* __restrict__ Ap) {
  __shared__ float s_end_all[EDGE_WAVES][FN_MAX_NT];
  __shared__ float s_T[FN_MAX_NT];
  __shared__ float s_fix[EDGE_WAVES][4];
  __shared__ float s_mod[EDGE_WAVES][SCREEN_FLOATS];
  __shared__ GeoLDS<float> s_geo[EDGE_WAVES];
  extern __shared__ float s_tab[];  // EDGE_WAVES * nsph * (n_obs + n_caps) floats
  for (int t = threadIdx.x; t < a.n_t; t += blockDim.x) s_T[t] = a.grid[t];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t e = xcd_edge(blockIdx.x, a.k, a.E / a.k);
  if (e < 0) return;
  search_edge<PAT, MODE, false>(a, e, e, *Ap, s_end_all[wave], s_T, s_fix[wave], s_mod[wave],
                                &s_geo[wave], s_tab + wave * Ap->nsph * (a.n_obs + a.n_caps));
}

// Two-phase screened search, phase 1: the triage, one wavefront per edge,
// four per workgroup (light: no full evaluation, no post-checks).
template <int PAT, int MODE>
__global__ __launch_bounds__(256) void edge_triage_kernel(EdgeArgs a,
                                                          const ArmConst<float>* __restrict__ Ap) {
  __shared__ float s_T[FN_MAX_NT];
  __shared__ float s_mod[4][SCREEN_FLOATS];
  __shared__ float s_x[4][2 * FN_STATE];
  for (int t = threadIdx.x; t < a.n_t; t += blockDim.x) s_T[t] = a.grid[t];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t e = (int64_t)blockIdx.x * 4 + wave;
  if (e >= a.E) return;
  triage_edge<PAT, MODE>(a, e, *Ap, s_T, s_mod[wave], s_x[wave]);
}

// Ordered two-phase search (form 3), between the triage and the search: a
// counting sort of the open edges, heaviest bin first.  Bin of an open-slot
// count (1..n_t): TRI_BINS equal ranges.
__device__ __forceinline__ int tri_bin(int open, int n_t) {
  return min((open - 1) * TRI_BINS / n_t, TRI_BINS - 1);
}

// Bin counts of the open edges of each block's chunk of edges (an LDS
// histogram; no global atomics).
__global__ __launch_bounds__(256) void tri_hist_kernel(const int32_t* __restrict__ items,
                                                       int64_t E, int64_t chunk, int n_t,
                                                       int32_t* __restrict__ hist) {
  __shared__ int h[TRI_BINS];
  if (threadIdx.x < TRI_BINS) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(E, lo + chunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const int v = items[i];
    if (v > 0) atomicAdd(&h[tri_bin(v, n_t)], 1);
  }
  __syncthreads();
  if (threadIdx.x < TRI_BINS) hist[(size_t)blockIdx.x * TRI_BINS + threadIdx.x] = h[threadIdx.x];
}

// Places of each block's open edges: an edge of bin b goes after every edge
// of the heavier bins and of bin b in the earlier blocks (each block sums
// the bin counts itself; within a block and bin the places are taken by LDS
// atomics in no fixed order, which changes no result).  Block 0 writes the
// number of open edges to *n_open.
__global__ __launch_bounds__(256) void tri_scatter_kernel(const int32_t* __restrict__ items,
                                                          int64_t E, int64_t chunk, int n_t,
                                                          const int32_t* __restrict__ hist,
                                                          int nblk, int32_t* __restrict__ order,
                                                          int32_t* __restrict__ n_open) {
  static_assert(TRI_BINS == 64, "one bin per lane of the first wavefront");
  __shared__ int s_tot[4][TRI_BINS], s_bef[4][TRI_BINS];
  __shared__ int s_cur[TRI_BINS];
  const int t = threadIdx.x, bin = t & (TRI_BINS - 1), part = t >> 6;
  int tot = 0, bef = 0;
  for (int j = part; j < nblk; j += 4) {
    const int v = hist[(size_t)j * TRI_BINS + bin];
    tot += v;
    if (j < (int)blockIdx.x) bef += v;
  }
  s_tot[part][bin] = tot;
  s_bef[part][bin] = bef;
  __syncthreads();
  if (t < TRI_BINS) {
    // lane = bin: the count of bins bin..63 by a suffix scan over the lanes
    const int n = s_tot[0][bin] + s_tot[1][bin] + s_tot[2][bin] + s_tot[3][bin];
    int x = n;
#pragma unroll
    for (int off = 1; off < TRI_BINS; off <<= 1) {
      const int y = __shfl_down(x, off);
      if (bin + off < TRI_BINS) x += y;
    }
    s_cur[bin] = x - n + s_bef[0][bin] + s_bef[1][bin] + s_bef[2][bin] + s_bef[3][bin];
    if (blockIdx.x == 0 && t == 0) *n_open = x;  // lane 0: every bin
  }
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(E, lo + chunk);
  for (int64_t i = lo + t; i < hi; i += blockDim.x) {
    const int v = items[i];
    if (v > 0) order[atomicAdd(&s_cur[tri_bin(v, n_t)], 1)] = (int32_t)i;
  }
}

// Two-phase screened search, phase 2: the search of the edges the triage
// left open; ORDERED: workgroup w takes the w-th edge of the sorted order
// (form 3), else the one-kernel grid's order, where wavefronts of finished
// edges end at once (form 2).
template <int PAT, int MODE, bool ORDERED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void
edge_search_open_kernel(EdgeArgs a, const ArmConst<float>* __restrict__ Ap) {
  __shared__ float s_end[FN_MAX_NT];
  __shared__ float s_T[FN_MAX_NT];
  __shared__ float s_fix[4];
  __shared__ float s_mod[SCREEN_FLOATS];
  __shared__ GeoLDS<float> s_geo;
  extern __shared__ float s_tab[];  // nsph * (n_obs + n_caps) floats
  int64_t e;
  if constexpr (ORDERED) {
    const int n_open = __builtin_amdgcn_readfirstlane(a.tri_hist[TRI_MAX_BLOCKS * TRI_BINS]);
    if ((int64_t)blockIdx.x >= n_open) return;
    e = __builtin_amdgcn_readfirstlane(a.tri_order[blockIdx.x]);
  } else {
    e = xcd_edge(blockIdx.x, a.k, a.E / a.k);
    if (e < 0 || __builtin_amdgcn_readfirstlane(a.tri_items[e]) < 0) return;
  }
  for (int t = threadIdx.x; t < a.n_t; t += blockDim.x) s_T[t] = a.grid[t];
  __syncthreads();
  search_edge<PAT, MODE, false>(a, e, e, *Ap, s_end, s_T, s_fix, s_mod, &s_geo, s_tab);
}

// ---------------------------------------------------------------------------
// Fixed-duration check (goal branch of Algorithm 1; recheck of a sent plan)
// ---------------------------------------------------------------------------
template <int PAT>
__global__ __launch_bounds__(256) void edge_check_kernel(const float* __restrict__ x0,
                                                         const float* __restrict__ x1,
                                                         const float* __restrict__ Tv, int64_t E,
                                                         int S, World w,
                                                         const ArmConst<float>* __restrict__ Ap,
                                                         uint16_t* out_st, float* out_rho,
                                                         float* out_tau) {
  __shared__ GeoLDS<float> s_geo[4];
  extern __shared__ float s_tab[];  // 4 * nsph * (n_obs + n_caps) floats
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t e = (int64_t)blockIdx.x * 4 + wave;
  if (e >= E) return;
  const ArmConst<float>& A = *Ap;
  const int lane = lane_id();
  EdgeState<float> ES;
  bool finite = true;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    const float q0 = x0[e * FN_STATE + i], v0 = x0[e * FN_STATE + NJ + i];
    const float q1 = x1[e * FN_STATE + i], v1 = x1[e * FN_STATE + NJ + i];
    finite = finite && isfinite(q0) && isfinite(v0) && isfinite(q1) && isfinite(v1);
    ES.q0[i] = q0;
    ES.qd0[i] = v0;
    ES.dq[i] = q1 - q0;
    ES.d2[i] = v1 - v0;
  }
  const float T = Tv[e];
  int st = 0;
  if (!finite || !isfinite(T)) st = FN_S_BAD_INPUT;
  else if (!(T > 0.f)) st = FN_S_NONE;
  if (st) {
    if (lane == 0) {
      out_st[e] = (uint16_t)st;
      for (int r = 0; r < 5; ++r) out_rho[5 * e + r] = 0.f;
    }
    if (out_tau)
      for (int t = lane; t < S * NJ; t += WAVE) out_tau[(size_t)e * S * NJ + t] = 0.f;
    return;
  }
  const float invT = 1.f / T;
  float rt_all = 0.f, rp_all = 0.f;
  for (int s0 = 0; s0 < S; s0 += WAVE) {
    const int s = s0 + lane;
    if (s < S) {
      float tau[NJ], rt, rp;
      eval_point<float, PAT>(A, ES, T, invT, float(s) / float(S - 1), rt, rp, tau);
      rt_all = fmaxf(rt_all, rt);
      rp_all = fmaxf(rp_all, rp);
      if (out_tau)
#pragma unroll
        for (int i = 0; i < NJ; ++i) out_tau[((size_t)e * S + s) * NJ + i] = tau[i];
    }
  }
  const float rt = wave_max(rt_all), rp = wave_max(rp_all);
  float rv, rq, rc;
  // clearance only when every limit check passes (Alg. 1)
  post_checks<float, PAT>(A, ES, T, S, w, &s_geo[wave], s_tab + wave * A.nsph * world_size(w),
                          rt <= 1.f && rp <= 1.f ? 1.f : -1.f, rv, rq, rc);
  if (lane == 0) {
    int s2 = post_status(rv, rq, rc);
    if (rt > 1.f || rp > 1.f) s2 |= FN_S_NONE;
    out_st[e] = (uint16_t)s2;
    out_rho[5 * e + 0] = rt;
    out_rho[5 * e + 1] = rp;
    out_rho[5 * e + 2] = rv;
    out_rho[5 * e + 3] = rq;
    out_rho[5 * e + 4] = rc;
  }
}

// ---------------------------------------------------------------------------
// Self-collision pairs of the fixed-duration check (the full-resolution
// recheck, Sec. IV-E), for edges whose limit checks passed: one wavefront
// per edge, lane = sample (chunks of 64), every sphere centre of the lane's
// pose in LDS ([3][nsph][64], conflict-free per lane), then the pairs'
// smallest d^2 / (r_a + r_b + margin)^2.  Merges into the check's clearance
// ratio (the larger of the two) and status (COLL | SELF when above 1).
// ---------------------------------------------------------------------------
template <int PAT>
__global__ __launch_bounds__(64) void edge_self_kernel(
    const float* __restrict__ x0, const float* __restrict__ x1, const float* __restrict__ Tv,
    int64_t E, int S, const int16_t* __restrict__ pairs, int n_pairs, float margin_self,
    const ArmConst<float>* __restrict__ Ap, uint16_t* __restrict__ out_st,
    float* __restrict__ out_rho) {
  extern __shared__ float s_self[];  // local centres [4][nsph], centres [3][nsph][64], 1/need^2
  const int64_t e = blockIdx.x;
  if (e >= E) return;
  const uint16_t st = out_st[e];
  if (st & (FN_S_NONE | FN_S_VEL | FN_S_POS | FN_S_BAD_INPUT)) return;  // not evaluated
  const ArmConst<float>& A = *Ap;
  const int lane = lane_id(), ns = A.nsph;
  float* loc = s_self;
  float* cx = loc + 4 * ns;
  float* cy = cx + ns * WAVE;
  float* cz = cy + ns * WAVE;
  float* inv = cz + ns * WAVE;
  for (int t = lane; t < ns; t += WAVE) {
    loc[4 * t] = A.sphx[t];
    loc[4 * t + 1] = A.sphy[t];
    loc[4 * t + 2] = A.sphz[t];
    loc[4 * t + 3] = A.sphr[t];
  }
  for (int p = lane; p < n_pairs; p += WAVE) {
    const float need = A.sphr[pairs[2 * p]] + A.sphr[pairs[2 * p + 1]] + margin_self;
    inv[p] = __builtin_amdgcn_rcpf(need * need);
  }
  EdgeState<float> ES;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    ES.q0[i] = x0[e * FN_STATE + i];
    ES.qd0[i] = x0[e * FN_STATE + NJ + i];
    ES.dq[i] = x1[e * FN_STATE + i] - ES.q0[i];
    ES.d2[i] = x1[e * FN_STATE + NJ + i] - ES.qd0[i];
  }
  const float T = Tv[e];
  __builtin_amdgcn_wave_barrier();
  float best = INFINITY;
  for (int s0 = 0; s0 < S; s0 += WAVE) {
    const int s = s0 + lane;
    const bool act = s < S;
    if (act) {
      float sg[NJ], sd[NJ], sdd[NJ], sn[NJ], cs[NJ];
      cubic_point(ES, T, 1.f / T, float(s) / float(S - 1), sg, sd, sdd);
#pragma unroll
      for (int i = 0; i < NJ; ++i) sincos_r(sg[i], sn[i], cs[i]);
      sphere_centres<float, PAT>(A, sn, cs, 0, 1, loc, [&](int k, float x, float y, float z) {
        cx[k * WAVE + lane] = x;
        cy[k * WAVE + lane] = y;
        cz[k * WAVE + lane] = z;
      });
    }
    __builtin_amdgcn_wave_barrier();
    if (act)
      for (int p = 0; p < n_pairs; ++p) {
        const int a = pairs[2 * p] * WAVE + lane, b = pairs[2 * p + 1] * WAVE + lane;
        const float dx = cx[a] - cx[b], dy = cy[a] - cy[b], dz = cz[a] - cz[b];
        best = fminf(best, (dx * dx + dy * dy + dz * dz) * inv[p]);
      }
    __builtin_amdgcn_wave_barrier();
  }
  const float mn = wave_min(best);
  const float rs = mn < INFINITY ? 1.f / sqrtf(mn) : 0.f;
  if (lane == 0) {
    out_rho[5 * e + 4] = fmaxf(out_rho[5 * e + 4], rs);
    if (rs > 1.f) out_st[e] = (uint16_t)(st | FN_S_COLL | FN_S_SELF);
  }
}

// ---------------------------------------------------------------------------
// Multi-round N-ary refinement below the grid result (Sec. IV-D after
// Def. 7).  One wavefront per edge; lanes over (point, sample) as in the
// search: a pass evaluates G = 64 / Sw points of a round, a round the N - 1
// interior points t_i = lo + i (hi - lo) / N in ceil((N - 1) / G) passes, the
// first feasible point in ascending order ending it.  At most REFINE_ROUNDS
// rounds (a round cuts the width N-fold, so only a width below the FP32
// resolution of T could need more).
// ---------------------------------------------------------------------------
constexpr int REFINE_ROUNDS = 64;

template <int PAT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void
edge_refine_kernel(EdgeArgs a, const int16_t* __restrict__ j_in, int n_ary, float eps,
                   const ArmConst<float>* __restrict__ Ap, float* __restrict__ out_T,
                   uint16_t* __restrict__ out_st, float* __restrict__ out_rho,
                   int32_t* __restrict__ out_rounds, int32_t* __restrict__ out_work) {
  __shared__ GeoLDS<float> s_geo;
  extern __shared__ float s_tab[];  // nsph * (n_obs + n_caps) floats
  const int64_t e = xcd_edge(blockIdx.x, a.k, a.E / a.k);
  if (e < 0) return;
  const ArmConst<float>& A = *Ap;
  const int lane = lane_id();
  auto put = [&](float T, int st, float r0, float r1, float r2, float r3, int rounds, int work) {
    if (lane == 0) {
      out_T[e] = T;
      out_st[e] = (uint16_t)st;
      out_rho[4 * e] = r0;
      out_rho[4 * e + 1] = r1;
      out_rho[4 * e + 2] = r2;
      out_rho[4 * e + 3] = r3;
      if (out_rounds) out_rounds[e] = rounds;
      if (out_work) out_work[e] = work;
    }
  };
  const int j = j_in[e];
  EdgeState<float> ES;
  int st0;
  if (!load_edge(a, e, ES, st0)) {
    put(NAN, st0, 0.f, 0.f, 0.f, 0.f, 0, 0);
    return;
  }
  if (j < 0 || j >= a.n_t) {
    put(NAN, FN_S_NONE, 0.f, 0.f, 0.f, 0.f, 0, 0);
    return;
  }
  const int S = a.S, Sw = a.Sw, G = WAVE / Sw, g = lane / Sw;
  const float u = lane_u(lane, Sw, S);
  const bool s_ok = (lane & (Sw - 1)) < S;
  float hi = a.grid[j], lo = j > 0 ? a.grid[j - 1] : 0.f;
  int rounds = 0, work = 0;
  while (hi - lo > eps && rounds < REFINE_ROUNDS) {
    const float wd = (hi - lo) / float(n_ary);
    int first = n_ary;
    for (int i0 = 1; i0 < n_ary && first == n_ary; i0 += G) {
      const int i = i0 + g;
      const bool act = s_ok && i < n_ary;
      float r = 0.f;
      if (act) {
        const float T = lo + float(i) * wd;
        r = eval_rho<float, PAT>(A, ES, T, __builtin_amdgcn_rcpf(T), u);
      }
      work += __popcll(__ballot(act));
      r = group_max(r, Sw);
      for (int q = 0; q < G && i0 + q < n_ary; ++q)
        if (readlane(r, q * Sw) <= 1.f) {
          first = i0 + q;
          break;
        }
    }
    const float nlo = lo + float(first - 1) * wd;
    const float nhi = first < n_ary ? lo + float(first) * wd : hi;
    lo = nlo;
    hi = nhi;
    ++rounds;
  }
  // ratio at the result, then the post-checks there (clearance only when
  // the limit checks pass)
  float r = 0.f;
  if (lane < S) r = eval_rho<float, PAT>(A, ES, hi, __builtin_amdgcn_rcpf(hi), float(lane) / float(S - 1));
  work += S;
  const float rho = wave_max(r);
  float rv, rq, rc;
  post_checks<float, PAT>(A, ES, hi, S, world_of(a), &s_geo, s_tab, 1.f, rv, rq, rc);
  put(hi, post_status(rv, rq, rc), rho, rv, rq, rc, rounds, work);
}

// FP64 stage grid: one wavefront per SIMD at most (its FP64 recursion holds
// 512 registers per lane), each looping over queue entries; more workgroups
// than SIMDs would only queue up empty waves behind the working ones
static unsigned recheck_waves(int64_t E) { return (unsigned)(E < RECHECK_WAVES ? (E > 0 ? E : 1) : RECHECK_WAVES); }

// model kernel (screening modes), search kernel between the timing events,
// FP64 stage
template <int PAT, int MODE>
static void launch_search(fn_ctx* c, const EdgeArgs& a, int ti, hipStream_t s) {
  const int64_t E = a.E, B = a.E / a.k;
  // the model kernel also clears the queue length
  if (MODE != FN_SEARCH_PLAIN)
    hipLaunchKernelGGL(edge_model_kernel<PAT>, dim3((unsigned)(((E + B) * 8 + 255) / 256)),
                       dim3(256), 0, s, a, c->arm32);
  else
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, a.q_count, 1);
  if (ti >= 0) (void)hipEventRecord(c->tev[2 * ti], s);
  const size_t tab = (size_t)EDGE_WAVES * c->desc.n_spheres * (a.n_obs + a.n_caps) * sizeof(float);
  // two phases when asked for, or by default (ordered) for large searches
  int form = c->tune.edge_form > 0 ? c->tune.edge_form : (E >= TRIAGE_MIN_EDGES ? 3 : 1);
  if (form == 3 && E > INT32_MAX) form = 2;  // the order holds int32 edge ids
  if (MODE != FN_SEARCH_PLAIN && form >= 2) {
    hipLaunchKernelGGL((edge_triage_kernel<PAT, MODE>), dim3((unsigned)((E + 3) / 4)), dim3(256),
                       0, s, a, c->arm32);
    if (form == 3) {
      const int64_t chunk = std::max(TRI_MIN_CHUNK, (E + TRI_MAX_BLOCKS - 1) / TRI_MAX_BLOCKS);
      const int nblk = (int)((E + chunk - 1) / chunk);
      int32_t* n_open = a.tri_hist + TRI_MAX_BLOCKS * TRI_BINS;
      hipLaunchKernelGGL(tri_hist_kernel, dim3(nblk), dim3(256), 0, s, a.tri_items, E, chunk,
                         a.n_t, a.tri_hist);
      hipLaunchKernelGGL(tri_scatter_kernel, dim3(nblk), dim3(256), 0, s, a.tri_items, E, chunk,
                         a.n_t, a.tri_hist, nblk, a.tri_order, n_open);
      hipLaunchKernelGGL((edge_search_open_kernel<PAT, MODE, true>), dim3((unsigned)E), dim3(64),
                         tab, s, a, c->arm32);
    } else {
      hipLaunchKernelGGL((edge_search_open_kernel<PAT, MODE, false>),
                         dim3((unsigned)xcd_grid(B, a.k)), dim3(64), tab, s, a, c->arm32);
    }
  } else {
    hipLaunchKernelGGL((edge_time_kernel<PAT, MODE>), dim3((unsigned)xcd_grid(B, a.k)),
                       dim3(64 * EDGE_WAVES), tab, s, a, c->arm32);
  }
  if (ti >= 0) (void)hipEventRecord(c->tev[2 * ti + 1], s);
  hipLaunchKernelGGL(edge_recheck_kernel<PAT>, dim3(recheck_waves(E)), dim3(64),
                     (size_t)c->desc.n_spheres * (a.n_obs + a.n_caps) * sizeof(double), s, a,
                     ProbTable{0, nullptr, nullptr}, c->arm64);
}

template <int PAT>
static void launch_search_mode(fn_ctx* c, const EdgeArgs& a, int ti, hipStream_t s) {
  switch (a.mode) {
    case FN_SEARCH_PLAIN: launch_search<PAT, FN_SEARCH_PLAIN>(c, a, ti, s); break;
    case FN_SEARCH_SCREEN: launch_search<PAT, FN_SEARCH_SCREEN>(c, a, ti, s); break;
    default: launch_search<PAT, FN_SEARCH_WINDOW>(c, a, ti, s); break;
  }
}

static int pow2_at_least(int s) {
  int w = 1;
  while (w < s) w <<= 1;
  return w;
}

int check_obstacles(const fn_obstacles* obs, const char* who) {
  if (!obs) return FN_OK;
  if (obs->n < 0 || obs->n > FN_MAX_OBS) return fail(FN_E_SHAPE, "%s: %d obstacles (max %d)", who, obs->n, FN_MAX_OBS);
  if (obs->n > 0 && !obs->spheres) return fail(FN_E_ARG, "%s: NULL obstacle array", who);
  if (obs->n_caps < 0 || obs->n_caps > FN_MAX_CAPS || obs->n + obs->n_caps > FN_MAX_OBS)
    return fail(FN_E_SHAPE, "%s: %d capsules with %d spheres (max %d capsules, %d obstacles)", who,
                obs->n_caps, obs->n, FN_MAX_CAPS, FN_MAX_OBS);
  if (obs->n_caps > 0 && !obs->capsules) return fail(FN_E_ARG, "%s: NULL capsule array", who);
  if (!(obs->margin >= 0.f)) return fail(FN_E_ARG, "%s: clearance margin must be >= 0", who);
  return FN_OK;
}

}  // namespace fn

using namespace fn;

namespace fn {

// Checks the arguments of an edge search and launches it with the given
// scratch (the FP64-stage counter and queue, the endpoint models).
// max_edges: the most edges that scratch holds.
int edge_time_run(fn_ctx* c, const float* tree, int64_t ld, int32_t n_nodes, const float* cand,
                  int32_t B, const int32_t* nbr, int32_t k, const fn_search* sr,
                  const fn_obstacles* obs, const fn_edge_out* out, void* stream,
                  const EdgeScratch& sc, int64_t max_edges, const char* who, bool timed) {
  if (!c || !sr || !out) return fail(FN_E_ARG, "%s: NULL context, search or out", who);
  if (B < 0 || k < 1 || k > FN_MAX_K) return fail(FN_E_SHAPE, "%s: B = %d, k = %d", who, B, k);
  const int64_t E = (int64_t)B * k;
  if (E > max_edges) return fail(FN_E_SHAPE, "%s: %lld edges (cap %lld)", who, (long long)E, (long long)max_edges);
  if (n_nodes < 0) return fail(FN_E_SHAPE, "%s: n_nodes = %d", who, n_nodes);
  if (sr->n_t < 1 || sr->n_t > FN_MAX_NT) return fail(FN_E_SHAPE, "%s: n_t = %d (1..%d)", who, sr->n_t, FN_MAX_NT);
  if (sr->samples < 2 || sr->samples > FN_MAX_SAMPLES) return fail(FN_E_SHAPE, "%s: S = %d (2..%d)", who, sr->samples, FN_MAX_SAMPLES);
  if (sr->mode < FN_SEARCH_PLAIN || sr->mode > FN_SEARCH_WINDOW) return fail(FN_E_ARG, "%s: mode %d", who, sr->mode);
  if (sr->mode == FN_SEARCH_WINDOW && sr->win_half < 0) return fail(FN_E_ARG, "%s: window mode needs win_half >= 0", who);
  int rc = check_obstacles(obs, who);
  if (rc) return rc;
  if (E == 0) return FN_OK;  // nothing to read or write: the arrays may be NULL
  if (sr->mode == FN_SEARCH_WINDOW && !sr->win_lo) return fail(FN_E_ARG, "%s: window mode needs win_lo", who);
  if (!cand || !nbr || !sr->grid || !out->j || !out->status || !out->margin || (n_nodes > 0 && !tree))
    return fail(FN_E_ARG, "%s: NULL array", who);
  if (ld < n_nodes) return fail(FN_E_ARG, "%s: ld < n_nodes", who);
  EdgeArgs a{};
  a.tree = tree; a.ld = ld; a.n_nodes = n_nodes; a.cand = cand; a.nbr = nbr; a.k = k; a.E = E;
  a.grid = sr->grid; a.n_t = sr->n_t; a.S = sr->samples; a.Sw = pow2_at_least(sr->samples);
  a.mode = sr->mode; a.win_half = sr->win_half; a.j_max = sr->j_max; a.win_lo = sr->win_lo;
  a.obs = obs ? obs->spheres : nullptr; a.n_obs = obs ? obs->n : 0; a.margin_c = obs ? obs->margin : 0.f;
  a.caps = obs ? obs->capsules : nullptr; a.n_caps = obs ? obs->n_caps : 0;
  a.out_j = out->j; a.out_st = out->status; a.out_m = out->margin; a.out_rho = out->rho4;
  a.out_work = out->work; a.out_scr = out->screened;
  a.q_count = sc.q_count; a.queue = sc.queue; a.model_e = sc.model_e; a.model_c = sc.model_c;
  a.tri_items = sc.tri_items;
  a.tri_order = sc.tri_items + max_edges;
  a.tri_hist = sc.tri_items + 2 * max_edges;
  hipStream_t s = (hipStream_t)stream;
  const int ti = timed && c->timing && c->n_timed < FN_MAX_TIMED ? c->n_timed++ : -1;
  if (c->pattern == PAT_FR3) launch_search_mode<PAT_FR3>(c, a, ti, s);
  else launch_search_mode<PAT_GENERIC>(c, a, ti, s);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, who);
}

}  // namespace fn

extern "C" int edge_time_batch(fn_ctx* c, const float* tree, int64_t ld, int32_t n_nodes,
                               const float* cand, int32_t B, const int32_t* nbr, int32_t k,
                               const fn_search* sr, const fn_obstacles* obs,
                               const fn_edge_out* out, void* stream) {
  if (!c) return fail(FN_E_ARG, "edge_time_batch: NULL context");
  const EdgeScratch sc{c->q_count, c->queue, c->model_e, c->model_c, c->tri_items};
  return edge_time_run(c, tree, ld, n_nodes, cand, B, nbr, k, sr, obs, out, stream, sc,
                       c->caps.max_edges, "edge_time_batch", true);
}

extern "C" int edge_check(fn_ctx* c, const float* x0, const float* x1, const float* T, int64_t E,
                          int32_t S, const fn_obstacles* obs, uint16_t* out_status,
                          float* out_rho5, float* out_tau, void* stream) {
  if (!c) return fail(FN_E_ARG, "edge_check: NULL context");
  if (E < 0 || E > c->caps.max_edges) return fail(FN_E_SHAPE, "edge_check: E = %lld (cap %lld)", (long long)E, (long long)c->caps.max_edges);
  if (S < 2 || S > 4096) return fail(FN_E_SHAPE, "edge_check: S = %d (2..4096)", S);
  int rc = check_obstacles(obs, "edge_check");
  if (rc) return rc;
  if (E == 0) return FN_OK;
  if (!x0 || !x1 || !T || !out_status || !out_rho5) return fail(FN_E_ARG, "edge_check: NULL array");
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid((unsigned)((E + 3) / 4));
  World w{};
  if (obs) w = World{obs->spheres, obs->n, obs->capsules, obs->n_caps, obs->margin};
  const size_t tab = (size_t)4 * c->desc.n_spheres * world_size(w) * sizeof(float);
  if (c->pattern == PAT_FR3)
    hipLaunchKernelGGL(edge_check_kernel<PAT_FR3>, grid, dim3(256), tab, s, x0, x1, T, E, S, w, c->arm32, out_status, out_rho5, out_tau);
  else
    hipLaunchKernelGGL(edge_check_kernel<PAT_GENERIC>, grid, dim3(256), tab, s, x0, x1, T, E, S, w, c->arm32, out_status, out_rho5, out_tau);
  if (c->n_self > 0) {
    // the arm's self-collision pairs, one wavefront per edge
    const int ns = c->desc.n_spheres;
    const size_t lds = (size_t)(4 * ns + 3 * ns * WAVE + c->n_self) * sizeof(float);
    if (c->pattern == PAT_FR3)
      hipLaunchKernelGGL(edge_self_kernel<PAT_FR3>, dim3((unsigned)E), dim3(64), lds, s, x0, x1, T, E, S, c->self_pairs, c->n_self, c->margin_self, c->arm32, out_status, out_rho5);
    else
      hipLaunchKernelGGL(edge_self_kernel<PAT_GENERIC>, dim3((unsigned)E), dim3(64), lds, s, x0, x1, T, E, S, c->self_pairs, c->n_self, c->margin_self, c->arm32, out_status, out_rho5);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "edge_check launch");
}

extern "C" int fn_set_self_pairs(fn_ctx* c, const int32_t* pairs, int32_t n, float margin) {
  if (!c) return fail(FN_E_ARG, "fn_set_self_pairs: NULL context");
  if (n < 0 || n > FN_MAX_SELF_PAIRS) return fail(FN_E_SHAPE, "fn_set_self_pairs: %d pairs (max %d)", n, FN_MAX_SELF_PAIRS);
  if (n > 0 && !pairs) return fail(FN_E_ARG, "fn_set_self_pairs: NULL pairs");
  if (!(margin >= 0.f)) return fail(FN_E_ARG, "fn_set_self_pairs: margin must be >= 0");
  int16_t h[2 * FN_MAX_SELF_PAIRS];
  for (int p = 0; p < n; ++p) {
    const int a = pairs[2 * p], b = pairs[2 * p + 1];
    if (a < 0 || b < 0 || a >= c->desc.n_spheres || b >= c->desc.n_spheres || a == b)
      return fail(FN_E_ARG, "fn_set_self_pairs: pair %d = (%d, %d) (spheres 0..%d, distinct)", p, a, b, c->desc.n_spheres - 1);
    // sphere indices as the caller gave them, mapped to the link-sorted order
    h[2 * p] = (int16_t)c->sphere_order[a];
    h[2 * p + 1] = (int16_t)c->sphere_order[b];
  }
  if (n > 0) {
    const hipError_t e = hipMemcpy(c->self_pairs, h, sizeof(int16_t) * 2 * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "fn_set_self_pairs");
  }
  c->n_self = n;
  c->margin_self = margin;
  return FN_OK;
}

extern "C" int edge_refine(fn_ctx* c, const float* tree, int64_t ld, int32_t n_nodes,
                           const float* cand, int32_t B, const int32_t* nbr, int32_t k,
                           const int16_t* j_in, const fn_refine* r, const fn_obstacles* obs,
                           float* out_T, uint16_t* out_status, float* out_rho4,
                           int32_t* out_rounds, int32_t* out_work, void* stream) {
  if (!c || !r) return fail(FN_E_ARG, "edge_refine: NULL context or refinement");
  if (B < 0 || k < 1 || k > FN_MAX_K) return fail(FN_E_SHAPE, "edge_refine: B = %d, k = %d", B, k);
  const int64_t E = (int64_t)B * k;
  if (n_nodes < 0) return fail(FN_E_SHAPE, "edge_refine: n_nodes = %d", n_nodes);
  if (r->n_t < 1 || r->n_t > FN_MAX_NT) return fail(FN_E_SHAPE, "edge_refine: n_t = %d (1..%d)", r->n_t, FN_MAX_NT);
  if (r->samples < 2 || r->samples > FN_MAX_SAMPLES) return fail(FN_E_SHAPE, "edge_refine: S = %d (2..%d)", r->samples, FN_MAX_SAMPLES);
  if (r->n_ary < 2 || r->n_ary > 1024) return fail(FN_E_ARG, "edge_refine: N = %d (2..1024)", r->n_ary);
  if (!(r->eps > 0.f)) return fail(FN_E_ARG, "edge_refine: eps must be > 0");
  int rc = check_obstacles(obs, "edge_refine");
  if (rc) return rc;
  if (E == 0) return FN_OK;
  if (!cand || !nbr || !j_in || !r->grid || !out_T || !out_status || !out_rho4 || (n_nodes > 0 && !tree))
    return fail(FN_E_ARG, "edge_refine: NULL array");
  if (ld < n_nodes) return fail(FN_E_ARG, "edge_refine: ld < n_nodes");
  EdgeArgs a{};
  a.tree = tree; a.ld = ld; a.n_nodes = n_nodes; a.cand = cand; a.nbr = nbr; a.k = k; a.E = E;
  a.grid = r->grid; a.n_t = r->n_t; a.S = r->samples; a.Sw = pow2_at_least(r->samples);
  a.obs = obs ? obs->spheres : nullptr; a.n_obs = obs ? obs->n : 0; a.margin_c = obs ? obs->margin : 0.f;
  a.caps = obs ? obs->capsules : nullptr; a.n_caps = obs ? obs->n_caps : 0;
  hipStream_t s = (hipStream_t)stream;
  const size_t tab = (size_t)c->desc.n_spheres * (a.n_obs + a.n_caps) * sizeof(float);
  const dim3 grid((unsigned)xcd_grid(B, k));
  if (c->pattern == PAT_FR3)
    hipLaunchKernelGGL(edge_refine_kernel<PAT_FR3>, grid, dim3(64), tab, s, a, j_in, r->n_ary,
                       r->eps, c->arm32, out_T, out_status, out_rho4, out_rounds, out_work);
  else
    hipLaunchKernelGGL(edge_refine_kernel<PAT_GENERIC>, grid, dim3(64), tab, s, a, j_in, r->n_ary,
                       r->eps, c->arm32, out_T, out_status, out_rho4, out_rounds, out_work);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "edge_refine launch");
}
