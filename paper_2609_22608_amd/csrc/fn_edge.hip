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
  __shared__ float s_mod[EDGE_WAVES][2 * MODEL_FLOATS];
  __shared__ GeoLDS<float> s_geo[EDGE_WAVES];
  extern __shared__ float s_tab[];  // EDGE_WAVES * nsph * n_obs floats
  for (int t = threadIdx.x; t < a.n_t; t += blockDim.x) s_T[t] = a.grid[t];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t e = xcd_edge(blockIdx.x, a.k, a.E / a.k);
  if (e < 0) return;
  search_edge<PAT, MODE, false>(a, e, e, *Ap, s_end_all[wave], s_T, s_fix[wave], s_mod[wave],
                                &s_geo[wave], s_tab + wave * Ap->nsph * a.n_obs);
}

// ---------------------------------------------------------------------------
// Fixed-duration check (goal branch of Algorithm 1; recheck of a sent plan)
// ---------------------------------------------------------------------------
template <int PAT>
__global__ __launch_bounds__(256) void edge_check_kernel(const float* __restrict__ x0,
                                                         const float* __restrict__ x1,
                                                         const float* __restrict__ Tv, int64_t E,
                                                         int S, const float* __restrict__ obs,
                                                         int n_obs, float margin_c,
                                                         const ArmConst<float>* __restrict__ Ap,
                                                         uint16_t* out_st, float* out_rho,
                                                         float* out_tau) {
  __shared__ GeoLDS<float> s_geo[4];
  extern __shared__ float s_tab[];  // 4 * nsph * n_obs floats
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
  post_checks<float, PAT>(A, ES, T, S, obs, n_obs, margin_c, &s_geo[wave],
                          s_tab + wave * A.nsph * n_obs, rt <= 1.f && rp <= 1.f ? 1.f : -1.f,
                          rv, rq, rc);
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
  const size_t tab = (size_t)EDGE_WAVES * c->desc.n_spheres * a.n_obs * sizeof(float);
  hipLaunchKernelGGL((edge_time_kernel<PAT, MODE>), dim3((unsigned)xcd_grid(B, a.k)),
                     dim3(64 * EDGE_WAVES), tab, s, a, c->arm32);
  if (ti >= 0) (void)hipEventRecord(c->tev[2 * ti + 1], s);
  hipLaunchKernelGGL(edge_recheck_kernel<PAT>, dim3(recheck_waves(E)), dim3(64),
                     (size_t)c->desc.n_spheres * a.n_obs * sizeof(double), s, a,
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
  if (sr->mode == FN_SEARCH_WINDOW && (!sr->win_lo || sr->win_half < 0)) return fail(FN_E_ARG, "%s: window mode needs win_lo and win_half >= 0", who);
  int rc = check_obstacles(obs, who);
  if (rc) return rc;
  if (E == 0) return FN_OK;
  if (!cand || !nbr || !sr->grid || !out->j || !out->status || !out->margin || (n_nodes > 0 && !tree))
    return fail(FN_E_ARG, "%s: NULL array", who);
  if (ld < n_nodes) return fail(FN_E_ARG, "%s: ld < n_nodes", who);
  EdgeArgs a{};
  a.tree = tree; a.ld = ld; a.n_nodes = n_nodes; a.cand = cand; a.nbr = nbr; a.k = k; a.E = E;
  a.grid = sr->grid; a.n_t = sr->n_t; a.S = sr->samples; a.Sw = pow2_at_least(sr->samples);
  a.mode = sr->mode; a.win_half = sr->win_half; a.j_max = sr->j_max; a.win_lo = sr->win_lo;
  a.obs = obs ? obs->spheres : nullptr; a.n_obs = obs ? obs->n : 0; a.margin_c = obs ? obs->margin : 0.f;
  a.out_j = out->j; a.out_st = out->status; a.out_m = out->margin; a.out_rho = out->rho4;
  a.out_work = out->work; a.out_scr = out->screened;
  a.q_count = sc.q_count; a.queue = sc.queue; a.model_e = sc.model_e; a.model_c = sc.model_c;
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
  const EdgeScratch sc{c->q_count, c->queue, c->model_e, c->model_c};
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
  if (S > FN_MAX_SAMPLES && obs && obs->n > 0)
    return fail(FN_E_SHAPE, "edge_check: clearance needs S <= %d", FN_MAX_SAMPLES);
  if (E == 0) return FN_OK;
  if (!x0 || !x1 || !T || !out_status || !out_rho5) return fail(FN_E_ARG, "edge_check: NULL array");
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid((unsigned)((E + 3) / 4));
  const float* ob = obs ? obs->spheres : nullptr;
  const int no = obs ? obs->n : 0;
  const float mg = obs ? obs->margin : 0.f;
  const size_t tab = (size_t)4 * c->desc.n_spheres * no * sizeof(float);
  if (c->pattern == PAT_FR3)
    hipLaunchKernelGGL(edge_check_kernel<PAT_FR3>, grid, dim3(256), tab, s, x0, x1, T, E, S, ob, no, mg, c->arm32, out_status, out_rho5, out_tau);
  else
    hipLaunchKernelGGL(edge_check_kernel<PAT_GENERIC>, grid, dim3(256), tab, s, x0, x1, T, E, S, ob, no, mg, c->arm32, out_status, out_rho5, out_tau);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "edge_check launch");
}
