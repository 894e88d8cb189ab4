// fn_edge.hip -- minimum feasible time of every edge on the T grid (Def. 7,
// Algorithm 1 free-candidate branch), the post-checks at that time (Def. 6
// rho_v, position limits, clearance of Sec. IV-E), and the fixed-duration
// check of the goal branch.
//
// One wavefront per edge.  The 64 lanes are mapped over (slot, sample)
// pairs: a pass evaluates G = 64 / Sw slots at once (Sw = S rounded up to a
// power of two), every lane one point of Eq. (4) along the cubic of Eq. (6).
// A slot's ratio is the max over its lane group (xor shuffles); slots are
// decided in ascending order, so the first feasible slot of the grid is the
// result whatever order the work is done in.
//
// Search modes (same result, different work):
//  PLAIN  -- ascending passes over full slots, stop at the first feasible.
//  SCREEN -- first the two endpoint samples (u = 0, 1) of every slot, 32
//            slots per pass; a slot whose endpoint ratio exceeds 1 + BAND is
//            infeasible for certain and never evaluated in full.  Then full
//            passes over the remaining slots in ascending order.
//  WINDOW -- the surrogate's window [lo, lo + 2h]: slots below it are
//            screened (the certificate), the window is evaluated in full, the
//            slots above it are screened only if the window holds no
//            feasible slot.  "Hit" = the result lies in the window (or the
//            network predicted no feasible slot and there is none).
//
// Every FP32 ratio within BAND of 1 that a decision rests on sends the edge
// to the FP64 stage (edge_recheck), which resumes it from that slot.
#include <hip/hip_runtime.h>

#include "fn_ctx.h"

namespace fn {

struct EdgeArgs {
  const float* __restrict__ tree;
  int64_t ld;
  int n_nodes;
  const float* __restrict__ cand;
  const int32_t* __restrict__ nbr;
  int k;
  int64_t E;
  const float* __restrict__ grid;
  int n_t, S, Sw, mode, win_half;
  const int16_t* __restrict__ j_max;
  const int16_t* __restrict__ win_lo;
  const float* __restrict__ obs;
  int n_obs;
  float margin_c;
  int16_t* out_j;
  uint16_t* out_st;
  float* out_m;
  float* out_rho;
  int32_t* out_work;
  int32_t* q_count;
  QEntry* queue;
};

// queue phase bits
constexpr int PH_POST = 1;        // only the post-checks are left
constexpr int PH_BELOW_FULL = 2;  // window mode: a slot below the window was evaluated in full

template <typename R>
__device__ __forceinline__ bool load_edge(const EdgeArgs& a, int64_t e, EdgeState<R>& S,
                                          int& status) {
  const int64_t b = e / a.k;
  const int p = a.nbr[e];
  status = 0;
  if (p < 0) {
    status = FN_S_NO_PARENT;
    return false;
  }
  if (p >= a.n_nodes) {
    status = FN_S_BAD_INPUT;
    return false;
  }
  bool finite = true;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    const float q0 = a.tree[(size_t)i * a.ld + p];
    const float v0 = a.tree[(size_t)(NJ + i) * a.ld + p];
    const float q1 = a.cand[b * FN_STATE + i];
    const float v1 = a.cand[b * FN_STATE + NJ + i];
    finite = finite && isfinite(q0) && isfinite(v0) && isfinite(q1) && isfinite(v1);
    S.q0[i] = R(q0);
    S.qd0[i] = R(v0);
    S.dq[i] = R(q1) - R(q0);
    S.d2[i] = R(v1) - R(v0);
  }
  if (!finite) status = FN_S_BAD_INPUT;
  return finite;
}

__device__ __forceinline__ float lane_u(int lane, int Sw, int S) {
  const int s = lane & (Sw - 1);
  return s < S ? float(s) / float(S - 1) : 0.f;
}

// Post-checks at duration T (Def. 6 rho_v; position limits; clearance):
// returns (rho_v, rho_q, rho_c) in every lane.
template <typename R, int PAT>
__device__ void post_checks(const ArmConst<R>& A, const EdgeState<R>& E, R T, int S,
                            const float* __restrict__ obs, int n_obs, float margin_c, R& rv,
                            R& rq, R& rc) {
  const int lane = lane_id();
  R v = 0, q = 0;
  // lane i < 7 checks joint i (register selects keep the edge state in VGPRs)
  R q0 = 0, qd0 = 0, dq = 0, d2v = 0;
#pragma unroll
  for (int i = 0; i < NJ; ++i)
    if (lane == i) {
      q0 = E.q0[i];
      qd0 = E.qd0[i];
      dq = E.dq[i];
      d2v = E.d2[i];
    }
  if (lane < NJ) joint_post(A, lane, q0, qd0, dq, d2v, T, v, q);
  // clearance: lane = (sample, sphere part); the parts split each link's
  // spheres so that all 64 lanes work when S < 64
  R best = 0;
  if (n_obs > 0) {
    int Sw = 1;
    while (Sw < S) Sw <<= 1;
    const int nparts = Sw >= WAVE ? 1 : WAVE / Sw;
    const int s = lane & (Sw - 1), part = lane / Sw;
    if (s < S && part < nparts) {
      const R u = R(s) / R(S - 1);
      R sg[NJ], sd[NJ], sdd[NJ], sn[NJ], cs[NJ];
      cubic_point(E, T, R(1) / T, u, sg, sd, sdd);
#pragma unroll
      for (int i = 0; i < NJ; ++i) sincos_r(sg[i], sn[i], cs[i]);
      sphere_centres<R, PAT>(A, sn, cs, part, nparts, [&](int k, R x, R y, R z) {
        const R ra = A.sphr[k] + R(margin_c);
        for (int o = 0; o < n_obs; ++o) {
          const R dx = x - R(obs[4 * o]), dy = y - R(obs[4 * o + 1]), dz = z - R(obs[4 * o + 2]);
          const R need = ra + R(obs[4 * o + 3]);
          const R d2 = dx * dx + dy * dy + dz * dz;
          const R r2 = d2 > R(0) ? fdiv(need * need, d2) : R(INFINITY);
          best = rmax(best, r2);
        }
      });
    }
  }
  if constexpr (sizeof(R) == 4) {
    rv = wave_max(float(v));
    rq = wave_max(float(q));
    rc = sqrtf(wave_max(float(best)));
  } else {
    rv = wave_max(double(v));
    rq = wave_max(double(q));
    rc = sqrt(wave_max(double(best)));
  }
}

__device__ __forceinline__ bool near_one(float r) { return fabsf(r - 1.f) <= BAND; }

// Final status bits from the post-check ratios.
template <typename R>
__device__ __forceinline__ int post_status(R rv, R rq, R rc) {
  int st = 0;
  if (rv > R(1)) st |= FN_S_VEL;
  if (rq > R(1)) st |= FN_S_POS;
  if (rc > R(1)) st |= FN_S_COLL;
  return st;
}

__device__ __forceinline__ void write_out(const EdgeArgs& a, int64_t e, int j, int st, float m,
                                          float r0, float r1, float r2, float r3, int work) {
  if (lane_id() == 0) {
    a.out_j[e] = (int16_t)j;
    a.out_st[e] = (uint16_t)st;
    a.out_m[e] = m;
    if (a.out_rho) {
      a.out_rho[4 * e + 0] = r0;
      a.out_rho[4 * e + 1] = r1;
      a.out_rho[4 * e + 2] = r2;
      a.out_rho[4 * e + 3] = r3;
    }
    if (a.out_work) a.out_work[e] = work;
  }
}

__device__ __forceinline__ void push_queue(const EdgeArgs& a, int64_t e, int j, int phase,
                                           float m, int work) {
  if (lane_id() == 0) {
    const int slot = atomicAdd(a.q_count, 1);
    QEntry q;
    q.edge = (int32_t)e;
    q.j = (int16_t)j;
    q.phase = (int16_t)phase;
    q.margin = m;
    q.work = work;
    a.queue[slot] = q;
  }
}

// ---------------------------------------------------------------------------
// FP32 search kernel
//
// The search of every mode is a short list of stages, each a slot range
// that is either screened (endpoint samples) or scanned (full slots in
// ascending order, certified slots skipped):
//   PLAIN : scan [0, jmax]
//   SCREEN: screen [0, jmax], scan [0, jmax]
//   WINDOW: screen [0, lo-1], scan [0, lo-1], scan [lo, hi],
//           screen [hi+1, jmax], scan [hi+1, jmax]
// One loop walks the stages so that the evaluation of Eq. (4) has a single
// call site.
// ---------------------------------------------------------------------------
enum { ST_SCREEN = 0, ST_SCAN = 1, ST_END = 2 };

__device__ __forceinline__ void stage_of(int mode, int st, int jmax, int lo, int hi, int& type,
                                         int& a, int& b, bool& below) {
  below = false;
  type = ST_END;
  a = 0;
  b = -1;
  if (mode == FN_SEARCH_PLAIN) {
    if (st == 0) { type = ST_SCAN; a = 0; b = jmax; }
  } else if (mode == FN_SEARCH_SCREEN) {
    if (st == 0) { type = ST_SCREEN; a = 0; b = jmax; }
    if (st == 1) { type = ST_SCAN; a = 0; b = jmax; }
  } else {
    switch (st) {
      case 0: type = ST_SCREEN; a = 0; b = lo - 1; break;
      case 1: type = ST_SCAN; a = 0; b = lo - 1; below = true; break;
      case 2: type = ST_SCAN; a = lo; b = hi; break;
      case 3: type = ST_SCREEN; a = hi + 1; b = jmax; break;
      case 4: type = ST_SCAN; a = hi + 1; b = jmax; break;
      default: break;
    }
  }
}

// Slots still to be evaluated in full: bit j of word j / 64.
struct SlotMask {
  uint64_t w0, w1, w2, w3;
  __device__ __forceinline__ uint64_t get(int i) const {
    return i == 0 ? w0 : i == 1 ? w1 : i == 2 ? w2 : w3;
  }
  __device__ __forceinline__ void clear(int i, uint64_t m) {
    if (i == 0) w0 &= ~m;
    else if (i == 1) w1 &= ~m;
    else if (i == 2) w2 &= ~m;
    else w3 &= ~m;
  }
  // lowest set slot in [j, hi], or -1
  __device__ __forceinline__ int next(int j, int hi) const {
    while (j <= hi) {
      const int w = j >> 6;
      const uint64_t bits = get(w) & (~0ull << (j & 63));
      if (bits) {
        const int t = (w << 6) + __ffsll((long long)bits) - 1;
        return t <= hi ? t : -1;
      }
      j = (w + 1) << 6;
    }
    return -1;
  }
};

template <int PAT>
__global__ __launch_bounds__(256) void edge_time_kernel(EdgeArgs a,
                                                        const ArmConst<float>* __restrict__ Ap) {
  __shared__ float s_end_all[4][FN_MAX_NT];
  __shared__ float s_T[FN_MAX_NT];
  // the block's four edges share the grid: stage it once
  for (int t = threadIdx.x; t < a.n_t; t += blockDim.x) s_T[t] = a.grid[t];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t e = (int64_t)blockIdx.x * 4 + wave;
  if (e >= a.E) return;
  const ArmConst<float>& A = *Ap;
  const int lane = lane_id();
  float* s_end = s_end_all[wave];

  EdgeState<float> ES;
  int st0;
  if (!load_edge(a, e, ES, st0)) {
    write_out(a, e, -1, st0, st0 == FN_S_NO_PARENT ? INFINITY : 0.f, 0, 0, 0, 0, 0);
    return;
  }
  int jmax = a.n_t - 1;
  if (a.j_max) jmax = min(jmax, (int)a.j_max[e]);
  if (jmax < 0) {
    write_out(a, e, -1, FN_S_NONE, INFINITY, 0, 0, 0, 0, 0);
    return;
  }
  const int S = a.S, Sw = a.Sw, G = WAVE / Sw;
  const int g = lane / Sw;
  const float u_full = lane_u(lane, Sw, S);
  const bool s_ok = (lane & (Sw - 1)) < S;

  for (int j = lane; j < a.n_t; j += WAVE) s_end[j] = -1.f;  // -1: not screened
  __builtin_amdgcn_wave_barrier();
  SlotMask todo{~0ull, ~0ull, ~0ull, ~0ull};

  int wlo = 0, whi = -1;
  if (a.mode == FN_SEARCH_WINDOW) {
    wlo = min(max((int)a.win_lo[e], 0), jmax + 1);
    whi = min(wlo + 2 * a.win_half, jmax);
  }

  int work = 0;
  float marg = INFINITY;  // over fully evaluated slots up to the result
  float last = 0.f;
  int jstar = -1;
  float rho_star = 0.f;
  bool below_full = false;
  bool queued = false;

  int stage = 0, type, sa, sb;
  bool below;
  stage_of(a.mode, stage, jmax, wlo, whi, type, sa, sb, below);
  int j = sa;
  while (type != ST_END) {
    if (j > sb) {
      ++stage;
      stage_of(a.mode, stage, jmax, wlo, whi, type, sa, sb, below);
      j = sa;
      continue;
    }
    // lanes of this pass: slot `my` (or -1) and normalised time u
    int my = -1, cnt = 0;
    float u = u_full;
    if (type == ST_SCREEN) {
      // lane l: slot j + (l & 31), endpoint u = 0 (l < 32) or u = 1
      const int jj = j + (lane & 31);
      my = jj <= sb ? jj : -1;
      u = lane >= 32 ? 1.f : 0.f;
      cnt = min(WAVE / 2, sb - j + 1);
      j += WAVE / 2;
    } else {
      // next G slots still to be evaluated; lane group g takes the g-th
      while (cnt < G) {
        const int t = todo.next(j, sb);
        if (t < 0) {
          j = sb + 1;
          break;
        }
        if (cnt == g) my = t;
        ++cnt;
        j = t + 1;
      }
      if (cnt == 0) continue;  // range exhausted
      if (!s_ok) my = -1;
      if (below) below_full = true;
    }
    const bool act = my >= 0;
    float r = 0.f;
    if (act) {
      const float T = s_T[my];
      r = eval_rho<float, PAT>(A, ES, T, __builtin_amdgcn_rcpf(T), u);
    }
    work += __popcll(__ballot(act));
    if (type == ST_SCREEN) {
      r = fmaxf(r, __shfl_xor(r, 32));
      if (act && lane < 32) s_end[my] = r;
      // slots certified infeasible leave the to-do mask: bit t of the ballot
      // is slot j0 + t, and the pass may straddle two 64-slot words
      const int j0 = j - WAVE / 2;
      const uint64_t bits = __ballot(act && lane < 32 && r > 1.f + BAND) & 0xffffffffull;
      const int w0 = j0 >> 6, sh = j0 & 63;
      todo.clear(w0, bits << sh);
      if (sh > 32) todo.clear(w0 + 1, bits >> (64 - sh));
      continue;
    }
    r = group_max(r, Sw);
    bool done = false;
    for (int q = 0; q < cnt; ++q) {
      const float rho = __shfl(r, q * Sw);
      const int jq = __shfl(my, q * Sw);
      if (near_one(rho)) {
        // decided in FP64: hand the edge over at slot jq
        float m = INFINITY;
        for (int t = lane; t < jq; t += WAVE)
          if (s_end[t] > 1.f + BAND) m = fminf(m, s_end[t] - 1.f);
        m = fminf(marg, wave_min(m));
        push_queue(a, e, jq, below_full ? PH_BELOW_FULL : 0, m, work);
        queued = done = true;
        break;
      }
      marg = fminf(marg, fabsf(rho - 1.f));
      last = rho;
      if (rho <= 1.f) {
        jstar = jq;
        rho_star = rho;
        done = true;
        break;
      }
    }
    if (done) break;
  }
  if (queued) return;
  __builtin_amdgcn_wave_barrier();
  // certified-infeasible margin of the screened slots below the result
  const int lim = jstar >= 0 ? jstar : jmax + 1;
  float mc = INFINITY;
  for (int t = lane; t < lim; t += WAVE)
    if (s_end[t] > 1.f + BAND) mc = fminf(mc, s_end[t] - 1.f);
  float m = fminf(marg, wave_min(mc));
  int winbits = 0;
  if (a.mode == FN_SEARCH_WINDOW) {
    // hit: the result lies in the predicted window (or none was predicted
    // and none exists); BELOW: a slot under the window needed a full pass
    const bool hit = (jstar >= 0 && jstar >= wlo && jstar <= whi) || (jstar < 0 && wlo > jmax);
    winbits = (hit ? FN_S_WIN_HIT : FN_S_WIN_MISS) | (below_full ? FN_S_WIN_BELOW : 0);
  }
  if (jstar < 0) {
    // ratio of the last slot: its full value, else its screened endpoint value
    const float lastv = s_end[jmax] > 1.f + BAND ? s_end[jmax] : last;
    write_out(a, e, -1, FN_S_NONE | winbits, m, lastv, 0, 0, 0, work);
    return;
  }
  float rv, rq, rc;
  const float T = s_T[jstar];
  post_checks<float, PAT>(A, ES, T, S, a.obs, a.n_obs, a.margin_c, rv, rq, rc);
  if (near_one(rv) || near_one(rq) || (a.n_obs > 0 && near_one(rc))) {
    push_queue(a, e, jstar, PH_POST | (below_full ? PH_BELOW_FULL : 0), m, work);
    return;
  }
  m = fminf(m, fminf(fabsf(rv - 1.f), fminf(fabsf(rq - 1.f), fabsf(rc - 1.f))));
  write_out(a, e, jstar, post_status(rv, rq, rc) | winbits, m, rho_star, rv, rq, rc, work);
}

// ---------------------------------------------------------------------------
// FP64 stage: every queued edge resumes at its slot with full slots in
// ascending order; a slot whose FP32 ratio is within BAND of 1 is decided by
// its FP64 ratio; post-checks are done in FP64.
// ---------------------------------------------------------------------------
template <int PAT>
__global__ __launch_bounds__(64) void edge_recheck_kernel(EdgeArgs a,
                                                          const ArmConst<float>* __restrict__ Ap,
                                                          const ArmConst<double>* __restrict__ Dp) {
  const int n = *a.q_count;
  const ArmConst<float>& A = *Ap;
  const ArmConst<double>& D = *Dp;
  const int lane = lane_id();
  for (int qi = blockIdx.x; qi < n; qi += gridDim.x) {
    const QEntry q = a.queue[qi];
    const int64_t e = q.edge;
    EdgeState<float> ES;
    EdgeState<double> ED;
    int st0;
    load_edge(a, e, ES, st0);
    load_edge(a, e, ED, st0);
    int jmax = a.n_t - 1;
    if (a.j_max) jmax = min(jmax, (int)a.j_max[e]);
    const int S = a.S;
    int work = q.work;
    float marg = q.margin;
    int jstar = -1;
    double rho_star = 0;
    float last = 0;
    if (q.phase & PH_POST) {
      jstar = q.j;
      const double T = a.grid[jstar];
      rho_star = 0;
      // the slot ratio itself is reported from FP32 (it was outside the band)
      const float Tf = a.grid[jstar];
      float r = 0.f;
      if (lane < S) r = eval_rho<float, PAT>(A, ES, Tf, 1.f / Tf, float(lane) / float(S - 1));
      rho_star = wave_max(r);
      (void)T;
    } else {
      for (int j = q.j; j <= jmax; ++j) {
        const float Tf = a.grid[j];
        float r = 0.f;
        if (lane < S) r = eval_rho<float, PAT>(A, ES, Tf, 1.f / Tf, float(lane) / float(S - 1));
        float rho = wave_max(r);
        work += S;
        double rho_d = rho;
        if (near_one(rho)) {
          const double T = (double)Tf;
          double rd = 0.0;
          if (lane < S) rd = eval_rho<double, PAT>(D, ED, T, 1.0 / T, double(lane) / double(S - 1));
          rho_d = wave_max(rd);
        }
        marg = fminf(marg, (float)fabs(rho_d - 1.0));
        last = (float)rho_d;
        if (rho_d <= 1.0) {
          jstar = j;
          rho_star = rho_d;
          break;
        }
      }
    }
    int winbits = 0;
    if (a.mode == FN_SEARCH_WINDOW) {
      const int wlo = min(max((int)a.win_lo[e], 0), jmax + 1);
      const int whi = min(wlo + 2 * a.win_half, jmax);
      const bool below = (q.phase & PH_BELOW_FULL) != 0;
      const bool hit = (jstar >= 0 && jstar >= wlo && jstar <= whi) || (jstar < 0 && wlo > jmax);
      winbits = (hit ? FN_S_WIN_HIT : FN_S_WIN_MISS) | (below ? FN_S_WIN_BELOW : 0);
    }
    if (jstar < 0) {
      write_out(a, e, -1, FN_S_NONE | FN_S_RECHECK64 | winbits, marg, last, 0, 0, 0, work);
      continue;
    }
    double rv, rq, rc;
    post_checks<double, PAT>(D, ED, (double)a.grid[jstar], S, a.obs, a.n_obs, a.margin_c, rv, rq,
                             rc);
    const float m = fminf(marg, (float)fmin(fabs(rv - 1.0), fmin(fabs(rq - 1.0), fabs(rc - 1.0))));
    write_out(a, e, jstar, post_status(rv, rq, rc) | FN_S_RECHECK64 | winbits, m, (float)rho_star,
              (float)rv, (float)rq, (float)rc, work);
  }
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
  post_checks<float, PAT>(A, ES, T, S, obs, n_obs, margin_c, rv, rq, rc);
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

// waves of the FP64 stage: one per queued edge up to 4096 (the queue
// length is known only on the device)
static unsigned recheck_waves(int64_t E) { return (unsigned)(E < 4096 ? (E > 0 ? E : 1) : 4096); }

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

extern "C" int edge_time_batch(fn_ctx* c, const float* tree, int64_t ld, int32_t n_nodes,
                               const float* cand, int32_t B, const int32_t* nbr, int32_t k,
                               const fn_search* sr, const fn_obstacles* obs,
                               const fn_edge_out* out, void* stream) {
  if (!c || !sr || !out) return fail(FN_E_ARG, "edge_time_batch: NULL context, search or out");
  if (B < 0 || k < 1 || k > FN_MAX_K) return fail(FN_E_SHAPE, "edge_time_batch: B = %d, k = %d", B, k);
  const int64_t E = (int64_t)B * k;
  if (E > c->caps.max_edges) return fail(FN_E_SHAPE, "edge_time_batch: %lld edges (cap %lld)", (long long)E, (long long)c->caps.max_edges);
  if (n_nodes < 0) return fail(FN_E_SHAPE, "edge_time_batch: n_nodes = %d", n_nodes);
  if (sr->n_t < 1 || sr->n_t > FN_MAX_NT) return fail(FN_E_SHAPE, "edge_time_batch: n_t = %d (1..%d)", sr->n_t, FN_MAX_NT);
  if (sr->samples < 2 || sr->samples > FN_MAX_SAMPLES) return fail(FN_E_SHAPE, "edge_time_batch: S = %d (2..%d)", sr->samples, FN_MAX_SAMPLES);
  if (sr->mode < FN_SEARCH_PLAIN || sr->mode > FN_SEARCH_WINDOW) return fail(FN_E_ARG, "edge_time_batch: mode %d", sr->mode);
  if (sr->mode == FN_SEARCH_WINDOW && (!sr->win_lo || sr->win_half < 0)) return fail(FN_E_ARG, "edge_time_batch: window mode needs win_lo and win_half >= 0");
  int rc = check_obstacles(obs, "edge_time_batch");
  if (rc) return rc;
  if (E == 0) return FN_OK;
  if (!cand || !nbr || !sr->grid || !out->j || !out->status || !out->margin || (n_nodes > 0 && !tree))
    return fail(FN_E_ARG, "edge_time_batch: NULL array");
  if (ld < n_nodes) return fail(FN_E_ARG, "edge_time_batch: ld < n_nodes");
  EdgeArgs a;
  a.tree = tree; a.ld = ld; a.n_nodes = n_nodes; a.cand = cand; a.nbr = nbr; a.k = k; a.E = E;
  a.grid = sr->grid; a.n_t = sr->n_t; a.S = sr->samples; a.Sw = pow2_at_least(sr->samples);
  a.mode = sr->mode; a.win_half = sr->win_half; a.j_max = sr->j_max; a.win_lo = sr->win_lo;
  a.obs = obs ? obs->spheres : nullptr; a.n_obs = obs ? obs->n : 0; a.margin_c = obs ? obs->margin : 0.f;
  a.out_j = out->j; a.out_st = out->status; a.out_m = out->margin; a.out_rho = out->rho4;
  a.out_work = out->work; a.q_count = c->q_count; a.queue = c->queue;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, c->q_count, 1);
  const dim3 grid((unsigned)((E + 3) / 4));
  if (c->pattern == PAT_FR3) {
    hipLaunchKernelGGL(edge_time_kernel<PAT_FR3>, grid, dim3(256), 0, s, a, c->arm32);
    hipLaunchKernelGGL(edge_recheck_kernel<PAT_FR3>, dim3(recheck_waves(E)), dim3(64), 0, s, a, c->arm32, c->arm64);
  } else {
    hipLaunchKernelGGL(edge_time_kernel<PAT_GENERIC>, grid, dim3(256), 0, s, a, c->arm32);
    hipLaunchKernelGGL(edge_recheck_kernel<PAT_GENERIC>, dim3(recheck_waves(E)), dim3(64), 0, s, a, c->arm32, c->arm64);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "edge_time_batch launch");
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
  if (c->pattern == PAT_FR3)
    hipLaunchKernelGGL(edge_check_kernel<PAT_FR3>, grid, dim3(256), 0, s, x0, x1, T, E, S, ob, no, mg, c->arm32, out_status, out_rho5, out_tau);
  else
    hipLaunchKernelGGL(edge_check_kernel<PAT_GENERIC>, grid, dim3(256), 0, s, x0, x1, T, E, S, ob, no, mg, c->arm32, out_status, out_rho5, out_tau);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "edge_check launch");
}
