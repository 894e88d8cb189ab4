// fn_edge.h -- device side of the edge search: arguments, the per-edge
// search of one wavefront (minimum feasible time on the T grid, Def. 7,
// Algorithm 1; post-checks of Def. 6 rho_v, position limits and clearance of
// Sec. IV-E) and its FP64 stage.  Used by the single-problem kernels
// (fn_edge.hip) and the batched multi-problem kernels (fn_batch.hip).
//
// Search modes (same result, different work):
//  PLAIN  -- ascending passes over full slots, stop at the first feasible.
//  SCREEN -- first the two endpoint samples (u = 0, 1) of every slot, 64
//            slots per pass, from the endpoint models (the torque there is
//            affine in the acceleration, so a slot costs two 7x7 products
//            instead of two Newton-Euler passes); a slot whose endpoint
//            ratio exceeds 1 + BAND is infeasible for certain and never
//            evaluated in full.  Then full passes over the remaining slots
//            in ascending order.
//  WINDOW -- every slot is screened first, as in SCREEN; the surrogate's
//            window [lo, lo + 2h] then starts no lower than the first slot
//            the screen leaves open (slots below it are certified
//            infeasible, so no window needs them), and the open slots are
//            scanned below, inside and above the window in ascending order.
//            The work equals SCREEN's; "hit" = the result lies in the window
//            (or the network predicted no feasible slot and there is none).
// Every FP32 ratio within BAND of 1 that a decision rests on sends the edge
// to the FP64 stage.  At the first slot in the band the search does not
// stop: it goes on to the next candidate slot and post-checks both in FP32,
// so that the FP64 stage only has FP64 decisions left (see QEntry).
#pragma once

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
  const float* __restrict__ caps;  // obstacle capsules [n_caps][7] = (p0, p1, radius)
  int n_caps;
  int16_t* out_j;
  uint16_t* out_st;
  float* out_m;
  float* out_rho;
  int32_t* out_work;
  int16_t* out_scr;  // slots screened by the endpoint models, or NULL
  // endpoint models (MODEL_FLOATS each): of edge e's parent state at
  // model_e + e * MODEL_FLOATS, of candidate b at model_c + b * MODEL_FLOATS;
  // needed by the SCREEN and WINDOW modes
  float* model_e;
  float* model_c;
  int32_t* q_count;
  QEntry* queue;
  // batched problems: device node count (overrides n_nodes when set), and the
  // goal branch of Algorithm 1 -- candidates with kind 1 are checked once at
  // T = t_req[b] - t_node[parent] instead of searched
  const int32_t* __restrict__ n_nodes_dev;
  const int32_t* __restrict__ kind;
  const float* __restrict__ t_req;
  const float* __restrict__ t_node;
  float* out_T;  // duration of the result (grid slot or fixed T), or NULL
  // anytime loop (Algorithm 1): a free edge searches only the slots with
  // t(parent) + T <= *t_best; NULL: no bound
  const float* __restrict__ t_best;
  // two-phase screened search: each edge's number of open slots after the
  // triage (-1: finished by the triage); the ordered form's edge order and
  // per-block bin counts, the open-edge count at tri_hist[TRI_MAX_BLOCKS *
  // TRI_BINS]
  int32_t* tri_items;
  int32_t* tri_order;
  int32_t* tri_hist;
};

// ---------------------------------------------------------------------------
// Two-phase screened search.  The triage screens every slot of an edge with
// the endpoint models and finishes the edges on which it leaves no open
// slot (no feasible slot: the same outputs the one-kernel search writes for
// them); the search then runs on the other edges only.  About half of the
// one-iteration shape's edges end at the triage.
// ---------------------------------------------------------------------------
// default form 3 from this many edges (measured faster than forms 1 and 2 at
// 32,768 and 1,048,576 edges), form 1 below
constexpr int64_t TRIAGE_MIN_EDGES = 1 << 15;
// The ordered form's counting sort (fn_edge.hip): per-block bin counts of
// the open-slot counts, then each open edge's place in the order.
__global__ void tri_hist_kernel(const int32_t* __restrict__ items, int64_t E, int64_t chunk,
                                int n_t, int32_t* __restrict__ hist);
__global__ void tri_scatter_kernel(const int32_t* __restrict__ items, int64_t E, int64_t chunk,
                                   int n_t, const int32_t* __restrict__ hist, int nblk,
                                   int32_t* __restrict__ order, int32_t* __restrict__ n_open);
__device__ __forceinline__ int nodes_of(const EdgeArgs& a) {
  return a.n_nodes_dev ? *a.n_nodes_dev : a.n_nodes;
}

// Largest slot j <= jmax with t(parent) + Tg[j] <= t_best in FP32 (the sums
// grow with j), -1 when there is none; jmax unchanged without a bound.
// Edge e's parent index must be valid.
__device__ __forceinline__ int bound_slots(const EdgeArgs& a, int64_t e, const float* Tg,
                                           int jmax) {
  if (!a.t_best) return jmax;
  const float tb = *a.t_best;
  const float tp = a.t_node[a.nbr[e]];
  int lo = -1, hi = jmax;  // slot lo passes (or -1); slots above hi fail
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tp + Tg[mid] <= tb) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// queue phase bits
constexpr int PH_POST = 1;        // only the post-checks are left
constexpr int PH_BELOW_FULL = 2;  // window mode: a slot below the window was evaluated in full
constexpr int PH_J2_NEAR = 4;     // slot j2 is within the band too

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
  if (p >= nodes_of(a)) {
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

// The obstacles an edge is checked against (Sec. IV-E): spheres [n_obs][4]
// = (centre, radius) and capsules [n_caps][7] = (segment ends p0, p1,
// radius), with the clearance margin.
struct World {
  const float* __restrict__ obs;
  int n_obs;
  const float* __restrict__ caps;
  int n_caps;
  float margin;
};
__host__ __device__ __forceinline__ int world_size(const World& w) { return w.n_obs + w.n_caps; }

// LDS of one wavefront for the clearance check: every sphere as (x, y, z
// in its link frame, radius + margin), every obstacle sphere as (x, y, z,
// radius), every capsule as (p0, p1 - p0, 1 / |p1 - p0|^2, radius).
template <typename R>
struct GeoLDS {
  R sph[4 * FN_MAX_SPHERES];
  R obs[4 * FN_MAX_OBS];
  R caps[8 * FN_MAX_CAPS];
};

// Velocity taper (Def. 6 rho_v) and position limits at duration T: lane
// 8 i + p evaluates candidate extremum p of joint i (joint_point), and the
// wave maxima give (rho_v, rho_q) in every lane.
template <typename R>
__device__ void joint_checks(const ArmConst<R>& A, const EdgeState<R>& E, R T, R& rv, R& rq) {
  const int lane = lane_id();
  const int ji = lane >> 3, p = lane & 7;
  R v = 0, q = 0;
  // register selects keep the edge state in VGPRs
  R q0 = 0, qd0 = 0, dq = 0, d2v = 0;
#pragma unroll
  for (int i = 0; i < NJ; ++i)
    if (ji == i) {
      q0 = E.q0[i];
      qd0 = E.qd0[i];
      dq = E.dq[i];
      d2v = E.d2[i];
    }
  if (ji < NJ) joint_point(A, ji, p, q0, qd0, dq, d2v, T, v, q);
  rv = wave_max(v);
  rq = wave_max(q);
}

// Clearance (Sec. IV-E) at duration T: rho_c = max over samples, arm spheres
// and obstacles of (r_a + margin + r_o) / distance, in every lane; the
// distance to a capsule is the distance to its segment.  The sphere and
// obstacle tables are staged in LDS first, so the (sphere, obstacle) loops
// read broadcast LDS instead of waiting on a memory load per pair.  Lane =
// (sample, sphere part): the parts split each link's spheres so that all 64
// lanes work when S < 64; above 64 samples the lanes take them in chunks.
// tab (LDS, nsph * (n_obs + n_caps) values) receives 1 / (r_a + margin +
// r_o)^2 of every (sphere, obstacle) pair (FP32: hardware reciprocal, within
// 1 ulp; FP64: IEEE division), and the loops keep the smallest d^2 / (r_a +
// margin + r_o)^2 (a product and a minimum per pair instead of a division);
// rho_c is its inverse square root.
template <typename R, int PAT>
__device__ void clearance(const ArmConst<R>& A, const EdgeState<R>& E, R T, int S, const World& w,
                          GeoLDS<R>* geo, R* tab, R& rc) {
  constexpr bool F32 = sizeof(R) == 4;
  const int lane = lane_id();
  const int n_obs = w.n_obs, n_caps = w.n_caps, nt = n_obs + n_caps;
  for (int t = lane; t < A.nsph; t += WAVE) {
    geo->sph[4 * t] = A.sphx[t];
    geo->sph[4 * t + 1] = A.sphy[t];
    geo->sph[4 * t + 2] = A.sphz[t];
    geo->sph[4 * t + 3] = A.sphr[t] + R(w.margin);
  }
  for (int t = lane; t < 4 * n_obs; t += WAVE) geo->obs[t] = R(w.obs[t]);
  for (int t = lane; t < n_caps; t += WAVE) {
    const float* c = w.caps + 7 * t;
    const R dx = R(c[3]) - R(c[0]), dy = R(c[4]) - R(c[1]), dz = R(c[5]) - R(c[2]);
    const R dd = dx * dx + dy * dy + dz * dz;
    R* g = geo->caps + 8 * t;
    g[0] = R(c[0]);
    g[1] = R(c[1]);
    g[2] = R(c[2]);
    g[3] = dx;
    g[4] = dy;
    g[5] = dz;
    if constexpr (F32) g[6] = dd > 0.f ? __builtin_amdgcn_rcpf(dd) : 0.f;
    else g[6] = dd > 0.0 ? 1.0 / dd : 0.0;
    g[7] = R(c[6]);
  }
  __builtin_amdgcn_wave_barrier();
  {
    // 1 / need^2 per (sphere, obstacle) pair: the hardware reciprocal in
    // FP32, an IEEE division in FP64; lane = (obstacle o, sphere offset k0),
    // WAVE / nt spheres per step
    const int kstep = WAVE / nt, o = lane % nt, k0 = lane / nt;
    if (k0 < kstep)
      for (int k = k0; k < A.nsph; k += kstep) {
        const R need = geo->sph[4 * k + 3] + (o < n_obs ? geo->obs[4 * o + 3]
                                                          : geo->caps[8 * (o - n_obs) + 7]);
        if constexpr (F32) tab[k * nt + o] = __builtin_amdgcn_rcpf(need * need);
        else tab[k * nt + o] = R(1) / (need * need);
      }
    __builtin_amdgcn_wave_barrier();
  }
  // smallest d^2 / need^2 over the (sample, sphere, obstacle) triples
  R best = R(INFINITY);
  int Sw = 1;
  while (Sw < S) Sw <<= 1;
  const int nparts = Sw >= WAVE ? 1 : WAVE / Sw;
  const int part = Sw >= WAVE ? 0 : lane / Sw;
  for (int s0 = 0; s0 < S; s0 += (Sw >= WAVE ? WAVE : S)) {
    const int s = Sw >= WAVE ? s0 + lane : (lane & (Sw - 1));
    if (s < S && part < nparts) {
      const R u = R(s) / R(S - 1);
      R sg[NJ], sd[NJ], sdd[NJ], sn[NJ], cs[NJ];
      cubic_point(E, T, R(1) / T, u, sg, sd, sdd);
#pragma unroll
      for (int i = 0; i < NJ; ++i) sincos_r(sg[i], sn[i], cs[i]);
      const R* so = geo->obs;
      const R* sc = geo->caps;
      sphere_centres<R, PAT>(A, sn, cs, part, nparts, geo->sph, [&](int k, R x, R y, R z) {
        const R* tk = tab + k * nt;
#pragma unroll 4
        for (int o = 0; o < n_obs; ++o) {
          const R dx = x - so[4 * o], dy = y - so[4 * o + 1], dz = z - so[4 * o + 2];
          const R d2 = dx * dx + dy * dy + dz * dz;
          if constexpr (F32) best = fminf(best, d2 * tk[o]);
          else best = fmin(best, d2 * tk[o]);
        }
        for (int o = 0; o < n_caps; ++o) {
          // closest point of the segment: the projection clamped to [0, 1]
          const R* g = sc + 8 * o;
          const R wx = x - g[0], wy = y - g[1], wz = z - g[2];
          R t = (wx * g[3] + wy * g[4] + wz * g[5]) * g[6];
          t = t < R(0) ? R(0) : (t > R(1) ? R(1) : t);
          const R ex = wx - t * g[3], ey = wy - t * g[4], ez = wz - t * g[5];
          const R d2 = ex * ex + ey * ey + ez * ez;
          if constexpr (F32) best = fminf(best, d2 * tk[n_obs + o]);
          else best = fmin(best, d2 * tk[n_obs + o]);
        }
      });
    }
  }
  // d2 = 0 gives rho_c = +inf; no pair (no spheres) gives 0
  const R mn = wave_min(best);
  rc = mn < R(INFINITY) ? R(1) / sqrt(mn) : R(0);
  __builtin_amdgcn_wave_barrier();
}

// Post-checks at duration T: (rho_v, rho_q, rho_c) in every lane.  Alg. 1
// and-s the clearance into the edge's flag after the limit checks, so rho_c
// is evaluated only when rho_v and rho_q are at most `pass` (1 in FP64;
// 1 + BAND in FP32, where a ratio in the band is decided later in FP64) and
// is NaN (not evaluated) otherwise; 0 without obstacles.  tab: LDS for the
// FP32 clearance (nsph * (n_obs + n_caps) floats).
template <typename R, int PAT>
__device__ void post_checks(const ArmConst<R>& A, const EdgeState<R>& E, R T, int S,
                            const World& w, GeoLDS<R>* geo, float* tab, R pass, R& rv, R& rq,
                            R& rc) {
  joint_checks<R>(A, E, T, rv, rq);
  rc = R(NAN);
  if (rv <= pass && rq <= pass) {
    rc = R(0);
    if (world_size(w) > 0) clearance<R, PAT>(A, E, T, S, w, geo, tab, rc);
  }
}

// The obstacles of an edge launch.
__device__ __forceinline__ World world_of(const EdgeArgs& a) {
  return World{a.obs, a.n_obs, a.caps, a.n_caps, a.margin_c};
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
                                          float r0, float r1, float r2, float r3, int work,
                                          float T = 0.f) {
  if (lane_id() == 0) {
    if (a.out_T) a.out_T[e] = j >= 0 ? T : 0.f;
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

// Hands edge e over to the FP64 stage (see QEntry).
__device__ __forceinline__ void push_queue(const EdgeArgs& a, int64_t e, int j, int phase, int j2,
                                           float m, float m2, int work, float rho, float rho2,
                                           float v1, float q1, float c1, float v2, float q2,
                                           float c2, const SlotMask& todo, int wlo) {
  if (lane_id() == 0) {
    const int slot = atomicAdd(a.q_count, 1);
    QEntry q;
    q.edge = (int32_t)e;
    q.j = (int16_t)j;
    q.phase = (int16_t)phase;
    q.j2 = (int16_t)j2;
    q.wlo = (int16_t)wlo;
    q.work = work;
    q.margin = m;
    q.margin2 = m2;
    q.rho = rho;
    q.rho2 = rho2;
    q.post[0] = v1;
    q.post[1] = q1;
    q.post[2] = c1;
    q.post[3] = v2;
    q.post[4] = q2;
    q.post[5] = c2;
    q.pad2[0] = q.pad2[1] = 0;
    q.todo[0] = todo.w0;
    q.todo[1] = todo.w1;
    q.todo[2] = todo.w2;
    q.todo[3] = todo.w3;
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
//   WINDOW: screen [0, jmax], scan [0, lo-1], scan [lo, hi], scan [hi+1, jmax]
//           (lo raised to the first open slot once the screen is done)
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
      case 0: type = ST_SCREEN; a = 0; b = jmax; break;
      case 1: type = ST_SCAN; a = 0; b = lo - 1; below = true; break;
      case 2: type = ST_SCAN; a = lo; b = hi; break;
      case 3: type = ST_SCAN; a = hi + 1; b = jmax; break;
      default: break;
    }
  }
}

// Edges (wavefronts) per workgroup of the search kernels.
constexpr int EDGE_WAVES = 1;
// Largest grid of the FP64 stage (one wavefront per SIMD of the chip).
constexpr int RECHECK_WAVES = 1024;

// XCD-aware order of the search grid.  Workgroups are dealt to the 8 XCDs
// in turn (workgroup w runs on XCD w mod 8), so consecutive edges land on
// different L2s.  Workgroup w takes edge i of candidate b with
// b = 8 ((w div 8) div k) + w mod 8 and i = (w div 8) mod k: all k edges of a
// candidate run on one XCD, which then fetches the candidate's state and
// endpoint model once.  The grid has ceil(B / 8) 8 k workgroups; the ones
// past the last candidate return.  Returns -1 for those.
constexpr int N_XCD = 8;
__device__ __forceinline__ int64_t xcd_edge(int64_t w, int k, int64_t B) {
  static_assert(EDGE_WAVES == 1, "one edge per workgroup");
  const int64_t s = w / N_XCD;
  const int64_t b = (s / k) * N_XCD + (w % N_XCD);
  return b < B ? b * k + s % k : -1;
}
__host__ __forceinline__ int64_t xcd_grid(int64_t B, int k) {
  return (B + N_XCD - 1) / N_XCD * N_XCD * k;
}

// Fixed duration of a goal edge (Algorithm 1 goal branch): t_req of the
// candidate minus the parent's time-to-come.  Returns false for a free edge.
__device__ __forceinline__ bool fixed_T(const EdgeArgs& a, int64_t e, float& T) {
  if (!a.kind) return false;
  const int64_t b = e / a.k;
  if (a.kind[b] != 1) return false;
  const int p = a.nbr[e];
  T = a.t_req[b] - a.t_node[p];
  return true;
}

// Endpoint model of one state of an edge launch (8 lanes per state, lane
// `role`): st < E is the parent of edge st, st = E + b is candidate b.
// States that no screen reads are skipped: padded or invalid parents and
// goal candidates (their edges are checked at one fixed duration).
template <int PAT>
__device__ __forceinline__ void model_state(const EdgeArgs& a, int64_t st, int role,
                                            const ArmConst<float>& A) {
  float q[NJ], qd[NJ];
  float* dst;
  if (st < a.E) {
    const int64_t b = st / a.k;
    if (a.kind && a.kind[b] == 1) return;
    const int p = a.nbr[st];
    if (p < 0 || p >= nodes_of(a)) return;
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      q[i] = a.tree[(size_t)i * a.ld + p];
      qd[i] = a.tree[(size_t)(NJ + i) * a.ld + p];
    }
    dst = a.model_e + st * MODEL_FLOATS;
  } else {
    const int64_t b = st - a.E;
    if (a.kind && a.kind[b] == 1) return;
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      q[i] = a.cand[b * FN_STATE + i];
      qd[i] = a.cand[b * FN_STATE + NJ + i];
    }
    dst = a.model_c + b * MODEL_FLOATS;
  }
  float out[NJ];
  model_lane<float, PAT>(A, q, qd, role, out);
#pragma unroll
  for (int i = 0; i < NJ; ++i) dst[NJ * role + i] = out[i];
}

// The search of one edge by one wavefront (see the stage list above).
// eq: the edge's id in the FP64-stage queue; s_end: this wavefront's
// FN_MAX_NT floats of LDS; s_T: the grid in LDS; s_fix: four floats of LDS;
// s_mod: SCREEN_FLOATS floats of LDS; geo, tab: the clearance tables (LDS;
// tab: nsph * n_obs floats).
// MODE is the search mode (a
// compile-time constant, so each mode is its own kernel); GOALS: edges of
// goal candidates (kind 1) are checked at their fixed duration.
// Inlined into each kernel: a call would spill the live state of the search
// to a stack frame of ~600 bytes per lane.
template <int PAT, int MODE, bool GOALS>
__device__ __forceinline__ void search_edge(const EdgeArgs& a, int64_t e, int64_t eq,
                                            const ArmConst<float>& A,
                            float* s_end, const float* s_T, float* s_fix, float* s_mod,
                            GeoLDS<float>* geo, float* tab) {
  const int lane = lane_id();
  if (a.out_scr && lane == 0) a.out_scr[e] = 0;
  EdgeState<float> ES;
  int st0;
  if (!load_edge(a, e, ES, st0)) {
    write_out(a, e, -1, st0, st0 == FN_S_NO_PARENT ? INFINITY : 0.f, 0, 0, 0, 0, 0);
    return;
  }
  // goal edges: one slot at the fixed duration
  float Tfix;
  const bool fixed = GOALS && fixed_T(a, e, Tfix);
  const float* Tg = s_T;
  int n_t = a.n_t, mode = MODE;
  if (fixed) {
    if (!isfinite(Tfix)) {
      write_out(a, e, -1, FN_S_BAD_INPUT, 0.f, 0, 0, 0, 0, 0);
      return;
    }
    if (!(Tfix > 0.f)) {
      write_out(a, e, -1, FN_S_NONE, INFINITY, 0, 0, 0, 0, 0);
      return;
    }
    if (lane == 0) s_fix[0] = Tfix;
    __builtin_amdgcn_wave_barrier();
    Tg = s_fix;
    n_t = 1;
    mode = FN_SEARCH_PLAIN;
  }
  int jmax = n_t - 1;
  if (a.j_max && !fixed) jmax = min(jmax, (int)a.j_max[e]);
  if (!fixed) jmax = bound_slots(a, e, Tg, jmax);
  if (jmax < 0) {
    // no slot to search: the window is empty and so is the result (a hit)
    write_out(a, e, -1, FN_S_NONE | (mode == FN_SEARCH_WINDOW ? FN_S_WIN_HIT : 0), INFINITY, 0,
              0, 0, 0, 0);
    return;
  }
  const int S = a.S, Sw = a.Sw, G = WAVE / Sw;
  const int g = lane / Sw;
  const float u_full = lane_u(lane, Sw, S);
  const bool s_ok = (lane & (Sw - 1)) < S;

  for (int j = lane; j < n_t; j += WAVE) s_end[j] = -1.f;  // -1: not screened
  if (mode != FN_SEARCH_PLAIN && lane < MODEL_FLOATS) {
    s_mod[lane] = a.model_e[e * MODEL_FLOATS + lane];
    s_mod[MODEL_FLOATS + lane] = a.model_c[(e / a.k) * MODEL_FLOATS + lane];
  }
  __builtin_amdgcn_wave_barrier();
  if (mode != FN_SEARCH_PLAIN) {
    endpoint_table(lane, ES, s_mod, s_mod + MODEL_FLOATS, s_mod + 2 * MODEL_FLOATS);
    __builtin_amdgcn_wave_barrier();
  }
  SlotMask todo{~0ull, ~0ull, ~0ull, ~0ull};

  int wlo = 0, whi = -1;
  if (mode == FN_SEARCH_WINDOW) {
    wlo = min(max((int)a.win_lo[e], 0), jmax + 1);
    whi = min(wlo + 2 * a.win_half, jmax);
  }

  int work = 0, scr = 0;
  float marg = INFINITY;  // over fully evaluated slots up to the result
  float last = 0.f;
  int jstar = -1;
  float rho_star = 0.f;
  bool below_full = false;
  // the first slot whose FP32 ratio is within the band is decided in FP64 by
  // the next stage, and the search goes on above it in case it is
  // infeasible; that slot, its ratio and the margin below it wait in LDS
  // (s_fix[1..3]; rarely used, so they hold no registers in the loop)
  if (lane == 0) s_fix[1] = __int_as_float(-1);

  int stage = 0, type, sa, sb;
  bool below;
  stage_of(mode, stage, jmax, wlo, whi, type, sa, sb, below);
  int j = sa;
  while (type != ST_END) {
    if (j > sb) {
      if (mode == FN_SEARCH_WINDOW && stage == 0) {
        // every slot is screened: the window starts no lower than the first
        // slot the screen leaves open
        const int f0 = todo.next(0, jmax);
        wlo = max(wlo, f0 < 0 ? jmax + 1 : f0);
        whi = min(wlo + 2 * a.win_half, jmax);
      }
      ++stage;
      stage_of(mode, stage, jmax, wlo, whi, type, sa, sb, below);
      j = sa;
      continue;
    }
    // lanes of this pass: slot `my` (or -1) and normalised time u
    int my = -1, cnt = 0;
    float u = u_full;
    if (type == ST_SCREEN) {
      // lane l: slot j + l, both endpoints from the models
      const int j0 = j;
      const int jj = j + lane;
      my = jj <= sb ? jj : -1;
      j += WAVE;
      const bool act = my >= 0;
      float r = 0.f;
      if (act) {
        const float T = Tg[my];
        r = endpoint_ratio(A, ES, s_mod, s_mod + MODEL_FLOATS, s_mod + 2 * MODEL_FLOATS,
                           __builtin_amdgcn_rcpf(T));
        s_end[my] = r;
      }
      scr += __popcll(__ballot(act));
      // slots certified infeasible leave the to-do mask: bit t of the ballot
      // is slot j0 + t, and the pass may straddle two 64-slot words
      const uint64_t bits = __ballot(act && r > 1.f + BAND);
      const int w0 = j0 >> 6, sh = j0 & 63;
      todo.clear(w0, bits << sh);
      if (sh > 0 && w0 < 3) todo.clear(w0 + 1, bits >> (64 - sh));
      continue;
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
      const float T = Tg[my];
      r = eval_rho<float, PAT>(A, ES, T, __builtin_amdgcn_rcpf(T), u);
    }
    work += __popcll(__ballot(act));
    // the plain search is bound by VALU issue: its group maxima go through
    // the LDS; the screened searches are latency-bound: DPP
    r = MODE == FN_SEARCH_PLAIN ? group_max_lds(r, Sw) : group_max(r, Sw);
    bool done = false;
    for (int q = 0; q < cnt; ++q) {
      // lane q * Sw holds group q's slot and ratio (a scalar read, no LDS)
      const float rho = readlane(r, q * Sw);
      const int jq = __builtin_amdgcn_readlane(my, q * Sw);
      if (near_one(rho)) {
        __builtin_amdgcn_wave_barrier();
        if (__builtin_amdgcn_readfirstlane(__float_as_int(s_fix[1])) >= 0) {
          // a second slot within the band ends the FP32 search
          jstar = jq;
          rho_star = rho;
          done = true;
          break;
        }
        float m = INFINITY;
        for (int t = lane; t < jq; t += WAVE)
          if (s_end[t] > 1.f + BAND) m = fminf(m, s_end[t] - 1.f);
        m = fminf(marg, wave_min(m));
        if (lane == 0) {
          s_fix[1] = __int_as_float(jq);
          s_fix[2] = rho;
          s_fix[3] = m;
        }
        __builtin_amdgcn_wave_barrier();
        marg = INFINITY;  // from here: the slots above it
        continue;
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
  if (a.out_scr && lane == 0) a.out_scr[e] = (int16_t)scr;
  __builtin_amdgcn_wave_barrier();
  const int jn = __builtin_amdgcn_readfirstlane(__float_as_int(s_fix[1]));
  // certified-infeasible margin of the screened slots below the result
  // (above jn when a slot within the band was met)
  const int lim = jstar >= 0 ? jstar : jmax + 1;
  float mc = INFINITY;
  for (int t = jn + 1 + lane; t < lim; t += WAVE)
    if (s_end[t] > 1.f + BAND) mc = fminf(mc, s_end[t] - 1.f);
  float m = fminf(marg, wave_min(mc));
  int winbits = 0;
  if (mode == FN_SEARCH_WINDOW) {
    // hit: the result lies in the predicted window (or none was predicted
    // and none exists); BELOW: a slot under the window needed a full pass
    const bool hit = (jstar >= 0 && jstar >= wlo && jstar <= whi) || (jstar < 0 && wlo > jmax);
    winbits = (hit ? FN_S_WIN_HIT : FN_S_WIN_MISS) | (below_full ? FN_S_WIN_BELOW : 0);
  }
  // ratio of the last slot: its full value, else its screened endpoint value
  const float lastv = jstar < 0 && s_end[jmax] > 1.f + BAND ? s_end[jmax] : last;
  if (jstar < 0 && jn < 0) {
    write_out(a, e, -1, FN_S_NONE | winbits, m, lastv, 0, 0, 0, work);
    return;
  }
  // FP32 post-checks at jn (the result if FP64 finds it feasible) and at
  // jstar (one call site; plain registers, no array, so nothing goes to
  // scratch memory)
  float v1 = 0.f, q1 = 0.f, c1 = 0.f, rv = 0.f, rq = 0.f, rc = 0.f;
#pragma unroll 1
  for (int pass = jn >= 0 ? 0 : 1; pass < 2; ++pass) {
    const int js = pass == 0 ? jn : jstar;
    if (js < 0) break;
    float pv, pq, pc;
    post_checks<float, PAT>(A, ES, Tg[js], S, world_of(a), geo, tab, 1.f + BAND, pv, pq, pc);
    if (pass == 0) {
      v1 = pv; q1 = pq; c1 = pc;
    } else {
      rv = pv; rq = pq; rc = pc;
    }
  }
  const int ph_b = below_full ? PH_BELOW_FULL : 0;
  if (jn >= 0) {
    const bool j2near = jstar >= 0 && near_one(rho_star);
    push_queue(a, eq, jn, ph_b | (j2near ? PH_J2_NEAR : 0), jstar, s_fix[3], m, work, s_fix[2],
               jstar >= 0 ? rho_star : lastv, v1, q1, c1, rv, rq, rc, todo, wlo);
    return;
  }
  if (near_one(rv) || near_one(rq) || (a.n_obs + a.n_caps > 0 && near_one(rc))) {
    push_queue(a, eq, jstar, PH_POST | ph_b, -1, m, INFINITY, work, rho_star, 0.f, rv, rq, rc, 0.f,
               0.f, 0.f, todo, wlo);
    return;
  }
  m = fminf(m, fminf(fabsf(rv - 1.f), fminf(fabsf(rq - 1.f), fabsf(rc - 1.f))));
  write_out(a, e, jstar, post_status(rv, rq, rc) | winbits, m, rho_star, rv, rq, rc, work,
            Tg[jstar]);
}

// Triage (two-phase screened search): the screen of search_edge over every
// slot up to jmax of one edge whose parent index p, states x (parent 14
// floats, candidate 14 floats) and endpoint models are in LDS; with no open
// slot the edge is finished exactly as search_edge finishes it (count -1),
// else its open-slot count is recorded.  The parent checks and the
// state differences are load_edge's.
template <int PAT, int MODE>
__device__ void triage_one(const EdgeArgs& a, int64_t e, int p, const ArmConst<float>& A,
                           const float* s_T, float* s_mod, const float* x) {
  const int lane = lane_id();
  if (lane == 0) a.tri_items[e] = -1;
  int st0 = p < 0 ? FN_S_NO_PARENT : p >= nodes_of(a) ? FN_S_BAD_INPUT : 0;
  EdgeState<float> ES;
  if (st0 == 0) {
    bool finite = true;
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      const float q0 = x[i], v0 = x[NJ + i], q1 = x[FN_STATE + i], v1 = x[FN_STATE + NJ + i];
      finite = finite && isfinite(q0) && isfinite(v0) && isfinite(q1) && isfinite(v1);
      ES.q0[i] = q0;
      ES.qd0[i] = v0;
      ES.dq[i] = q1 - q0;
      ES.d2[i] = v1 - v0;
    }
    if (!finite) st0 = FN_S_BAD_INPUT;
  }
  if (st0 != 0) {
    if (a.out_scr && lane == 0) a.out_scr[e] = 0;
    write_out(a, e, -1, st0, st0 == FN_S_NO_PARENT ? INFINITY : 0.f, 0, 0, 0, 0, 0);
    return;
  }
  int jmax = a.n_t - 1;
  if (a.j_max) jmax = min(jmax, (int)a.j_max[e]);
  jmax = bound_slots(a, e, s_T, jmax);
  if (jmax < 0) {
    if (a.out_scr && lane == 0) a.out_scr[e] = 0;
    write_out(a, e, -1, FN_S_NONE | (MODE == FN_SEARCH_WINDOW ? FN_S_WIN_HIT : 0), INFINITY, 0,
              0, 0, 0, 0);
    return;
  }
  endpoint_table(lane, ES, s_mod, s_mod + MODEL_FLOATS, s_mod + 2 * MODEL_FLOATS);
  __builtin_amdgcn_wave_barrier();
  int open = 0;
  float mc = INFINITY, lastv = 0.f;
  for (int j0 = 0; j0 <= jmax; j0 += WAVE) {
    const int jj = j0 + lane;
    const bool act = jj <= jmax;
    float r = 0.f;
    if (act) {
      const float T = s_T[jj];
      r = endpoint_ratio(A, ES, s_mod, s_mod + MODEL_FLOATS, s_mod + 2 * MODEL_FLOATS,
                         __builtin_amdgcn_rcpf(T));
    }
    const bool cert = act && r > 1.f + BAND;
    open += __popcll(__ballot(act && !cert));
    if (cert) mc = fminf(mc, r - 1.f);
    if (jj == jmax) lastv = r;
  }
  if (open == 0) {
    const float m = wave_min(mc);
    const float lv = readlane(lastv, jmax & (WAVE - 1));
    if (a.out_scr && lane == 0) a.out_scr[e] = (int16_t)(jmax + 1);
    write_out(a, e, -1, FN_S_NONE | (MODE == FN_SEARCH_WINDOW ? FN_S_WIN_HIT : 0), m, lv, 0, 0,
              0, 0);
    return;
  }
  if (lane == 0) a.tri_items[e] = open;
}

// Triage of one edge by one wavefront: parent index, states and endpoint
// models into LDS (s_mod: SCREEN_FLOATS floats, s_x: 2 * FN_STATE
// floats), then triage_one.
template <int PAT, int MODE>
__device__ void triage_edge(const EdgeArgs& a, int64_t e, const ArmConst<float>& A,
                            const float* s_T, float* s_mod, float* s_x) {
  const int lane = lane_id();
  const int p = a.nbr[e];
  const int64_t b = e / a.k;
  if (lane < MODEL_FLOATS) {
    s_mod[lane] = a.model_e[e * MODEL_FLOATS + lane];
    s_mod[MODEL_FLOATS + lane] = a.model_c[b * MODEL_FLOATS + lane];
  }
  if (lane < FN_STATE) {
    s_x[FN_STATE + lane] = a.cand[b * FN_STATE + lane];
    if (p >= 0 && p < nodes_of(a)) s_x[lane] = a.tree[(size_t)lane * a.ld + p];
  }
  __builtin_amdgcn_wave_barrier();
  triage_one<PAT, MODE>(a, e, p, A, s_T, s_mod, s_x);
}

// Slot ratio of Eq. (7) in FP64 at the S samples (lanes < S), in every lane.
template <int PAT>
__device__ __forceinline__ double rho64(const ArmConst<double>& D, const EdgeState<double>& ED,
                                        float Tf, int S) {
  const int lane = lane_id();
  const double T = (double)Tf;
  double r = 0.0;
  if (lane < S) r = eval_rho<double, PAT>(D, ED, T, 1.0 / T, double(lane) / double(S - 1));
  return wave_max(r);
}

// FP64 stage of one queued edge (one wavefront; FP64 arithmetic only, see
// QEntry).  Phase 0: slot j is decided in FP64; if it is infeasible the
// result is j2 (decided in FP64 too when it is within the band), and in the
// rare case that j2 fails as well the search goes on over the uncertified
// slots above it in FP64.  Post-check ratios within the band of 1 are
// recomputed in FP64 (all of them after the FP64 walk).
template <int PAT>
__device__ void recheck_edge(const EdgeArgs& a, int64_t e, const QEntry& q,
                             const ArmConst<double>& D, float* s_fix, GeoLDS<double>* geo,
                             double* tab) {
  const int lane = lane_id();
  EdgeState<double> ED;
  int st0;
  load_edge(a, e, ED, st0);
  float Tfix;
  const bool fixed = fixed_T(a, e, Tfix);
  if (fixed && lane == 0) s_fix[0] = Tfix;
  __builtin_amdgcn_wave_barrier();
  const float* Tg = fixed ? s_fix : a.grid;
  int jmax = fixed ? 0 : a.n_t - 1;
  if (a.j_max && !fixed) jmax = min(jmax, (int)a.j_max[e]);
  if (!fixed) jmax = bound_slots(a, e, Tg, jmax);
  const int S = a.S;
  int work = q.work;
  float m = q.margin;
  int jstar = -1;
  float rho_star = 0.f, last = 0.f;
  // post-check ratios at the result: the search's FP32 values, or FP64
  // values after the FP64 walk (exact)
  double rv = 0.0, rq = 0.0, rc = 0.0;
  bool exact = false;
  int pick = -1;  // which FP32 post-check triple applies: 0 (slot j), 3 (slot j2)
  if (q.phase & PH_POST) {
    jstar = q.j;
    rho_star = q.rho;  // outside the band: the FP32 value stands
    pick = 0;
  } else {
    const double r0 = rho64<PAT>(D, ED, Tg[q.j], S);
    m = fminf(m, (float)fabs(r0 - 1.0));
    if (r0 <= 1.0) {
      jstar = q.j;
      rho_star = (float)r0;
      pick = 0;
    } else {
      m = fminf(m, q.margin2);
      if (q.j2 < 0) {
        last = q.j == jmax ? (float)r0 : q.rho2;
      } else if (!(q.phase & PH_J2_NEAR)) {
        jstar = q.j2;
        rho_star = q.rho2;
        pick = 3;
      } else {
        const double r2 = rho64<PAT>(D, ED, Tg[q.j2], S);
        m = fminf(m, (float)fabs(r2 - 1.0));
        last = (float)r2;
        if (r2 <= 1.0) {
          jstar = q.j2;
          rho_star = (float)r2;
          pick = 3;
        } else {
          const SlotMask todo{q.todo[0], q.todo[1], q.todo[2], q.todo[3]};
          int lastj = q.j2;
          for (int t = todo.next(q.j2 + 1, jmax); t >= 0; t = todo.next(t + 1, jmax)) {
            const double rd = rho64<PAT>(D, ED, Tg[t], S);
            work += S;
            m = fminf(m, (float)fabs(rd - 1.0));
            last = (float)rd;
            lastj = t;
            if (rd <= 1.0) {
              jstar = t;
              rho_star = (float)rd;
              exact = true;
              break;
            }
          }
          // the last slot was certified: report its ratio
          if (jstar < 0 && lastj != jmax) last = (float)rho64<PAT>(D, ED, Tg[jmax], S);
        }
      }
    }
  }
  int winbits = 0;
  if (a.mode == FN_SEARCH_WINDOW && !fixed) {
    const int wlo = q.wlo;  // raised to the first open slot by the search
    const int whi = min(wlo + 2 * a.win_half, jmax);
    const bool below = (q.phase & PH_BELOW_FULL) != 0;
    const bool hit = (jstar >= 0 && jstar >= wlo && jstar <= whi) || (jstar < 0 && wlo > jmax);
    winbits = (hit ? FN_S_WIN_HIT : FN_S_WIN_MISS) | (below ? FN_S_WIN_BELOW : 0);
  }
  if (jstar < 0) {
    write_out(a, e, -1, FN_S_NONE | FN_S_RECHECK64 | winbits, m, last, 0, 0, 0, work);
    return;
  }
  if (pick >= 0) {
    rv = q.post[pick];
    rq = q.post[pick + 1];
    rc = q.post[pick + 2];
  }
  // limit ratios within the band of 1 (all, after the FP64 walk) in FP64
  const bool nv = exact || near_one((float)rv), nq = exact || near_one((float)rq);
  const double T = (double)Tg[jstar];
  if (nv || nq) {
    double dv, dq;
    joint_checks<double>(D, ED, T, dv, dq);
    if (nv) rv = dv;
    if (nq) rq = dq;
  }
  // clearance only for an edge that passes the limit checks (Alg. 1); in
  // FP64 when its FP32 value is in the band or missing, or after the walk
  if (rv > 1.0 || rq > 1.0) rc = NAN;
  else if (a.n_obs + a.n_caps == 0) rc = 0.0;
  else if (exact || isnan(rc) || near_one((float)rc))
    clearance<double, PAT>(D, ED, T, S, world_of(a), geo, tab, rc);
  m = fminf(m, (float)fmin(fabs(rv - 1.0), fmin(fabs(rq - 1.0), fabs(rc - 1.0))));
  write_out(a, e, jstar, post_status(rv, rq, rc) | FN_S_RECHECK64 | winbits, m, rho_star,
            (float)rv, (float)rq, (float)rc, work, Tg[jstar]);
}

// Several problems in one launch: edge ranges per problem (prefix offsets,
// n + 1 entries) and each problem's arguments, on the device.
struct ProbTable {
  int n;
  const int64_t* __restrict__ edge_off;
  const EdgeArgs* __restrict__ args;
};

// problem of a global edge id (binary search over the offsets)
__device__ __forceinline__ int problem_of(const ProbTable& pt, int64_t eg) {
  int lo = 0, hi = pt.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pt.edge_off[mid] <= eg) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// FP64 stage over the queue; pt.n == 0: one problem (a).  Dynamic LDS: the
// clearance table, nsph * (largest obstacle count) doubles.
template <int PAT>
__global__ __launch_bounds__(64) void edge_recheck_kernel(EdgeArgs a, ProbTable pt,
                                                          const ArmConst<double>* __restrict__ Dp) {
  __shared__ float s_fix[1];
  __shared__ GeoLDS<double> s_geo;
  extern __shared__ double s_tab64[];
  const int n = *a.q_count;
  for (int qi = blockIdx.x; qi < n; qi += gridDim.x) {
    const QEntry q = a.queue[qi];
    const EdgeArgs* ap = &a;
    int64_t e = q.edge;
    if (pt.n > 0) {
      const int p = problem_of(pt, q.edge);
      ap = pt.args + p;
      e -= pt.edge_off[p];
    }
    recheck_edge<PAT>(*ap, e, q, *Dp, s_fix, &s_geo, s_tab64);
  }
}

}  // namespace fn
