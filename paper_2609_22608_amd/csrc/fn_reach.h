// fn_reach.h -- the earliest reach time of Eq. (8) (Sec. IV-D, arrival-time
// pruning) for one tree node.
//
// With the ballistic flight of Eq. (1), p - x(T) = c0 + c1 T + c2 T^2
// (c0 = p - x0, c1 = -v0, c2 = -g/2).  For T >= t_n the condition
// t_n + |p - x(T)| / V <= T is G(T) <= 0 with the quartic
//     G(T) = |p - x(T)|^2 - V^2 (T - t_n)^2.
// T_n is the first T of [a, b] = [max(t_enter, t_n), t_fall] with G <= 0:
// a itself when G(a) <= 0, else the first root of G.  G'' is a quadratic,
// so its roots split [a, b] into pieces where G' is monotone; the sign
// changes of G' on them (found by bisection) split [a, b] into pieces where
// G is monotone, and the first piece whose right end has G <= 0 holds the
// root, again found by bisection.  G and G' are evaluated from the geometry
// (not from expanded coefficients) to avoid cancellation.
//
// The routine is written for R = float (the pass over every node) and
// R = double (the recheck of nodes whose FP32 decision is close to its
// boundary): it reports the smallest |G| at the points that decide the
// outcome (a, the critical points, b) and the slope of G at the root.
#pragma once

#include <hip/hip_runtime.h>

namespace fn {

// flight layout: x0[3], v0[3], g[3], t_enter, t_fall
constexpr int FLIGHT_FLOATS = 11;

template <typename R>
struct ReachGeo {
  R c0[3], c1[3], c2[3];
  R v2, tn;
  __device__ R G(R T) const {
    const R dx = c0[0] + T * (c1[0] + T * c2[0]);
    const R dy = c0[1] + T * (c1[1] + T * c2[1]);
    const R dz = c0[2] + T * (c1[2] + T * c2[2]);
    const R s = T - tn;
    return dx * dx + dy * dy + dz * dz - v2 * s * s;
  }
  // G'(T) / 2
  __device__ R dG(R T) const {
    R acc = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      acc += (c0[i] + T * (c1[i] + T * c2[i])) * (c1[i] + R(2) * T * c2[i]);
    return acc - v2 * (T - tn);
  }
};

// Bisection on (l, r] for the crossing of a predicate that is false at l
// and true at r; runs until the interval stops shrinking and returns the
// right end.
template <typename R, typename F>
__device__ __forceinline__ R bisect(R l, R r, F&& past) {
  for (int it = 0; it < 64; ++it) {
    const R m = R(0.5) * (l + r);
    if (!(m > l && m < r)) break;
    if (past(m)) r = m;
    else l = m;
  }
  return r;
}

template <typename R>
__device__ __forceinline__ R rnan() {
  if constexpr (sizeof(R) == 4) return __builtin_nanf("");
  else return __builtin_nan("");
}

// T_n of Eq. (8) for blade point p and node time tn (NaN when it does not
// exist).  gmin: smallest |G| at a, the critical points and b (how close the
// outcome came to changing); slope: |G'| at the root (infinite when T_n = a
// or when there is none).
template <typename R>
__device__ __forceinline__ R reach_time_dev(const R p[3], R tn, const float* __restrict__ fl,
                                            R v_tip, R& gmin, R& slope) {
  const R inf = R(1) / R(0);
  gmin = inf;
  slope = inf;
  const R a = tn > R(fl[9]) ? tn : R(fl[9]), b = R(fl[10]);
  if (!(a <= b)) return rnan<R>();
  ReachGeo<R> g;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    g.c0[i] = p[i] - R(fl[i]);
    g.c1[i] = -R(fl[3 + i]);
    g.c2[i] = R(-0.5) * R(fl[6 + i]);
  }
  g.v2 = v_tip * v_tip;
  g.tn = tn;
  const R ga = g.G(a);
  gmin = ga < 0 ? -ga : ga;
  if (ga <= R(0)) return a;
  // G''/2 = q2 T^2 + q1 T + q0
  R c22 = 0, c12 = 0, c11 = 0, c02 = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    c22 += g.c2[i] * g.c2[i];
    c12 += g.c1[i] * g.c2[i];
    c11 += g.c1[i] * g.c1[i];
    c02 += g.c0[i] * g.c2[i];
  }
  const R q2 = R(6) * c22, q1 = R(6) * c12, q0 = c11 + R(2) * c02 - g.v2;
  // break points of G' monotonicity inside (a, b)
  R brk[4];
  int nb = 0;
  brk[nb++] = a;
  if (q2 != R(0)) {
    const R disc = q1 * q1 - R(4) * q2 * q0;
    if (disc > R(0)) {
      const R sq = sqrt(disc);
      const R qq = R(-0.5) * (q1 + (q1 >= R(0) ? sq : -sq));
      R r1 = qq / q2, r2 = qq != R(0) ? q0 / qq : r1;
      if (r1 > r2) { const R t = r1; r1 = r2; r2 = t; }
      if (r1 > a && r1 < b) brk[nb++] = r1;
      if (r2 > a && r2 < b && r2 != r1) brk[nb++] = r2;
    }
  } else if (q1 != R(0)) {
    const R r1 = -q0 / q1;
    if (r1 > a && r1 < b) brk[nb++] = r1;
  }
  brk[nb++] = b;
  // critical points of G: sign changes of G' on the monotone pieces of G'
  R pts[5];
  int np = 0;
  pts[np++] = a;
  for (int s = 0; s + 1 < nb; ++s) {
    const R l = brk[s], r = brk[s + 1];
    const R gl = g.dG(l), gr = g.dG(r);
    if ((gl < R(0)) != (gr < R(0))) {
      const bool up = gl < R(0);  // G' rises through zero
      const R c = bisect<R>(l, r, [&](R m) { return up ? g.dG(m) >= R(0) : g.dG(m) < R(0); });
      if (c > pts[np - 1] && c < b) pts[np++] = c;
    }
  }
  pts[np++] = b;
  // first monotone piece of G whose right end reaches G <= 0
  for (int s = 1; s < np; ++s) {
    const R gr = g.G(pts[s]);
    const R ag = gr < 0 ? -gr : gr;
    gmin = ag < gmin ? ag : gmin;
    if (gr <= R(0)) {
      const R T = bisect<R>(pts[s - 1], pts[s], [&](R m) { return g.G(m) <= R(0); });
      const R d = R(2) * g.dG(T);
      slope = d < 0 ? -d : d;
      return T;
    }
  }
  return rnan<R>();
}

// Whether an FP32 reach time may be on the wrong side of its decision: the
// outcome at a, at a critical point or at b was within tol_g of flipping,
// the root is shallow, or T_n lies within 1e-3 s of the bound t_best (pass
// NaN for no bound).  tol_g scales with the size of the terms of G.
__device__ __forceinline__ bool reach_ambiguous(float T, float gmin, float slope, float t_best,
                                                float scale) {
  const float tol_g = 1e-4f * (1.f + scale);
  if (gmin <= tol_g) return true;
  if (T == T && slope < 1e-2f) return true;
  return T == T && t_best == t_best && fabsf(T - t_best) <= 1e-3f;
}

}  // namespace fn
