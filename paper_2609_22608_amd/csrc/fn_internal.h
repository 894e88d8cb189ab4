// fn_internal.h -- device-side building blocks of the edge-timing library:
// the per-context arm constant block, the cubic edge of Eq. (6), the torque
// model of Eqs. (4)-(5) as recursive Newton-Euler in link frames, and the
// ratios of Eq. (7).  Everything is templated on the arithmetic type so that
// the FP32 bulk path and the FP64 near-limit recheck share one formulation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fruitninja.h"

namespace fn {

constexpr int NJ = 7;
constexpr int WAVE = 64;
// A ratio within BAND of 1 is not decided in FP32.
constexpr float BAND = 1e-3f;

// Twist pattern of a modified-DH arm as 7 base-4 digits: 0: alpha = 0,
// 1: +pi/2, 2: -pi/2.  PAT_GENERIC selects runtime cos/sin of alpha.
constexpr int PAT_GENERIC = -1;
constexpr int pat_digit(int pat, int i) {
  int p = pat;
  for (int k = 0; k < i; ++k) p /= 4;
  return p % 4;
}
// 0, -pi/2, +pi/2, +pi/2, -pi/2, +pi/2, +pi/2 (Panda/FR3-like chain)
constexpr int PAT_FR3 = 0 + 2 * 4 + 1 * 16 + 1 * 64 + 2 * 256 + 1 * 1024 + 1 * 4096;

// Per-link constants, contiguous so that one scalar load fetches a link.
template <typename R>
struct alignas(16 * sizeof(R)) LinkConst {
  R px, py, pz;     // origin of frame i in frame i-1
  R m;
  R rcx, rcy, rcz;  // COM in frame i
  R Ix, Iy, Iz;     // diagonal inertia about the COM
  R Im;             // reflected rotor inertia
  R psi1, fk2, psi3;  // friction: fk2 = -psi2 log2(e)
  R f0;             // psi1 / (1 + exp(-psi2 psi3)): friction at rest, subtracted
  R inv_taumax;
};

template <typename R>
struct ArmConst {
  LinkConst<R> L[NJ];
  int32_t terms;
  int32_t pattern;        // twist pattern code (or -1 when some twist is general)
  R ca[NJ], sa[NJ];       // cos / sin of alpha_{i-1}
  R inv_wmax;
  R qmin[NJ], qmax[NJ], qcen[NJ], inv_qhalf[NJ], qdmax[NJ], two_acc[NJ];
  R vd0[3];               // base acceleration: -g when gravity is on
  int32_t nsph;
  int32_t sph_first[NJ + 1];  // spheres of link i+1: [sph_first[i], sph_first[i+1])
  int32_t sph_link[FN_MAX_SPHERES];
  R sphx[FN_MAX_SPHERES], sphy[FN_MAX_SPHERES], sphz[FN_MAX_SPHERES], sphr[FN_MAX_SPHERES];
  R taumax[NJ];           // torque limits and power limit (the controller's clips)
  R wmax;
};

// ---------------------------------------------------------------------------
// scalar helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincos_r(float x, float& s, float& c) {
  // v_sin_f32 / v_cos_f32 take revolutions
  const float r = x * 0.15915494309189535f;
  s = __builtin_amdgcn_sinf(r);
  c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void sincos_r(double x, double& s, double& c) {
  sincos(x, &s, &c);  // one argument reduction for both
}
__device__ __forceinline__ float logistic_neg(float k2x) {
  // 1 / (1 + 2^(k2x)) with k2x = -psi2 (qd + psi3) log2(e)
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(k2x));
}
__device__ __forceinline__ double logistic_neg(double k2x) {
  return 1.0 / (1.0 + exp2(k2x));
}
template <typename R>
__device__ __forceinline__ R rabs(R x) { return x < R(0) ? -x : x; }
// a / b: hardware reciprocal (1 ulp) in FP32, IEEE division in FP64
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
// square root of x >= 0: the hardware square root (1 ulp) in FP32, IEEE in
// FP64
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
template <typename R>
__device__ __forceinline__ R rmax(R a, R b) { return a > b ? a : b; }
// Larger of two FP32 ratios, each non-negative or a NaN from arithmetic
// (sign clear): their bit patterns as signed integers order like the values
// and a NaN lies above +inf, so one integer max gives the maximum and keeps
// a NaN (the slot then fails every "<= 1" test), with no compare-and-select
// and no canonicalising of the operands.
__device__ __forceinline__ float ratio_max(float a, float b) {
  return __int_as_float(max(__float_as_int(a), __float_as_int(b)));
}

// ---------------------------------------------------------------------------
// Rotation by ^{i-1}R_i = Rx(alpha) Rz(theta) and its transpose, with the
// twist folded in at compile time when it is 0 or +-pi/2.
// ---------------------------------------------------------------------------
template <typename R, int PAT, int I>
__device__ __forceinline__ void rotT(const ArmConst<R>& A, R c, R s, R vx, R vy, R vz, R& ox,
                                     R& oy, R& oz) {
  // u = Rx(alpha)^T v
  R ux = vx, uy, uz;
  if constexpr (PAT != PAT_GENERIC && pat_digit(PAT, I) == 0) {
    uy = vy; uz = vz;
  } else if constexpr (PAT != PAT_GENERIC && pat_digit(PAT, I) == 1) {
    uy = vz; uz = -vy;
  } else if constexpr (PAT != PAT_GENERIC && pat_digit(PAT, I) == 2) {
    uy = -vz; uz = vy;
  } else {
    const R ca = A.ca[I], sa = A.sa[I];
    uy = ca * vy + sa * vz;
    uz = ca * vz - sa * vy;
  }
  // o = Rz(theta)^T u
  ox = c * ux + s * uy;
  oy = c * uy - s * ux;
  oz = uz;
}
template <typename R, int PAT, int I>
__device__ __forceinline__ void rot(const ArmConst<R>& A, R c, R s, R vx, R vy, R vz, R& ox,
                                    R& oy, R& oz) {
  // u = Rz(theta) v ; o = Rx(alpha) u
  const R ux = c * vx - s * vy;
  const R uy = s * vx + c * vy;
  const R uz = vz;
  ox = ux;
  if constexpr (PAT != PAT_GENERIC && pat_digit(PAT, I) == 0) {
    oy = uy; oz = uz;
  } else if constexpr (PAT != PAT_GENERIC && pat_digit(PAT, I) == 1) {
    oy = -uz; oz = uy;
  } else if constexpr (PAT != PAT_GENERIC && pat_digit(PAT, I) == 2) {
    oy = uz; oz = -uy;
  } else {
    const R ca = A.ca[I], sa = A.sa[I];
    oy = ca * uy - sa * uz;
    oz = sa * uy + ca * uz;
  }
}

// ---------------------------------------------------------------------------
// Eq. (4): rigid-body inverse dynamics by recursive Newton-Euler in link
// frames (outward: angular velocity/acceleration and linear acceleration of
// every frame, Newton-Euler force/moment of every link about its COM;
// inward: force and moment transmitted at every joint), plus armature and
// the sigmoid friction of Eq. (5).  sn/cs: sin/cos of q.
// ---------------------------------------------------------------------------
// Rigid-body part only, with the base acceleration (vd0x, vd0y, vd0z) given:
// -g for the torque model, 0 for columns of the mass matrix.
template <typename R, int PAT>
__device__ __forceinline__ void rnea_rigid(const ArmConst<R>& A, const R* sn, const R* cs,
                                           const R* qd, const R* qdd, R vd0x, R vd0y, R vd0z,
                                           R* tau) {
  const bool rigid = (A.terms & FN_T_RIGID) != 0;
  R Fx[NJ], Fy[NJ], Fz[NJ], Nx[NJ], Ny[NJ], Nz[NJ];
  R wx = 0, wy = 0, wz = 0, ax = 0, ay = 0, az = 0;  // w_{i-1}, wd_{i-1}
  R vx = vd0x, vy = vd0y, vz = vd0z;                  // vd_{i-1}
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    const R c = cs[i], s = sn[i];
    const R px = A.L[i].px, py = A.L[i].py, pz = A.L[i].pz;
    // t = wd x p + w x (w x p) + vd   (frame i-1)
    const R wpx = wy * pz - wz * py, wpy = wz * px - wx * pz, wpz = wx * py - wy * px;
    const R tx = (ay * pz - az * py) + (wy * wpz - wz * wpy) + vx;
    const R ty = (az * px - ax * pz) + (wz * wpx - wx * wpz) + vy;
    const R tz = (ax * py - ay * px) + (wx * wpy - wy * wpx) + vz;
    R nvx, nvy, nvz, rwx, rwy, rwz, rax, ray, raz;
    switch (i) {  // compile-time link index after unrolling
#define FN_ROT3(II)                                              \
  case II:                                                       \
    rotT<R, PAT, II>(A, c, s, tx, ty, tz, nvx, nvy, nvz);        \
    rotT<R, PAT, II>(A, c, s, wx, wy, wz, rwx, rwy, rwz);        \
    rotT<R, PAT, II>(A, c, s, ax, ay, az, rax, ray, raz);        \
    break;
      FN_ROT3(0) FN_ROT3(1) FN_ROT3(2) FN_ROT3(3) FN_ROT3(4) FN_ROT3(5) FN_ROT3(6)
#undef FN_ROT3
    }
    const R q1 = qd[i];
    wx = rwx; wy = rwy; wz = rwz + q1;
    ax = rax + rwy * q1; ay = ray - rwx * q1; az = raz + qdd[i];
    vx = nvx; vy = nvy; vz = nvz;
    // COM acceleration and the link's Newton-Euler wrench
    const R rx = A.L[i].rcx, ry = A.L[i].rcy, rz = A.L[i].rcz;
    const R wrx = wy * rz - wz * ry, wry = wz * rx - wx * rz, wrz = wx * ry - wy * rx;
    const R cx = (ay * rz - az * ry) + (wy * wrz - wz * wry) + vx;
    const R cy = (az * rx - ax * rz) + (wz * wrx - wx * wrz) + vy;
    const R cz = (ax * ry - ay * rx) + (wx * wry - wy * wrx) + vz;
    const R mm = A.L[i].m;
    Fx[i] = mm * cx; Fy[i] = mm * cy; Fz[i] = mm * cz;
    const R Iwx = A.L[i].Ix * wx, Iwy = A.L[i].Iy * wy, Iwz = A.L[i].Iz * wz;
    Nx[i] = A.L[i].Ix * ax + (wy * Iwz - wz * Iwy);
    Ny[i] = A.L[i].Iy * ay + (wz * Iwx - wx * Iwz);
    Nz[i] = A.L[i].Iz * az + (wx * Iwy - wy * Iwx);
  }
  R fx = 0, fy = 0, fz = 0, nx = 0, ny = 0, nz = 0;  // f_{i+1}, n_{i+1} in frame i+1
#pragma unroll
  for (int i = NJ - 1; i >= 0; --i) {
    R Rfx = 0, Rfy = 0, Rfz = 0, Rnx = 0, Rny = 0, Rnz = 0;
    if (i + 1 < NJ) {
      const R c = cs[i + 1], s = sn[i + 1];
      switch (i + 1) {
#define FN_ROT2(II)                                              \
  case II:                                                       \
    rot<R, PAT, II>(A, c, s, fx, fy, fz, Rfx, Rfy, Rfz);         \
    rot<R, PAT, II>(A, c, s, nx, ny, nz, Rnx, Rny, Rnz);         \
    break;
        FN_ROT2(1) FN_ROT2(2) FN_ROT2(3) FN_ROT2(4) FN_ROT2(5) FN_ROT2(6)
#undef FN_ROT2
      }
      // + p_{i+1} x (R f_{i+1})
      const R px = A.L[i + 1].px, py = A.L[i + 1].py, pz = A.L[i + 1].pz;
      Rnx += py * Rfz - pz * Rfy;
      Rny += pz * Rfx - px * Rfz;
      Rnz += px * Rfy - py * Rfx;
    }
    const R rx = A.L[i].rcx, ry = A.L[i].rcy, rz = A.L[i].rcz;
    fx = Rfx + Fx[i]; fy = Rfy + Fy[i]; fz = Rfz + Fz[i];
    nx = Nx[i] + Rnx + (ry * Fz[i] - rz * Fy[i]);
    ny = Ny[i] + Rny + (rz * Fx[i] - rx * Fz[i]);
    nz = Nz[i] + Rnz + (rx * Fy[i] - ry * Fx[i]);
    tau[i] = rigid ? nz : R(0);
  }
}

// Eq. (5) friction of joint i at velocity v, zero at rest.
template <typename R>
__device__ __forceinline__ R friction(const ArmConst<R>& A, int i, R v) {
  return A.L[i].psi1 * logistic_neg(A.L[i].fk2 * (v + A.L[i].psi3)) - A.L[i].f0;
}

template <typename R, int PAT>
__device__ __forceinline__ void rnea(const ArmConst<R>& A, const R* sn, const R* cs,
                                     const R* qd, const R* qdd, R* tau) {
  rnea_rigid<R, PAT>(A, sn, cs, qd, qdd, A.vd0[0], A.vd0[1], A.vd0[2], tau);
  const bool arm = (A.terms & FN_T_ARMATURE) != 0;
  const bool fric = (A.terms & FN_T_FRICTION) != 0;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    if (arm) tau[i] += A.L[i].Im * qdd[i];
    if (fric) tau[i] += friction(A, i, qd[i]);
  }
}

// ---------------------------------------------------------------------------
// Endpoint model.  At u = 0 and u = 1 the cubic's position and velocity are
// the boundary states, whatever T is; only the acceleration depends on T.
// The torque of Eq. (4)-(5) is affine in the acceleration,
//   tau(qdd) = b + (M + diag(Im)) qdd,  b = rigid(q, qd, 0) + friction(qd),
// so one model per boundary state gives the endpoint torques of every slot.
// A model is 56 floats: column c of M + diag(Im) at [7c, 7c + 7), b at
// [49, 56).  Lane `role` 0..6 of a state computes column `role` (unit
// acceleration, zero velocity, no gravity, no friction); role 7 computes b.
// ---------------------------------------------------------------------------
constexpr int MODEL_FLOATS = 56;

template <typename R, int PAT>
__device__ __forceinline__ void model_lane(const ArmConst<R>& A, const R* q, const R* qd, int role,
                                           R* out) {
  R sn[NJ], cs[NJ], v[NJ], acc[NJ];
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    sincos_r(q[i], sn[i], cs[i]);
    v[i] = role == NJ ? qd[i] : R(0);
    acc[i] = i == role ? R(1) : R(0);
  }
  const bool col = role < NJ;
  rnea_rigid<R, PAT>(A, sn, cs, v, acc, col ? R(0) : A.vd0[0], col ? R(0) : A.vd0[1],
                     col ? R(0) : A.vd0[2], out);
  const bool arm = (A.terms & FN_T_ARMATURE) != 0;
  const bool fric = (A.terms & FN_T_FRICTION) != 0;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    if (col && arm && i == role) out[i] += A.L[i].Im;
    if (!col && fric) out[i] += friction(A, i, qd[i]);
  }
}


// ---------------------------------------------------------------------------
// Eq. (6) in the normalised time u = t / T:
//   sigma = q0 + u (qd0 T + u (A2 + u A3)),  A2 = 3 d1 - d2 T,  A3 = d2 T - 2 d1,
//   d1 = q1 - q0 - qd0 T,  d2 = qd1 - qd0.
// ---------------------------------------------------------------------------
template <typename R>
struct EdgeState {
  R q0[NJ], qd0[NJ], dq[NJ], d2[NJ];  // dq = q1 - q0
};

template <typename R>
__device__ __forceinline__ void cubic_point(const EdgeState<R>& E, R T, R invT, R u, R* sg,
                                            R* sd, R* sdd) {
  const R invT2 = invT * invT;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    const R v0T = E.qd0[i] * T;
    const R d1 = E.dq[i] - v0T;
    const R A2 = R(3) * d1 - E.d2[i] * T;
    const R A3 = E.d2[i] * T - R(2) * d1;
    sg[i] = E.q0[i] + u * (v0T + u * (A2 + u * A3));
    sd[i] = E.qd0[i] + u * (R(2) * A2 + R(3) * A3 * u) * invT;
    sdd[i] = (R(2) * A2 + R(6) * A3 * u) * invT2;
  }
}

// One evaluation point of Def. 6: torque ratio max_i |tau_i| / taumax_i and
// power ratio |sum_i tau_i sd_i| / W_max at normalised time u of duration T.
template <typename R, int PAT>
__device__ __forceinline__ void eval_point(const ArmConst<R>& A, const EdgeState<R>& E, R T,
                                           R invT, R u, R& rt, R& rp, R* tau_out) {
  R sg[NJ], sd[NJ], sdd[NJ], sn[NJ], cs[NJ], tau[NJ];
  cubic_point(E, T, invT, u, sg, sd, sdd);
#pragma unroll
  for (int i = 0; i < NJ; ++i) sincos_r(sg[i], sn[i], cs[i]);
  rnea<R, PAT>(A, sn, cs, sd, sdd, tau);
  R t = 0, pw = 0;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    if constexpr (sizeof(R) == 4) t = ratio_max(t, fabsf(tau[i]) * A.L[i].inv_taumax);
    else t = rmax(t, rabs(tau[i]) * A.L[i].inv_taumax);
    pw += tau[i] * sd[i];
    if (tau_out) tau_out[i] = tau[i];
  }
  rt = t;
  if constexpr (sizeof(R) == 4) rp = fabsf(pw) * A.inv_wmax;
  else rp = rabs(pw) * A.inv_wmax;
}
template <typename R, int PAT>
__device__ __forceinline__ R eval_rho(const ArmConst<R>& A, const EdgeState<R>& E, R T, R invT,
                                      R u) {
  R rt, rp;
  eval_point<R, PAT>(A, E, T, invT, u, rt, rp, nullptr);
  if constexpr (sizeof(R) == 4) return ratio_max(rt, rp);
  else return rmax(rt, rp);
}

// Screen of a slot from the two endpoint models (m0: state q0, qd0; m1:
// state q1, qd1 = qd0 + d2; each the columns of M + diag(I_m) and the bias
// b, MODEL_FLOATS floats).  At an endpoint the torque is b + M qdd, and the
// cubic's endpoint accelerations are affine in 1 / T^2 and 1 / T:
//   qdd(0) = 6 dq / T^2 - (6 qd0 + 2 d2) / T,
//   qdd(1) = -6 dq / T^2 + (6 qd0 + 4 d2) / T,
// so per edge P0 = M0 (6 dq), Q0 = M0 (6 qd0 + 2 d2), P1 = M1 (6 dq) and
// Q1 = M1 (6 qd0 + 4 d2) give both endpoint torques of any duration with two
// FMAs per joint.  SCREEN_FLOATS of LDS per wavefront hold the two models
// and these 28 coefficients.
constexpr int SCREEN_FLOATS = 2 * MODEL_FLOATS + 32;

// The coefficients of one edge into tab (LDS): lane 7 w + i (w < 4) of the
// wavefront forms coefficient w (P0, Q0, P1, Q1) of joint i.  The caller
// orders the LDS writes before the reads (a wave barrier).
__device__ __forceinline__ void endpoint_table(int lane, const EdgeState<float>& E,
                                               const float* __restrict__ m0,
                                               const float* __restrict__ m1, float* tab) {
  if (lane < 4 * NJ) {
    const int w = lane / NJ, i = lane - NJ * w;
    const float* m = w < 2 ? m0 : m1;
    const float kd = w == 1 ? 2.f : 4.f;
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
      const float v = (w & 1) ? fmaf(kd, E.d2[c], 6.f * E.qd0[c]) : 6.f * E.dq[c];
      s = fmaf(m[NJ * c + i], v, s);
    }
    tab[lane] = s;
  }
}

// Larger of the torque and power ratios (Def. 6) at u = 0 and u = 1 of
// duration 1 / invT from the endpoint models (biases at m0[49..], m1[49..])
// and the edge's coefficients (endpoint_table); all read from LDS at the
// same address in every lane.
__device__ __forceinline__ float endpoint_ratio(const ArmConst<float>& A, const EdgeState<float>& E,
                                                const float* __restrict__ m0,
                                                const float* __restrict__ m1,
                                                const float* __restrict__ tab, float invT) {
  const float invT2 = invT * invT;
  float r = 0.f, p0 = 0.f, p1 = 0.f;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    const float t0 = fmaf(tab[i], invT2, fmaf(-tab[NJ + i], invT, m0[49 + i]));
    const float t1 = fmaf(-tab[2 * NJ + i], invT2, fmaf(tab[3 * NJ + i], invT, m1[49 + i]));
    r = fmaxf(r, fmaxf(fabsf(t0), fabsf(t1)) * A.L[i].inv_taumax);
    p0 = fmaf(t0, E.qd0[i], p0);
    p1 = fmaf(t1, E.qd0[i] + E.d2[i], p1);
  }
  return fmaxf(r, fmaxf(fabsf(p0), fabsf(p1)) * A.inv_wmax);
}

// Velocity taper of Def. 1 (braking law) and the ratio |v| / taper.
template <typename R>
__device__ __forceinline__ R vel_ratio(const ArmConst<R>& A, int i, R q, R v) {
  if (v == R(0)) return R(0);
  const R dist = v >= R(0) ? (A.qmax[i] - q) : (q - A.qmin[i]);
  R lim = fsqrt(A.two_acc[i] * rmax(R(0), dist));
  lim = lim < A.qdmax[i] ? lim : A.qdmax[i];
  if (!(lim > R(0))) return R(INFINITY);
  return fdiv(rabs(v), lim);
}

// One candidate extremum of joint i's cubic at duration T (boundary state
// (q0, qd0), dq = q1 - q0, d2 = qd1 - qd0): point p = 0, 1, 2 are the
// velocity peaks (t = 0, t = T, vertex of the quadratic velocity), p = 3, 4,
// 5, 6 the position extrema (t = 0, t = T, real roots of the velocity in
// [0, T]).  v receives the velocity-taper ratio of a velocity point, q the
// position ratio of a position point, 0 for the other kind or a point that
// does not exist; rho_v and rho_q are the maxima over the 7 points of every
// joint.  Every lane runs the same instructions (the point is selected, not
// branched on), so a wavefront evaluates all 49 (joint, point) pairs at the
// latency of one.
template <typename R>
__device__ __forceinline__ void joint_point(const ArmConst<R>& A, int i, int p, R q0, R qd0, R dq,
                                            R d2v, R T, R& v, R& q) {
  // quotients and roots: fdiv / fsqrt (1 ulp in FP32, IEEE in FP64); each
  // quotient is used only where its divisor is nonzero, and a candidate time
  // off by an ulp moves its value by far less (the derivative vanishes at an
  // extremum)
  const R invT = fdiv(R(1), T);
  const R c0 = q0, c1 = qd0;
  const R d1 = dq - c1 * T;
  const R c2 = (R(3) * d1 * invT - d2v) * invT;
  const R c3 = (d2v - R(2) * d1 * invT) * invT * invT;
  // velocity vertex
  const R tv = fdiv(-c2, R(3) * c3);
  const bool tv_ok = c3 != R(0) && tv > R(0) && tv < T;
  // roots of the velocity 3 c3 t^2 + 2 c2 t + c1
  const R qa = R(3) * c3, qb = R(2) * c2, qc = c1;
  const R tl = fdiv(-qc, qb);  // qa = 0: the linear root
  const bool tl_ok = qb != R(0) && tl >= R(0) && tl <= T;
  const R disc = qb * qb - R(4) * qa * qc;
  const R sq = fsqrt(disc >= R(0) ? disc : R(0));
  const R qq = R(-0.5) * (qb + (qb >= R(0) ? sq : -sq));
  const R t1 = fdiv(qq, qa), t2 = fdiv(qc, qq);
  const bool quad = qa != R(0) && disc >= R(0) && qq != R(0);
  const bool t1_ok = quad && t1 >= R(0) && t1 <= T;
  const bool t2_ok = quad && t2 >= R(0) && t2 <= T;
  R t = R(0);
  bool ok = p <= 6;
  if (p == 1 || p == 4) t = T;
  if (p == 2) {
    t = tv;
    ok = tv_ok;
  }
  if (p == 5) {
    t = qa == R(0) ? tl : t1;
    ok = qa == R(0) ? tl_ok : t1_ok;
  }
  if (p == 6) {
    t = t2;
    ok = qa != R(0) && t2_ok;
  }
  const R pt = c0 + t * (c1 + t * (c2 + t * c3));
  const R vt = c1 + t * (R(2) * c2 + R(3) * c3 * t);
  const R rvel = vel_ratio(A, i, pt, vt);
  const R rpos = rabs(pt - A.qcen[i]) * A.inv_qhalf[i];
  v = ok && p <= 2 ? rvel : R(0);
  q = ok && p >= 3 ? rpos : R(0);
}

// Modified-DH frame chain at configuration (sn, cs): after frame i + 1 is
// formed, fn(i, r, o) receives its world rotation (rows r[0..8]) and origin.
template <typename R, int PAT, typename F>
__device__ __forceinline__ void frame_chain(const ArmConst<R>& A, const R* sn, const R* cs,
                                            F&& fn) {
  // world rotation of frame i (rows) and its origin
  R r00 = 1, r01 = 0, r02 = 0, r10 = 0, r11 = 1, r12 = 0, r20 = 0, r21 = 0, r22 = 1;
  R ox = 0, oy = 0, oz = 0;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    // origin_i = origin_{i-1} + R_{i-1} p_i
    const R px = A.L[i].px, py = A.L[i].py, pz = A.L[i].pz;
    ox += r00 * px + r01 * py + r02 * pz;
    oy += r10 * px + r11 * py + r12 * pz;
    oz += r20 * px + r21 * py + r22 * pz;
    // R_i = R_{i-1} Rx(alpha) Rz(theta)
    R a0, a1, a2, b0, b1, b2, c0, c1, c2;  // rows after Rx
    switch (i) {
#define FN_RX(II)                                                             \
  case II:                                                                   \
    if constexpr (PAT != PAT_GENERIC && pat_digit(PAT, II) == 0) {            \
      a0 = r00; a1 = r01; a2 = r02; b0 = r10; b1 = r11; b2 = r12;             \
      c0 = r20; c1 = r21; c2 = r22;                                           \
    } else if constexpr (PAT != PAT_GENERIC && pat_digit(PAT, II) == 1) {     \
      a0 = r00; a1 = r02; a2 = -r01; b0 = r10; b1 = r12; b2 = -r11;           \
      c0 = r20; c1 = r22; c2 = -r21;                                          \
    } else if constexpr (PAT != PAT_GENERIC && pat_digit(PAT, II) == 2) {     \
      a0 = r00; a1 = -r02; a2 = r01; b0 = r10; b1 = -r12; b2 = r11;           \
      c0 = r20; c1 = -r22; c2 = r21;                                          \
    } else {                                                                  \
      const R ca = A.ca[II], sa = A.sa[II];                                   \
      a0 = r00; a1 = r01 * ca + r02 * sa; a2 = r02 * ca - r01 * sa;           \
      b0 = r10; b1 = r11 * ca + r12 * sa; b2 = r12 * ca - r11 * sa;           \
      c0 = r20; c1 = r21 * ca + r22 * sa; c2 = r22 * ca - r21 * sa;           \
    }                                                                         \
    break;
      FN_RX(0) FN_RX(1) FN_RX(2) FN_RX(3) FN_RX(4) FN_RX(5) FN_RX(6)
#undef FN_RX
    }
    const R c = cs[i], s = sn[i];
    r00 = a0 * c + a1 * s; r01 = a1 * c - a0 * s; r02 = a2;
    r10 = b0 * c + b1 * s; r11 = b1 * c - b0 * s; r12 = b2;
    r20 = c0 * c + c1 * s; r21 = c1 * c - c0 * s; r22 = c2;
    const R r[9] = {r00, r01, r02, r10, r11, r12, r20, r21, r22};
    fn(i, r, ox, oy, oz);
  }
}

// World-frame centres of the collision spheres at configuration (sn, cs),
// streamed link by link: fn(k, x, y, z) is called for the spheres
// k = first + part, first + part + nparts, ... of every link, so that
// `nparts` lane groups share the spheres of one pose.  sph: sphere k's
// centre in its link frame at sph[4k .. 4k + 2].
template <typename R, int PAT, typename F>
__device__ __forceinline__ void sphere_centres(const ArmConst<R>& A, const R* sn, const R* cs,
                                               int part, int nparts, const R* sph, F&& fn) {
  frame_chain<R, PAT>(A, sn, cs, [&](int i, const R* r, R ox, R oy, R oz) {
    for (int k = A.sph_first[i] + part; k < A.sph_first[i + 1]; k += nparts) {
      const R lx = sph[4 * k], ly = sph[4 * k + 1], lz = sph[4 * k + 2];
      fn(k, ox + r[0] * lx + r[1] * ly + r[2] * lz, oy + r[3] * lx + r[4] * ly + r[5] * lz,
         oz + r[6] * lx + r[7] * ly + r[8] * lz);
    }
  });
}

// World position of the point (lx, ly, lz) of the last link's frame.
template <typename R, int PAT>
__device__ __forceinline__ void last_link_point(const ArmConst<R>& A, const R* sn, const R* cs,
                                                R lx, R ly, R lz, R& x, R& y, R& z) {
  frame_chain<R, PAT>(A, sn, cs, [&](int i, const R* r, R ox, R oy, R oz) {
    if (i == NJ - 1) {
      x = ox + r[0] * lx + r[1] * ly + r[2] * lz;
      y = oy + r[3] * lx + r[4] * ly + r[5] * lz;
      z = oz + r[6] * lx + r[7] * ly + r[8] * lz;
    }
  });
}

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }
// Value of lane (lane ^ J) for J = 1..16 without the LDS where DPP can do
// it: quad permutations for 1 and 2; for 4 the half-row mirror (lane ^ 7)
// then the quad reversal (^ 3); for 8 the row mirror (^ 15) then the
// half-row mirror; 16 by LDS swizzle.  Every lane must be active.
template <int J>
__device__ __forceinline__ int xlane(int v) {
  if constexpr (J == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xf, 0xf, true);  // quad_perm 1,0,3,2
  else if constexpr (J == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xf, 0xf, true);  // 2,3,0,1
  else if constexpr (J == 4)
    return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xf, 0xf, true), 0x1B, 0xf,
                                    0xf, true);
  else if constexpr (J == 8)
    return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x140, 0xf, 0xf, true), 0x141, 0xf,
                                    0xf, true);
  else return __builtin_amdgcn_ds_swizzle(v, (16 << 10) | 0x1f);
}
template <int J>
__device__ __forceinline__ float xlane(float v) {
  return __int_as_float(xlane<J>(__float_as_int(v)));
}
template <int J>
__device__ __forceinline__ double xlane(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = xlane<J>((int)(b & 0xffffffff)), hi = xlane<J>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Reductions over the wave (the result in every lane; called with every lane
// active): exchanges within each half, then the two halves' lane 0.
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, xlane<1>(v));
  v = fmaxf(v, xlane<2>(v));
  v = fmaxf(v, xlane<4>(v));
  v = fmaxf(v, xlane<8>(v));
  v = fmaxf(v, xlane<16>(v));
  return fmaxf(readlane(v, 0), readlane(v, 32));
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, xlane<1>(v));
  v = fmax(v, xlane<2>(v));
  v = fmax(v, xlane<4>(v));
  v = fmax(v, xlane<8>(v));
  v = fmax(v, xlane<16>(v));
  return fmax(readlane(v, 0), readlane(v, 32));
}
__device__ __forceinline__ float wave_min(float v) {
  v = fminf(v, xlane<1>(v));
  v = fminf(v, xlane<2>(v));
  v = fminf(v, xlane<4>(v));
  v = fminf(v, xlane<8>(v));
  v = fminf(v, xlane<16>(v));
  return fminf(readlane(v, 0), readlane(v, 32));
}
__device__ __forceinline__ double wave_min(double v) {
  v = fmin(v, xlane<1>(v));
  v = fmin(v, xlane<2>(v));
  v = fmin(v, xlane<4>(v));
  v = fmin(v, xlane<8>(v));
  v = fmin(v, xlane<16>(v));
  return fmin(readlane(v, 0), readlane(v, 32));
}
// Ratio maxima over aligned groups of `width` lanes (width a wave-uniform
// power of two <= 64; every value a ratio, see ratio_max).  Through LDS
// permutes (no VALU moves, for VALU-bound loops) or by lane exchanges.
__device__ __forceinline__ float group_max_lds(float v, int width) {
  for (int o = 1; o < width; o <<= 1) v = ratio_max(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float group_max(float v, int width) {
  if (width >= 32) {
    // the common widths (32 and 64 samples) under one wave-uniform test
    v = ratio_max(v, xlane<1>(v));
    v = ratio_max(v, xlane<2>(v));
    v = ratio_max(v, xlane<4>(v));
    v = ratio_max(v, xlane<8>(v));
    v = ratio_max(v, xlane<16>(v));
    if (width > 32) v = ratio_max(readlane(v, 0), readlane(v, 32));
    return v;
  }
  if (width > 1) v = ratio_max(v, xlane<1>(v));
  if (width > 2) v = ratio_max(v, xlane<2>(v));
  if (width > 4) v = ratio_max(v, xlane<4>(v));
  if (width > 8) v = ratio_max(v, xlane<8>(v));
  if (width > 16) v = ratio_max(v, xlane<16>(v));
  return v;
}

}  // namespace fn
