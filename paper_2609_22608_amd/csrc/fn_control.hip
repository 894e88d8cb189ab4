// fn_control.hip -- the 1 kHz tracking controller of Sec. IV-F, batched:
// for every instance the cubic of Eq. (6) refitted from the measured state
// to the rendezvous gives the desired acceleration of Eq. (9), clipped to
// the velocity taper, and the torque of Eq. (4) at that acceleration is
// clipped to the slew, torque and power limits.  One lane per instance
// (a recursive Newton-Euler pass in registers, FP32).
#include <hip/hip_runtime.h>

#include <cmath>

#include "fn_ctx.h"

namespace fn {

struct Slew {
  float d[NJ];  // largest torque change per period, slew_i * dt
};

template <int PAT>
__global__ __launch_bounds__(256) void control_kernel(
    int64_t n, const float* __restrict__ q, const float* __restrict__ qd,
    const float* __restrict__ tau_prev, const float* __restrict__ qg,
    const float* __restrict__ qdg, const float* __restrict__ Th, float dt, Slew sl,
    const ArmConst<float>* __restrict__ Ap, float* __restrict__ out_tau,
    float* __restrict__ out_qdd, uint16_t* __restrict__ out_st) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const ArmConst<float>& A = *Ap;
  float x[NJ], v[NJ], p[NJ], g[NJ], w[NJ];
  const float T = Th[e];
  bool ok = isfinite(T) && T > 0.f;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    x[i] = q[e * NJ + i];
    v[i] = qd[e * NJ + i];
    p[i] = tau_prev[e * NJ + i];
    g[i] = qg[e * NJ + i];
    w[i] = qdg[e * NJ + i];
    ok = ok && isfinite(x[i]) && isfinite(v[i]) && isfinite(p[i]) && isfinite(g[i]) &&
         isfinite(w[i]);
  }
  if (!ok) {
#pragma unroll
    for (int i = 0; i < NJ; ++i) out_tau[e * NJ + i] = out_qdd[e * NJ + i] = 0.f;
    out_st[e] = FN_C_BAD;
    return;
  }
  int st = 0;
  // quotients and roots by the hardware reciprocal and square root (1 ulp)
  const float invT = __builtin_amdgcn_rcpf(T);
  const float inv_dt = __builtin_amdgcn_rcpf(dt);
  float a[NJ], sn[NJ], cs[NJ], tau[NJ];
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    // Eq. (9): initial acceleration of the refitted cubic
    float ai = 6.f * (g[i] - x[i]) * invT * invT - (4.f * v[i] + 2.f * w[i]) * invT;
    // the velocity after one period stays inside the taper of Def. 1
    const float vp = fminf(A.qdmax[i], fsqrt(A.two_acc[i] * fmaxf(0.f, A.qmax[i] - x[i])));
    const float vm = fminf(A.qdmax[i], fsqrt(A.two_acc[i] * fmaxf(0.f, x[i] - A.qmin[i])));
    const float lo = (-vm - v[i]) * inv_dt, hi = (vp - v[i]) * inv_dt;
    if (ai < lo) {
      ai = lo;
      st |= FN_C_ACC;
    } else if (ai > hi) {
      ai = hi;
      st |= FN_C_ACC;
    }
    a[i] = ai;
    sincos_r(x[i], sn[i], cs[i]);
  }
  rnea<float, PAT>(A, sn, cs, v, a, tau);
  float pw = 0.f;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    float t = tau[i];
    if (t > p[i] + sl.d[i]) {
      t = p[i] + sl.d[i];
      st |= FN_C_SLEW;
    } else if (t < p[i] - sl.d[i]) {
      t = p[i] - sl.d[i];
      st |= FN_C_SLEW;
    }
    if (t > A.taumax[i]) {
      t = A.taumax[i];
      st |= FN_C_TORQUE;
    } else if (t < -A.taumax[i]) {
      t = -A.taumax[i];
      st |= FN_C_TORQUE;
    }
    tau[i] = t;
    pw += t * v[i];
  }
  const float apw = fabsf(pw);
  const float scale = apw > A.wmax ? fdiv(A.wmax, apw) : 1.f;
  if (apw > A.wmax) st |= FN_C_POWER;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    out_tau[e * NJ + i] = tau[i] * scale;
    out_qdd[e * NJ + i] = a[i];
  }
  out_st[e] = (uint16_t)st;
}

}  // namespace fn

using namespace fn;

extern "C" int fn_control(fn_ctx* c, int64_t n, const float* q, const float* qd,
                          const float* tau_prev, const float* qg, const float* qdg, const float* T,
                          float dt, const double* slew, float* out_tau, float* out_qdd,
                          uint16_t* out_status, void* stream) {
  if (!c || !slew) return fail(FN_E_ARG, "fn_control: NULL context or slew limits");
  if (n < 0 || n > ((int64_t)1 << 40)) return fail(FN_E_SHAPE, "fn_control: n = %lld", (long long)n);
  if (!(dt > 0.f) || !std::isfinite(dt)) return fail(FN_E_ARG, "fn_control: dt must be > 0");
  Slew sl;
  for (int i = 0; i < NJ; ++i) {
    if (!(slew[i] >= 0.0)) return fail(FN_E_ARG, "fn_control: slew limit of joint %d must be >= 0", i);
    sl.d[i] = (float)(slew[i] * (double)dt);
  }
  if (n == 0) return FN_OK;
  if (!q || !qd || !tau_prev || !qg || !qdg || !T || !out_tau || !out_qdd || !out_status)
    return fail(FN_E_ARG, "fn_control: NULL array");
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (c->pattern == PAT_FR3)
    hipLaunchKernelGGL(control_kernel<PAT_FR3>, grid, dim3(256), 0, s, n, q, qd, tau_prev, qg, qdg,
                       T, dt, sl, c->arm32, out_tau, out_qdd, out_status);
  else
    hipLaunchKernelGGL(control_kernel<PAT_GENERIC>, grid, dim3(256), 0, s, n, q, qd, tau_prev, qg,
                       qdg, T, dt, sl, c->arm32, out_tau, out_qdd, out_status);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "fn_control launch");
}
