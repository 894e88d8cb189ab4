// fn_risk.h -- the risk objective of Eq. (2) with the terms of Eq. (3)
// (Sec. IV-B), evaluated in FP32.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/fruitninja.h"

namespace fn {

// log Phi(z) = log(erfc(-z / sqrt 2) / 2).  For z < -4 erfc(x), x = -z / sqrt 2,
// loses relative accuracy in FP32 and underflows below x ~ 10; there the
// scaled complementary error function carries the tail:
// log erfc(x) = log erfcx(x) - x^2.
__device__ __forceinline__ float log_phi_dev(float z) {
  const float x = -z * 0.70710678118654752f;
  if (z > -4.f) return logf(0.5f * erfcf(x));
  return logf(0.5f * erfcxf(x)) - x * x;
}

// J = w_v min(v_rel, v_target) + w_p log P_object + w_r log P_inrange
//   + w_x log P_arm, with P_object = erf(r / (sigma sqrt 2)),
// P_inrange = Phi((t_fall - T) / sigma_t), sigma_t = sigma / |xdot_z(t_fall)|,
// log P_arm = -lambda (nu - nu0)_+ T (1 - nu0 / nu).
__device__ __forceinline__ float risk_eval(const fn_risk& w, float t, float v_rel, float nu,
                                           float vz0, float tf) {
  float sg;
  if (w.sigma_mode == 1) {
    sg = (float)w.s0 + (float)w.s1 * t;
  } else {
    const float a = (float)w.sp, b = (float)w.sv * t, c = 0.5f * (float)w.sa * t * t;
    sg = sqrtf(a * a + b * b + c * c);
  }
  const float x = (float)w.r / (sg * 1.41421356237309515f);
  // log erf(x): directly for small x, through erfc where erf is close to 1
  const float lpo = x < 0.5f ? logf(erff(x)) : log1pf(-erfcf(x));
  // The vertical speed at t_fall vanishes near the apex of the flight, where
  // vz0 + gz t_fall cancels; one FP64 FMA keeps it to a single FP32 rounding.
  const float xdz = (float)fma(w.gz, (double)tf, (double)vz0);
  const float st = sg / fabsf(xdz);
  const float lpr = log_phi_dev((tf - t) / st);
  const float nu0 = (float)w.nu0;
  const float lpa = nu > nu0 ? -(float)w.lam * (nu - nu0) * t * (1.f - nu0 / nu) : 0.f;
  const float vr = fminf(v_rel, (float)w.vtarget);
  return (float)w.wv * vr + (float)w.wp * lpo + (float)w.wr * lpr + (float)w.wx * lpa;
}

}  // namespace fn
