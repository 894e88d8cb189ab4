// fn_risk.h -- the risk objective of Eq. (2) with the terms of Eq. (3)
// (Sec. IV-B), evaluated in FP64.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/fruitninja.h"

namespace fn {

// log Phi(z) = log(erfc(-z / sqrt 2) / 2); below -30 erfc underflows, so the
// scaled complementary error function carries the tail:
// erfc(x) = erfcx(x) exp(-x^2)
__device__ __forceinline__ double log_phi_dev(double z) {
  if (z > -30.0) return log(0.5 * erfc(-z * 0.70710678118654752));
  const double x = -z * 0.70710678118654752;
  return log(0.5 * erfcx(x)) - x * x;
}

// J = w_v min(v_rel, v_target) + w_p log P_object + w_r log P_inrange
//   + w_x log P_arm, with P_object = erf(r / (sigma sqrt 2)),
// P_inrange = Phi((t_fall - T) / sigma_t), sigma_t = sigma / |xdot_z(t_fall)|,
// log P_arm = -lambda (nu - nu0)_+ T (1 - nu0 / nu).
__device__ __forceinline__ double risk_eval(const fn_risk& w, double t, double v_rel, double nu,
                                            double vz0, double tf) {
  double sg;
  if (w.sigma_mode == 1) {
    sg = w.s0 + w.s1 * t;
  } else {
    const double a = w.sp, b = w.sv * t, c = 0.5 * w.sa * t * t;
    sg = sqrt(a * a + b * b + c * c);
  }
  const double x = w.r / (sg * 1.4142135623730951);
  const double lpo = x < 0.5 ? log(erf(x)) : log1p(-erfc(x));
  const double xdz = vz0 + w.gz * tf;
  const double st = sg / fabs(xdz);
  const double lpr = log_phi_dev((tf - t) / st);
  const double lpa = nu > w.nu0 ? -w.lam * (nu - w.nu0) * t * (1.0 - w.nu0 / nu) : 0.0;
  const double vr = fmin(v_rel, w.vtarget);
  return w.wv * vr + w.wp * lpo + w.wr * lpr + w.wx * lpa;
}

}  // namespace fn
