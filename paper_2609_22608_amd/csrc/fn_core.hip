// fn_core.hip -- context lifecycle, error reporting, the per-context arm
// constant block, and the risk objective of Eqs. (2)-(3).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "fn_ctx.h"
#include "fn_risk.h"

namespace fn {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(FN_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

// Twist pattern code (see PAT_FR3) or PAT_GENERIC.
static int twist_pattern(const fn_arm_desc* d, int digits[NJ]) {
  const double hp = 1.5707963267948966;
  int pat = 0, mul = 1;
  bool generic = false;
  for (int i = 0; i < NJ; ++i) {
    const double a = d->alpha[i];
    int dg;
    if (std::fabs(a) < 1e-9) dg = 0;
    else if (std::fabs(a - hp) < 1e-9) dg = 1;
    else if (std::fabs(a + hp) < 1e-9) dg = 2;
    else { dg = 3; generic = true; }
    digits[i] = dg;
    pat += dg * mul;
    mul *= 4;
  }
  return generic ? PAT_GENERIC : pat;
}

// Derives the constant blocks on the device from the FP64 description, in
// FP64, and rounds the FP32 copy from it.
template <typename R>
__device__ void fill_arm(const fn_arm_desc* d, const int* digits, int pattern, ArmConst<R>* A) {
  A->terms = d->terms;
  A->pattern = pattern;
  for (int i = 0; i < NJ; ++i) {
    double ca, sa;
    switch (digits[i]) {
      case 0: ca = 1.0; sa = 0.0; break;
      case 1: ca = 0.0; sa = 1.0; break;
      case 2: ca = 0.0; sa = -1.0; break;
      default: ca = cos(d->alpha[i]); sa = sin(d->alpha[i]); break;
    }
    A->ca[i] = R(ca);
    A->sa[i] = R(sa);
    A->L[i].px = R(d->a[i]);
    A->L[i].py = R(-sa * d->d[i]);
    A->L[i].pz = R(ca * d->d[i]);
    A->L[i].m = R(d->m[i]);
    A->L[i].rcx = R(d->rc[i][0]);
    A->L[i].rcy = R(d->rc[i][1]);
    A->L[i].rcz = R(d->rc[i][2]);
    A->L[i].Ix = R(d->inertia[i][0]);
    A->L[i].Iy = R(d->inertia[i][1]);
    A->L[i].Iz = R(d->inertia[i][2]);
    A->L[i].Im = R(d->Im[i]);
    A->L[i].psi1 = R(d->psi1[i]);
    A->L[i].psi3 = R(d->psi3[i]);
    A->L[i].fk2 = R(-d->psi2[i] * 1.4426950408889634);
    A->L[i].f0 = R(d->psi1[i] / (1.0 + exp(-d->psi2[i] * d->psi3[i])));
    A->L[i].inv_taumax = R(1.0 / d->taumax[i]);
    A->taumax[i] = R(d->taumax[i]);
    A->qmin[i] = R(d->qmin[i]);
    A->qmax[i] = R(d->qmax[i]);
    A->qcen[i] = R(0.5 * (d->qmax[i] + d->qmin[i]));
    A->inv_qhalf[i] = R(2.0 / (d->qmax[i] - d->qmin[i]));
    A->qdmax[i] = R(d->qdmax[i]);
    A->two_acc[i] = R(2.0 * d->acc[i]);
  }
  A->inv_wmax = R(1.0 / d->wmax);
  A->wmax = R(d->wmax);
  const bool grav = (d->terms & FN_T_GRAVITY) != 0;
  for (int r = 0; r < 3; ++r) A->vd0[r] = grav ? R(-d->g[r]) : R(0);
  A->nsph = d->n_spheres;
  // spheres arrive sorted by link: prefix offsets per link
  for (int i = 0; i <= NJ; ++i) A->sph_first[i] = 0;
  for (int k = 0; k < d->n_spheres; ++k) A->sph_first[d->sphere_link[k]] += 1;
  for (int i = 1; i <= NJ; ++i) A->sph_first[i] += A->sph_first[i - 1];
  for (int k = 0; k < d->n_spheres; ++k) {
    A->sph_link[k] = d->sphere_link[k];
    A->sphx[k] = R(d->sphere[k][0]);
    A->sphy[k] = R(d->sphere[k][1]);
    A->sphz[k] = R(d->sphere[k][2]);
    A->sphr[k] = R(d->sphere[k][3]);
  }
}

__global__ void arm_prepare_kernel(const fn_arm_desc* d, Digits dg, int pattern,
                                   ArmConst<float>* a32, ArmConst<double>* a64) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    fill_arm<double>(d, dg.v, pattern, a64);
    fill_arm<float>(d, dg.v, pattern, a32);
  }
}

__global__ void risk_kernel(fn_risk w, const float* T, const float* v_rel, const float* nu,
                            const float* vz0, const float* t_fall, int n, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = (float)risk_eval(w, T[i], v_rel[i], nu[i], vz0[i], t_fall[i]);
}

__global__ void zero_i32_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace fn

using namespace fn;

extern "C" const char* fn_last_error(void) { return g_err.c_str(); }
extern "C" const char* fn_version(void) { return "fruitninja-mi355x 0.1 (gfx950)"; }

extern "C" int fn_create(const fn_arm_desc* arm, const fn_caps* caps, fn_ctx** out) {
  if (!arm || !caps || !out) return fail(FN_E_ARG, "fn_create: NULL argument");
  *out = nullptr;
  if (arm->n != NJ) return fail(FN_E_UNSUPPORTED, "fn_create: n = %d, only 7 joints supported", arm->n);
  if (arm->n_spheres < 0 || arm->n_spheres > FN_MAX_SPHERES)
    return fail(FN_E_UNSUPPORTED, "fn_create: %d spheres (max %d)", arm->n_spheres, FN_MAX_SPHERES);
  for (int k = 0; k < arm->n_spheres; ++k)
    if (arm->sphere_link[k] < 1 || arm->sphere_link[k] > NJ)
      return fail(FN_E_ARG, "fn_create: sphere %d on link %d (must be 1..7)", k, arm->sphere_link[k]);
  for (int i = 0; i < NJ; ++i) {
    if (!(arm->taumax[i] > 0) || !(arm->qdmax[i] > 0) || !(arm->qmax[i] > arm->qmin[i]) ||
        !(arm->acc[i] >= 0) || !(arm->m[i] >= 0))
      return fail(FN_E_ARG, "fn_create: joint %d has invalid limits or mass", i);
  }
  if (!(arm->wmax > 0)) return fail(FN_E_ARG, "fn_create: wmax must be > 0");
  if (caps->max_nodes < 0 || caps->max_batch < 0 || caps->max_k < 1 || caps->max_k > FN_MAX_K ||
      caps->max_edges < 0 || caps->max_problems < 0 || caps->max_problems > 4096)
    return fail(FN_E_SHAPE, "fn_create: invalid caps");

  fn_ctx* c = new fn_ctx();
  std::memset(c, 0, sizeof(*c));
  (void)hipGetDevice(&c->device);
  c->n_cu = 0;
  (void)hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (c->n_cu <= 0) c->n_cu = 256;
  c->caps = *caps;
  // spheres sorted by link (stable), as the device FK streams them per link
  c->desc = *arm;
  {
    int w = 0;
    for (int l = 1; l <= NJ; ++l)
      for (int k = 0; k < arm->n_spheres; ++k)
        if (arm->sphere_link[k] == l) {
          c->sphere_order[k] = w;
          c->desc.sphere_link[w] = l;
          for (int r = 0; r < 4; ++r) c->desc.sphere[w][r] = arm->sphere[k][r];
          ++w;
        }
  }
  Digits dg;
  c->pattern = twist_pattern(&c->desc, dg.v);

  hipError_t e;
  fn_arm_desc* d_desc = nullptr;
#define FN_ALLOC(ptr, bytes)                                              \
  do {                                                                    \
    e = hipMalloc((void**)&(ptr), (bytes) > 0 ? (bytes) : 16);            \
    if (e != hipSuccess) {                                                \
      fn_destroy(c);                                                      \
      if (d_desc) (void)hipFree(d_desc);                                     \
      return fail(FN_E_NOMEM, "fn_create: hipMalloc(%zu): %s", (size_t)(bytes), hipGetErrorString(e)); \
    }                                                                     \
  } while (0)
  FN_ALLOC(d_desc, sizeof(fn_arm_desc));
  FN_ALLOC(c->arm32, sizeof(ArmConst<float>));
  FN_ALLOC(c->arm64, sizeof(ArmConst<double>));
  // kNN partial lists of every (query, node chunk)
  const size_t kl = knn_scratch_entries(caps->max_batch, caps->max_k, caps->max_problems);
  FN_ALLOC(c->knn_d, kl * sizeof(float));
  FN_ALLOC(c->knn_i, kl * sizeof(int32_t));
  FN_ALLOC(c->knn_y, knn_scratch_entries(caps->max_batch, 0, caps->max_problems) * sizeof(float));
  // near-limit queue: counter + one entry per edge
  FN_ALLOC(c->q_count, 64 * sizeof(int32_t));
  FN_ALLOC(c->queue, (size_t)(caps->max_edges > 0 ? caps->max_edges : 1) * sizeof(QEntry));
  FN_ALLOC(c->model_e, (size_t)caps->max_edges * MODEL_FLOATS * sizeof(float));
  FN_ALLOC(c->model_c, (size_t)caps->max_batch * MODEL_FLOATS * sizeof(float));
  FN_ALLOC(c->tri_items, tri_ints(caps->max_edges > 0 ? caps->max_edges : 1) * sizeof(int32_t));
  FN_ALLOC(c->self_pairs, (size_t)2 * FN_MAX_SELF_PAIRS * sizeof(int16_t));
#undef FN_ALLOC
  {
    const int brc = batch_alloc(c);
    if (brc) {
      (void)hipFree(d_desc);
      fn_destroy(c);
      return brc;
    }
  }
  {
    // address of this device's scratch array of edge_time_batch_noalloc
    const int src = static_scratch_init();
    if (src) {
      (void)hipFree(d_desc);
      fn_destroy(c);
      return src;
    }
  }
  e = hipMemcpy(d_desc, &c->desc, sizeof(fn_arm_desc), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d_desc);
    fn_destroy(c);
    return hip_fail(e, "fn_create: copy arm");
  }
  hipLaunchKernelGGL(arm_prepare_kernel, dim3(1), dim3(64), 0, 0, d_desc, dg, c->pattern,
                     c->arm32, c->arm64);
  e = hipDeviceSynchronize();
  (void)hipFree(d_desc);
  if (e != hipSuccess) {
    fn_destroy(c);
    return hip_fail(e, "fn_create: arm constants");
  }
  *out = c;
  return FN_OK;
}

extern "C" int fn_kernel_timing(fn_ctx* c, int enable) {
  if (!c) return fail(FN_E_ARG, "fn_kernel_timing: NULL context");
  if (enable && !c->timing) {
    for (int i = 0; i < 2 * FN_MAX_TIMED; ++i) {
      const hipError_t e = hipEventCreate(&c->tev[i]);
      if (e != hipSuccess) {
        for (int j = 0; j < i; ++j) (void)hipEventDestroy(c->tev[j]);
        return hip_fail(e, "fn_kernel_timing: event");
      }
    }
    c->timing = true;
    c->n_timed = 0;
  } else if (!enable && c->timing) {
    (void)hipDeviceSynchronize();
    for (int i = 0; i < 2 * FN_MAX_TIMED; ++i) (void)hipEventDestroy(c->tev[i]);
    c->timing = false;
    c->n_timed = 0;
  }
  return FN_OK;
}

extern "C" int fn_kernel_times(fn_ctx* c, float* out_ms, int32_t max, int32_t* n_out) {
  if (!c || !n_out || (max > 0 && !out_ms)) return fail(FN_E_ARG, "fn_kernel_times: NULL argument");
  *n_out = 0;
  if (!c->timing) return FN_OK;
  const int n = c->n_timed < max ? c->n_timed : max;
  for (int i = 0; i < n; ++i) {
    hipError_t e = hipEventSynchronize(c->tev[2 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&out_ms[i], c->tev[2 * i], c->tev[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "fn_kernel_times");
  }
  *n_out = n;
  c->n_timed = 0;
  return FN_OK;
}

extern "C" void fn_destroy(fn_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  if (c->timing)
    for (int i = 0; i < 2 * FN_MAX_TIMED; ++i) (void)hipEventDestroy(c->tev[i]);
  batch_free(c);
  (void)hipFree(c->arm32);
  (void)hipFree(c->arm64);
  (void)hipFree(c->knn_d);
  (void)hipFree(c->knn_i);
  (void)hipFree(c->knn_y);
  (void)hipFree(c->q_count);
  (void)hipFree(c->queue);
  (void)hipFree(c->model_e);
  (void)hipFree(c->tri_items);
  (void)hipFree(c->model_c);
  (void)hipFree(c->self_pairs);
  delete c;
}

extern "C" int risk_score(fn_ctx* ctx, const fn_risk* w, const float* T, const float* v_rel,
                          const float* nu, const float* vz0, const float* t_fall, int32_t n,
                          float* out_J, void* stream) {
  if (!ctx || !w) return fail(FN_E_ARG, "risk_score: NULL context or weights");
  if (n < 0) return fail(FN_E_SHAPE, "risk_score: n = %d", n);
  if (n == 0) return FN_OK;
  if (!T || !v_rel || !nu || !vz0 || !t_fall || !out_J)
    return fail(FN_E_ARG, "risk_score: NULL array");
  if (w->sigma_mode != 0 && w->sigma_mode != 1)
    return fail(FN_E_ARG, "risk_score: sigma_mode %d", w->sigma_mode);
  hipLaunchKernelGGL(risk_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, *w, T,
                     v_rel, nu, vz0, t_fall, n, out_J);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FN_OK : hip_fail(e, "risk_score launch");
}
