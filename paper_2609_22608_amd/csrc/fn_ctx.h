// fn_ctx.h -- host-side context shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fn_internal.h"

namespace fn {

// kNN: most node chunks one query tile is split into
constexpr int KNN_MAX_SPLIT = 64;

struct Digits {
  int v[NJ];
};

// An edge whose decision hit a ratio within BAND of 1: the FP64 stage
// resumes it at slot j (phase 0) or redoes its post-checks (phase 1).
struct QEntry {
  int32_t edge;
  int16_t j;
  int16_t phase;
  float margin;
  int32_t work;
};

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* where);

__global__ void zero_i32_kernel(int32_t* p, int n);



// entries of the kNN partial-list scratch for these caps
// Largest kNN scan grid a tuning may ask for (waves); the partial-list
// scratch is sized for it.
constexpr int KNN_TARGET_MAX = 16384;
size_t knn_scratch_entries(int max_batch, int max_k, int max_problems);
// list length a kNN launch uses for k
// (k + 4 spare entries per node chunk, so that near ties at the k-th
// distance almost never force the exact rescan; 33 for k > 12)
inline int knn_k1(int k) { return k <= 12 ? k + 4 : 33; }

}  // namespace fn

struct fn_ctx;
int batch_alloc(fn_ctx* c);
void batch_free(fn_ctx* c);

struct fn_batch;

struct fn_ctx {
  int device;
  fn_tuning tune;     // launch mappings (0 = defaults)
  fn_batch* batch;    // batched-iteration state (NULL when max_problems = 0)
  int pattern;  // twist pattern code or PAT_GENERIC
  fn_caps caps;
  fn_arm_desc desc;  // host copy, spheres sorted by link
  fn::ArmConst<float>* arm32;
  fn::ArmConst<double>* arm64;
  float* knn_d;
  int32_t* knn_i;
  float* knn_y;  // per (query, chunk): max |y|^2 of the chunk
  int32_t* q_count;  // [0]: queue length
  fn::QEntry* queue;
  // endpoint models: of every edge's parent [max_edges][56], of every
  // candidate [max_batch][56]
  float* model_e;
  float* model_c;
  // kernel timing: event pairs around the search kernel of timed calls
  bool timing;
  int n_timed;
  hipEvent_t tev[2 * FN_MAX_TIMED];
};
