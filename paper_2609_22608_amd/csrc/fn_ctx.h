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

// An edge whose decision rests on a ratio within BAND of 1, handed to the
// FP64 stage.  Phase 0: slot j is the first slot whose FP32 ratio is within
// the band; the FP32 search went on to j2, the first slot above j that is
// feasible in FP32 or again within the band (PH_J2_NEAR), or -1 when there is
// none.  Phase 1 (PH_POST): j is the result and a post-check ratio at j is
// within the band.  FP32 post-check ratios (rho_v, rho_q, rho_c) come along
// for j (post[0..2]) and j2 (post[3..5]).
struct QEntry {
  int32_t edge;
  int16_t j;
  int16_t phase;
  int16_t j2;
  int16_t wlo;       // window mode: lowest slot of the window
  int32_t work;      // evaluated sample lanes of the FP32 search
  float margin;      // smallest |rho - 1| of the slots below j
  float margin2;     // the same over the slots in (j, j2], FP32
  float rho;         // FP32 ratio of slot j
  float rho2;        // FP32 ratio of slot j2 (of the last slot when j2 = -1)
  float post[6];
  uint32_t pad2[2];
  uint64_t todo[4];  // slots not certified infeasible (bit t: slot t)
};
static_assert(sizeof(QEntry) == 96, "queue entry layout");

// Ordered two-phase search (form 3): between the triage and the search, a
// counting sort puts the open edges in descending order of their open-slot
// count (TRI_BINS equal ranges over 1..n_t), so that the longest searches
// start first and the short ones fill in behind them instead of a few long
// ones starting last.  The sort runs over at most TRI_MAX_BLOCKS blocks of
// at least TRI_MIN_CHUNK edges each.
constexpr int TRI_BINS = 64;
constexpr int TRI_MAX_BLOCKS = 256;
constexpr int64_t TRI_MIN_CHUNK = 1024;
// ints of the two-phase scratch for max_edges edges: the open-slot counts
// [max_edges], the order [max_edges], the per-block bin counts
// [TRI_MAX_BLOCKS][TRI_BINS] and the open-edge count (64 ints)
__host__ __device__ constexpr size_t tri_ints(int64_t max_edges) {
  return 2 * (size_t)max_edges + (size_t)TRI_MAX_BLOCKS * TRI_BINS + 64;
}

// Scratch of one edge search: the FP64-stage counter (first int32; the
// search's first kernel clears it) and queue (one entry per edge), the
// endpoint models of every edge's parent and of every candidate.
struct EdgeScratch {
  int32_t* q_count;  // the FP64-stage queue length (64 ints)
  QEntry* queue;
  float* model_e;
  float* model_c;
  int32_t* tri_items;  // [tri_ints(max edges)]: the two-phase search's counts, order, bins
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
// (at least k + 4 spare entries per node chunk, so that near ties at the
// k-th distance almost never force the exact rescan: k + 4 up to k = 12,
// then 20, 24 and 33 for k up to 16, 20 and 32)
inline int knn_k1(int k) { return k <= 12 ? k + 4 : (k <= 16 ? 20 : (k <= 20 ? 24 : 33)); }

}  // namespace fn

struct fn_ctx;
int batch_alloc(fn_ctx* c);
void batch_free(fn_ctx* c);
// scratch of edge_time_batch_noalloc on the current device (fn_static.hip)
int static_scratch_init();

namespace fn {
int edge_time_run(fn_ctx* c, const float* tree, int64_t ld, int32_t n_nodes, const float* cand,
                  int32_t B, const int32_t* nbr, int32_t k, const fn_search* sr,
                  const fn_obstacles* obs, const fn_edge_out* out, void* stream,
                  const EdgeScratch& sc, int64_t max_edges, const char* who, bool timed);
}  // namespace fn

struct fn_batch;

struct fn_ctx {
  int device;
  int n_cu;           // compute units of the device
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
  int32_t* tri_items;  // [max_edges]: open-slot counts of the two-phase search
  // endpoint models: of every edge's parent [max_edges][56], of every
  // candidate [max_batch][56]
  float* model_e;
  float* model_c;
  // self-collision pairs of the fixed-duration check (link-sorted sphere
  // indices, device [FN_MAX_SELF_PAIRS][2]) and the caller's sphere index ->
  // link-sorted index
  int16_t* self_pairs;
  int n_self;
  float margin_self;
  int sphere_order[FN_MAX_SPHERES];
  // kernel timing: event pairs around the search kernel of timed calls
  bool timing;
  int n_timed;
  hipEvent_t tev[2 * FN_MAX_TIMED];
};
