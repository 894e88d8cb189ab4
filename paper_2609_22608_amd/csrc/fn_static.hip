// fn_static.hip -- edge_time_batch_noalloc: the edge search with its scratch
// in a file-scope device array, for callers that cannot allocate device
// memory (code under graph capture, tight serving loops).
//
// The array holds, for at most FN_NOALLOC_MAX_EDGES edges: the FP64-stage
// counter (256 bytes), its queue (one 96-byte entry per edge), the
// endpoint models of every edge's parent and of every candidate (56 floats
// each) and the two-phase search's open-slot counts and edge order (8 bytes
// per edge, and 64 KiB of bin counts).  Each device holds its own copy for
// the life of the process; its address is taken once per device with
// hipGetSymbolAddress (at fn_create,
// or at the first call on a device), and only that address is used on the
// host.  Every call on one device shares the array: calls that overlap in
// time on one device (other streams, other threads) race.  The counter is
// cleared by the search's first kernel, so nothing needs clearing between
// calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fn_ctx.h"

namespace {

constexpr size_t kCounterBytes = 256;
constexpr size_t kQueueBytes = (size_t)FN_NOALLOC_MAX_EDGES * sizeof(fn::QEntry);
constexpr size_t kModelBytes = (size_t)FN_NOALLOC_MAX_EDGES * fn::MODEL_FLOATS * sizeof(float);
constexpr size_t kTriageBytes = fn::tri_ints(FN_NOALLOC_MAX_EDGES) * sizeof(int32_t);
constexpr size_t kScratchBytes = kCounterBytes + kQueueBytes + 2 * kModelBytes + kTriageBytes;
static_assert(kQueueBytes % 256 == 0 && kModelBytes % 256 == 0 && kTriageBytes % 256 == 0,
              "256-byte aligned parts");

// never named in host code except by hipGetSymbolAddress below
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's array (taken once), or NULL with the
// error set.
unsigned char* scratch_of_current(int* rc) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *rc = fn::hip_fail(e, "edge_time_batch_noalloc: hipGetDevice");
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *rc = fn::fail(FN_E_UNSUPPORTED, "edge_time_batch_noalloc: device %d (max %d)", dev, kMaxDevices);
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_lock);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *rc = fn::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                         "edge_time_batch_noalloc: hipGetSymbolAddress(scratch)");
      return nullptr;
    }
    g_ptr[dev] = p;
  }
  *rc = FN_OK;
  return static_cast<unsigned char*>(g_ptr[dev]);
}

}  // namespace

// Takes the current device's scratch address (called by fn_create).
int static_scratch_init() {
  int rc = FN_OK;
  scratch_of_current(&rc);
  return rc;
}

extern "C" size_t fn_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int edge_time_batch_noalloc(fn_ctx* c, const float* tree, int64_t ld, int32_t n_nodes,
                                       const float* cand, int32_t B, const int32_t* nbr,
                                       int32_t k, const fn_search* sr, const fn_obstacles* obs,
                                       const fn_edge_out* out, void* stream) {
  if (!c) return fn::fail(FN_E_ARG, "edge_time_batch_noalloc: NULL context");
  int rc = FN_OK;
  unsigned char* p = scratch_of_current(&rc);
  if (!p) return rc;
  const fn::EdgeScratch sc{reinterpret_cast<int32_t*>(p),
                           reinterpret_cast<fn::QEntry*>(p + kCounterBytes),
                           reinterpret_cast<float*>(p + kCounterBytes + kQueueBytes),
                           reinterpret_cast<float*>(p + kCounterBytes + kQueueBytes + kModelBytes),
                           reinterpret_cast<int32_t*>(p + kCounterBytes + kQueueBytes + 2 * kModelBytes)};
  return fn::edge_time_run(c, tree, ld, n_nodes, cand, B, nbr, k, sr, obs, out, stream, sc,
                           FN_NOALLOC_MAX_EDGES, "edge_time_batch_noalloc", false);
}
