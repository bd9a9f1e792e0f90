// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <new>
#include <string>

#include "gm.h"

namespace gm {

// ---------------------------------------------------------------------------
// Errors. Every exported function returns through these helpers so the
// thread-local message always matches the status.
// ---------------------------------------------------------------------------
gm_status fail(gm_status st, const char* fmt, ...);
gm_status ok();

struct HipError {
  hipError_t err;
  const char* what;
  int line;
};

#define GM_HIP(expr)                                                          \
  do {                                                                        \
    hipError_t _e = (expr);                                                   \
    if (_e != hipSuccess) throw ::gm::HipError{_e, #expr, __LINE__};          \
  } while (0)

// ---------------------------------------------------------------------------
// Device buffers
// ---------------------------------------------------------------------------
struct OutOfMemory {
  size_t bytes;
};

// A valid request the library cannot serve (reported as GM_EUNSUPPORTED).
struct Unsupported {
  const char* what;
};

// Device allocation that throws OutOfMemory / HipError.
void* dmalloc(size_t bytes);
void dfree(void* p);

template <class T>
T* dalloc(size_t count) {
  return static_cast<T*>(dmalloc(count * sizeof(T) + (count == 0 ? 16 : 0)));
}

// Counters of the last frontier-program run.
struct RunStats {
  int32_t supersteps = 0;
  int32_t push_supersteps = 0;
  int32_t pull_supersteps = 0;
  unsigned long long edges_scanned = 0;  // out-edges of the vertices that sent
};

struct Tuning {
  // BFS: pull superstep when the frontier holds more than n / pull_div vertices
  uint32_t pull_div = 128;
  // supersteps launched before the first host check of the frontier size;
  // each later batch doubles, up to 64
  uint32_t superstep_batch = 4;
  // workgroups of the push kernels (plain and batched SSSP)
  uint32_t push_blocks = 2048;
  // batched PPR: in-edges per work item
  uint32_t ppr_chunk = 128;
  // TC: owners whose in-list is at most this long use a per-wavefront table
  uint32_t tc_wave_max = 512;
  // TC: partner-list elements per wavefront / workgroup work item
  uint32_t tc_wave_work = 1u << 14;
  uint32_t tc_block_work = 1u << 23;
  // PageRank / PPR pull: messages of the first pr_hot labels read from LDS
  uint32_t pr_hot = 40960;
  // GM_VARIANT_* bits: alternative schedules for ablation
  uint32_t variant = 0;
};

// Per-run outcome recorded on the device by a captured plan.
struct PlanResult {
  int32_t iters;       // supersteps that started with an active vertex
  int32_t converged;   // 1 if no vertex was left active
  unsigned long long edges;  // out-edges of the vertices that sent
};

// Neighbour-index arrays hold this many extra entries after the last edge,
// so that kernels may read the aligned 64-byte line holding an edge whole
// (triangle counting reads aligned 32-byte units).
constexpr int64_t kIdxPad = 16;

// Most supersteps a captured BFS/SSSP run records.
constexpr int kMaxPlanSteps = 64;

}  // namespace gm

struct gm_graph_s {
  uint64_t magic;
  int64_t n = 0;
  int64_t m = 0;
  int32_t wtype = GM_W_NONE;
  uint32_t prep = 0;
  uint32_t layouts = 0;
  int device = 0;
  int64_t max_out = 0, max_in = 0;
  int64_t n_src = 0;  // vertices with out-degree > 0
  int64_t n_dst = 0;  // vertices with in-degree > 0 (0 without the in-layout)
  // out-adjacency (CSR of G; the columns of G^T in the paper's terms)
  uint32_t* out_off = nullptr;
  int32_t* out_idx = nullptr;
  void* out_w = nullptr;
  // in-adjacency (CSC of G)
  uint32_t* in_off = nullptr;
  int32_t* in_idx = nullptr;
  void* in_w = nullptr;
  uint32_t* in_eid = nullptr;  // canonical (CSR) edge id of each in-edge
  float* inv_outdeg = nullptr; // 1/outdeg, 0 for dangling vertices
  int64_t device_bytes = 0;
  void* min_ws = nullptr;    // frontier workspace of the min programs (minprog.hip)
  void* pr_sched = nullptr;  // pull schedule of the dense programs (pagerank.hip)
  void* tc_plan = nullptr;   // receiver lists of the triangle count (tc.hip)
  void* batch_ws = nullptr;  // workspace of the batched programs (batched.hip)
  void* cf_plan = nullptr;   // work items of the rating passes (cf.hip)
  void* vjp_plan = nullptr;  // row schedule of the PageRank adjoint (prgrad.hip)
  // bipartite rating graphs (gm_bipartite_from_coo): rows = users, cols = items;
  // out_* is the CSR by row, in_* the CSC by column, ratings in *_val.
  bool bipartite = false;
  int64_t n_rows = 0, n_cols = 0;
  uint8_t* out_val = nullptr;
  uint8_t* in_val = nullptr;
  gm::RunStats last_stats;
  gm::Tuning tune;
  // Bumped whenever a workspace buffer is freed or replaced, so that captured
  // plans holding its address can tell they are stale.
  uint64_t ws_gen = 0;
};

namespace gm {

constexpr uint64_t kGraphMagic = 0x4752'4150'484d'4154ull;  // "GRAPHMAT"

// Runs f, turning the library's exceptions into a status and message.
template <class F>
gm_status guarded(F&& f) {
  try {
    return f();
  } catch (const OutOfMemory& e) {
    return fail(GM_ENOMEM, "device allocation of %zu bytes failed", e.bytes);
  } catch (const Unsupported& e) {
    return fail(GM_EUNSUPPORTED, "%s", e.what);
  } catch (const HipError& e) {
    return fail(GM_EHIP, "%s: %s (%s:%d)", e.what, hipGetErrorString(e.err), __FILE__, e.line);
  } catch (const std::bad_alloc&) {
    return fail(GM_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(GM_EHIP, "unexpected internal error");
  }
}


// Handle registry (graph handles are validated on every call).
bool graph_live(gm_graph g);
void graph_register(gm_graph g);
// GM_OK when the calling thread's current device holds g, else GM_EINVAL
// with its message; HIP failures throw HipError (call inside guarded()).
gm_status check_device(gm_graph g);
void graph_unregister(gm_graph g);

// Device-side graph construction (graph_build.hip).
void build_graph(gm_graph g, const int32_t* src, const int32_t* dst, const void* w, int64_t m_in,
                 hipStream_t s);
void free_graph_memory(gm_graph g);

// PageRank family (pagerank.hip).
void ensure_pull_schedule(gm_graph g, hipStream_t s);
// Allocation-free PageRank: size of its fixed device array, whether g's pull
// layout exists, the bytes a run on g needs from the array, and the run.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
bool pull_schedule_ready(gm_graph g);
size_t pagerank_noalloc_bytes(gm_graph g);
void run_pagerank_noalloc(gm_graph g, float r, int32_t iters, float* rank, hipStream_t s);
void run_pagerank(gm_graph g, float r, int32_t iters, float* rank, int32_t seed, hipStream_t s);

// Min programs (minprog.hip). Returns supersteps done.
// The first frontier is `bitmap` (n bits) when non-NULL, else the ids.
// order: GM_ORDER_* (the edges messages travel along).
int32_t run_min_program(gm_graph g, int kind, int order, const int32_t* ids, int64_t count,
                        const uint32_t* bitmap, int32_t max_iters, uint32_t* prop,
                        int32_t* active_out, hipStream_t s, RunStats* stats);
void free_min_workspace(gm_graph g);
void free_pull_schedule(gm_graph g);

// Triangle counting (tc.hip): counts[v] += triangles whose largest vertex is
// v; *total_host (optional) = sum of counts after the call (synchronises).
void run_triangle_count(gm_graph g, unsigned long long* counts, unsigned long long* total_host,
                        hipStream_t s);
void zero_counts(unsigned long long* a, int64_t n, hipStream_t s);
void free_tc_plan(gm_graph g);

// Batched programs (batched.hip); return supersteps run.
int32_t run_batched_bfs(gm_graph g, const int32_t* sources, int k, int32_t max_iters,
                        int32_t* level, hipStream_t s);
int32_t run_batched_sssp(gm_graph g, const int32_t* sources, int k, int32_t max_iters,
                         uint32_t* dist, hipStream_t s);
void run_batched_ppr(gm_graph g, const int32_t* seeds, int k, float r, int32_t iters, float* out,
                     hipStream_t s);
void free_batch(gm_graph g);

// Collaborative filtering (cf.hip).
void build_bipartite(gm_graph g, const int32_t* row, const int32_t* col, const uint8_t* val,
                     int64_t m, hipStream_t s);
void run_cf_forward(gm_graph g, int K, const float* PU, const float* PV, float lambda,
                    double* loss_dev, hipStream_t s);
void run_cf_backward(gm_graph g, int K, const float* PU, const float* PV, float lambda, float scale,
                     float* gPU, float* gPV, hipStream_t s);
void run_cf_gd(gm_graph g, int K, float* PU, float* PV, float lambda, float gamma, int32_t iters,
               double* loss_hist, hipStream_t s);
void free_cf_plan(gm_graph g);

// Weighted PageRank with history and its edge-weight VJP (pagerank.hip,
// prgrad.hip). hist is (T + 1) x n in the caller's labels.
void run_pagerank_history(gm_graph g, const float* w, float r, int32_t T, float* hist,
                          hipStream_t s);
void run_pagerank_vjp(gm_graph g, const float* w, float r, int32_t T, const float* hist,
                      const float* grad_out, float* grad_w, hipStream_t s);
void free_vjp_plan(gm_graph g);

// The frontier workspace of the plain BFS/SSSP/degree runs and, when the
// tuning asks for the degree order, their relabelled adjacency along
// out-edges (with BFS's pull layout).
void prepare_plain_min_program(gm_graph g, int kind, hipStream_t s);

// Captured-run building blocks (no allocation, no host synchronisation once
// the prepare_* call for the same graph and shape has run).
void prepare_min_program(gm_graph g, hipStream_t s);
void enqueue_min_program(gm_graph g, int kind, const int32_t* ids, int64_t count, int32_t steps,
                         uint32_t* prop, PlanResult* res, hipStream_t s);
void prepare_batched(gm_graph g, int kind, int k, hipStream_t s);
void enqueue_batched(gm_graph g, int kind, const int32_t* sources, int k, int32_t steps, float r,
                     void* block, PlanResult* res, hipStream_t s);
void prepare_triangle_count(gm_graph g, hipStream_t s);
void enqueue_pagerank(gm_graph g, float r, int32_t iters, float* rank, hipStream_t s);
// res <- {iters, 1, edges}
void set_plan_result(PlanResult* res, int32_t iters, unsigned long long edges, hipStream_t s);
void fill_f32(float* p, int64_t n, float v, hipStream_t s);

// Tuning checks and the scratch-output runs of the autotuner (plan.hip,
// minprog.hip).
void init_min_prop(gm_graph g, int kind, const int32_t* ids, int64_t count, uint32_t* prop,
                   hipStream_t s);

// Block-diagonal union of graphs (union.hip).
void build_union(gm_graph u, const gm_graph* parts, int32_t count, hipStream_t s);

// Fill n uint32 words with v on stream s (a kernel, safe under graph capture).
void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);

// Validate device ids in [0, n): returns false if any is out of range.
bool ids_in_range(const int32_t* ids, int64_t count, int64_t n, hipStream_t s);

}  // namespace gm
