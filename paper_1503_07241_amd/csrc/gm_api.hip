// Exported C ABI: argument validation, handle registry, error reporting and
// dispatch to the kernels. No device work is enqueued before a call's
// arguments have been checked.
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "gm_internal.h"

namespace gm {

namespace {
thread_local char g_msg[512] = "";
std::mutex g_reg_mu;
std::unordered_set<gm_graph>* g_reg = nullptr;
std::mutex g_fault_mu;
long g_alloc_count = 0;     // allocations since GM_FAULT_ALLOC last changed
std::string* g_fault_env = nullptr;  // its value when last read
}  // namespace

gm_status fail(gm_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
  va_end(ap);
  return st;
}

gm_status ok() {
  g_msg[0] = '\0';
  return GM_OK;
}

// Device allocations go through here. GM_FAULT_ALLOC=k makes the k-th
// allocation after the variable was set (or changed) fail, for tests of the
// error paths; it is read at every allocation, so a process can set, change
// and clear it between calls.
void* dmalloc(size_t bytes) {
  {
    std::lock_guard<std::mutex> lk(g_fault_mu);
    const char* e = getenv("GM_FAULT_ALLOC");
    const std::string now = e ? e : "";
    if (!g_fault_env) g_fault_env = new std::string();
    if (now != *g_fault_env) {
      *g_fault_env = now;
      g_alloc_count = 0;
    }
    const long at = e ? atol(e) : -1;
    ++g_alloc_count;
    if (at > 0 && g_alloc_count == at) throw OutOfMemory{bytes};
  }
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    throw OutOfMemory{bytes};
  }
  if (e != hipSuccess) throw HipError{e, "hipMalloc", __LINE__};
  return p;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

bool graph_live(gm_graph g) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  return g && g_reg && g_reg->count(g) && g->magic == kGraphMagic;
}

void graph_register(gm_graph g) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  if (!g_reg) g_reg = new std::unordered_set<gm_graph>();
  g_reg->insert(g);
}

void graph_unregister(gm_graph g) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  if (g_reg) g_reg->erase(g);
}

gm_status check_device(gm_graph g) {
  int dev = 0;
  GM_HIP(hipGetDevice(&dev));
  if (dev != g->device)
    return fail(GM_EINVAL, "graph lives on device %d, current is %d", g->device, dev);
  return GM_OK;
}

}  // namespace gm

using namespace gm;

extern "C" {

const char* gm_last_error(void) { return g_msg; }

const char* gm_version(void) { return "graphmat-mi355x 0.1 (gfx950)"; }

gm_status gm_graph_from_coo(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                            const void* w, int32_t wtype, uint32_t prep, uint32_t layouts,
                            void* stream, gm_graph* out) {
  if (!out) return fail(GM_EINVAL, "out is NULL");
  *out = nullptr;
  if (n <= 0 || n > INT32_MAX) return fail(GM_EINVAL, "n = %lld outside [1, 2^31-1]", (long long)n);
  if (m < 0) return fail(GM_EINVAL, "m = %lld is negative", (long long)m);
  if (m > 0 && (!src || !dst)) return fail(GM_EINVAL, "src/dst is NULL");
  if (wtype != GM_W_NONE && wtype != GM_W_U32 && wtype != GM_W_F32)
    return fail(GM_EINVAL, "unknown wtype %d", wtype);
  if ((wtype == GM_W_NONE) != (w == nullptr) && m > 0)
    return fail(GM_EINVAL, "w must be NULL exactly when wtype is GM_W_NONE");
  if (prep & ~(uint32_t)(GM_PREP_DROP_SELF_LOOPS | GM_PREP_SYMMETRIZE | GM_PREP_UPPER_DAG))
    return fail(GM_EINVAL, "unknown prep bits 0x%x", prep);
  if (layouts == 0 || (layouts & ~(uint32_t)(GM_LAYOUT_OUT | GM_LAYOUT_IN)))
    return fail(GM_EINVAL, "layouts 0x%x: need GM_LAYOUT_OUT and/or GM_LAYOUT_IN", layouts);
  for (int64_t e = 0; e < m; ++e) {
    if ((uint32_t)src[e] >= (uint64_t)n || (uint32_t)dst[e] >= (uint64_t)n)
      return fail(GM_EINVAL, "edge %lld (%d -> %d) has an id outside [0, %lld)", (long long)e,
                  src[e], dst[e], (long long)n);
  }
  if (wtype == GM_W_F32) {
    const float* wf = static_cast<const float*>(w);
    for (int64_t e = 0; e < m; ++e)
      if (!std::isfinite(wf[e]))
        return fail(GM_EINVAL, "weight of edge %lld is not finite", (long long)e);
  }
  gm_graph g = nullptr;
  return guarded([&]() -> gm_status {
    int dev = 0;
    GM_HIP(hipGetDevice(&dev));
    g = new gm_graph_s();
    g->magic = kGraphMagic;
    g->n = n;
    g->wtype = wtype;
    g->prep = prep;
    g->layouts = layouts | GM_LAYOUT_OUT;
    g->device = dev;
    try {
      build_graph(g, src, dst, w, m, static_cast<hipStream_t>(stream));
    } catch (...) {
      free_graph_memory(g);
      delete g;
      throw;
    }
    graph_register(g);
    *out = g;
    return ok();
  });
}

gm_status gm_graph_get_info(gm_graph g, gm_graph_info* info) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (!info) return fail(GM_EINVAL, "info is NULL");
  info->n = g->n;
  info->m = g->m;
  info->max_out = g->max_out;
  info->max_in = g->max_in;
  info->wtype = g->wtype;
  info->prep = g->prep;
  info->layouts = g->layouts;
  info->device = g->device;
  info->device_bytes = g->device_bytes;
  info->n_src = g->n_src;
  info->n_dst = g->n_dst;
  return ok();
}

gm_status gm_graph_edges(gm_graph g, int32_t* src, int32_t* dst, void* w) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (w && g->wtype == GM_W_NONE) return fail(GM_EINVAL, "graph has no edge values");
  return guarded([&]() -> gm_status {
    // a rating graph's out-adjacency has one row per user, ids are columns
    const int64_t n = g->bipartite ? g->n_rows : g->n, m = g->m;
    if (dst && m > 0) GM_HIP(hipMemcpy(dst, g->out_idx, m * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (w && m > 0) GM_HIP(hipMemcpy(w, g->out_w, m * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (src && m > 0) {
      uint32_t* off = new uint32_t[n + 1];
      const hipError_t e = hipMemcpy(off, g->out_off, (n + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        delete[] off;
        throw HipError{e, "hipMemcpy", __LINE__};
      }
      for (int64_t v = 0; v < n; ++v)
        for (uint32_t i = off[v]; i < off[v + 1]; ++i) src[i] = (int32_t)v;
      delete[] off;
    }
    return ok();
  });
}

gm_status gm_graph_destroy(gm_graph g) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  graph_unregister(g);
  free_min_workspace(g);
  free_pull_schedule(g);
  free_tc_plan(g);
  free_batch(g);
  free_cf_plan(g);
  free_vjp_plan(g);
  free_graph_memory(g);
  g->magic = 0;
  delete g;
  return ok();
}

gm_status gm_graph_prepare(gm_graph g, const gm_program* prog, void* stream) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (!prog) return fail(GM_EINVAL, "prog is NULL");
  if (g->bipartite) return fail(GM_EUNSUPPORTED, "rating graphs take the CF calls only");
  const int kind = prog->kind;
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (kind) {
    case GM_PROG_BFS:
    case GM_PROG_DEGREE:
      break;
    case GM_PROG_SSSP:
      if (g->wtype != GM_W_U32) return fail(GM_EUNSUPPORTED, "SSSP needs uint32 edge weights");
      break;
    case GM_PROG_PAGERANK:
    case GM_PROG_PPR:
      if (!(g->layouts & GM_LAYOUT_IN)) return fail(GM_EUNSUPPORTED, "PageRank needs GM_LAYOUT_IN");
      break;
    case GM_PROG_TC:
      if (!(g->prep & GM_PREP_UPPER_DAG) || !(g->layouts & GM_LAYOUT_IN))
        return fail(GM_EUNSUPPORTED, "triangle counting needs GM_PREP_UPPER_DAG and GM_LAYOUT_IN");
      break;
    default:
      return fail(GM_EINVAL, "unknown program kind %d", kind);
  }
  return guarded([&]() -> gm_status {
    if (const gm_status st = check_device(g)) return st;
    if (kind == GM_PROG_BFS || kind == GM_PROG_SSSP || kind == GM_PROG_DEGREE) {
      prepare_plain_min_program(g, kind, s);
    } else if (kind == GM_PROG_TC) {
      prepare_triangle_count(g, s);
    } else {
      ensure_pull_schedule(g, s);
      GM_HIP(hipStreamSynchronize(s));
    }
    return ok();
  });
}

gm_status gm_graph_release(gm_graph g) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  return guarded([&]() -> gm_status {
    if (const gm_status st = check_device(g)) return st;
    GM_HIP(hipDeviceSynchronize());  // nothing enqueued may still use the buffers
    free_min_workspace(g);
    free_pull_schedule(g);
    free_tc_plan(g);
    free_batch(g);
    free_cf_plan(g);
    free_vjp_plan(g);
    return ok();
  });
}

gm_status gm_run_vertex_program(gm_graph g, const gm_program* prog, const gm_frontier* frontier,
                                int32_t max_iters, void* vprop, int32_t* active_out,
                                int32_t* iters_done, void* stream) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (!prog) return fail(GM_EINVAL, "prog is NULL");
  if (!vprop) return fail(GM_EINVAL, "vprop is NULL");
  if (g->bipartite) return fail(GM_EUNSUPPORTED, "rating graphs take the CF calls only");
  const int kind = prog->kind;
  if (kind != GM_PROG_BFS && kind != GM_PROG_SSSP && kind != GM_PROG_PAGERANK &&
      kind != GM_PROG_PPR && kind != GM_PROG_TC && kind != GM_PROG_DEGREE)
    return fail(GM_EINVAL, "unknown program kind %d", kind);
  const int order = prog->order;
  if (order != GM_ORDER_OUT && order != GM_ORDER_IN && order != GM_ORDER_ALL)
    return fail(GM_EINVAL, "unknown order %d", order);
  const bool frontier_prog = kind == GM_PROG_BFS || kind == GM_PROG_SSSP || kind == GM_PROG_DEGREE;
  if (order != GM_ORDER_OUT && !frontier_prog)
    return fail(GM_EUNSUPPORTED, "order %d: this program runs along out-edges only", order);
  if (order != GM_ORDER_OUT && !(g->layouts & GM_LAYOUT_IN))
    return fail(GM_EUNSUPPORTED, "GM_ORDER_IN / GM_ORDER_ALL need GM_LAYOUT_IN");
  if (prog->flags != 0) return fail(GM_EINVAL, "flags must be 0");
  if (kind == GM_PROG_DEGREE) {
    if (frontier) return fail(GM_EINVAL, "the degree program takes no frontier (all vertices send)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return guarded([&]() -> gm_status {
      if (const gm_status st = check_device(g)) return st;
      // one superstep: every vertex sends once, nobody changes afterwards
      const int32_t it = run_min_program(g, kind, order, nullptr, 0, nullptr, 1,
                                         static_cast<uint32_t*>(vprop), active_out, s,
                                         &g->last_stats);
      if (iters_done) *iters_done = it;
      return ok();
    });
  }
  if (kind == GM_PROG_TC) {
    if (frontier) return fail(GM_EINVAL, "triangle counting takes no frontier (all vertices send)");
    if (!(g->prep & GM_PREP_UPPER_DAG) || !(g->layouts & GM_LAYOUT_IN))
      return fail(GM_EUNSUPPORTED, "triangle counting needs GM_PREP_UPPER_DAG and GM_LAYOUT_IN");
    return guarded([&]() -> gm_status {
      if (const gm_status st = check_device(g)) return st;
      run_triangle_count(g, static_cast<unsigned long long*>(vprop), nullptr,
                         static_cast<hipStream_t>(stream));
      if (active_out) fill_u32(reinterpret_cast<uint32_t*>(active_out), g->n, 0u,
                               static_cast<hipStream_t>(stream));
      g->last_stats = RunStats{};
      g->last_stats.supersteps = 1;
      g->last_stats.push_supersteps = 1;
      g->last_stats.edges_scanned = (unsigned long long)g->m;
      if (iters_done) *iters_done = 1;
      return ok();
    });
  }
  const bool dense = kind == GM_PROG_PAGERANK || kind == GM_PROG_PPR;
  if (dense) {
    if (max_iters <= 0) return fail(GM_EINVAL, "PageRank needs max_iters > 0");
    if (!(prog->r >= 0.0f && prog->r <= 1.0f)) return fail(GM_EINVAL, "r outside [0, 1]");
    if (!(g->layouts & GM_LAYOUT_IN)) return fail(GM_EUNSUPPORTED, "PageRank needs GM_LAYOUT_IN");
  }
  if (kind == GM_PROG_SSSP && g->wtype != GM_W_U32)
    return fail(GM_EUNSUPPORTED, "SSSP needs uint32 edge weights");
  const uint32_t* bitmap = nullptr;
  if (!dense || kind == GM_PROG_PPR) {
    if (!frontier) return fail(GM_EINVAL, "frontier is NULL");
    if (frontier->bitmap) {
      if (frontier->ids || frontier->count != 0)
        return fail(GM_EINVAL, "frontier: give ids or a bitmap, not both");
      if (kind == GM_PROG_PPR) return fail(GM_EINVAL, "PPR takes its seed from frontier ids");
      bitmap = frontier->bitmap;
    } else {
      if (frontier->count < 0 || frontier->count > g->n)
        return fail(GM_EINVAL, "frontier count %lld outside [0, n]", (long long)frontier->count);
      if (frontier->count > 0 && !frontier->ids) return fail(GM_EINVAL, "frontier ids NULL");
      if (kind == GM_PROG_PPR && frontier->count < 1) return fail(GM_EINVAL, "PPR needs a seed");
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() -> gm_status {
    if (const gm_status st = check_device(g)) return st;
    if (frontier && !bitmap && frontier->count > 0 &&
        !ids_in_range(frontier->ids, frontier->count, g->n, s))
      return fail(GM_EINVAL, "frontier id outside [0, n)");
    int32_t it = 0;
    if (dense) {
      int32_t seed = -1;
      if (kind == GM_PROG_PPR) {
        GM_HIP(hipMemcpyAsync(&seed, frontier->ids, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GM_HIP(hipStreamSynchronize(s));
      }
      run_pagerank(g, prog->r, max_iters, static_cast<float*>(vprop), seed, s);
      if (active_out) {
        // every vertex stays active in a dense program
        fill_u32(reinterpret_cast<uint32_t*>(active_out), g->n, 1u, s);
      }
      it = max_iters;
      g->last_stats = RunStats{};
      g->last_stats.supersteps = it;
      g->last_stats.pull_supersteps = it;
      g->last_stats.edges_scanned = (unsigned long long)g->m * it;
    } else {
      it = run_min_program(g, kind, order, bitmap ? nullptr : frontier->ids,
                           bitmap ? 0 : frontier->count, bitmap, max_iters,
                           static_cast<uint32_t*>(vprop), active_out, s, &g->last_stats);
    }
    if (iters_done) *iters_done = it;
    return ok();
  });
}

gm_status gm_triangle_count(gm_graph g, uint64_t* counts, uint64_t* total, void* stream) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (g->bipartite) return fail(GM_EUNSUPPORTED, "rating graphs take the CF calls only");
  if (!(g->prep & GM_PREP_UPPER_DAG) || !(g->layouts & GM_LAYOUT_IN))
    return fail(GM_EUNSUPPORTED, "triangle counting needs GM_PREP_UPPER_DAG and GM_LAYOUT_IN");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() -> gm_status {
    if (const gm_status st = check_device(g)) return st;
    unsigned long long* c = reinterpret_cast<unsigned long long*>(counts);
    unsigned long long* own = nullptr;
    if (!c) own = c = dalloc<unsigned long long>(g->n);
    try {
      zero_counts(c, g->n, s);
      unsigned long long t = 0;
      run_triangle_count(g, c, &t, s);
      if (total) *total = t;
    } catch (...) {
      dfree(own);
      throw;
    }
    if (own) {
      GM_HIP(hipStreamSynchronize(s));
      dfree(own);
    }
    return ok();
  });
}

gm_status gm_run_batched(gm_graph g, const gm_program* prog, const int32_t* sources, int32_t k,
                         int32_t max_iters, void* vprop_block, int32_t* iters_done, void* stream) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (!prog || !sources || !vprop_block) return fail(GM_EINVAL, "prog/sources/vprop_block is NULL");
  if (g->bipartite) return fail(GM_EUNSUPPORTED, "rating graphs take the CF calls only");
  const int kind = prog->kind;
  if (prog->order != GM_ORDER_OUT) return fail(GM_EINVAL, "only GM_ORDER_OUT is supported");
  if (prog->flags != 0) return fail(GM_EINVAL, "flags must be 0");
  if (kind == GM_PROG_BFS || kind == GM_PROG_SSSP) {
    if (k < 1 || k > 64) return fail(GM_EINVAL, "k = %d outside [1, 64]", k);
  } else if (kind == GM_PROG_PPR) {
    if (k < 1 || k > 256) return fail(GM_EINVAL, "k = %d outside [1, 256]", k);
    if (max_iters <= 0) return fail(GM_EINVAL, "PPR needs max_iters > 0");
    if (!(prog->r >= 0.0f && prog->r <= 1.0f)) return fail(GM_EINVAL, "r outside [0, 1]");
    if (!(g->layouts & GM_LAYOUT_IN)) return fail(GM_EUNSUPPORTED, "PPR needs GM_LAYOUT_IN");
  } else {
    return fail(GM_EINVAL, "batched runs support BFS, SSSP and PPR (kind %d)", kind);
  }
  if ((int64_t)k * g->n > ((int64_t)1 << 40)) return fail(GM_EUNSUPPORTED, "n * k too large");
  if (kind == GM_PROG_SSSP && g->wtype != GM_W_U32)
    return fail(GM_EUNSUPPORTED, "SSSP needs uint32 edge weights");
  const bool sym = (g->prep & (GM_PREP_SYMMETRIZE | GM_PREP_UPPER_DAG)) == GM_PREP_SYMMETRIZE;
  if (kind == GM_PROG_BFS && !sym && !(g->layouts & GM_LAYOUT_IN))
    return fail(GM_EUNSUPPORTED, "batched BFS on a directed graph needs GM_LAYOUT_IN");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() -> gm_status {
    if (const gm_status st = check_device(g)) return st;
    if (!ids_in_range(sources, k, g->n, s)) return fail(GM_EINVAL, "source id outside [0, n)");
    int32_t it = 0;
    if (kind == GM_PROG_BFS)
      it = run_batched_bfs(g, sources, k, max_iters, static_cast<int32_t*>(vprop_block), s);
    else if (kind == GM_PROG_SSSP)
      it = run_batched_sssp(g, sources, k, max_iters, static_cast<uint32_t*>(vprop_block), s);
    else {
      run_batched_ppr(g, sources, k, prog->r, max_iters, static_cast<float*>(vprop_block), s);
      it = max_iters;
    }
    if (iters_done) *iters_done = it;
    return ok();
  });
}

gm_status gm_bipartite_from_coo(int64_t n_rows, int64_t n_cols, int64_t m, const int32_t* row,
                                const int32_t* col, const uint8_t* val, void* stream,
                                gm_graph* out) {
  if (!out) return fail(GM_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_rows <= 0 || n_cols <= 0 || n_rows > INT32_MAX || n_cols > INT32_MAX)
    return fail(GM_EINVAL, "n_rows/n_cols outside [1, 2^31-1]");
  if (m < 0) return fail(GM_EINVAL, "m is negative");
  if (m > (int64_t)UINT32_MAX) return fail(GM_EUNSUPPORTED, "more than 2^32-1 ratings");
  if (m > 0 && (!row || !col || !val)) return fail(GM_EINVAL, "row/col/val is NULL");
  for (int64_t e = 0; e < m; ++e)
    if ((uint32_t)row[e] >= (uint64_t)n_rows || (uint32_t)col[e] >= (uint64_t)n_cols)
      return fail(GM_EINVAL, "rating %lld (%d, %d) outside the matrix", (long long)e, row[e], col[e]);
  return guarded([&]() -> gm_status {
    int dev = 0;
    GM_HIP(hipGetDevice(&dev));
    gm_graph g = new gm_graph_s();
    g->magic = kGraphMagic;
    g->bipartite = true;
    g->n_rows = n_rows;
    g->n_cols = n_cols;
    g->n = n_rows + n_cols;
    g->layouts = GM_LAYOUT_OUT | GM_LAYOUT_IN;
    g->device = dev;
    try {
      build_bipartite(g, row, col, val, m, static_cast<hipStream_t>(stream));
    } catch (...) {
      free_graph_memory(g);
      delete g;
      throw;
    }
    graph_register(g);
    *out = g;
    return ok();
  });
}

static gm_status check_cf(gm_graph g, int32_t K, const float* PU, const float* PV, float lambda) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (!g->bipartite) return fail(GM_EUNSUPPORTED, "CF needs a rating graph (gm_bipartite_from_coo)");
  if (K < 1 || K > 64) return fail(GM_EINVAL, "K = %d outside [1, 64]", K);
  if (!PU || !PV) return fail(GM_EINVAL, "PU/PV is NULL");
  if (!(lambda >= 0.0f) || !std::isfinite(lambda)) return fail(GM_EINVAL, "lambda must be >= 0");
  return GM_OK;
}

gm_status gm_cf_forward(gm_graph g, int32_t K, const float* PU, const float* PV, float lambda,
                        double* loss, void* stream) {
  const gm_status st = check_cf(g, K, PU, PV, lambda);
  if (st != GM_OK) return st;
  if (!loss) return fail(GM_EINVAL, "loss is NULL");
  return guarded([&]() -> gm_status {
    if (const gm_status st = check_device(g)) return st;
    run_cf_forward(g, K, PU, PV, lambda, loss, static_cast<hipStream_t>(stream));
    return ok();
  });
}

gm_status gm_cf_backward(gm_graph g, int32_t K, const float* PU, const float* PV, float lambda,
                         float scale, float* gPU, float* gPV, void* stream) {
  const gm_status st = check_cf(g, K, PU, PV, lambda);
  if (st != GM_OK) return st;
  if (!gPU && !gPV) return fail(GM_EINVAL, "gPU and gPV are both NULL");
  if (!std::isfinite(scale)) return fail(GM_EINVAL, "scale is not finite");
  return guarded([&]() -> gm_status {
    if (const gm_status st = check_device(g)) return st;
    run_cf_backward(g, K, PU, PV, lambda, scale, gPU, gPV, static_cast<hipStream_t>(stream));
    return ok();
  });
}

gm_status gm_cf_gd(gm_graph g, int32_t K, float* PU, float* PV, float lambda, float gamma,
                   int32_t iters, double* loss_hist, void* stream) {
  const gm_status st = check_cf(g, K, PU, PV, lambda);
  if (st != GM_OK) return st;
  if (iters < 0) return fail(GM_EINVAL, "iters = %d is negative", iters);
  if (!(gamma >= 0.0f) || !std::isfinite(gamma)) return fail(GM_EINVAL, "gamma must be >= 0");
  return guarded([&]() -> gm_status {
    if (const gm_status st = check_device(g)) return st;
    run_cf_gd(g, K, PU, PV, lambda, gamma, iters, loss_hist, static_cast<hipStream_t>(stream));
    return ok();
  });
}

static gm_status check_prw(gm_graph g, const float* w, float r, int32_t T) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (g->bipartite) return fail(GM_EUNSUPPORTED, "rating graphs take the CF calls only");
  if (!(g->layouts & GM_LAYOUT_IN)) return fail(GM_EUNSUPPORTED, "needs GM_LAYOUT_IN");
  if (!w && g->m > 0) return fail(GM_EINVAL, "w is NULL");  // unread without edges
  if (!(r >= 0.0f && r <= 1.0f)) return fail(GM_EINVAL, "r outside [0, 1]");
  if (T < 1) return fail(GM_EINVAL, "T must be >= 1");
  return GM_OK;
}

gm_status gm_pagerank_forward_w(gm_graph g, const float* w, float r, int32_t T, float* hist,
                                void* stream) {
  const gm_status st = check_prw(g, w, r, T);
  if (st != GM_OK) return st;
  if (!hist) return fail(GM_EINVAL, "hist is NULL");
  return guarded([&]() -> gm_status {
    if (const gm_status st = check_device(g)) return st;
    run_pagerank_history(g, w, r, T, hist, static_cast<hipStream_t>(stream));
    return ok();
  });
}

gm_status gm_pagerank_vjp_w(gm_graph g, const float* w, float r, int32_t T, const float* hist,
                            const float* grad_out, float* grad_w, void* stream) {
  const gm_status st = check_prw(g, w, r, T);
  if (st != GM_OK) return st;
  if (!hist || !grad_out || (!grad_w && g->m > 0))
    return fail(GM_EINVAL, "hist/grad_out/grad_w is NULL");
  return guarded([&]() -> gm_status {
    if (const gm_status st = check_device(g)) return st;
    run_pagerank_vjp(g, w, r, T, hist, grad_out, grad_w, static_cast<hipStream_t>(stream));
    return ok();
  });
}

gm_status gm_run_multi_graph(const gm_graph* graphs, int32_t count, const gm_program* prog,
                             const int32_t* sources, void* const* vprops, int32_t max_iters,
                             int32_t* iters_done, void* stream) {
  if (!graphs || !vprops || !prog) return fail(GM_EINVAL, "graphs/vprops/prog is NULL");
  if (count < 1) return fail(GM_EINVAL, "count = %d < 1", count);
  const int kind = prog->kind;
  if (kind == GM_PROG_PPR) return fail(GM_EUNSUPPORTED, "PPR is not run over several graphs");
  if (kind != GM_PROG_BFS && kind != GM_PROG_SSSP && kind != GM_PROG_PAGERANK &&
      kind != GM_PROG_TC)
    return fail(GM_EINVAL, "unknown program kind %d", kind);
  const bool frontier_prog = kind == GM_PROG_BFS || kind == GM_PROG_SSSP;
  if (frontier_prog && !sources) return fail(GM_EINVAL, "sources is NULL");
  if (!frontier_prog && sources) return fail(GM_EINVAL, "PageRank and TC take no sources");
  std::vector<int64_t> base(count + 1, 0);
  std::vector<int32_t> ids;
  for (int32_t i = 0; i < count; ++i) {
    if (!graph_live(graphs[i])) return fail(GM_ESTATE, "graph %d is not live", i);
    if (!vprops[i]) return fail(GM_EINVAL, "vprops[%d] is NULL", i);
    base[i + 1] = base[i] + graphs[i]->n;
    if (frontier_prog) {
      if (sources[i] < -1 || sources[i] >= graphs[i]->n)
        return fail(GM_EINVAL, "sources[%d] = %d outside [-1, n_%d)", i, sources[i], i);
      if (sources[i] >= 0) ids.push_back((int32_t)(base[i] + sources[i]));
    }
  }
  gm_graph u = nullptr;
  if (const gm_status st = gm_graph_union(graphs, count, stream, &u)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t elem = kind == GM_PROG_TC ? 8 : 4;
  void* prop = nullptr;
  int32_t* dids = nullptr;
  gm_status st = guarded([&]() -> gm_status {
    prop = dmalloc((size_t)base[count] * elem);
    dids = dalloc<int32_t>(ids.size());
    if (!ids.empty())
      GM_HIP(hipMemcpyAsync(dids, ids.data(), ids.size() * 4, hipMemcpyHostToDevice, s));
    for (int32_t i = 0; i < count; ++i)
      GM_HIP(hipMemcpyAsync(static_cast<char*>(prop) + base[i] * elem, vprops[i],
                            (size_t)graphs[i]->n * elem, hipMemcpyDeviceToDevice, s));
    return GM_OK;
  });
  if (st == GM_OK) {
    const gm_frontier fr{dids, (int64_t)ids.size(), nullptr};
    st = gm_run_vertex_program(u, prog, frontier_prog ? &fr : nullptr, max_iters, prop, nullptr,
                               iters_done, stream);
  }
  if (st == GM_OK) {
    st = guarded([&]() -> gm_status {
      for (int32_t i = 0; i < count; ++i)
        GM_HIP(hipMemcpyAsync(vprops[i], static_cast<char*>(prop) + base[i] * elem,
                              (size_t)graphs[i]->n * elem, hipMemcpyDeviceToDevice, s));
      GM_HIP(hipStreamSynchronize(s));
      return ok();
    });
  } else {
    (void)hipStreamSynchronize(s);
  }
  dfree(prop);
  dfree(dids);
  char msg[sizeof(g_msg)];
  std::snprintf(msg, sizeof(msg), "%s", g_msg);  // destroying the union clears it
  gm_graph_destroy(u);
  return st == GM_OK ? ok() : fail(st, "%s", msg);
}

static_assert(kNoallocScratchBytes == GM_NOALLOC_SCRATCH_BYTES,
              "the header states the array's size");

gm_status gm_pagerank_noalloc(gm_graph g, float r, int32_t iters, float* rank, void* stream) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (!rank) return fail(GM_EINVAL, "rank is NULL");
  if (g->bipartite) return fail(GM_EUNSUPPORTED, "rating graphs take the CF calls only");
  if (!(g->layouts & GM_LAYOUT_IN)) return fail(GM_EUNSUPPORTED, "PageRank needs GM_LAYOUT_IN");
  if (iters <= 0) return fail(GM_EINVAL, "PageRank needs iters > 0");
  if (!(r >= 0.0f && r <= 1.0f)) return fail(GM_EINVAL, "r outside [0, 1]");
  return guarded([&]() -> gm_status {
    if (const gm_status st = check_device(g)) return st;
    if (!pull_schedule_ready(g))
      return fail(GM_ESTATE, "the pull layout is not built: call gm_graph_prepare first");
    const size_t need = pagerank_noalloc_bytes(g);
    if (need > kNoallocScratchBytes)
      return fail(GM_EUNSUPPORTED, "a run on this graph needs %zu bytes of scratch; the "
                  "allocation-free array holds %zu", need, kNoallocScratchBytes);
    run_pagerank_noalloc(g, r, iters, rank, static_cast<hipStream_t>(stream));
    return ok();
  });
}

gm_status gm_last_run_stats(gm_graph g, gm_run_stats* out) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (!out) return fail(GM_EINVAL, "out is NULL");
  out->supersteps = g->last_stats.supersteps;
  out->push_supersteps = g->last_stats.push_supersteps;
  out->pull_supersteps = g->last_stats.pull_supersteps;
  out->edges_scanned = (int64_t)g->last_stats.edges_scanned;
  return ok();
}

}  // extern "C"
