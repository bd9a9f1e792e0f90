// Mixed batches, captured runs and tuning (C ABI).
//
//  - gm_graph_union: the graphs of a mixed batch as one block-diagonal graph
//    (union.hip), so one generalized SpMV per superstep serves all of them.
//  - gm_plan_*: a sequence of runs recorded once as a HIP graph and replayed
//    with a single launch. Every superstep of Alg. 2 is enqueued up front; the
//    frontier test that ends a run happens on the device (a superstep whose
//    frontier is empty does no work), so no host round trip separates the
//    supersteps. Outputs are initialised inside the recording.
//  - gm_autotune: coordinate descent over the schedule parameters of a
//    program, timed with HIP events on the caller's stream.
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <unordered_set>
#include <vector>

#include "gm_internal.h"

namespace gm {
namespace {

__global__ void put_result(PlanResult* r, int32_t iters, unsigned long long edges) {
  r->iters = iters;
  r->converged = 1;
  r->edges = edges;
}

}  // namespace

void set_plan_result(PlanResult* res, int32_t iters, unsigned long long edges, hipStream_t s) {
  put_result<<<1, 1, 0, s>>>(res, iters, edges);
  GM_HIP(hipGetLastError());
}

void fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  uint32_t bits;
  std::memcpy(&bits, &v, 4);
  fill_u32(reinterpret_cast<uint32_t*>(p), n, bits, s);
}

}  // namespace gm

struct gm_plan_s {
  uint64_t magic = 0;
  int device = 0;
  std::vector<gm_plan_run> runs;
  std::vector<uint64_t> gens;  // workspace generation of each run's graph at capture
  gm::PlanResult* res = nullptr;
  gm::PlanResult* host_res = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool launched = false;
};

namespace gm {
namespace {

constexpr uint64_t kPlanMagic = 0x504c'414e'4752'4150ull;
std::mutex g_plan_mu;
std::unordered_set<gm_plan>* g_plans = nullptr;

bool plan_live(gm_plan p) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  return p && g_plans && g_plans->count(p) && p->magic == kPlanMagic;
}

void free_plan(gm_plan p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  dfree(p->res);
  if (p->host_res) (void)hipHostFree(p->host_res);
  p->magic = 0;
  delete p;
}

bool sym_graph(gm_graph g) {
  return (g->prep & (GM_PREP_SYMMETRIZE | GM_PREP_UPPER_DAG)) == GM_PREP_SYMMETRIZE;
}

// Validation of one plan run (no device work).
gm_status check_run(const gm_plan_run& r, int i) {
  gm_graph g = r.g;
  if (!graph_live(g)) return fail(GM_ESTATE, "run %d: graph handle is not live", i);
  if (g->bipartite) return fail(GM_EUNSUPPORTED, "run %d: rating graphs take the CF calls only", i);
  const gm_program& p = r.prog;
  if (p.order != GM_ORDER_OUT) return fail(GM_EINVAL, "run %d: only GM_ORDER_OUT is supported", i);
  if (p.flags != 0) return fail(GM_EINVAL, "run %d: flags must be 0", i);
  if (!r.vprop) return fail(GM_EINVAL, "run %d: vprop is NULL", i);
  const int kind = p.kind;
  if (kind == GM_PROG_SSSP && g->wtype != GM_W_U32)
    return fail(GM_EUNSUPPORTED, "run %d: SSSP needs uint32 edge weights", i);
  if (r.batched) {
    if (kind == GM_PROG_BFS || kind == GM_PROG_SSSP) {
      if (r.count < 1 || r.count > 64) return fail(GM_EINVAL, "run %d: k outside [1, 64]", i);
      if (r.max_iters < 1 || r.max_iters > kMaxPlanSteps)
        return fail(GM_EINVAL, "run %d: max_iters outside [1, %d]", i, kMaxPlanSteps);
      if (kind == GM_PROG_BFS && !sym_graph(g) && !(g->layouts & GM_LAYOUT_IN))
        return fail(GM_EUNSUPPORTED, "run %d: batched BFS on a directed graph needs GM_LAYOUT_IN", i);
    } else if (kind == GM_PROG_PPR) {
      if (r.count < 1 || r.count > 256) return fail(GM_EINVAL, "run %d: k outside [1, 256]", i);
      if (r.max_iters < 1) return fail(GM_EINVAL, "run %d: PPR needs max_iters > 0", i);
      if (!(p.r >= 0.0f && p.r <= 1.0f)) return fail(GM_EINVAL, "run %d: r outside [0, 1]", i);
      if (!(g->layouts & GM_LAYOUT_IN)) return fail(GM_EUNSUPPORTED, "run %d: PPR needs GM_LAYOUT_IN", i);
    } else {
      return fail(GM_EINVAL, "run %d: batched runs support BFS, SSSP and PPR", i);
    }
    if (r.count * g->n > ((int64_t)1 << 40)) return fail(GM_EUNSUPPORTED, "run %d: n * k too large", i);
    if (!r.ids) return fail(GM_EINVAL, "run %d: ids is NULL", i);
    return GM_OK;
  }
  switch (kind) {
    case GM_PROG_BFS:
    case GM_PROG_SSSP:
      if (r.max_iters < 1 || r.max_iters > kMaxPlanSteps)
        return fail(GM_EINVAL, "run %d: max_iters outside [1, %d]", i, kMaxPlanSteps);
      if (r.count < 0 || r.count > g->n) return fail(GM_EINVAL, "run %d: count outside [0, n]", i);
      if (r.count > 0 && !r.ids) return fail(GM_EINVAL, "run %d: ids is NULL", i);
      return GM_OK;
    case GM_PROG_PAGERANK:
      if (r.max_iters < 1) return fail(GM_EINVAL, "run %d: PageRank needs max_iters > 0", i);
      if (!(p.r >= 0.0f && p.r <= 1.0f)) return fail(GM_EINVAL, "run %d: r outside [0, 1]", i);
      if (!(g->layouts & GM_LAYOUT_IN))
        return fail(GM_EUNSUPPORTED, "run %d: PageRank needs GM_LAYOUT_IN", i);
      return GM_OK;
    case GM_PROG_TC:
      if (!(g->prep & GM_PREP_UPPER_DAG) || !(g->layouts & GM_LAYOUT_IN))
        return fail(GM_EUNSUPPORTED, "run %d: triangle counting needs GM_PREP_UPPER_DAG and GM_LAYOUT_IN", i);
      return GM_OK;
    case GM_PROG_PPR:
      return fail(GM_EUNSUPPORTED, "run %d: plain PPR is not recorded; use a batched run with k = 1", i);
    default:
      return fail(GM_EINVAL, "run %d: unknown program kind %d", i, kind);
  }
}

// Allocate (outside the capture) everything run r needs.
void prepare_run(const gm_plan_run& r, hipStream_t s) {
  gm_graph g = r.g;
  const int kind = r.prog.kind;
  if (r.batched)
    prepare_batched(g, kind, (int)r.count, s);
  else if (kind == GM_PROG_BFS || kind == GM_PROG_SSSP)
    prepare_min_program(g, s);
  else if (kind == GM_PROG_PAGERANK)
    ensure_pull_schedule(g, s);
  else
    prepare_triangle_count(g, s);
}

void enqueue_run(const gm_plan_run& r, PlanResult* res, hipStream_t s) {
  gm_graph g = r.g;
  const int kind = r.prog.kind;
  if (r.batched) {
    enqueue_batched(g, kind, r.ids, (int)r.count, r.max_iters, r.prog.r, r.vprop, res, s);
  } else if (kind == GM_PROG_BFS || kind == GM_PROG_SSSP) {
    enqueue_min_program(g, kind, r.ids, r.count, r.max_iters, static_cast<uint32_t*>(r.vprop),
                        res, s);
  } else if (kind == GM_PROG_PAGERANK) {
    enqueue_pagerank(g, r.prog.r, r.max_iters, static_cast<float*>(r.vprop), s);
    set_plan_result(res, r.max_iters, (unsigned long long)g->m * r.max_iters, s);
  } else {
    unsigned long long* c = static_cast<unsigned long long*>(r.vprop);
    zero_counts(c, g->n, s);
    run_triangle_count(g, c, nullptr, s);
    set_plan_result(res, 1, (unsigned long long)g->m, s);
  }
}

// ---------------------------------------------------------------- tuning --
struct Range {
  uint32_t lo, hi;
};

gm_status check_tuning(const gm_tuning& t) {
  struct F {
    const char* name;
    uint32_t v;
    Range r;
  } f[] = {{"pull_div", t.pull_div, {1, 65536}},
           {"superstep_batch", t.superstep_batch, {1, 64}},
           {"push_blocks", t.push_blocks, {64, 65536}},
           {"ppr_chunk", t.ppr_chunk, {64, 65536}},
           {"tc_wave_max", t.tc_wave_max, {64, 512}},
           {"tc_wave_work", t.tc_wave_work, {256, 1u << 24}},
           {"tc_block_work", t.tc_block_work, {256, 1u << 26}},
           {"pr_hot", t.pr_hot, {0, 40960}},
           {"variant", t.variant, {0, 15}}};
  for (const F& x : f)
    if (x.v < x.r.lo || x.v > x.r.hi)
      return fail(GM_EINVAL, "%s = %u outside [%u, %u]", x.name, x.v, x.r.lo, x.r.hi);
  return GM_OK;
}

gm_tuning to_abi(const Tuning& t) {
  gm_tuning o;
  o.pull_div = t.pull_div;
  o.superstep_batch = t.superstep_batch;
  o.push_blocks = t.push_blocks;
  o.ppr_chunk = t.ppr_chunk;
  o.tc_wave_max = t.tc_wave_max;
  o.tc_wave_work = t.tc_wave_work;
  o.tc_block_work = t.tc_block_work;
  o.pr_hot = t.pr_hot;
  o.variant = t.variant;
  return o;
}

void from_abi(const gm_tuning& o, Tuning* t) {
  t->pull_div = o.pull_div;
  t->superstep_batch = o.superstep_batch;
  t->push_blocks = o.push_blocks;
  t->ppr_chunk = o.ppr_chunk;
  t->tc_wave_max = o.tc_wave_max;
  t->tc_wave_work = o.tc_wave_work;
  t->tc_block_work = o.tc_block_work;
  t->pr_hot = o.pr_hot;
  t->variant = o.variant;
}

// ---------------------------------------------------------------------------
// Autotuner cache: a JSON object of entries "key": {"field": value, ...},
// one entry per line, fields as in gm_tuning. Only that shape is read.
// ---------------------------------------------------------------------------
using TuneCache = std::map<std::string, gm_tuning>;

struct CacheParser {
  const std::string& t;
  size_t i = 0;
  bool ok = true;

  void ws() {
    while (i < t.size() && std::isspace((unsigned char)t[i])) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < t.size() && t[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  void need(char c) {
    if (!eat(c)) ok = false;
  }
  std::string str() {
    ws();
    std::string out;
    if (i >= t.size() || t[i] != '"') {
      ok = false;
      return out;
    }
    for (++i; i < t.size() && t[i] != '"'; ++i) out += t[i];
    if (i >= t.size()) ok = false;
    ++i;
    return out;
  }
  uint64_t num() {
    ws();
    uint64_t v = 0;
    const size_t b = i;
    while (i < t.size() && std::isdigit((unsigned char)t[i]) && v <= UINT32_MAX)
      v = v * 10 + (uint64_t)(t[i++] - '0');
    if (i == b || v > UINT32_MAX) ok = false;
    return v;
  }
};

// Entries of the file at path (an absent file is an empty cache); false if
// the text is not of the expected shape or a value is out of range.
bool read_cache(const char* path, TuneCache* out) {
  std::ifstream f(path);
  if (!f) return true;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  CacheParser p{text};
  p.need('{');
  if (!p.ok) return false;
  if (p.eat('}')) return true;
  do {
    const std::string key = p.str();
    p.need(':');
    p.need('{');
    gm_tuning t = to_abi(Tuning{});
    if (!p.eat('}')) {
      do {
        const std::string field = p.str();
        p.need(':');
        const uint32_t v = (uint32_t)p.num();
        if (field == "pull_div") t.pull_div = v;
        else if (field == "superstep_batch") t.superstep_batch = v;
        else if (field == "push_blocks") t.push_blocks = v;
        else if (field == "ppr_chunk") t.ppr_chunk = v;
        else if (field == "tc_wave_max") t.tc_wave_max = v;
        else if (field == "tc_wave_work") t.tc_wave_work = v;
        else if (field == "tc_block_work") t.tc_block_work = v;
        else if (field == "pr_hot") t.pr_hot = v;
        else if (field == "variant") t.variant = v;
        else p.ok = false;
      } while (p.ok && p.eat(','));
      p.need('}');
    }
    if (!p.ok || check_tuning(t) != GM_OK) return false;
    (*out)[key] = t;
  } while (p.eat(','));
  p.need('}');
  return p.ok;
}

bool write_cache(const char* path, const TuneCache& c) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << "{\n";
    size_t k = 0;
    for (const auto& e : c) {
      const gm_tuning& t = e.second;
      f << "  \"" << e.first << "\": {\"pull_div\": " << t.pull_div
        << ", \"superstep_batch\": " << t.superstep_batch << ", \"push_blocks\": " << t.push_blocks
        << ", \"ppr_chunk\": " << t.ppr_chunk << ", \"tc_wave_max\": " << t.tc_wave_max
        << ", \"tc_wave_work\": " << t.tc_wave_work << ", \"tc_block_work\": " << t.tc_block_work
        << ", \"pr_hot\": " << t.pr_hot << ", \"variant\": " << t.variant << "}"
        << (++k < c.size() ? "," : "") << "\n";
    }
    f << "}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

// Cache key: device architecture, program, and the graph's shape (log2 n,
// log2 of the average degree, rounded).
std::string cache_key(gm_graph g, int kind, bool batched, int64_t k) {
  hipDeviceProp_t prop;
  GM_HIP(hipGetDeviceProperties(&prop, g->device));
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  static const char* const names[] = {"?", "bfs", "sssp", "pagerank", "ppr", "tc"};
  const char* name = kind >= 1 && kind <= 5 ? names[kind] : names[0];
  const int ln = (int)std::lround(std::log2((double)std::max<int64_t>(g->n, 1)));
  const double avg = (double)std::max<int64_t>(g->m, 1) / (double)std::max<int64_t>(g->n, 1);
  const int ld = (int)std::lround(std::log2(avg));
  char buf[160];
  std::snprintf(buf, sizeof(buf), "%s|%s|batched=%d|k=%lld|log2n=%d|log2deg=%d", arch.c_str(), name,
                batched ? 1 : 0, (long long)k, ln, ld);
  return buf;
}

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  Events() {
    GM_HIP(hipEventCreate(&a));
    const hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
      (void)hipEventDestroy(a);
      throw HipError{e, "hipEventCreate", __LINE__};
    }
  }
  ~Events() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

struct Scratch {
  void* p = nullptr;
  ~Scratch() { dfree(p); }
};

// One tuning trial: the program run once on scratch outputs.
struct Trial {
  gm_graph g;
  int kind;
  bool batched;
  const int32_t* ids;
  int64_t count;
  int32_t max_iters;
  float r;
  void* out;
  void operator()(hipStream_t s) const {
    if (batched) {
      if (kind == GM_PROG_BFS)
        run_batched_bfs(g, ids, (int)count, max_iters, static_cast<int32_t*>(out), s);
      else if (kind == GM_PROG_SSSP)
        run_batched_sssp(g, ids, (int)count, max_iters, static_cast<uint32_t*>(out), s);
      else
        run_batched_ppr(g, ids, (int)count, r, max_iters, static_cast<float*>(out), s);
    } else if (kind == GM_PROG_BFS || kind == GM_PROG_SSSP) {
      uint32_t* prop = static_cast<uint32_t*>(out);
      init_min_prop(g, kind, ids, count, prop, s);
      RunStats st{};
      run_min_program(g, kind, GM_ORDER_OUT, ids, count, nullptr, max_iters, prop, nullptr, s,
                      &st);
    } else if (kind == GM_PROG_PAGERANK) {
      fill_f32(static_cast<float*>(out), g->n, 1.0f, s);
      run_pagerank(g, r, max_iters, static_cast<float*>(out), -1, s);
    } else {
      unsigned long long* c = static_cast<unsigned long long*>(out);
      zero_counts(c, g->n, s);
      run_triangle_count(g, c, nullptr, s);
    }
  }
};

// Median time (ms) of `trials` runs after one warm-up run.
float time_trial(const Trial& t, int trials, hipStream_t s, Events& ev) {
  t(s);
  GM_HIP(hipStreamSynchronize(s));
  std::vector<float> ms;
  for (int i = 0; i < trials; ++i) {
    GM_HIP(hipEventRecord(ev.a, s));
    t(s);
    GM_HIP(hipEventRecord(ev.b, s));
    GM_HIP(hipEventSynchronize(ev.b));
    float x = 0;
    GM_HIP(hipEventElapsedTime(&x, ev.a, ev.b));
    ms.push_back(x);
  }
  std::sort(ms.begin(), ms.end());
  return ms[ms.size() / 2];
}

}  // namespace
}  // namespace gm

using namespace gm;

extern "C" {

gm_status gm_graph_union(const gm_graph* parts, int32_t count, void* stream, gm_graph* out) {
  if (!out) return fail(GM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!parts) return fail(GM_EINVAL, "parts is NULL");
  if (count < 1) return fail(GM_EINVAL, "count = %d < 1", count);
  int64_t n = 0, m = 0;
  for (int32_t i = 0; i < count; ++i) {
    const gm_graph p = parts[i];
    if (!graph_live(p)) return fail(GM_ESTATE, "part %d is not a live graph", i);
    if (p->bipartite) return fail(GM_EUNSUPPORTED, "part %d is a rating graph", i);
    if (p->prep != parts[0]->prep || p->wtype != parts[0]->wtype ||
        p->layouts != parts[0]->layouts)
      return fail(GM_EINVAL, "part %d differs from part 0 in prep, wtype or layouts", i);
    n += p->n;
    m += p->m;
  }
  if (n > INT32_MAX) return fail(GM_EUNSUPPORTED, "%lld vertices in total", (long long)n);
  if (m > (int64_t)UINT32_MAX) return fail(GM_EUNSUPPORTED, "%lld edges in total", (long long)m);
  return guarded([&]() -> gm_status {
    int dev = 0;
    GM_HIP(hipGetDevice(&dev));
    for (int32_t i = 0; i < count; ++i)
      if (parts[i]->device != dev)
        return fail(GM_EINVAL, "part %d lives on device %d, current is %d", i, parts[i]->device, dev);
    gm_graph u = new gm_graph_s();
    u->magic = kGraphMagic;
    u->n = n;
    u->m = m;
    u->wtype = parts[0]->wtype;
    u->prep = parts[0]->prep;
    u->layouts = parts[0]->layouts;
    u->device = dev;
    for (int32_t i = 0; i < count; ++i) {
      u->max_out = std::max(u->max_out, parts[i]->max_out);
      u->max_in = std::max(u->max_in, parts[i]->max_in);
      u->n_src += parts[i]->n_src;
      u->n_dst += parts[i]->n_dst;
    }
    try {
      build_union(u, parts, count, static_cast<hipStream_t>(stream));
    } catch (...) {
      free_graph_memory(u);
      delete u;
      throw;
    }
    graph_register(u);
    *out = u;
    return ok();
  });
}

gm_status gm_plan_create(const gm_plan_run* runs, int32_t nruns, void* stream, gm_plan* out) {
  if (!out) return fail(GM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!runs) return fail(GM_EINVAL, "runs is NULL");
  if (nruns < 1) return fail(GM_EINVAL, "nruns = %d < 1", nruns);
  for (int32_t i = 0; i < nruns; ++i) {
    const gm_status st = check_run(runs[i], i);
    if (st != GM_OK) return st;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() -> gm_status {
    int dev = 0;
    GM_HIP(hipGetDevice(&dev));
    for (int32_t i = 0; i < nruns; ++i) {
      const gm_plan_run& r = runs[i];
      if (r.g->device != dev)
        return fail(GM_EINVAL, "run %d: graph lives on device %d, current is %d", i, r.g->device, dev);
      if (r.ids && r.count > 0 && !ids_in_range(r.ids, r.count, r.g->n, s))
        return fail(GM_EINVAL, "run %d: id outside [0, n)", i);
    }
    gm_plan p = new gm_plan_s();
    p->device = dev;
    hipStream_t cap = nullptr;
    try {
      p->runs.assign(runs, runs + nruns);
      p->res = dalloc<PlanResult>(nruns);
      void* h = nullptr;
      GM_HIP(hipHostMalloc(&h, nruns * sizeof(PlanResult), hipHostMallocDefault));
      p->host_res = static_cast<PlanResult*>(h);
      for (const gm_plan_run& r : p->runs) prepare_run(r, s);
      for (const gm_plan_run& r : p->runs) p->gens.push_back(r.g->ws_gen);
      GM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      GM_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
      try {
        for (int32_t i = 0; i < nruns; ++i) enqueue_run(p->runs[i], p->res + i, cap);
      } catch (...) {
        hipGraph_t tmp = nullptr;
        (void)hipStreamEndCapture(cap, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        throw;
      }
      GM_HIP(hipStreamEndCapture(cap, &p->graph));
      GM_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
      GM_HIP(hipStreamDestroy(cap));
      cap = nullptr;
    } catch (...) {
      if (cap) (void)hipStreamDestroy(cap);
      free_plan(p);
      throw;
    }
    p->magic = kPlanMagic;
    {
      std::lock_guard<std::mutex> lk(g_plan_mu);
      if (!g_plans) g_plans = new std::unordered_set<gm_plan>();
      g_plans->insert(p);
    }
    *out = p;
    return ok();
  });
}

gm_status gm_plan_launch(gm_plan p, void* stream) {
  if (!plan_live(p)) return fail(GM_ESTATE, "plan handle is not live");
  for (size_t i = 0; i < p->runs.size(); ++i) {
    const gm_graph g = p->runs[i].g;
    if (!graph_live(g)) return fail(GM_ESTATE, "run %zu: its graph was destroyed", i);
    if (g->ws_gen != p->gens[i])
      return fail(GM_ESTATE, "run %zu: the graph's workspace changed since the plan was created", i);
  }
  return guarded([&]() -> gm_status {
    GM_HIP(hipGraphLaunch(p->exec, static_cast<hipStream_t>(stream)));
    p->launched = true;
    return ok();
  });
}

gm_status gm_plan_results(gm_plan p, gm_plan_result* out, void* stream) {
  if (!plan_live(p)) return fail(GM_ESTATE, "plan handle is not live");
  if (!out) return fail(GM_EINVAL, "out is NULL");
  if (!p->launched) return fail(GM_ESTATE, "plan has not been launched");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() -> gm_status {
    const size_t k = p->runs.size();
    GM_HIP(hipMemcpyAsync(p->host_res, p->res, k * sizeof(PlanResult), hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < k; ++i) {
      out[i].iters_done = p->host_res[i].iters;
      out[i].converged = p->host_res[i].converged;
      out[i].edges_scanned = (int64_t)p->host_res[i].edges;
    }
    return ok();
  });
}

gm_status gm_plan_destroy(gm_plan p) {
  if (!plan_live(p)) return fail(GM_ESTATE, "plan handle is not live");
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans->erase(p);
  }
  free_plan(p);
  return ok();
}

gm_status gm_graph_get_tuning(gm_graph g, gm_tuning* out) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (!out) return fail(GM_EINVAL, "out is NULL");
  *out = to_abi(g->tune);
  return ok();
}

gm_status gm_graph_set_tuning(gm_graph g, const gm_tuning* t) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (!t) return fail(GM_EINVAL, "tuning is NULL");
  const gm_status st = check_tuning(*t);
  if (st != GM_OK) return st;
  const Tuning old = g->tune;
  from_abi(*t, &g->tune);
  // kernel-launch parameters are baked into captured plans too
  if (std::memcmp(&old, &g->tune, sizeof(Tuning)) != 0) ++g->ws_gen;
  return ok();
}

gm_status gm_autotune(gm_graph g, const gm_program* prog, int32_t batched, const int32_t* ids,
                      int64_t count, int32_t max_iters, int32_t trials, const char* cache_path,
                      gm_tuning* chosen, void* stream) {
  if (!graph_live(g)) return fail(GM_ESTATE, "graph handle is not live");
  if (!prog) return fail(GM_EINVAL, "prog is NULL");
  if (trials < 1 || trials > 100) return fail(GM_EINVAL, "trials = %d outside [1, 100]", trials);
  // Reuse the plan validation: the same rules as the corresponding call.
  gm_plan_run r{};
  r.g = g;
  r.prog = *prog;
  r.batched = batched ? 1 : 0;
  r.ids = ids;
  r.count = count;
  r.vprop = reinterpret_cast<void*>(1);  // outputs are the tuner's own
  const int kind = prog->kind;
  const bool fixed = kind == GM_PROG_PAGERANK || kind == GM_PROG_PPR;
  r.max_iters = fixed ? max_iters : 1;  // BFS/SSSP: any max_iters is accepted
  if (!batched && kind == GM_PROG_PPR)
    return fail(GM_EINVAL, "plain PPR has no parameters; tune the batched form");
  gm_status st = check_run(r, 0);
  if (st != GM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() -> gm_status {
    if (const gm_status dev_st = check_device(g)) return dev_st;
    if (ids && count > 0 && !ids_in_range(ids, count, g->n, s))
      return fail(GM_EINVAL, "id outside [0, n)");
    const int64_t k = batched ? count : 1;
    TuneCache cache;
    std::string key;
    if (cache_path) {
      if (!read_cache(cache_path, &cache))
        return fail(GM_EINVAL, "tuning cache %s: not an object of tuning entries", cache_path);
      key = cache_key(g, kind, batched != 0, k);
      const auto hit = cache.find(key);
      if (hit != cache.end()) {
        const Tuning before = g->tune;
        from_abi(hit->second, &g->tune);
        if (std::memcmp(&before, &g->tune, sizeof(Tuning)) != 0) ++g->ws_gen;
        if (chosen) *chosen = to_abi(g->tune);
        return ok();
      }
    }
    const size_t elem = kind == GM_PROG_TC ? 8 : 4;
    Scratch out;
    out.p = dmalloc((size_t)g->n * k * elem);
    Events ev;
    const Trial t{g, kind, batched != 0, ids, count, fixed ? max_iters : (max_iters > 0 ? max_iters : -1),
                  prog->r, out.p};
    // Candidate values per parameter, tuned in this order.
    struct Param {
      uint32_t Tuning::*field;
      std::vector<uint32_t> values;
    };
    std::vector<Param> params;
    if (!batched && kind == GM_PROG_BFS) {
      params.push_back({&Tuning::pull_div, {16, 32, 64, 128, 256, 512}});
      params.push_back({&Tuning::push_blocks, {512, 1024, 2048, 4096, 8192}});
      params.push_back({&Tuning::superstep_batch, {1, 2, 4, 8, 16}});
    } else if (!batched && kind == GM_PROG_SSSP) {
      // pull once the frontier's out-edges exceed m (never), m/2, m/4, m/8, m/16
      params.push_back({&Tuning::pull_div, {64, 128, 256, 512, 1024}});
      params.push_back({&Tuning::push_blocks, {512, 1024, 2048, 4096, 8192}});
      params.push_back({&Tuning::superstep_batch, {1, 2, 4, 8, 16}});
    } else if (batched && kind == GM_PROG_SSSP) {
      params.push_back({&Tuning::push_blocks, {512, 1024, 2048, 4096, 8192}});
    } else if (batched && kind == GM_PROG_PPR) {
      params.push_back({&Tuning::ppr_chunk, {128, 256, 512, 1024, 2048, 4096}});
    } else if (!batched && kind == GM_PROG_PAGERANK) {
      params.push_back({&Tuning::pr_hot, {0, 8192, 16384, 32768, 40960}});
    } else if (kind == GM_PROG_TC) {
      params.push_back({&Tuning::tc_wave_max, {128, 256, 512}});
      params.push_back({&Tuning::tc_wave_work, {1u << 12, 1u << 14, 1u << 16}});
      params.push_back({&Tuning::tc_block_work, {1u << 21, 1u << 23, 1u << 25}});
    }
    const Tuning before = g->tune;
    for (const Param& prm : params) {
      uint32_t best_v = g->tune.*prm.field;
      float best = time_trial(t, trials, s, ev);
      for (uint32_t v : prm.values) {
        if (v == best_v) continue;
        const uint32_t keep = g->tune.*prm.field;
        g->tune.*prm.field = v;
        const float ms = time_trial(t, trials, s, ev);
        if (ms < best) {
          best = ms;
          best_v = v;
        }
        g->tune.*prm.field = keep;
      }
      g->tune.*prm.field = best_v;
    }
    // rebuild the workspaces for the values kept
    t(s);
    GM_HIP(hipStreamSynchronize(s));
    if (std::memcmp(&before, &g->tune, sizeof(Tuning)) != 0) ++g->ws_gen;
    if (chosen) *chosen = to_abi(g->tune);
    if (cache_path) {
      cache[key] = to_abi(g->tune);
      if (!write_cache(cache_path, cache))
        return fail(GM_EINVAL, "tuning cache %s: cannot be written", cache_path);
    }
    return ok();
  });
}

}  // extern "C"
