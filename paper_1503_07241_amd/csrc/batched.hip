// Batched forms of the generalized SpMSpV: k sources (or personalised
// PageRank seeds) run together, so one read of the matrix serves all k
// frontiers (an SpMM with a dense n x k frontier block, semirings as in
// Sec. 3). Column s of every result equals the plain run from source s.
//
//  - BFS (k <= 64): the frontier of vertex v over all sources is one 64-bit
//    mask (REDUCE = or). Pull superstep: v ORs the masks of its neighbours
//    until every source that has not reached v is covered; new bits get
//    level t + 1.
//  - SSSP (k <= 64): distances are an n x k uint32 block. Active vertices
//    (any source changed) are compacted with a snapshot of their distance
//    rows (SEND); their out-edges are split evenly over wavefronts, lane s
//    relaxing source s (PROCESS msg + w, REDUCE/APPLY = atomic min) and the
//    sources that improved v are or-ed into v's next active mask.
//  - Personalised PageRank (k <= 256): messages are an n x k float block;
//    one wavefront reduces one destination row (all k seeds at once, lane
//    l holding seeds l, l + 64, ...), rows longer than the chunk size are split
//    into chunks combined by a second kernel, sums in double.
// Blocks are vertex-major: entry (v, s) at v * k + s.
#include <algorithm>
#include <vector>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kInfBfs = 0x7FFFFFFFu;
constexpr uint32_t kInfDist = 0xFFFFFFFFu;
constexpr int kEdgeUnroll = 4;     // rows in flight per wavefront

inline unsigned blocks_for(int64_t n, int64_t cap = 8192) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

__device__ inline unsigned long long full_mask(int k) {
  return k >= 64 ? ~0ull : ((1ull << k) - 1);
}

// ---------------------------------------------------------------- BFS -----
__global__ void bbfs_init(int64_t n, int k, const int32_t* __restrict__ src, int32_t* level,
                          unsigned long long* vis, unsigned long long* fr) {
  const int64_t total = n * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x)
    level[i] = (int32_t)kInfBfs;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    vis[v] = 0;
    fr[v] = 0;
  }
}

__global__ void bbfs_seed(int k, const int32_t* __restrict__ src, int32_t* level,
                          unsigned long long* vis, unsigned long long* fr) {
  for (int s = threadIdx.x; s < k; s += blockDim.x) {
    const int32_t v = src[s];
    level[(int64_t)v * k + s] = 0;
    atomicOr(&vis[v], 1ull << s);
    atomicOr(&fr[v], 1ull << s);
  }
}

__global__ __launch_bounds__(kThreads) void bbfs_pull(
    int64_t n, int k, int32_t t, const uint32_t* __restrict__ off, const int32_t* __restrict__ idx,
    const unsigned long long* __restrict__ fr, unsigned long long* __restrict__ vis,
    unsigned long long* __restrict__ fnext, int32_t* __restrict__ level,
    const unsigned int* __restrict__ prev, unsigned int* __restrict__ changed) {
  // a recorded superstep after the one that found nothing new does nothing
  if (prev && !*prev) return;
  const unsigned long long full = full_mask(k);
  int any = 0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long seen = vis[v];
    unsigned long long acc = 0;
    if (seen != full) {
      const uint32_t e1 = off[v + 1];
      for (uint32_t e = off[v]; e < e1; ++e) {
        acc |= fr[idx[e]];
        if ((acc | seen) == full) break;
      }
    }
    const unsigned long long nw = acc & ~seen;
    fnext[v] = nw;
    if (nw) {
      vis[v] = seen | nw;
      for (unsigned long long b = nw; b; b &= b - 1) level[v * k + (__ffsll((long long)b) - 1)] = t + 1;
      any = 1;
    }
  }
  // Every writer stores the same value: a plain store is enough.
  if (__syncthreads_or(any) && threadIdx.x == 0) *changed = 1u;
}

// ---------------------------------------------------------------- SSSP ----
struct BCtl {
  unsigned long long packed;  // (active vertices << 32) | their out-edges
};

__global__ void bsssp_init(int64_t n, int k, uint32_t* dist, unsigned long long* act,
                           unsigned long long* act2) {
  const int64_t total = n * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x)
    dist[i] = kInfDist;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    act[v] = 0;
    act2[v] = 0;
  }
}

__global__ void bsssp_seed(int k, const int32_t* __restrict__ src, uint32_t* dist,
                           unsigned long long* act) {
  for (int s = threadIdx.x; s < k; s += blockDim.x) {
    const int32_t v = src[s];
    dist[(int64_t)v * k + s] = 0;
    atomicOr(&act[v], 1ull << s);
  }
}

__device__ inline uint32_t wave_incl_scan(uint32_t x, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  return x;
}

// SEND: active masks -> queue (vertex, first edge, edge prefix) plus a
// snapshot of the active sources' distances (others INF); clears the masks.
__global__ __launch_bounds__(kThreads) void bsssp_send(
    int64_t n, int k, unsigned long long* __restrict__ act, const uint32_t* __restrict__ dist,
    const uint32_t* __restrict__ off, int32_t* __restrict__ q, uint32_t* __restrict__ qbeg,
    uint32_t* __restrict__ qest, uint32_t* __restrict__ qrow, BCtl* __restrict__ ctl) {
  __shared__ uint32_t sh[2 * kWaves];
  __shared__ unsigned long long base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t v0 = (int64_t)blockIdx.x * kThreads; v0 < n; v0 += (int64_t)gridDim.x * kThreads) {
    const int64_t v = v0 + threadIdx.x;
    const unsigned long long a = v < n ? act[v] : 0ull;
    const uint32_t cnt = a ? 1u : 0u;
    const uint32_t deg = a ? off[v + 1] - off[v] : 0u;
    const uint32_t ci = wave_incl_scan(cnt, lane), ei = wave_incl_scan(deg, lane);
    if (lane == 63) {
      sh[wave] = ci;
      sh[kWaves + wave] = ei;
    }
    __syncthreads();
    uint32_t cb = 0, eb = 0, ct = 0, et = 0;
    for (int i = 0; i < kWaves; ++i) {
      if (i < wave) {
        cb += sh[i];
        eb += sh[kWaves + i];
      }
      ct += sh[i];
      et += sh[kWaves + i];
    }
    if (threadIdx.x == 0 && ct) base = atomicAdd(&ctl->packed, ((unsigned long long)ct << 32) | et);
    __syncthreads();
    if (ct && a) {
      const unsigned long long bp = base;
      const uint32_t slot = (uint32_t)(bp >> 32) + cb + ci - cnt;
      q[slot] = (int32_t)v;
      qbeg[slot] = off[v];
      qest[slot] = (uint32_t)bp + eb + ei - deg;
      act[v] = 0;
      for (int s = 0; s < k; ++s)
        qrow[(int64_t)slot * k + s] = ((a >> s) & 1ull) ? dist[v * k + s] : kInfDist;
    }
    __syncthreads();
  }
}

// Relax the active vertices' out-edges, one edge per wavefront step with
// lane s handling source s; edges split evenly over wavefronts.
__global__ __launch_bounds__(kThreads) void bsssp_push(
    int k, const BCtl* __restrict__ ctl, const uint32_t* __restrict__ qbeg,
    const uint32_t* __restrict__ qest, const uint32_t* __restrict__ qrow,
    const int32_t* __restrict__ idx, const uint32_t* __restrict__ w, uint32_t* dist,
    unsigned long long* anext) {
  const uint32_t count = (uint32_t)(ctl->packed >> 32);
  const uint64_t E = (uint32_t)ctl->packed;
  if (count == 0 || E == 0) return;
  const int lane = threadIdx.x & 63;
  const uint64_t nw = (uint64_t)gridDim.x * kWaves;
  const uint64_t wid = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const uint32_t e_begin = (uint32_t)(E * wid / nw), e_end = (uint32_t)(E * (wid + 1) / nw);
  if (e_begin >= e_end) return;
  // 64-ary search for the slot holding edge e_begin.
  uint32_t lo = 0, hi = count;
  while (hi - lo > 64) {
    const uint32_t span = hi - lo;
    const uint32_t p = lo + (uint32_t)((uint64_t)span * lane / 64);
    const int last = 63 - __clzll(__ballot(qest[p] <= e_begin));
    const uint32_t nlo = lo + (uint32_t)((uint64_t)span * last / 64);
    hi = last == 63 ? hi : lo + (uint32_t)((uint64_t)span * (last + 1) / 64);
    lo = nlo;
  }
  {
    const uint32_t p = lo + lane;
    lo += 63 - __clzll(__ballot(p < hi && qest[p] <= e_begin));
  }
  uint32_t slot = lo;
  uint32_t slot_end = slot + 1 < count ? qest[slot + 1] : (uint32_t)E;
  for (uint32_t e = e_begin; e < e_end; e += kEdgeUnroll) {
    uint32_t sl[kEdgeUnroll], ed[kEdgeUnroll];
    bool ok[kEdgeUnroll];
#pragma unroll
    for (int u = 0; u < kEdgeUnroll; ++u) {
      const uint32_t ee = e + u;
      ok[u] = ee < e_end;
      if (ok[u]) {
        while (ee >= slot_end) {  // wave-uniform walk to the next slot
          ++slot;
          slot_end = slot + 1 < count ? qest[slot + 1] : (uint32_t)E;
        }
      }
      sl[u] = slot;
      ed[u] = ok[u] ? qbeg[slot] + (ee - qest[slot]) : 0u;
    }
    int32_t vv[kEdgeUnroll];
    uint32_t ww[kEdgeUnroll], m[kEdgeUnroll], cur[kEdgeUnroll];
#pragma unroll
    for (int u = 0; u < kEdgeUnroll; ++u) {
      vv[u] = ok[u] ? idx[ed[u]] : 0;
      ww[u] = ok[u] ? w[ed[u]] : 0u;
      m[u] = (ok[u] && lane < k) ? qrow[(int64_t)sl[u] * k + lane] : kInfDist;
    }
#pragma unroll
    for (int u = 0; u < kEdgeUnroll; ++u)
      cur[u] = (ok[u] && lane < k) ? dist[(int64_t)vv[u] * k + lane] : 0u;
#pragma unroll
    for (int u = 0; u < kEdgeUnroll; ++u) {
      bool better = false;
      if (ok[u] && lane < k && m[u] != kInfDist) {
        const uint32_t sum = m[u] + ww[u];
        const uint32_t cand = sum < m[u] ? kInfDist : sum;
        if (cand < cur[u]) {
          __hip_atomic_fetch_min(&dist[(int64_t)vv[u] * k + lane], cand, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
          better = true;
        }
      }
      const unsigned long long bm = __ballot(better);
      if (bm && lane == 0)
        __hip_atomic_fetch_or(&anext[vv[u]], bm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ void reset_bctl(BCtl* c) { c->packed = 0; }

// ---------------------------------------------------------------- PPR -----
struct PprItem {
  uint32_t row;
  uint32_t edge_begin;
  uint32_t edge_end;
  int32_t partial;  // partial-row slot for split rows, -1 otherwise
};

struct PprSplit {
  uint32_t row;
  uint32_t first;   // first partial slot
  uint32_t count;
  uint32_t pad;
};

template <int kPerLane>
__device__ inline void ppr_apply_row(int k, uint32_t v, const double (&acc)[kPerLane], float r,
                                     const int32_t* __restrict__ seeds, float inv,
                                     float* __restrict__ xout, float* __restrict__ pout) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < kPerLane; ++j) {
    const int s = lane + 64 * j;
    if (s < k) {
      const double tele = seeds[s] == (int32_t)v ? 1.0 : 0.0;
      const float pr = (float)((double)r * tele + (1.0 - (double)r) * acc[j]);
      xout[(int64_t)v * k + s] = pr * inv;
      if (pout) pout[(int64_t)v * k + s] = pr;
    }
  }
}

// One wavefront per work item (a row, or a chunk of a long row).
template <int kPerLane>
__global__ __launch_bounds__(kThreads) void bppr_pull(
    int k, const PprItem* __restrict__ items, int64_t nitems, const int32_t* __restrict__ idx,
    const float* __restrict__ x, const float* __restrict__ inv_outdeg,
    const int32_t* __restrict__ seeds, float r, float* __restrict__ xout,
    float* __restrict__ pout, double* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (it >= nitems) return;
  const PprItem item = items[it];
  double acc[kPerLane];
#pragma unroll
  for (int j = 0; j < kPerLane; ++j) acc[j] = 0.0;
  for (uint32_t e = item.edge_begin; e < item.edge_end; e += kEdgeUnroll) {
    int32_t u[kEdgeUnroll];
#pragma unroll
    for (int q = 0; q < kEdgeUnroll; ++q) u[q] = e + q < item.edge_end ? idx[e + q] : -1;
    float val[kEdgeUnroll][kPerLane];
#pragma unroll
    for (int q = 0; q < kEdgeUnroll; ++q)
#pragma unroll
      for (int j = 0; j < kPerLane; ++j) {
        const int s = lane + 64 * j;
        val[q][j] = (u[q] >= 0 && s < k) ? x[(int64_t)u[q] * k + s] : 0.0f;
      }
#pragma unroll
    for (int q = 0; q < kEdgeUnroll; ++q)
#pragma unroll
      for (int j = 0; j < kPerLane; ++j) acc[j] += (double)val[q][j];
  }
  if (item.partial >= 0) {
#pragma unroll
    for (int j = 0; j < kPerLane; ++j) {
      const int s = lane + 64 * j;
      if (s < k) partial[(int64_t)item.partial * k + s] = acc[j];
    }
  } else {
    ppr_apply_row<kPerLane>(k, item.row, acc, r, seeds, inv_outdeg[item.row], xout, pout);
  }
}

template <int kPerLane>
__global__ __launch_bounds__(kThreads) void bppr_finish(
    int k, const PprSplit* __restrict__ splits, int64_t nsplit, const double* __restrict__ partial,
    const float* __restrict__ inv_outdeg, const int32_t* __restrict__ seeds, float r,
    float* __restrict__ xout, float* __restrict__ pout) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (i >= nsplit) return;
  const PprSplit sp = splits[i];
  double acc[kPerLane];
#pragma unroll
  for (int j = 0; j < kPerLane; ++j) {
    acc[j] = 0.0;
    const int s = lane + 64 * j;
    if (s < k)
      for (uint32_t c = 0; c < sp.count; ++c) acc[j] += partial[(int64_t)(sp.first + c) * k + s];
  }
  ppr_apply_row<kPerLane>(k, sp.row, acc, r, seeds, inv_outdeg[sp.row], xout, pout);
}

// PPR^0 = e_s: x[v][s] = [v == seed_s] / outdeg(v).
__global__ void bppr_init(int64_t n, int k, const int32_t* __restrict__ seeds,
                          const float* __restrict__ inv_outdeg, float* __restrict__ x) {
  const int64_t total = n * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = i / k;
    const int s = (int)(i - v * k);
    x[i] = seeds[s] == (int32_t)v ? inv_outdeg[v] : 0.0f;
  }
}

struct Batch {
  // BFS
  unsigned long long* vis = nullptr;
  unsigned long long* fr[2] = {nullptr, nullptr};
  unsigned int* flags = nullptr;  // kMaxPlanSteps "changed" words
  unsigned int* host_flag = nullptr;
  // SSSP
  unsigned long long* act[2] = {nullptr, nullptr};
  int32_t* q = nullptr;
  uint32_t* qbeg = nullptr;
  uint32_t* qest = nullptr;
  uint32_t* qrow = nullptr;
  int64_t qrow_k = 0;
  BCtl* ctl = nullptr;  // kMaxPlanSteps records
  BCtl* host_ctl = nullptr;
  // PPR
  PprItem* items = nullptr;
  int64_t nitems = 0;
  PprSplit* splits = nullptr;
  int64_t nsplit = 0;
  int64_t npartial = 0;
  uint32_t items_chunk = 0;  // ppr chunk the items were built with
  double* partial = nullptr;
  int64_t partial_k = 0;
  float* xb[2] = {nullptr, nullptr};
  int64_t xb_k = 0;
};

Batch* batch(gm_graph g) { return static_cast<Batch*>(g->batch_ws); }

Batch* ensure_batch(gm_graph g) {
  if (!batch(g)) g->batch_ws = new Batch();
  return batch(g);
}

void free_ppr_items(gm_graph g, Batch* b) {
  dfree(b->items);
  dfree(b->splits);
  dfree(b->partial);
  b->items = nullptr;
  b->splits = nullptr;
  b->partial = nullptr;
  b->nitems = b->nsplit = b->npartial = b->partial_k = 0;
  ++g->ws_gen;
}

void ensure_ppr_items(gm_graph g, Batch* b, hipStream_t s) {
  const uint32_t chunk = g->tune.ppr_chunk;
  if (b->items && b->items_chunk == chunk) return;
  if (b->items) free_ppr_items(g, b);
  const int64_t n = g->n;
  std::vector<uint32_t> off(n + 1);
  GM_HIP(hipMemcpyAsync(off.data(), g->in_off, (n + 1) * 4, hipMemcpyDeviceToHost, s));
  GM_HIP(hipStreamSynchronize(s));
  std::vector<PprItem> items;
  std::vector<PprSplit> splits;
  int32_t np = 0;
  // long rows first so they start early
  std::vector<int64_t> order;
  for (int64_t v = 0; v < n; ++v)
    if (off[v + 1] - off[v] > chunk) order.push_back(v);
  std::sort(order.begin(), order.end(),
            [&](int64_t a, int64_t c) { return off[a + 1] - off[a] > off[c + 1] - off[c]; });
  std::vector<uint8_t> split(n, 0);
  for (int64_t v : order) {
    split[v] = 1;
    const uint32_t nch = (off[v + 1] - off[v] + chunk - 1) / chunk;
    splits.push_back({(uint32_t)v, (uint32_t)np, nch, 0});
    for (uint32_t c = 0; c < nch; ++c) {
      const uint32_t eb = off[v] + c * chunk;
      items.push_back({(uint32_t)v, eb, std::min(eb + chunk, off[v + 1]), np++});
    }
  }
  for (int64_t v = 0; v < n; ++v)
    if (!split[v]) items.push_back({(uint32_t)v, off[v], off[v + 1], -1});
  b->nitems = (int64_t)items.size();
  b->nsplit = (int64_t)splits.size();
  b->npartial = np;
  b->items_chunk = chunk;
  b->items = dalloc<PprItem>(items.size());
  b->splits = dalloc<PprSplit>(splits.size());
  GM_HIP(hipMemcpyAsync(b->items, items.data(), items.size() * sizeof(PprItem),
                        hipMemcpyHostToDevice, s));
  if (!splits.empty())
    GM_HIP(hipMemcpyAsync(b->splits, splits.data(), splits.size() * sizeof(PprSplit),
                          hipMemcpyHostToDevice, s));
  GM_HIP(hipStreamSynchronize(s));
}

void ensure_bfs_ws(Batch* b, int64_t n) {
  if (b->vis) return;
  b->vis = dalloc<unsigned long long>(n);
  b->fr[0] = dalloc<unsigned long long>(n);
  b->fr[1] = dalloc<unsigned long long>(n);
  b->flags = dalloc<unsigned int>(kMaxPlanSteps);
  void* h = nullptr;
  GM_HIP(hipHostMalloc(&h, sizeof(unsigned int), hipHostMallocDefault));
  b->host_flag = static_cast<unsigned int*>(h);
}

void ensure_sssp_ws(gm_graph g, Batch* b, int k) {
  const int64_t n = g->n;
  if (!b->act[0]) {
    b->act[0] = dalloc<unsigned long long>(2 * n);  // both masks in one buffer
    b->act[1] = b->act[0] + n;
    b->q = dalloc<int32_t>(n);
    b->qbeg = dalloc<uint32_t>(n);
    b->qest = dalloc<uint32_t>(n);
    b->ctl = dalloc<BCtl>(kMaxPlanSteps);
    void* h = nullptr;
    GM_HIP(hipHostMalloc(&h, sizeof(BCtl), hipHostMallocDefault));
    b->host_ctl = static_cast<BCtl*>(h);
  }
  if (b->qrow_k < k) {
    dfree(b->qrow);
    b->qrow = nullptr;
    ++g->ws_gen;
    b->qrow = dalloc<uint32_t>((size_t)n * k);
    b->qrow_k = k;
  }
}

void ensure_ppr_ws(gm_graph g, Batch* b, int k, hipStream_t s) {
  const int64_t n = g->n;
  ensure_ppr_items(g, b, s);
  if (b->xb_k < k) {
    dfree(b->xb[0]);
    dfree(b->xb[1]);
    b->xb[0] = b->xb[1] = nullptr;
    ++g->ws_gen;
    b->xb[0] = dalloc<float>((size_t)n * k);
    b->xb[1] = dalloc<float>((size_t)n * k);
    b->xb_k = k;
  }
  if (b->partial_k < k) {
    dfree(b->partial);
    b->partial = nullptr;
    ++g->ws_gen;
    b->partial = dalloc<double>((size_t)b->npartial * k);
    b->partial_k = k;
  }
}

// Pull adjacency of batched BFS: the out-lists of a symmetrised graph, else
// the in-lists.
void bfs_adjacency(gm_graph g, const uint32_t** off, const int32_t** idx) {
  const bool sym = (g->prep & (GM_PREP_SYMMETRIZE | GM_PREP_UPPER_DAG)) == GM_PREP_SYMMETRIZE;
  *off = sym ? g->out_off : g->in_off;
  *idx = sym ? g->out_idx : g->in_idx;
}

void bfs_init(gm_graph g, Batch* b, const int32_t* sources, int k, int32_t* level, hipStream_t s) {
  const int64_t n = g->n;
  bbfs_init<<<blocks_for(n * k), kThreads, 0, s>>>(n, k, sources, level, b->vis, b->fr[0]);
  bbfs_seed<<<1, 64, 0, s>>>(k, sources, level, b->vis, b->fr[0]);
  GM_HIP(hipGetLastError());
}

void bfs_superstep(gm_graph g, Batch* b, int k, int32_t t, int cur, int32_t* level,
                   const unsigned int* prev, unsigned int* changed, hipStream_t s) {
  const uint32_t* off;
  const int32_t* idx;
  bfs_adjacency(g, &off, &idx);
  bbfs_pull<<<blocks_for(g->n), kThreads, 0, s>>>(g->n, k, t, off, idx, b->fr[cur], b->vis,
                                                  b->fr[cur ^ 1], level, prev, changed);
  GM_HIP(hipGetLastError());
}

void sssp_init(gm_graph g, Batch* b, const int32_t* sources, int k, uint32_t* dist,
               hipStream_t s) {
  const int64_t n = g->n;
  bsssp_init<<<blocks_for(n * k), kThreads, 0, s>>>(n, k, dist, b->act[0], b->act[1]);
  bsssp_seed<<<1, 64, 0, s>>>(k, sources, dist, b->act[0]);
  GM_HIP(hipGetLastError());
}

void sssp_superstep(gm_graph g, Batch* b, int k, int cur, BCtl* ctl, uint32_t* dist,
                    hipStream_t s) {
  const int64_t n = g->n;
  reset_bctl<<<1, 1, 0, s>>>(ctl);
  bsssp_send<<<blocks_for(n, 4096), kThreads, 0, s>>>(n, k, b->act[cur], dist, g->out_off, b->q,
                                                      b->qbeg, b->qest, b->qrow, ctl);
  bsssp_push<<<g->tune.push_blocks, kThreads, 0, s>>>(
      k, ctl, b->qbeg, b->qest, b->qrow, g->out_idx, static_cast<const uint32_t*>(g->out_w), dist,
      b->act[cur ^ 1]);
  GM_HIP(hipGetLastError());
}

void ppr_supersteps(gm_graph g, Batch* b, const int32_t* seeds, int k, float r, int32_t iters,
                    float* out, hipStream_t s) {
  const int64_t n = g->n;
  bppr_init<<<blocks_for(n * k, 65536), kThreads, 0, s>>>(n, k, seeds, g->inv_outdeg, b->xb[0]);
  GM_HIP(hipGetLastError());
  const unsigned gi = (unsigned)((b->nitems + kWaves - 1) / kWaves);
  const unsigned gs = (unsigned)((b->nsplit + kWaves - 1) / kWaves);
  for (int32_t it = 0; it < iters; ++it) {
    const float* xin = b->xb[it & 1];
    float* xo = b->xb[(it + 1) & 1];
    float* po = it == iters - 1 ? out : nullptr;
    auto launch = [&](auto pull, auto finish) {
      if (gi > 0)
        pull<<<gi, kThreads, 0, s>>>(k, b->items, b->nitems, g->in_idx, xin, g->inv_outdeg, seeds,
                                     r, xo, po, b->partial);
      if (b->nsplit > 0)
        finish<<<gs, kThreads, 0, s>>>(k, b->splits, b->nsplit, b->partial, g->inv_outdeg, seeds,
                                       r, xo, po);
    };
    if (k <= 64)
      launch(bppr_pull<1>, bppr_finish<1>);
    else if (k <= 128)
      launch(bppr_pull<2>, bppr_finish<2>);
    else
      launch(bppr_pull<4>, bppr_finish<4>);
    GM_HIP(hipGetLastError());
  }
}

// Outcome of recorded batched BFS supersteps: superstep t found nothing new
// iff changed[t] == 0 (that superstep still counts, as in the plain run).
__global__ void bbfs_summary(const unsigned int* __restrict__ changed, int32_t steps,
                             PlanResult* res) {
  int32_t it = steps, conv = 0;
  for (int32_t t = 0; t < steps; ++t)
    if (!changed[t]) {
      it = t + 1;
      conv = 1;
      break;
    }
  res->iters = it;
  res->converged = conv;
  res->edges = 0;
}

// Outcome of recorded batched SSSP supersteps: the first superstep with no
// active vertex ends the run.
__global__ void bsssp_summary(const BCtl* __restrict__ ctl, int32_t steps, PlanResult* res) {
  int32_t it = steps;
  unsigned long long e = 0;
  for (int32_t t = 0; t < steps; ++t) {
    if ((ctl[t].packed >> 32) == 0) {
      it = t;
      break;
    }
    e += (uint32_t)ctl[t].packed;
  }
  res->iters = it;
  res->converged = 1;  // cleared by bsssp_finish if a vertex is still active
  res->edges = e;
}

// The run converged iff no vertex is left active; both masks are cleared for
// the next run. Every writer stores 0.
__global__ void bsssp_finish(unsigned long long* act, int64_t words, int32_t* converged) {
  bool any = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (act[i]) {
      any = true;
      act[i] = 0;
    }
  }
  if (any) *converged = 0;
}

}  // namespace

void free_batch(gm_graph g) {
  Batch* b = batch(g);
  if (!b) return;
  dfree(b->vis);
  dfree(b->fr[0]);
  dfree(b->fr[1]);
  dfree(b->flags);
  if (b->host_flag) (void)hipHostFree(b->host_flag);
  dfree(b->act[0]);
  dfree(b->q);
  dfree(b->qbeg);
  dfree(b->qest);
  dfree(b->qrow);
  dfree(b->ctl);
  if (b->host_ctl) (void)hipHostFree(b->host_ctl);
  dfree(b->items);
  dfree(b->splits);
  dfree(b->partial);
  dfree(b->xb[0]);
  dfree(b->xb[1]);
  delete b;
  g->batch_ws = nullptr;
  ++g->ws_gen;
}

int32_t run_batched_bfs(gm_graph g, const int32_t* sources, int k, int32_t max_iters,
                        int32_t* level, hipStream_t s) {
  Batch* b = ensure_batch(g);
  ensure_bfs_ws(b, g->n);
  bfs_init(g, b, sources, k, level, s);
  int cur = 0;
  int32_t t = 0;
  for (;; ++t) {
    if (max_iters > 0 && t >= max_iters) break;
    fill_u32(b->flags, 1, 0u, s);
    bfs_superstep(g, b, k, t, cur, level, nullptr, b->flags, s);
    GM_HIP(hipMemcpyAsync(b->host_flag, b->flags, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    cur ^= 1;
    if (!*b->host_flag) {
      ++t;  // this superstep scanned the deepest frontier and found nothing new
      break;
    }
  }
  return t;
}

int32_t run_batched_sssp(gm_graph g, const int32_t* sources, int k, int32_t max_iters,
                         uint32_t* dist, hipStream_t s) {
  Batch* b = ensure_batch(g);
  ensure_sssp_ws(g, b, k);
  sssp_init(g, b, sources, k, dist, s);
  int cur = 0;
  int32_t t = 0;
  for (;; ++t) {
    if (max_iters > 0 && t >= max_iters) break;
    sssp_superstep(g, b, k, cur, b->ctl, dist, s);
    GM_HIP(hipMemcpyAsync(b->host_ctl, b->ctl, sizeof(BCtl), hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    cur ^= 1;
    if ((b->host_ctl->packed >> 32) == 0) break;  // no vertex was active
  }
  // leave the workspace cleared for the next run
  fill_u32(reinterpret_cast<uint32_t*>(b->act[0]), 4 * g->n, 0u, s);
  GM_HIP(hipStreamSynchronize(s));
  return t;
}

void run_batched_ppr(gm_graph g, const int32_t* seeds, int k, float r, int32_t iters, float* out,
                     hipStream_t s) {
  Batch* b = ensure_batch(g);
  ensure_ppr_ws(g, b, k, s);
  ppr_supersteps(g, b, seeds, k, r, iters, out, s);
}

void prepare_batched(gm_graph g, int kind, int k, hipStream_t s) {
  Batch* b = ensure_batch(g);
  if (kind == GM_PROG_BFS)
    ensure_bfs_ws(b, g->n);
  else if (kind == GM_PROG_SSSP)
    ensure_sssp_ws(g, b, k);
  else
    ensure_ppr_ws(g, b, k, s);
  GM_HIP(hipStreamSynchronize(s));
}

void enqueue_batched(gm_graph g, int kind, const int32_t* sources, int k, int32_t steps, float r,
                     void* block, PlanResult* res, hipStream_t s) {
  Batch* b = batch(g);
  if (!b || steps < 1) throw Unsupported{"captured run not prepared"};
  if (kind == GM_PROG_BFS) {
    if (!b->vis || steps > kMaxPlanSteps) throw Unsupported{"captured run not prepared"};
    int32_t* level = static_cast<int32_t*>(block);
    bfs_init(g, b, sources, k, level, s);
    fill_u32(b->flags, steps, 0u, s);
    int cur = 0;
    for (int32_t t = 0; t < steps; ++t) {
      bfs_superstep(g, b, k, t, cur, level, t > 0 ? b->flags + t - 1 : nullptr, b->flags + t, s);
      cur ^= 1;
    }
    bbfs_summary<<<1, 1, 0, s>>>(b->flags, steps, res);
  } else if (kind == GM_PROG_SSSP) {
    if (!b->act[0] || b->qrow_k < k || steps > kMaxPlanSteps)
      throw Unsupported{"captured run not prepared"};
    uint32_t* dist = static_cast<uint32_t*>(block);
    sssp_init(g, b, sources, k, dist, s);
    int cur = 0;
    for (int32_t t = 0; t < steps; ++t) {
      sssp_superstep(g, b, k, cur, b->ctl + t, dist, s);
      cur ^= 1;
    }
    bsssp_summary<<<1, 1, 0, s>>>(b->ctl, steps, res);
    // all supersteps used: converged only if nothing is left active
    bsssp_finish<<<blocks_for(2 * g->n), kThreads, 0, s>>>(b->act[0], 2 * g->n, &res->converged);
  } else {
    if (!b->items || b->xb_k < k || b->partial_k < k) throw Unsupported{"captured run not prepared"};
    ppr_supersteps(g, b, sources, k, r, steps, static_cast<float*>(block), s);
    set_plan_result(res, steps, (unsigned long long)g->m * steps, s);
  }
  GM_HIP(hipGetLastError());
}

}  // namespace gm
