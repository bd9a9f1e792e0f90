// Reverse-mode derivative of weighted PageRank with respect to the edge
// weights (the transpose-direction, adjoint generalized SpMV).
//
// Forward (Eq. (1) with edge weights; deg = unweighted out-degree):
//   PR^{t+1}(v) = r + (1 - r) sum_{u -> v} w_uv PR^t(u) / deg(u).
// With upstream c = dL/dPR^T, abar^T = c, and for t = T-1 .. 0:
//   dL/dw_uv += (1 - r) PR^t(u) / deg(u) * abar^{t+1}(v)
//   abar^t(u) = (1 - r) / deg(u) * sum_{v: u -> v} w_uv abar^{t+1}(v)
// The second line is a pull over out-edges (rows of the CSR = columns of
// G^T), i.e. the product with the transposed matrix. Both lines are one
// kernel per step, one pass over the out-edges.
//
// Layout (built once per graph): vertices relabelled by decreasing
// out-degree (rows with out-edges are then [0, rows); RMAT's high
// out-degree vertices are also the most gathered destinations), the
// out-adjacency rebuilt in the new labels with each edge's caller (CSR) id,
// cut into equal edge tiles reduced by a segmented scan like PageRank's pull
// superstep. Per call the edge values are gathered into the relabelled
// order once, the gradient is accumulated there (a coalesced read-modify-
// write per edge and step) and scattered back to the caller's order at the
// end. Sums in double, in a fixed order.
#include <algorithm>
#include <vector>

#include "gm_internal.h"
#include "tiles.h"

namespace gm {
namespace {

using namespace tiles;

constexpr int kThreads = 256;

struct VjpPlan {
  int64_t n = 0, m = 0, rows = 0, ntiles = 0, ncross = 0, mpad = 0;
  int32_t* old_of = nullptr;    // new label -> caller's label
  int32_t* idx = nullptr;       // relabelled out-adjacency (new labels), padded with 0
  uint32_t* ceid = nullptr;     // caller's (CSR) id of each relabelled edge
  float* inv_outdeg = nullptr;  // new labels
  uint32_t* starts = nullptr;   // row-start bitmap of the relabelled edges
  uint32_t* tile_row = nullptr;
  Cross* cross = nullptr;
  double* head = nullptr;
  double* tail = nullptr;
  float* wv = nullptr;          // edge values in the relabelled order, padded with 0
  float* gv = nullptr;          // gradient in the relabelled order, padded
  float* cu = nullptr;          // per row: (1 - r) PR^t(u) / deg(u); n + 1 entries, 0 past rows
  float* abar[2] = {nullptr, nullptr};
  int cus = 0, lds_max = 0;
};

// One reverse step over the tiles: gradient of every edge and the row sums
// sum_v w_uv abar_next(v), APPLY abar_cur(u) = (1 - r) / deg(u) * sum. The
// row of every edge comes from a count scan of the row-start bitmap before
// the gathers, so that each edge's cu(row) is loaded with its message.
__global__ __launch_bounds__(kTileThreads) void vjp_tile(
    const int32_t* __restrict__ idx, const float* __restrict__ wv,
    const uint32_t* __restrict__ starts, const uint32_t* __restrict__ tile_row, int64_t ntiles,
    const float* __restrict__ abar_next, const float* __restrict__ cu,
    const float* __restrict__ inv_outdeg, float one_r, float* __restrict__ abar_cur,
    float* __restrict__ gv, double* __restrict__ head, double* __restrict__ tail, int hot_n) {
  extern __shared__ float hot[];  // hot_n floats
  load_hot(abar_next, hot, hot_n);
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * kTileWaves;
  const int sh = (lane & 7) * 4;  // this lane's 4 bits in its word of `starts`
  const char* ab = reinterpret_cast<const char*>(abar_next);
  const char* cb = reinterpret_cast<const char*>(cu);
  int64_t t = __builtin_amdgcn_readfirstlane(blockIdx.x * kTileWaves + (threadIdx.x >> 6));
  for (; t < ntiles; t += stride) {
    const int64_t e0 = t * kTile + lane * 4;
    v4i src[kRounds];
    v4f w[kRounds];
    uint32_t nib[kRounds], next[kRounds];
#pragma unroll
    for (int v = 0; v < kRounds; ++v) {
      const int64_t ev = e0 + v * 256;
      src[v] = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(idx + ev));
      w[v] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(wv + ev));
      const uint32_t fa = starts[ev >> 5], fb = starts[(ev >> 5) + 1];
      nib[v] = (fa >> sh) & 0xFu;  // bit q: edge q of the lane starts a row
      next[v] = sh == 28 ? (fb & 1u) : (fa >> (sh + 4)) & 1u;
    }
    const uint32_t row0 = tile_row[t];
    // A start at the tile's first edge opens row0 itself, not the next row.
    const int f0 = __builtin_amdgcn_readfirstlane((int)(nib[0] & 1u));
    // Row of edge (v, q): row0 + starts before it in the tile (exc[v] from
    // the lanes before, then the lane's own) - f0.
    uint32_t exc[kRounds];
    int ccarry = 0;
#pragma unroll
    for (int v = 0; v < kRounds; ++v)
      exc[v] = row0 + (uint32_t)(count_scan((int)__popc(nib[v]), ccarry, lane) - f0);
    const auto row_of = [&](int v, int q) {
      return exc[v] + (uint32_t)__popc(nib[v] & ((2u << q) - 1u));
    };
    float a[kRounds][4], cv[kRounds][4];
    v4f g[kRounds];
#pragma unroll
    for (int v = 0; v < kRounds; ++v) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t s = (uint32_t)src[v][q];
        const bool in_lds = s < (uint32_t)hot_n;
        const float gl = *reinterpret_cast<const float*>(ab + (in_lds ? 0u : s << 2));
        const float l = hot[in_lds ? s : 0u];
        a[v][q] = in_lds ? l : gl;
        cv[v][q] = *reinterpret_cast<const float*>(cb + (row_of(v, q) << 2));
      }
      g[v] = *reinterpret_cast<const v4f*>(gv + e0 + v * 256);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int v = 0; v < kRounds; ++v) {
#pragma unroll
      for (int q = 0; q < 4; ++q) g[v][q] = g[v][q] + cv[v][q] * a[v][q];
      *reinterpret_cast<v4f*>(gv + e0 + v * 256) = g[v];
    }
    Seg carry{0, 0.0};
    float yv[kRounds][4];  // row sums ending here (rounded once more when applied)
    uint32_t done = 0;  // bit 4v+q: edge (v, q) ends a row begun in the tile
#pragma unroll
    for (int v = 0; v < kRounds; ++v) {
      double s[4];
      s[0] = (double)w[v][0] * (double)a[v][0];
#pragma unroll
      for (int q = 1; q < 4; ++q)
        s[q] = ((nib[v] >> q) & 1u ? 0.0 : s[q - 1]) + (double)w[v][q] * (double)a[v][q];
      const Seg ex = seg_scan(Seg{(int)__popc(nib[v]), s[3]}, carry, lane);
      const uint32_t ends = (nib[v] >> 1) | (next[v] << 3);  // bit q: edge q ends its row
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        yv[v][q] = 0.0f;
        if ((ends >> q) & 1u) {
          const int lc = (int)__popc(nib[v] & ((2u << q) - 1u));  // starts at or before edge q
          const double y = lc > 0 ? s[q] : ex.s + s[q];
          if (ex.c + lc > 0) {
            yv[v][q] = (float)y;
            done |= 1u << (4 * v + q);
          } else {
            head[t] = y;
          }
        }
      }
      if (v == kRounds - 1 && lane == 63 && !(ends >> 3)) {
        const double y = nib[v] ? s[3] : ex.s + s[3];
        if (ex.c + (int)__popc(nib[v]) > 0)
          tail[t] = y;
        else
          head[t] = y;
      }
    }
    float inv[kRounds][4];
#pragma unroll
    for (int v = 0; v < kRounds; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        inv[v][q] = 0.0f;
        if ((done >> (4 * v + q)) & 1u) inv[v][q] = inv_outdeg[row_of(v, q)];
      }
#pragma unroll
    for (int v = 0; v < kRounds; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if ((done >> (4 * v + q)) & 1u)
          abar_cur[row_of(v, q)] = (float)((double)one_r * (double)inv[v][q] * yv[v][q]);
  }
}

// Rows spanning tiles ta..tb: tail[ta] + head[ta + 1] + ... + head[tb],
// summed by kCrossLanes lanes in a fixed order, then APPLY.
__global__ void vjp_cross(const Cross* __restrict__ cross, int64_t ncross,
                          const double* __restrict__ head, const double* __restrict__ tail,
                          const float* __restrict__ inv_outdeg, float one_r,
                          float* __restrict__ abar_cur) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t i = gid / kCrossLanes;
  const int j = (int)(gid % kCrossLanes);
  double acc = 0.0;
  Cross c{0, 0, 0, 0};
  if (i < ncross) {
    c = cross[i];
    if (j == 0) acc = tail[c.ta];
    for (uint32_t t = c.ta + 1 + j; t <= c.tb; t += kCrossLanes) acc += head[t];
  }
  for (int o = kCrossLanes >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (i < ncross && j == 0)
    abar_cur[c.row] = (float)((double)one_r * (double)inv_outdeg[c.row] * acc);
}

// cu(u) = (1 - r) PR^t(u) / deg(u) for the rows with out-edges.
__global__ void vjp_cu(const float* __restrict__ pr_t, const int32_t* __restrict__ old_of,
                       const float* __restrict__ inv_outdeg, int64_t rows, float one_r,
                       float* __restrict__ cu) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
       i += (int64_t)gridDim.x * blockDim.x)
    cu[i] = one_r * pr_t[old_of[i]] * inv_outdeg[i];
}

// out[i] = in[index[i]] (into the relabelled order).
__global__ void gather_f32(const float* __restrict__ in, const int32_t* __restrict__ index,
                           int64_t count, float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = in[index[i]];
}

// out[index[i]] = in[i] (back to the caller's edge order).
__global__ void scatter_f32(const float* __restrict__ in, const uint32_t* __restrict__ index,
                            int64_t count, float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[index[i]] = in[i];
}

__global__ void gather_w(const float* __restrict__ w, const uint32_t* __restrict__ ceid,
                         int64_t m, float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = w[ceid[i]];
}

// Relabelled out-edge k (new row i, the last with noff[i] <= k; caller's row
// old_of[i]): destination in new labels, caller's edge id. One thread per
// edge (a thread per row would serialise the hubs).
__global__ void build_edges(const uint32_t* __restrict__ off, const int32_t* __restrict__ out_idx,
                            const int32_t* __restrict__ old_of, const int32_t* __restrict__ new_of,
                            const uint32_t* __restrict__ noff, int64_t rows, int64_t m,
                            int32_t* __restrict__ idx, uint32_t* __restrict__ ceid) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
       k += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = rows;  // noff[lo] <= k < noff[hi]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (noff[mid] <= (uint64_t)k)
        lo = mid;
      else
        hi = mid;
    }
    const uint32_t e = off[old_of[lo]] + (uint32_t)(k - noff[lo]);
    idx[k] = new_of[out_idx[e]];
    ceid[k] = e;
  }
}

inline unsigned blocks_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

VjpPlan* plan(gm_graph g) { return static_cast<VjpPlan*>(g->vjp_plan); }

VjpPlan* ensure_plan(gm_graph g, hipStream_t st) {
  if (plan(g)) return plan(g);
  const int64_t n = g->n, m = g->m;
  if (n >= (int64_t)1 << 30) throw Unsupported{"PageRank reverse pass takes fewer than 2^30 vertices"};
  VjpPlan* p = new VjpPlan();
  g->vjp_plan = p;
  DeviceLayout L;
  try {
    // Vertices relabelled by decreasing out-degree (ties by label), tiles of
    // the relabelled out-adjacency.
    L = build_device_layout(g->out_off, n, m, (uint32_t)g->max_out, st);
    p->n = n;
    p->m = m;
    p->old_of = L.old_of;
    p->starts = L.starts;
    p->tile_row = L.tile_row;
    p->cross = L.cross;
    L.old_of = nullptr;  // owned by the plan from here on
    L.starts = nullptr;
    L.tile_row = nullptr;
    L.cross = nullptr;
    p->rows = L.rows;
    p->ntiles = L.ntiles;
    p->ncross = L.ncross;
    p->mpad = L.mpad;
    int dev = 0;
    GM_HIP(hipGetDevice(&dev));
    GM_HIP(hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, dev));
    GM_HIP(hipDeviceGetAttribute(&p->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    p->idx = dalloc<int32_t>(L.mpad);
    p->ceid = dalloc<uint32_t>(m);
    p->inv_outdeg = dalloc<float>(n);
    p->head = dalloc<double>(L.ntiles);
    p->tail = dalloc<double>(L.ntiles);
    p->wv = dalloc<float>(L.mpad);
    p->gv = dalloc<float>(L.mpad);
    p->cu = dalloc<float>(n + 1);
    p->abar[0] = dalloc<float>(n);
    p->abar[1] = dalloc<float>(n);
    if (L.mpad > m) {
      GM_HIP(hipMemsetAsync(p->idx + m, 0, (L.mpad - m) * 4, st));
      GM_HIP(hipMemsetAsync(p->wv + m, 0, (L.mpad - m) * 4, st));
    }
    GM_HIP(hipMemsetAsync(p->cu, 0, (n + 1) * 4, st));
    gather_f32<<<blocks_for(n), kThreads, 0, st>>>(g->inv_outdeg, p->old_of, n, p->inv_outdeg);
    if (L.rows > 0)
      build_edges<<<blocks_for(m), kThreads, 0, st>>>(g->out_off, g->out_idx, p->old_of, L.new_of,
                                                       L.noff, L.rows, m, p->idx, p->ceid);
    GM_HIP(hipGetLastError());
    GM_HIP(hipStreamSynchronize(st));
  } catch (...) {
    (void)hipStreamSynchronize(st);
    free_device_layout(&L);
    free_vjp_plan(g);
    throw;
  }
  free_device_layout(&L);  // the new labels and offsets were only needed for the edges
  return p;
}

// Workgroups of one vjp_tile launch: as many as fit on the device at once
// with `lds` bytes of LDS each, no more than there are tiles.
unsigned tile_grid(VjpPlan* p, size_t lds) {
  int per_cu = 0;
  GM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)vjp_tile,
                                                       kTileThreads, lds));
  const int64_t fit = (int64_t)std::max(per_cu, 1) * std::max(p->cus, 1);
  const int64_t want = (p->ntiles + kTileWaves - 1) / kTileWaves;
  return (unsigned)std::max<int64_t>(1, std::min(fit, want));
}

}  // namespace

void free_vjp_plan(gm_graph g) {
  VjpPlan* p = plan(g);
  if (!p) return;
  dfree(p->old_of);
  dfree(p->idx);
  dfree(p->ceid);
  dfree(p->inv_outdeg);
  dfree(p->starts);
  dfree(p->tile_row);
  dfree(p->cross);
  dfree(p->head);
  dfree(p->tail);
  dfree(p->wv);
  dfree(p->gv);
  dfree(p->cu);
  dfree(p->abar[0]);
  dfree(p->abar[1]);
  delete p;
  g->vjp_plan = nullptr;
  ++g->ws_gen;
}

void run_pagerank_vjp(gm_graph g, const float* w, float r, int32_t T, const float* hist,
                      const float* grad_out, float* grad_w, hipStream_t st) {
  VjpPlan* p = ensure_plan(g, st);
  const int64_t n = g->n, m = g->m;
  const float one_r = 1.0f - r;
  const int64_t hot_cap = std::min<int64_t>(kTileHotMax, p->lds_max / (int64_t)sizeof(float));
  const int hot_n = (int)std::min<int64_t>(std::min<int64_t>(g->tune.pr_hot, hot_cap), n);
  const size_t lds = (size_t)hot_n * sizeof(float);
  const unsigned grid = tile_grid(p, lds);
  fill_u32(reinterpret_cast<uint32_t*>(p->gv), p->mpad, 0u, st);
  if (m > 0) gather_w<<<blocks_for(m), kThreads, 0, st>>>(w, p->ceid, m, p->wv);
  gather_f32<<<blocks_for(n), kThreads, 0, st>>>(grad_out, p->old_of, n, p->abar[0]);  // abar^T = c
  // Rows without out-edges have abar = 0 from the first reverse step on.
  if (n > p->rows)
    fill_u32(reinterpret_cast<uint32_t*>(p->abar[1] + p->rows), n - p->rows, 0u, st);
  GM_HIP(hipGetLastError());
  int cur = 0;
  for (int32_t t = T - 1; t >= 0; --t) {
    const float* an = p->abar[cur];
    float* ac = p->abar[cur ^ 1];
    if (p->rows > 0)
      vjp_cu<<<blocks_for(p->rows), kThreads, 0, st>>>(hist + (int64_t)t * n, p->old_of,
                                                        p->inv_outdeg, p->rows, one_r, p->cu);
    if (p->ntiles > 0)
      vjp_tile<<<grid, kTileThreads, lds, st>>>(p->idx, p->wv, p->starts, p->tile_row, p->ntiles,
                                                an, p->cu, p->inv_outdeg, one_r, ac, p->gv,
                                                p->head, p->tail, hot_n);
    if (p->ncross > 0)
      vjp_cross<<<(unsigned)((p->ncross * kCrossLanes + kThreads - 1) / kThreads), kThreads, 0,
                  st>>>(p->cross, p->ncross, p->head, p->tail, p->inv_outdeg, one_r, ac);
    GM_HIP(hipGetLastError());
    if (t == T - 1 && n > p->rows)  // abar^T (= c) is consumed: its rows without out-edges go to 0
      fill_u32(reinterpret_cast<uint32_t*>(p->abar[cur] + p->rows), n - p->rows, 0u, st);
    cur ^= 1;
  }
  if (m > 0) scatter_f32<<<blocks_for(m), kThreads, 0, st>>>(p->gv, p->ceid, m, grad_w);
  GM_HIP(hipGetLastError());
}

}  // namespace gm
