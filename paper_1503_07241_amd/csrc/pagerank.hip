// PageRank (Sec. 3 I, Eq. (1)) and personalised PageRank as a pull-direction
// generalized SpMV over the in-adjacency, with APPLY and the next SEND fused
// into the same kernel.
//
// One superstep = one launch of pr_pull (+ pr_cross for rows that span
// tiles):
//   y_v   = sum_{u -> v} x_u (* w_uv)          PROCESS = msg (* w), REDUCE = +
//   PR_v  = r * tele(v) + (1 - r) * y_v        APPLY, for every vertex
//   x'_v  = PR_v / outdeg(v)                   SEND for the next superstep
// where x_u = PR_u / outdeg(u) is the message (0 for dangling vertices, which
// send nothing). Row sums are accumulated in double in a fixed order, so the
// result does not depend on scheduling.
//
// Dense layout (built once per graph, on first use): vertices are relabelled
// in decreasing in-degree order and the in-adjacency is rebuilt in the new
// labels. Rows with in-edges are then [0, rows) and the rest are written once
// per run; the edge stream is cut into equal tiles regardless of row lengths
// (a bitmap marks the first edge of each row), so every wavefront streams the
// same number of edges with fully coalesced loads; and the most frequently
// gathered messages (high-degree vertices, which in RMAT graphs have high in-
// and out-degree alike) sit together at low labels: the first of them (a
// tuning parameter, up to kHotMax) are copied to LDS by every workgroup and
// read from there, the next ones stay cache resident. The caller's rank
// vector is mapped into the new labels by the first SEND and back after the
// last APPLY.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "gm_internal.h"
#include "tiles.h"

// Scratch of the allocation-free PageRank entry point (gm_pagerank_noalloc):
// the two message buffers, PR and the per-tile partial sums of one run.
static __device__ __align__(256) unsigned char scratch[gm::kNoallocScratchBytes];

namespace gm {
namespace {

using namespace tiles;

constexpr int kThreads = 256;
constexpr int kPullThreads = kTileThreads;
constexpr int kPullWaves = kTileWaves;
constexpr int kHotMax = kTileHotMax;  // at most this many hot messages in LDS (160 KB)

struct Dense {
  int64_t n = 0, m = 0;
  int32_t* new_of = nullptr;    // old label -> new label
  int32_t* old_of = nullptr;    // new label -> old label
  int32_t* idx = nullptr;       // relabelled in-adjacency, padded to whole tiles with 0
  float* w = nullptr;           // edge values in the relabelled order (weighted graphs), padded
  uint32_t* ceid = nullptr;     // canonical (CSR) edge id of each relabelled in-edge
  float* wdyn = nullptr;        // caller-supplied edge values, relabelled per call, padded
  float* inv_outdeg = nullptr;  // new labels
  float* x[2] = {nullptr, nullptr};
  float* pr = nullptr;          // PR in new labels (last superstep)
  uint32_t* starts = nullptr;   // bit e set: edge e is the first of its row (and bit m)
  uint32_t* tile_row = nullptr; // row holding the first edge of each tile
  double* head = nullptr;       // per tile: sum of the part of a row begun before the tile
  double* tail = nullptr;       // per tile: sum of the part of a row that goes on after it
  Cross* cross = nullptr;
  uint32_t* roff = nullptr;     // row offsets of the relabelled in-adjacency (n + 1)
  int64_t ntiles = 0, ncross = 0;
  int64_t rows = 0;             // rows with in-edges: new labels [0, rows)
  int cus = 0;                  // compute units of the device
  int lds_max = 0;              // bytes of LDS a workgroup may use
};

// APPLY: PR_v from the sum y of its in-messages.
template <bool kPersonal>
__device__ inline float pr_value(uint32_t v, double y, float r, int32_t seed) {
  double tele = 1.0;
  if constexpr (kPersonal) tele = (int32_t)v == seed ? 1.0 : 0.0;
  return (float)((double)r * tele + (1.0 - (double)r) * y);
}

// APPLY and the next SEND of row v.
template <bool kPersonal>
__device__ inline void apply_row(uint32_t v, double y, float r, int32_t seed,
                                 const float* __restrict__ inv_outdeg, float* __restrict__ x_out,
                                 float* __restrict__ pr_out) {
  const float pr = pr_value<kPersonal>(v, y, r, seed);
  x_out[v] = pr * inv_outdeg[v];
  if (pr_out) pr_out[v] = pr;
}

// One superstep: y = A^T x (pull over in-edges), APPLY, next SEND.
//
// The relabelled in-edges are cut into tiles of kTile consecutive edges,
// whatever the rows; a wavefront takes a tile in kRounds rounds of 256
// edges, 4 consecutive ones per lane, so every index load is one coalesced
// 16-byte load per lane, and all of a tile's gathers are in flight at once
// (they, not the index stream, bound the kernel: most go to a different
// cache line each). Row sums are a segmented scan over the tile (in double,
// in a fixed order): the lane holding the last edge of a row that begins in
// the tile applies it; a row begun in an earlier tile leaves its part in
// head[t], one that goes on past the tile's end its part in tail[t], and
// pr_cross finishes those rows. Each workgroup first copies the messages of
// the hottest labels to LDS (hot_n of them; a label below hot_n is read from
// there, its global gather then reads x[0], one line shared by all such
// lanes). Gathers use 32-bit byte offsets, hence n < 2^30.
template <bool kWeighted>
struct TileLoad {
  v4i src[kRounds];
  v4f w[kRounds];
  uint32_t fa[kRounds], fb[kRounds];  // word of `starts` with the lane's bits, and the next
};

template <bool kWeighted>
__device__ inline void load_tile(TileLoad<kWeighted>& L, const int32_t* __restrict__ idx,
                                 const float* __restrict__ w, const uint32_t* __restrict__ starts,
                                 int64_t e) {
#pragma unroll
  for (int v = 0; v < kRounds; ++v) {
    const int64_t ev = e + v * 256;
    L.src[v] = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(idx + ev));
    if constexpr (kWeighted) L.w[v] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(w + ev));
    L.fa[v] = starts[ev >> 5];
    L.fb[v] = starts[(ev >> 5) + 1];
  }
}

template <bool kWeighted, bool kPersonal>
__global__ __launch_bounds__(kPullThreads) void pr_pull(
    const int32_t* __restrict__ idx, const float* __restrict__ w,
    const uint32_t* __restrict__ starts, const uint32_t* __restrict__ tile_row, int64_t ntiles,
    const float* __restrict__ x_in, const float* __restrict__ inv_outdeg, float r, int32_t seed,
    float* __restrict__ x_out, float* __restrict__ pr_out, double* __restrict__ head,
    double* __restrict__ tail, int hot_n) {
  extern __shared__ float hot[];  // hot_n floats
  load_hot(x_in, hot, hot_n);
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * kPullWaves;
  const int sh = (lane & 7) * 4;  // this lane's 4 bits in its word of `starts`
  const char* xb = reinterpret_cast<const char*>(x_in);
  int64_t t = __builtin_amdgcn_readfirstlane(blockIdx.x * kPullWaves + (threadIdx.x >> 6));
  if (t >= ntiles) return;
  TileLoad<kWeighted> cur;
  for (; t < ntiles; t += stride) {
    load_tile(cur, idx, w, starts, t * kTile + lane * 4);
    float val[kRounds][4];
#pragma unroll
    for (int v = 0; v < kRounds; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t s = (uint32_t)cur.src[v][q];
        const bool in_lds = s < (uint32_t)hot_n;
        const float g = *reinterpret_cast<const float*>(xb + (in_lds ? 0u : s << 2));
        const float l = hot[in_lds ? s : 0u];
        val[v][q] = in_lds ? l : g;
        if constexpr (kWeighted) val[v][q] *= cur.w[v][q];
      }
    uint32_t nib[kRounds], next[kRounds];
#pragma unroll
    for (int v = 0; v < kRounds; ++v) {
      nib[v] = (cur.fa[v] >> sh) & 0xFu;  // bit q: edge q of the lane starts a row
      next[v] = sh == 28 ? (cur.fb[v] & 1u) : (cur.fa[v] >> (sh + 4)) & 1u;
    }
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t row0 = tile_row[t];
    // A start at the tile's first edge opens row0 itself, not the next row.
    const int f0 = __builtin_amdgcn_readfirstlane((int)(nib[0] & 1u));
    Seg carry{0, 0.0};
    float prv[kRounds][4];
    uint32_t rowv[kRounds][4];
    uint32_t done = 0;  // bit 4v+q: edge (v, q) ends a row begun in the tile
#pragma unroll
    for (int v = 0; v < kRounds; ++v) {
      double s[4];
      s[0] = (double)val[v][0];
#pragma unroll
      for (int q = 1; q < 4; ++q)
        s[q] = ((nib[v] >> q) & 1u ? 0.0 : s[q - 1]) + (double)val[v][q];
      const Seg ex = seg_scan(Seg{(int)__popc(nib[v]), s[3]}, carry, lane);
      const uint32_t ends = (nib[v] >> 1) | (next[v] << 3);  // bit q: edge q ends its row
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        rowv[v][q] = row0;
        prv[v][q] = 0.0f;
        if ((ends >> q) & 1u) {
          const int lc = (int)__popc(nib[v] & ((2u << q) - 1u));  // starts at or before edge q
          const int c = ex.c + lc;                                 // ... since the tile's first
          const double y = lc > 0 ? s[q] : ex.s + s[q];
          if (c > 0) {
            rowv[v][q] = row0 + (uint32_t)(c - f0);
            prv[v][q] = pr_value<kPersonal>(rowv[v][q], y, r, seed);
            done |= 1u << (4 * v + q);
          } else {
            head[t] = y;
          }
        }
      }
      if (v == kRounds - 1 && lane == 63 && !(ends >> 3)) {
        const int c = ex.c + (int)__popc(nib[v]);
        const double y = nib[v] ? s[3] : ex.s + s[3];
        if (c > 0)
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
        if ((done >> (4 * v + q)) & 1u) inv[v][q] = inv_outdeg[rowv[v][q]];
      }
#pragma unroll
    for (int v = 0; v < kRounds; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if ((done >> (4 * v + q)) & 1u) {
          x_out[rowv[v][q]] = prv[v][q] * inv[v][q];
          if (pr_out) pr_out[rowv[v][q]] = prv[v][q];
        }
  }
}

// Rows spanning tiles ta..tb: tail[ta] + head[ta + 1] + ... + head[tb],
// summed by kCrossLanes lanes in a fixed order, then APPLY and SEND.
template <bool kPersonal>
__global__ void pr_cross(const Cross* __restrict__ cross, int64_t ncross,
                         const double* __restrict__ head, const double* __restrict__ tail,
                         const float* __restrict__ inv_outdeg, float r, int32_t seed,
                         float* __restrict__ x_out, float* __restrict__ pr_out) {
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
  if (i < ncross && j == 0) apply_row<kPersonal>(c.row, acc, r, seed, inv_outdeg, x_out, pr_out);
}

// Ablation variant of the superstep (GM_VARIANT_ROW_PULL): one thread per
// row sums its in-edges in order (no edge tiles, no LDS copy of the hottest
// messages), then APPLY and the next SEND.
template <bool kWeighted, bool kPersonal>
__global__ void pr_rowpull(const uint32_t* __restrict__ roff, const int32_t* __restrict__ idx,
                           const float* __restrict__ w, int64_t rows,
                           const float* __restrict__ x_in, const float* __restrict__ inv_outdeg,
                           float r, int32_t seed, float* __restrict__ x_out,
                           float* __restrict__ pr_out) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < rows;
       v += (int64_t)gridDim.x * blockDim.x) {
    double y = 0.0;
    const uint32_t e1 = roff[v + 1];
    for (uint32_t e = roff[v]; e < e1; ++e) {
      float x = x_in[idx[e]];
      if constexpr (kWeighted) x *= w[e];
      y += (double)x;
    }
    apply_row<kPersonal>((uint32_t)v, y, r, seed, inv_outdeg, x_out, pr_out);
  }
}

// Rows without in-edges: PR = r * tele(v) in every superstep after the first,
// so their APPLY and next SEND are written once per run instead of per
// superstep.
template <bool kPersonal>
__global__ void pr_const_rows(int64_t row_begin, int64_t nrows, float r, int32_t seed,
                              const float* __restrict__ inv_outdeg, float* __restrict__ x_out,
                              float* __restrict__ pr_out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nrows;
       i += (int64_t)gridDim.x * blockDim.x)
    apply_row<kPersonal>((uint32_t)(row_begin + i), 0.0, r, seed, inv_outdeg, x_out, pr_out);
}

// First SEND in new labels: x[i] = rank[old(i)] / outdeg.
__global__ void pr_send0(const float* __restrict__ rank, const int32_t* __restrict__ old_of,
                         const float* __restrict__ inv_outdeg, int64_t n, float* __restrict__ x) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = rank[old_of[i]] * inv_outdeg[i];
}

// rank[v] = pr[new(v)]: back to the caller's labels.
__global__ void pr_unpermute(const float* __restrict__ pr, const int32_t* __restrict__ new_of,
                             int64_t n, float* __restrict__ rank) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    rank[v] = pr[new_of[v]];
}

// Row of edge e in a CSR with offsets off (n + 1 entries): the last v with
// off[v] <= e.
__device__ inline int64_t row_of_edge(const uint32_t* __restrict__ off, int64_t n, uint32_t e) {
  int64_t lo = 0, hi = n;  // off[lo] <= e < off[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= e)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Relabelled in-adjacency keys: (new row << b | new source), value = in-edge
// id; one thread per edge (a thread per row would serialise the hubs).
__global__ void relabel_keys(const uint32_t* __restrict__ in_off, const int32_t* __restrict__ in_idx,
                             const int32_t* __restrict__ new_of, int64_t n, int64_t m, int b,
                             unsigned long long* __restrict__ keys, uint32_t* __restrict__ eid) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = row_of_edge(in_off, n, (uint32_t)e);
    keys[e] = ((unsigned long long)(uint32_t)new_of[v] << b) | (uint32_t)new_of[in_idx[e]];
    eid[e] = (uint32_t)e;
  }
}

__global__ void relabel_finish(const unsigned long long* __restrict__ keys,
                               const uint32_t* __restrict__ eid, int64_t m, int b,
                               const float* __restrict__ in_w, const uint32_t* __restrict__ in_eid,
                               int32_t* __restrict__ idx, float* __restrict__ w,
                               uint32_t* __restrict__ ceid) {
  const unsigned long long mask = (1ull << b) - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    idx[i] = (int32_t)(keys[i] & mask);
    if (w) w[i] = in_w[eid[i]];
    ceid[i] = in_eid[eid[i]];
  }
}

// Caller-supplied edge values (canonical order) -> relabelled order.
__global__ void gather_w(const float* __restrict__ w, const uint32_t* __restrict__ ceid, int64_t m,
                         float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = w[ceid[i]];
}

__global__ void gather_f32(const float* __restrict__ src, const int32_t* __restrict__ index,
                           int64_t n, float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = src[index[i]];
}

inline unsigned blocks_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

Dense* dense(gm_graph g) { return static_cast<Dense*>(g->pr_sched); }

template <class T>
struct DevBuf {
  T* p = nullptr;
  explicit DevBuf(size_t n) : p(dalloc<T>(n)) {}
  ~DevBuf() { dfree(p); }
};

}  // namespace

void free_pull_schedule(gm_graph g) {
  Dense* d = dense(g);
  if (!d) return;
  dfree(d->new_of);
  dfree(d->old_of);
  dfree(d->idx);
  dfree(d->w);
  dfree(d->ceid);
  dfree(d->wdyn);
  dfree(d->inv_outdeg);
  dfree(d->x[0]);
  dfree(d->x[1]);
  dfree(d->pr);
  dfree(d->starts);
  dfree(d->tile_row);
  dfree(d->head);
  dfree(d->tail);
  dfree(d->cross);
  dfree(d->roff);
  delete d;
  g->pr_sched = nullptr;
  ++g->ws_gen;
}

void ensure_pull_schedule(gm_graph g, hipStream_t st) {
  if (dense(g)) return;
  const int64_t n = g->n, m = g->m;
  if (n >= (int64_t)1 << 30) throw Unsupported{"PageRank pull takes fewer than 2^30 vertices"};
  Dense* d = new Dense();
  g->pr_sched = d;
  try {
    d->n = n;
    d->m = m;
    // Vertices relabelled by decreasing in-degree (ties by label): rows with
    // in-edges come first; tiles of kTile edges, the index stream padded to
    // whole tiles.
    const DeviceLayout L = build_device_layout(g->in_off, n, m, (uint32_t)g->max_in, st);
    d->new_of = L.new_of;
    d->old_of = L.old_of;
    d->roff = L.noff;
    d->starts = L.starts;
    d->tile_row = L.tile_row;
    d->cross = L.cross;
    d->rows = L.rows;
    d->ntiles = L.ntiles;
    d->ncross = L.ncross;
    const int64_t ntiles = L.ntiles, mpad = L.mpad;
    int dev = 0;
    GM_HIP(hipGetDevice(&dev));
    GM_HIP(hipDeviceGetAttribute(&d->cus, hipDeviceAttributeMultiprocessorCount, dev));
    GM_HIP(hipDeviceGetAttribute(&d->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    d->idx = dalloc<int32_t>(mpad);
    d->inv_outdeg = dalloc<float>(n);
    d->x[0] = dalloc<float>(n);
    d->x[1] = dalloc<float>(n);
    d->pr = dalloc<float>(n);
    d->head = dalloc<double>(ntiles);
    d->tail = dalloc<double>(ntiles);
    if (mpad > m) GM_HIP(hipMemsetAsync(d->idx + m, 0, (mpad - m) * 4, st));
    gather_f32<<<blocks_for(n), kThreads, 0, st>>>(g->inv_outdeg, d->old_of, n, d->inv_outdeg);
    GM_HIP(hipGetLastError());
    if (m > 0) {
      int b = 1;
      while ((1ll << b) < n) ++b;
      DevBuf<unsigned long long> k1(m), k2(m);
      DevBuf<uint32_t> e1(m), e2(m);
      relabel_keys<<<blocks_for(m), kThreads, 0, st>>>(g->in_off, g->in_idx, d->new_of, n, m, b,
                                                       k1.p, e1.p);
      GM_HIP(hipGetLastError());
      rocprim::double_buffer<unsigned long long> kb(k1.p, k2.p);
      rocprim::double_buffer<uint32_t> vb(e1.p, e2.p);
      size_t bytes = 0;
      GM_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kb, vb, (size_t)m, 0, 2 * b, st));
      void* tmp = dmalloc(bytes);
      const hipError_t err = rocprim::radix_sort_pairs(tmp, bytes, kb, vb, (size_t)m, 0, 2 * b, st);
      if (err == hipSuccess) (void)hipStreamSynchronize(st);
      dfree(tmp);
      GM_HIP(err);
      if (g->wtype == GM_W_F32) {
        d->w = dalloc<float>(mpad);
        if (mpad > m) GM_HIP(hipMemsetAsync(d->w + m, 0, (mpad - m) * 4, st));
      }
      d->ceid = dalloc<uint32_t>(m);
      relabel_finish<<<blocks_for(m), kThreads, 0, st>>>(kb.current(), vb.current(), m, b,
                                                         static_cast<const float*>(g->in_w),
                                                         g->in_eid, d->idx, d->w, d->ceid);
      GM_HIP(hipGetLastError());
    }
    GM_HIP(hipStreamSynchronize(st));
  } catch (...) {
    free_pull_schedule(g);
    throw;
  }
}

// Workgroups of one pr_pull launch: as many as fit on the device at once
// with `lds` bytes of LDS each (the kernel strides over the tiles), no more
// than there are tiles.
static unsigned pull_grid(Dense* d, size_t lds, bool weighted, bool personal) {
  const void* k = weighted ? (personal ? (const void*)pr_pull<true, true> : (const void*)pr_pull<true, false>)
                           : (personal ? (const void*)pr_pull<false, true> : (const void*)pr_pull<false, false>);
  int per_cu = 0;
  GM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kPullThreads, lds));
  const int64_t fit = (int64_t)std::max(per_cu, 1) * std::max(d->cus, 1);
  const int64_t want = (d->ntiles + kPullWaves - 1) / kPullWaves;
  return (unsigned)std::max<int64_t>(1, std::min(fit, want));
}

namespace {

// The per-run vectors of a PageRank run: the two message buffers, PR in the
// new labels and the per-tile partial sums (the graph's own, or the fixed
// scratch array of the allocation-free entry point).
struct Vecs {
  float* x[2];
  float* pr;
  double* head;
  double* tail;
};

Vecs own_vecs(Dense* d) { return Vecs{{d->x[0], d->x[1]}, d->pr, d->head, d->tail}; }

}  // namespace

// Supersteps of (personalised, optionally weighted) PageRank from the rank
// vector `rank0` (caller labels). w: relabelled edge values or NULL. After
// the last superstep the ranks go to `rank_out`; with `hist` (T + 1 rows),
// PR^t is also written to row t for t = 1..iters.
static void pagerank_driver(gm_graph g, Dense* d, const Vecs& v, float r, int32_t iters,
                            const float* rank0, int32_t seed_new, const float* w, float* hist,
                            float* rank_out, hipStream_t st) {
  const int64_t n = g->n;
  const bool weighted = w != nullptr;
  const bool personal = seed_new >= 0;
  pr_send0<<<blocks_for(n), kThreads, 0, st>>>(rank0, d->old_of, d->inv_outdeg, n, v.x[0]);
  GM_HIP(hipGetLastError());
  const int64_t c0 = d->rows, n0 = n - d->rows;
  auto const_rows = [&](float* xo, float* po) {
    if (n0 == 0) return;
    if (personal)
      pr_const_rows<true><<<blocks_for(n0), kThreads, 0, st>>>(c0, n0, r, seed_new, d->inv_outdeg,
                                                                xo, po);
    else
      pr_const_rows<false><<<blocks_for(n0), kThreads, 0, st>>>(c0, n0, r, seed_new,
                                                                 d->inv_outdeg, xo, po);
    GM_HIP(hipGetLastError());
  };
  const int64_t hot_cap = std::min<int64_t>(kHotMax, d->lds_max / (int64_t)sizeof(float));
  const int hot_n = (int)std::min<int64_t>(std::min<int64_t>(g->tune.pr_hot, hot_cap), n);
  const size_t lds = (size_t)hot_n * sizeof(float);
  const unsigned grid = pull_grid(d, lds, weighted, personal);
  const_rows(v.x[1], v.pr);
  for (int32_t it = 0; it < iters; ++it) {
    const float* xin = v.x[it & 1];
    float* xout = v.x[(it + 1) & 1];
    float* pout = (hist || it == iters - 1) ? v.pr : nullptr;
    auto launch = [&](auto kern) {
      if (d->ntiles > 0)
        kern<<<grid, kPullThreads, lds, st>>>(d->idx, w, d->starts, d->tile_row, d->ntiles, xin,
                                              d->inv_outdeg, r, seed_new, xout, pout, v.head,
                                              v.tail, hot_n);
    };
    if (g->tune.variant & GM_VARIANT_ROW_PULL) {
      auto rows = [&](auto kern) {
        if (d->rows > 0)
          kern<<<blocks_for(d->rows), kThreads, 0, st>>>(d->roff, d->idx, w, d->rows, xin,
                                                         d->inv_outdeg, r, seed_new, xout, pout);
      };
      if (weighted && personal)
        rows(pr_rowpull<true, true>);
      else if (weighted)
        rows(pr_rowpull<true, false>);
      else if (personal)
        rows(pr_rowpull<false, true>);
      else
        rows(pr_rowpull<false, false>);
    } else if (weighted && personal)
      launch(pr_pull<true, true>);
    else if (weighted)
      launch(pr_pull<true, false>);
    else if (personal)
      launch(pr_pull<false, true>);
    else
      launch(pr_pull<false, false>);
    if (d->ncross > 0 && !(g->tune.variant & GM_VARIANT_ROW_PULL)) {
      const unsigned fb = (unsigned)((d->ncross * kCrossLanes + kThreads - 1) / kThreads);
      if (personal)
        pr_cross<true><<<fb, kThreads, 0, st>>>(d->cross, d->ncross, v.head, v.tail,
                                                 d->inv_outdeg, r, seed_new, xout, pout);
      else
        pr_cross<false><<<fb, kThreads, 0, st>>>(d->cross, d->ncross, v.head, v.tail,
                                                  d->inv_outdeg, r, seed_new, xout, pout);
    }
    GM_HIP(hipGetLastError());
    if (it == 0) const_rows(v.x[0], nullptr);  // x[0] held PR^0 messages until now
    if (hist) {
      pr_unpermute<<<blocks_for(n), kThreads, 0, st>>>(v.pr, d->new_of, n, hist + (it + 1) * n);
      GM_HIP(hipGetLastError());
    }
  }
  if (rank_out) {
    pr_unpermute<<<blocks_for(n), kThreads, 0, st>>>(v.pr, d->new_of, n, rank_out);
    GM_HIP(hipGetLastError());
  }
}

void run_pagerank(gm_graph g, float r, int32_t iters, float* rank, int32_t seed, hipStream_t st) {
  ensure_pull_schedule(g, st);
  Dense* d = dense(g);
  int32_t seed_new = -1;
  if (seed >= 0) {
    GM_HIP(hipMemcpyAsync(&seed_new, d->new_of + seed, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GM_HIP(hipStreamSynchronize(st));
  }
  pagerank_driver(g, d, own_vecs(d), r, iters, rank, seed_new,
                  g->wtype == GM_W_F32 ? d->w : nullptr, nullptr, rank, st);
}

// PR^0 = 1 for every vertex, then `iters` supersteps (no allocation and no
// host synchronisation once the pull schedule exists).
void enqueue_pagerank(gm_graph g, float r, int32_t iters, float* rank, hipStream_t st) {
  Dense* d = dense(g);
  if (!d) throw Unsupported{"captured run not prepared"};
  fill_f32(rank, g->n, 1.0f, st);
  pagerank_driver(g, d, own_vecs(d), r, iters, rank, -1, g->wtype == GM_W_F32 ? d->w : nullptr,
                  nullptr, rank, st);
}

void run_pagerank_history(gm_graph g, const float* w, float r, int32_t T, float* hist,
                          hipStream_t st) {
  ensure_pull_schedule(g, st);
  Dense* d = dense(g);
  if (!d->wdyn) {
    const int64_t mpad = d->ntiles * kTile;
    d->wdyn = dalloc<float>(mpad);
    if (mpad > g->m) GM_HIP(hipMemsetAsync(d->wdyn + g->m, 0, (mpad - g->m) * 4, st));
  }
  if (g->m > 0) {
    gather_w<<<blocks_for(g->m), kThreads, 0, st>>>(w, d->ceid, g->m, d->wdyn);
    GM_HIP(hipGetLastError());
  }
  pagerank_driver(g, d, own_vecs(d), r, T, hist, -1, d->wdyn, hist, nullptr, st);
}

// ---------------------------------------------------------------------------
// Allocation-free PageRank: the per-run vectors live in `scratch` (one copy
// per device, held until the process ends) instead of the graph's workspace.
// Host code reaches the array only through the address hipGetSymbolAddress
// returns for the current device, kept per device.
// ---------------------------------------------------------------------------
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

bool pull_schedule_ready(gm_graph g) { return dense(g) != nullptr; }

size_t pagerank_noalloc_bytes(gm_graph g) {
  const Dense* d = dense(g);
  return 3 * align256((size_t)g->n * 4) + 2 * align256((size_t)std::max<int64_t>(d->ntiles, 1) * 8);
}

void run_pagerank_noalloc(gm_graph g, float r, int32_t iters, float* rank, hipStream_t st) {
  Dense* d = dense(g);
  if (!d) throw Unsupported{"pull layout not built"};
  if (g->device < 0 || g->device >= kMaxDevices) throw Unsupported{"device ordinal out of range"};
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[g->device]) {
      void* ptr = nullptr;
      GM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));  // the current device's copy
      g_scratch_ptr[g->device] = ptr;
    }
    base = static_cast<char*>(g_scratch_ptr[g->device]);
  }
  const size_t xv = align256((size_t)g->n * 4);
  const size_t tv = align256((size_t)std::max<int64_t>(d->ntiles, 1) * 8);
  Vecs v;
  v.x[0] = reinterpret_cast<float*>(base);
  v.x[1] = reinterpret_cast<float*>(base + xv);
  v.pr = reinterpret_cast<float*>(base + 2 * xv);
  v.head = reinterpret_cast<double*>(base + 3 * xv);
  v.tail = reinterpret_cast<double*>(base + 3 * xv + tv);
  pagerank_driver(g, d, v, r, iters, rank, -1, g->wtype == GM_W_F32 ? d->w : nullptr, nullptr,
                  rank, st);
}

}  // namespace gm
