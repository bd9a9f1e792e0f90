// BFS (Sec. 3 II, Eq. (2)) and SSSP (Sec. 3 V, Eq. (8)): vertex programs whose
// REDUCE is min, run as supersteps of Alg. 2 on a sparse frontier.
//
// The frontier is a bitvector over the vertices (the sparse-vector layout the
// paper adopts, Sec. 4.4.2). Superstep t:
//   send_count, send_write
//                 compact the frontier bitvector into a queue of active
//                 vertices (in vertex order) and snapshot each one's message
//                 x_u = prop(u) (SEND_MESSAGE), its first out-edge, and the
//                 exclusive prefix sum of out-degrees over the queue. Counts,
//                 edge totals and the smallest/largest message go to a small
//                 per-superstep control record, which also decides the
//                 superstep's direction; a pull superstep needs no queue (an
//                 SSSP pull gets a dense message snapshot instead).
//   push_kernel   walks the out-edges of the queued vertices (the columns of
//                 G^T present in x, Alg. 1). The concatenated edge lists are
//                 cut into equal ranges, one per wavefront, so hubs and
//                 low-degree vertices cost the same per edge; a wavefront
//                 finds its first vertex by a 64-ary search of the prefix sum.
//                 Each edge (u, v, w) forms PROCESS(x_u, w) and REDUCEs it
//                 into prop(v) with an atomic min, which is also APPLY
//                 (min(prop, y)); a vertex whose value dropped gets its bit in
//                 the next frontier.
//   pull_kernel   (BFS, large frontier, all frontier levels equal) instead
//                 lets every vertex whose level exceeds the frontier level + 1
//                 look for an in-neighbour in the frontier. Levels are
//                 unique, so the result is the same as pushing.
//   pull_min_tiles (SSSP, frontier with many out-edges) instead lets every
//                 vertex take the min over all its in-edges of PROCESS applied
//                 to a dense snapshot of the frontier's messages (the max
//                 value for inactive sources), with no atomics on the edges.
// The push and pull kernels of a superstep are both launched; each reads the
// control record written by send_write and only the selected one works (a
// batch of supersteps the host expects to push only launches no pull
// kernel). Messages are snapshotted before the product and min is exact and
// order-free, so every superstep leaves exactly the state of Alg. 2. The
// push's atomic min returns the old value, which tells whether the target
// changed; the pull applies a row with a plain store when one wavefront
// holds all of its in-edges.
#include <algorithm>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kUnroll = 4;  // edge rounds in flight per wavefront
constexpr uint32_t kInfBfs = 0x7FFFFFFFu;
constexpr int kMaxCtl = 64;  // control records per launch batch (one more is allocated)
constexpr uint64_t kMinWaveEdges = 512;  // push: fewest edges per working wavefront

template <class T>
struct DevBuf {  // a temporary device array, freed at scope exit
  T* p = nullptr;
  explicit DevBuf(int64_t count) : p(dalloc<T>(count)) {}
  ~DevBuf() { dfree(p); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

struct Ctl {
  unsigned long long packed;  // (queued vertices << 32) | their out-edges
  unsigned int msg_min;       // smallest message of the frontier
  unsigned int msg_max;       // largest message of the frontier
};

struct Workspace {
  int64_t n = 0;
  int32_t* q = nullptr;       // active vertices
  uint32_t* qmsg = nullptr;   // their messages
  uint32_t* qbeg = nullptr;   // their first out-edge
  uint32_t* qest = nullptr;   // exclusive prefix sum of out-degrees
  uint32_t* bits[2] = {nullptr, nullptr};
  Ctl* ctl = nullptr;         // kMaxCtl records
  struct SendInfo* sinfo = nullptr;  // per-workgroup SEND totals (kSendBlocksMax)
  Ctl* host_ctl = nullptr;    // pinned mirror
  // GM_ORDER_ALL adjacency (built on first use): off = out_off + in_off,
  // each vertex's out-list followed by its in-list (values alike)
  uint32_t* all_off = nullptr;
  int32_t* all_idx = nullptr;
  uint32_t* all_w = nullptr;
  struct Relab* rl = nullptr;  // degree-ordered copy for the plain runs (built on first use)
  uint32_t* snap = nullptr;    // SSSP pull: frontier messages, the max value elsewhere (n)
  struct PullTiles* pt = nullptr;  // SSSP pull: tile layout of the pulled adjacency
};

// Tile layout of the SSSP pull over one adjacency (built on first use): the
// row-start bitmap over its edges (and bit m), its rows with edges in order,
// and for each tile of kPullTile edges the index in that list of the row
// holding the tile's first edge.
struct PullTiles {
  const uint32_t* for_off = nullptr;  // offsets of the adjacency it describes
  uint32_t* starts = nullptr;
  uint32_t* rows = nullptr;
  uint32_t* tile_row = nullptr;
  int64_t ntiles = 0, nrows = 0;
  // The message snapshot is kept in rank order: vertices by decreasing
  // out-degree (vert_of[rank] = vertex), so that the most gathered messages
  // share cache lines and the hot_n first ranks are the LDS hot set; tidx is
  // the adjacency's index array in ranks, padded to whole tiles with 0
  uint32_t* vert_of = nullptr;
  int32_t* tidx = nullptr;
  int hot_n = 0;
  int cus = 0;  // compute units (one 1,024-lane workgroup each)
  ~PullTiles() {
    dfree(starts);
    dfree(rows);
    dfree(tile_row);
    dfree(tidx);
    dfree(vert_of);
  }
};

// The adjacency a superstep pushes messages along: out-edges (GM_ORDER_OUT),
// in-edges (GM_ORDER_IN), or both (GM_ORDER_ALL: each vertex's out-list
// followed by its in-list, built once per graph).
struct Adj {
  const uint32_t* off;
  const int32_t* idx;
  const uint32_t* w;
};

// What a superstep reads: the adjacency it pushes along and, for BFS and
// SSSP along out-edges, the in-adjacency (with its values) a pull superstep
// scans (pull_ok false: never pulls).
struct View {
  Adj push;
  Adj pull;
  bool pull_ok;
};

// A device-owned adjacency (offsets, targets padded by kIdxPad, values).
struct OwnedAdj {
  uint32_t* off = nullptr;
  int32_t* idx = nullptr;
  uint32_t* w = nullptr;
  Adj view() const { return Adj{off, idx, w}; }
  void release() {
    dfree(off);
    dfree(idx);
    dfree(w);
    off = nullptr;
    idx = nullptr;
    w = nullptr;
  }
};

// Degree-ordered relabelling of the plain runs (GM_VARIANT_DEGREE_ORDER):
// vertices numbered by decreasing in-degree (out-degree without the
// in-layout), ties by label, and the adjacency rebuilt in the new labels.
// The values a superstep reads and lowers at random (prop of every edge's
// target) then cluster at low labels, where the hottest share few cache
// lines, whatever order the caller's labels come in. Each run maps the
// caller's values and frontier in and its results back; supersteps,
// frontiers and results are those of the caller's labels, permuted.
struct Relab {
  int32_t* new_of = nullptr;   // caller label -> new label
  int32_t* old_of = nullptr;   // new label -> caller label
  uint32_t* prop = nullptr;    // the run's vertex values in new labels
  int32_t* ids = nullptr;      // the run's frontier ids in new labels (list variant)
  int32_t* active = nullptr;   // the run's final frontier in new labels
  OwnedAdj out, in, all;       // each built on first use
};


// Direction of a superstep, from its control record: BFS pulls when more
// than n / pull_div vertices are active (all at one level), SSSP when the
// frontier's out-edges exceed 64 m / pull_div (half the edges at the
// default 128; pull_div 1: never).
__host__ __device__ inline bool use_pull(const Ctl& c, int kind, bool pull_ok, int64_t n,
                                         int64_t m, uint32_t pull_div) {
  const uint64_t count = c.packed >> 32;
  if (!pull_ok || count == 0) return false;
  if (kind == GM_PROG_BFS)
    return c.msg_min == c.msg_max && count > (uint64_t)(n / (int64_t)pull_div);
  if (kind == GM_PROG_SSSP)
    return (uint64_t)(uint32_t)c.packed * pull_div > 64 * (uint64_t)m;
  return false;
}

// Whether the batch after superstep `c` (preceded by `p`) may pull: its
// frontier (vertices for BFS, out-edges for SSSP) is within a factor 8 of
// the pull threshold, or within 64 and still growing by more than a
// quarter per superstep. A batch that may not pull is enqueued without pull
// kernels (every superstep of it pushes, with the same results).
inline bool near_pull(const Ctl& c, const Ctl& p, int kind, int64_t n, int64_t m,
                      uint32_t pull_div) {
  uint64_t x, xp;
  double thr;
  if (kind == GM_PROG_BFS) {
    x = c.packed >> 32;
    xp = p.packed >> 32;
    thr = (double)(n / (int64_t)pull_div);
  } else if (kind == GM_PROG_SSSP) {
    x = (uint32_t)c.packed;
    xp = (uint32_t)p.packed;
    thr = 64.0 * (double)m / (double)pull_div;
  } else {
    return false;
  }
  const bool growing = 4 * x > 5 * xp;
  return 8.0 * (double)x > thr || (growing && 64.0 * (double)x > thr);
}

template <int kKind>
__device__ inline uint32_t process(uint32_t msg, uint32_t w) {
  if constexpr (kKind == GM_PROG_DEGREE) {
    return 1u;  // every edge carries a one (Fig. 1: degree as an SpMV with a ones vector)
  } else if constexpr (kKind == GM_PROG_SSSP) {
    const uint32_t s = msg + w;
    return s < msg ? 0xFFFFFFFFu : s;  // saturating add
  } else {
    return msg >= kInfBfs ? kInfBfs : msg + 1;
  }
}

__device__ inline uint32_t wave_incl_scan(uint32_t x, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  return x;
}

// Block-wide exclusive scan of one value per thread; returns the exclusive
// prefix and writes the block total to *total.
__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t* sh, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(x, lane);
  if (lane == 63) sh[wave] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int i = 0; i < kWaves; ++i) {
    if (i < wave) base += sh[i];
    tot += sh[i];
  }
  __syncthreads();
  *total = tot;
  return base + incl - x;
}

__global__ __launch_bounds__(kThreads) void seed_bits(const int32_t* __restrict__ ids,
                                                      int64_t count, uint32_t* bits) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = ids[i];
    atomicOr(&bits[v >> 5], 1u << (v & 31));
  }
}

// The caller's frontier bitvector (Sec. 4.4.2) as the first frontier; bits
// at or past n are dropped.
__global__ __launch_bounds__(kThreads) void seed_bitmap(const uint32_t* __restrict__ in,
                                                        int64_t words, int64_t n, uint32_t* bits) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t left = n - 32 * i;  // vertices in this word, >= 1
    bits[i] = in[i] & (left >= 32 ? 0xFFFFFFFFu : (1u << left) - 1u);
  }
}

// Every vertex active (the first frontier of the degree program).
__global__ __launch_bounds__(kThreads) void seed_all(int64_t words, int64_t n, uint32_t* bits) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t left = n - 32 * i;
    bits[i] = left >= 32 ? 0xFFFFFFFFu : (1u << left) - 1u;
  }
}

// SEND: frontier bitvector -> queue (vertex, message, first edge, edge prefix),
// in two launches with no atomics on a shared address (which device-scope
// atomics, performed past the per-XCD caches, serialise): send_count gives
// each workgroup's contiguous range of words its totals (active vertices,
// their out-edges, smallest and largest message) and clears the other
// bitvector (the frontier before this one, into which this superstep's
// product writes the next); send_write places each workgroup's vertices
// after those of the workgroups before it, so the queue is in vertex order,
// and its first workgroup writes the superstep's control record. A thread
// takes one 32-bit word; for a nonzero word it reads the 33 offsets around
// its 32 vertices at once (independent loads, unrolled), so that a dense
// word costs one memory round trip, not one per set bit.
constexpr int kSendBlocksMax = 1024;

struct SendInfo {
  uint32_t cnt, edges, mn, mx;
};

// Words [w_begin, w_end) of workgroup b when the words are cut into
// contiguous ranges of `chunk` (a multiple of kThreads).
__device__ inline void send_range(int64_t words, int64_t chunk, int64_t* w_begin, int64_t* w_end) {
  *w_begin = (int64_t)blockIdx.x * chunk;
  *w_end = *w_begin + chunk < words ? *w_begin + chunk : words;
}

// Out-degree sum of the set bits of `word` (vertices v0..v0+31), with the
// 33 offsets around them left in o.
__device__ inline uint32_t word_edges(uint32_t word, int64_t v0, int64_t n,
                                      const uint32_t* __restrict__ off, uint32_t (&o)[33]) {
#pragma unroll
  for (int k = 0; k <= 32; ++k) o[k] = off[v0 + k < n ? v0 + k : n];
  uint32_t edges = 0;
#pragma unroll
  for (int k = 0; k < 32; ++k) edges += (word >> k) & 1u ? o[k + 1] - o[k] : 0u;
  return edges;
}

__global__ __launch_bounds__(kThreads) void send_count(
    const uint32_t* __restrict__ bits, uint32_t* __restrict__ other, int64_t words, int64_t n,
    int64_t chunk, const uint32_t* __restrict__ prop, const uint32_t* __restrict__ off,
    SendInfo* __restrict__ info) {
  __shared__ uint32_t sh[4 * kWaves];
  int64_t wb, we;
  send_range(words, chunk, &wb, &we);
  uint32_t cnt = 0, edges = 0, mn = 0xFFFFFFFFu, mx = 0;
  for (int64_t wi = wb + threadIdx.x; wi < we; wi += kThreads) {
    const uint32_t word = bits[wi];
    other[wi] = 0u;
    if (!word) continue;
    const int64_t v0 = wi * 32;
    uint32_t o[33];
    cnt += __popc(word);
    edges += word_edges(word, v0, n, off, o);
    uint32_t msg[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) msg[k] = (word >> k) & 1u ? prop[v0 + k] : 0u;
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if ((word >> k) & 1u) {
        mn = msg[k] < mn ? msg[k] : mn;
        mx = msg[k] > mx ? msg[k] : mx;
      }
  }
  for (int o = 32; o > 0; o >>= 1) {
    cnt += __shfl_xor(cnt, o, 64);
    edges += __shfl_xor(edges, o, 64);
    const uint32_t a = __shfl_xor(mn, o, 64), c = __shfl_xor(mx, o, 64);
    mn = a < mn ? a : mn;
    mx = c > mx ? c : mx;
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[wave] = cnt;
    sh[kWaves + wave] = edges;
    sh[2 * kWaves + wave] = mn;
    sh[3 * kWaves + wave] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    SendInfo t{0, 0, 0xFFFFFFFFu, 0};
    for (int i = 0; i < kWaves; ++i) {
      t.cnt += sh[i];
      t.edges += sh[kWaves + i];
      t.mn = sh[2 * kWaves + i] < t.mn ? sh[2 * kWaves + i] : t.mn;
      t.mx = sh[3 * kWaves + i] > t.mx ? sh[3 * kWaves + i] : t.mx;
    }
    info[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kThreads) void send_write(
    const uint32_t* __restrict__ bits, int64_t words, int64_t n, int64_t chunk,
    const uint32_t* __restrict__ prop, const uint32_t* __restrict__ off,
    const SendInfo* __restrict__ info, int32_t* __restrict__ q, uint32_t* __restrict__ qmsg,
    uint32_t* __restrict__ qbeg, uint32_t* __restrict__ qest, Ctl* __restrict__ ctl, int kind,
    int64_t m, bool pull_ok, uint32_t pull_div, uint32_t* __restrict__ snap,
    const uint32_t* __restrict__ vert_of) {
  __shared__ uint32_t sh[2 * kWaves];
  __shared__ uint32_t red[4][kWaves];
  // The superstep's totals (all workgroups: the control record and the
  // direction) and this workgroup's place (the workgroups before it).
  uint32_t cb = 0, eb = 0, ca = 0, ea = 0, mn = 0xFFFFFFFFu, mx = 0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += kThreads) {
    const SendInfo t = info[i];
    ca += t.cnt;
    ea += t.edges;
    mn = t.mn < mn ? t.mn : mn;
    mx = t.mx > mx ? t.mx : mx;
    if (i < (int)blockIdx.x) {
      cb += t.cnt;
      eb += t.edges;
    }
  }
  uint32_t ctot, etot;
  (void)block_excl_scan(cb, sh, &ctot);
  (void)block_excl_scan(eb, sh + kWaves, &etot);
  for (int o = 32; o > 0; o >>= 1) {
    ca += __shfl_xor(ca, o, 64);
    ea += __shfl_xor(ea, o, 64);
    const uint32_t a = __shfl_xor(mn, o, 64), c = __shfl_xor(mx, o, 64);
    mn = a < mn ? a : mn;
    mx = c > mx ? c : mx;
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = ca;
    red[1][threadIdx.x >> 6] = ea;
    red[2][threadIdx.x >> 6] = mn;
    red[3][threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  Ctl c{0, 0xFFFFFFFFu, 0};
  uint32_t call = 0, eall = 0;
  for (int i = 0; i < kWaves; ++i) {
    call += red[0][i];
    eall += red[1][i];
    c.msg_min = red[2][i] < c.msg_min ? red[2][i] : c.msg_min;
    c.msg_max = red[3][i] > c.msg_max ? red[3][i] : c.msg_max;
  }
  c.packed = ((unsigned long long)call << 32) | eall;
  if (blockIdx.x == 0 && threadIdx.x == 0) *ctl = c;
  // A pull superstep reads no queue: the frontier bits, the control record
  // and, for SSSP, the message snapshot in rank order (snap[r] = x_v of
  // v = vert_of[r] for a frontier vertex, the max value, which PROCESS keeps,
  // for any other), written here instead (this workgroup: the ranks of its
  // range of words).
  if (use_pull(c, kind, pull_ok, n, m, pull_div)) {
    if (snap) {
      int64_t wb, we;
      send_range(words, chunk, &wb, &we);
      const int64_t re = we * 32 < n ? we * 32 : n;
      for (int64_t r = wb * 32 + threadIdx.x; r < re; r += kThreads) {
        const uint32_t v = vert_of[r];
        snap[r] = (bits[v >> 5] >> (v & 31)) & 1u ? prop[v] : 0xFFFFFFFFu;
      }
    }
    return;
  }
  uint32_t slot0 = ctot, est0 = etot;
  int64_t wb, we;
  send_range(words, chunk, &wb, &we);
  for (int64_t w0 = wb; w0 < we; w0 += kThreads) {
    const int64_t wi = w0 + threadIdx.x;
    const uint32_t word = wi < we ? bits[wi] : 0u;
    if (!__syncthreads_or(word != 0u)) continue;  // no active vertex in these words
    const int64_t v0 = wi * 32;
    uint32_t o[33];
    const uint32_t edges = word ? word_edges(word, v0, n, off, o) : 0u;
    uint32_t ct, et;
    const uint32_t cex = block_excl_scan(word ? (uint32_t)__popc(word) : 0u, sh, &ct);
    const uint32_t eex = block_excl_scan(edges, sh + kWaves, &et);
    if (word) {
      uint32_t slot = slot0 + cex;
      uint32_t est = est0 + eex;
      uint32_t msg[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) msg[k] = (word >> k) & 1u ? prop[v0 + k] : 0u;
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        if ((word >> k) & 1u) {
          q[slot] = (int32_t)(v0 + k);
          qmsg[slot] = msg[k];
          qbeg[slot] = o[k];
          qest[slot] = est;
          est += o[k + 1] - o[k];
          ++slot;
        }
      }
    }
    slot0 += ct;
    est0 += et;
  }
}

// SEND of the list-frontier variant: the frontier is a sorted list of count
// distinct vertices; one thread per entry, queue slots in list order.
__global__ __launch_bounds__(kThreads) void send_list_kernel(
    const uint32_t* __restrict__ lst, int64_t count, const uint32_t* __restrict__ prop,
    const uint32_t* __restrict__ off, int32_t* __restrict__ q, uint32_t* __restrict__ qmsg,
    uint32_t* __restrict__ qbeg, uint32_t* __restrict__ qest, Ctl* __restrict__ ctl) {
  __shared__ uint32_t sh[2 * kWaves];
  __shared__ unsigned long long base_packed;
  for (int64_t i0 = (int64_t)blockIdx.x * kThreads; i0 < count;
       i0 += (int64_t)gridDim.x * kThreads) {
    const int64_t i = i0 + threadIdx.x;
    const bool live = i < count;
    const uint32_t v = live ? lst[i] : 0u;
    const uint32_t b = live ? off[v] : 0u;
    const uint32_t deg = live ? off[v + 1] - b : 0u;
    uint32_t ctot, etot;
    const uint32_t cex = block_excl_scan(live ? 1u : 0u, sh, &ctot);
    const uint32_t eex = block_excl_scan(deg, sh + kWaves, &etot);
    if (threadIdx.x == 0)
      base_packed = atomicAdd(&ctl->packed, ((unsigned long long)ctot << 32) | etot);
    __syncthreads();
    const unsigned long long bp = base_packed;
    __syncthreads();
    if (live) {
      const uint32_t slot = (uint32_t)(bp >> 32) + cex;
      q[slot] = (int32_t)v;
      qmsg[slot] = prop[v];
      qbeg[slot] = b;
      qest[slot] = (uint32_t)bp + eex;
    }
  }
}

__global__ void list_to_active(const uint32_t* __restrict__ lst, int64_t count,
                               int32_t* __restrict__ active) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    active[lst[i]] = 1;
}

__global__ void ids_to_u32(const int32_t* __restrict__ ids, int64_t count, uint32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (uint32_t)ids[i];
}

// PROCESS + REDUCE(min) + APPLY(min) of one edge. A cached read of v's value
// (the value at kernel start or a later, lower one: values only drop) filters
// out most edges; the others do an atomic min, and v is marked changed
// exactly when the value the atomic replaced was larger than cand.
__device__ inline void relax(uint32_t cand, int32_t v, uint32_t* prop, uint32_t* next) {
  if (cand < __hip_atomic_load(&prop[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT)) {
    const uint32_t old =
        __hip_atomic_fetch_min(&prop[v], cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cand < old)
      __hip_atomic_fetch_or(&next[v >> 5], 1u << (v & 31), __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
  }
}

// relax() with the next frontier as a bitvector (list == NULL) or, for the
// list-frontier variant, as an appended list of lowered vertices (a vertex
// lowered twice appears twice; the list is sorted and made unique later).
__device__ inline void relax_to(uint32_t cand, int32_t v, uint32_t* prop, uint32_t* next,
                                uint32_t* list, unsigned int* list_count) {
  if (!list) {
    relax(cand, v, prop, next);
    return;
  }
  if (cand < __hip_atomic_load(&prop[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT)) {
    const uint32_t old =
        __hip_atomic_fetch_min(&prop[v], cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cand < old) list[atomicAdd(list_count, 1u)] = (uint32_t)v;
  }
}

template <int kKind>
__global__ __launch_bounds__(kThreads) void push_kernel(
    const Ctl* __restrict__ ctlp, int64_t n, int64_t m, bool pull_ok, uint32_t pull_div,
    const uint32_t* __restrict__ qmsg, const uint32_t* __restrict__ qbeg,
    const uint32_t* __restrict__ qest, const int32_t* __restrict__ idx,
    const uint32_t* __restrict__ w, uint32_t* prop, uint32_t* next, uint32_t* list = nullptr,
    unsigned int* list_count = nullptr) {
  const Ctl c = *ctlp;
  if (use_pull(c, kKind, pull_ok, n, m, pull_div)) return;
  const uint32_t count = (uint32_t)(c.packed >> 32);
  const uint64_t E = (uint32_t)c.packed;
  if (count == 0 || E == 0) return;
  const int lane = threadIdx.x & 63;
  // at least kMinWaveEdges edges per working wavefront: a small frontier
  // keeps the others idle instead of spreading a few edges over all of them
  const uint64_t nw = std::min<uint64_t>((uint64_t)gridDim.x * kWaves,
                                         (E + kMinWaveEdges - 1) / kMinWaveEdges);
  const uint64_t wid = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (wid >= nw) return;
  const uint32_t e_begin = (uint32_t)(E * wid / nw);
  const uint32_t e_end = (uint32_t)(E * (wid + 1) / nw);
  if (e_begin >= e_end) return;
  // 64-ary search for the last slot whose edge prefix is <= e_begin (slot 0
  // has prefix 0, so lane 0's sample always qualifies).
  uint32_t lo = 0, hi = count;  // answer in [lo, hi)
  while (hi - lo > 64) {
    const uint32_t span = hi - lo;
    const uint32_t p = lo + (uint32_t)((uint64_t)span * lane / 64);
    const unsigned long long m = __ballot(qest[p] <= e_begin);
    const int last = 63 - __clzll(m);
    const uint32_t nlo = lo + (uint32_t)((uint64_t)span * last / 64);
    hi = last == 63 ? hi : lo + (uint32_t)((uint64_t)span * (last + 1) / 64);
    lo = nlo;
  }
  {
    const uint32_t p = lo + lane;
    lo += 63 - __clzll(__ballot(p < hi && qest[p] <= e_begin));
  }
  // Walk windows of 64 queue slots; lane j of a window holds slot s0 + j.
  uint32_t e = e_begin;
  for (uint32_t s0 = lo; e < e_end; s0 += 64) {
    const uint32_t s = s0 + lane;
    const bool valid = s < count;
    const uint32_t est = valid ? qest[s] : (uint32_t)E;
    const uint32_t beg = valid ? qbeg[s] : 0u;
    const uint32_t msg = valid ? qmsg[s] : 0u;
    const uint32_t win_end = s0 + 64 < count ? qest[s0 + 64] : (uint32_t)E;
    const uint32_t stop = win_end < e_end ? win_end : e_end;
    for (; e < stop; e += 64 * kUnroll) {
      uint32_t cand[kUnroll];
      uint32_t eidx[kUnroll];
      int32_t dst[kUnroll];
      bool act[kUnroll];
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        const uint32_t ee = e + k * 64 + lane;
        act[k] = ee < stop;
        int j = 0;  // owner: the last lane whose prefix is <= ee
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
          const uint32_t ex = __shfl(est, j + step, 64);
          if (ex <= ee) j += step;
        }
        const uint32_t ej = __shfl(est, j, 64);
        const uint32_t bj = __shfl(beg, j, 64);
        cand[k] = __shfl(msg, j, 64);
        eidx[k] = bj + (ee - ej);
      }
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) dst[k] = act[k] ? idx[eidx[k]] : 0;
      if constexpr (kKind == GM_PROG_SSSP) {
        uint32_t ww[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) ww[k] = act[k] ? w[eidx[k]] : 0u;
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) cand[k] = process<kKind>(cand[k], ww[k]);
      } else {
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) cand[k] = process<kKind>(cand[k], 0u);
      }
      if constexpr (kKind == GM_PROG_DEGREE) {  // REDUCE + (APPLY: the sum itself)
#pragma unroll
        for (int k = 0; k < kUnroll; ++k)
          if (act[k])
            __hip_atomic_fetch_add(&prop[dst[k]], cand[k], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
      } else {
#pragma unroll
        for (int k = 0; k < kUnroll; ++k)
          if (act[k]) relax_to(cand[k], dst[k], prop, next, list, list_count);
      }
    }
    e = stop;
  }
}

// Ablation variant of the push (GM_VARIANT_VERTEX_PUSH): one thread per
// queued vertex walks all its out-edges, so a hub's edges are one thread's
// serial work (no load balancing).
template <int kKind>
__global__ __launch_bounds__(kThreads) void push_vertex_kernel(
    const Ctl* __restrict__ ctlp, int64_t n, int64_t m, bool pull_ok, uint32_t pull_div,
    const uint32_t* __restrict__ qmsg, const uint32_t* __restrict__ qbeg,
    const uint32_t* __restrict__ qest, const int32_t* __restrict__ idx,
    const uint32_t* __restrict__ w, uint32_t* prop, uint32_t* next, uint32_t* list,
    unsigned int* list_count) {
  const Ctl c = *ctlp;
  if (use_pull(c, kKind, pull_ok, n, m, pull_div)) return;
  const uint32_t count = (uint32_t)(c.packed >> 32);
  const uint32_t E = (uint32_t)c.packed;
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < count;
       s += gridDim.x * blockDim.x) {
    const uint32_t beg = qbeg[s];
    const uint32_t deg = (s + 1 < count ? qest[s + 1] : E) - qest[s];
    const uint32_t msg = qmsg[s];
    for (uint32_t e = beg; e < beg + deg; ++e) {
      const uint32_t cand = process<kKind>(msg, kKind == GM_PROG_SSSP ? w[e] : 0u);
      relax_to(cand, idx[e], prop, next, list, list_count);
    }
  }
}

// BFS pull superstep over all vertices (frontier levels uniform).
__global__ __launch_bounds__(kThreads) void pull_kernel(
    const Ctl* __restrict__ ctlp, int64_t n, int64_t m, bool pull_ok, uint32_t pull_div,
    const uint32_t* __restrict__ off, const int32_t* __restrict__ idx,
    const uint32_t* __restrict__ cur, uint32_t* prop, uint32_t* next) {
  const Ctl c = *ctlp;
  if (!use_pull(c, GM_PROG_BFS, pull_ok, n, m, pull_div)) return;
  const uint32_t cand = c.msg_min >= kInfBfs ? kInfBfs : c.msg_min + 1;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    bool hit = false;
    if (v < n && cand < prop[v]) {
      const uint32_t e1 = off[v + 1];
      for (uint32_t e = off[v]; e < e1; ++e) {
        const int32_t u = idx[e];
        if (cur[u >> 5] & (1u << (u & 31))) {
          hit = true;
          break;
        }
      }
      if (hit) prop[v] = cand;
    }
    // 64 consecutive vertices = two whole words owned by this wavefront
    const unsigned long long m = __ballot(hit);
    const int64_t word0 = (base + (threadIdx.x & ~63)) >> 5;
    if (lane == 0 && (uint32_t)m) atomicOr(&next[word0], (uint32_t)m);
    if (lane == 32 && (uint32_t)(m >> 32)) atomicOr(&next[word0 + 1], (uint32_t)(m >> 32));
  }
}

// Segmented-min state of a run of in-edges: c = row starts in it, s = min of
// the candidates after the last of them (of all, if c = 0). Joining an
// earlier run with a later one is associative.
struct MinSeg {
  int c;
  uint32_t s;
};

__device__ inline MinSeg mseg_join(MinSeg a, MinSeg b) {
  return {a.c + b.c, b.c > 0 ? b.s : min(a.s, b.s)};
}

template <int kCtrl>
__device__ inline MinSeg mseg_dpp(MinSeg old, MinSeg v) {
  return {__builtin_amdgcn_update_dpp(old.c, v.c, kCtrl, 0xF, 0xF, false),
          (uint32_t)__builtin_amdgcn_update_dpp((int)old.s, (int)v.s, kCtrl, 0xF, 0xF, false)};
}

__device__ inline MinSeg mseg_lane(MinSeg v, int lane) {
  return {__builtin_amdgcn_readlane(v.c, lane),
          (uint32_t)__builtin_amdgcn_readlane((int)v.s, lane)};
}

// Wavefront scan of one round: each lane's exclusive prefix (earlier lanes
// and the carry of the earlier rounds); carry moves on to the round's end.
__device__ inline MinSeg mseg_scan(MinSeg own, MinSeg& carry, int lane) {
  constexpr MinSeg id{0, 0xFFFFFFFFu};
  MinSeg x = own;  // inclusive within rows of 16 lanes (row_shr 1, 2, 4, 8)
  x = mseg_join(mseg_dpp<0x111>(id, x), x);
  x = mseg_join(mseg_dpp<0x112>(id, x), x);
  x = mseg_join(mseg_dpp<0x114>(id, x), x);
  x = mseg_join(mseg_dpp<0x118>(id, x), x);
  const MinSeg p1 = mseg_join(carry, mseg_lane(x, 15));
  const MinSeg p2 = mseg_join(p1, mseg_lane(x, 31));
  const MinSeg p3 = mseg_join(p2, mseg_lane(x, 47));
  const int row = lane >> 4;
  const MinSeg before = row == 0 ? carry : row == 1 ? p1 : row == 2 ? p2 : p3;
  const MinSeg incl = mseg_join(before, x);
  carry = mseg_lane(incl, 63);
  return mseg_dpp<0x111>(before, incl);  // the row's first lane takes `before`
}

// APPLY of a row's minimum y: lower prop(v) and put v in the next frontier.
// kOwned: no other wavefront touches v in this superstep (plain store).
template <bool kOwned>
__device__ inline void apply_min(uint32_t v, uint32_t y, uint32_t* prop, uint32_t* next) {
  if (y >= prop[v]) return;
  if constexpr (kOwned) {
    prop[v] = y;
  } else {
    if (y >= __hip_atomic_fetch_min(&prop[v], y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
  atomicOr(&next[v >> 5], 1u << (v & 31));
}

// SSSP pull superstep: every vertex v takes the min of PROCESS(snap[u], w)
// over its in-edges (u, v, w) and APPLYs it: the state the push superstep
// leaves, since the messages are the same snapshot and min is exact and
// order-free. The in-adjacency is cut into tiles of kPullTile edges
// whatever the rows (a bitmap marks each row's first edge; rows without
// in-edges are skipped by a list of the rows that have some); a wavefront
// takes a tile in four rounds of 256 edges, four consecutive ones per lane
// (16-byte index and weight loads, all sixteen gathers in flight at once).
// Sources are numbered by rank (decreasing out-degree), the snapshot held in
// that order: each workgroup (one per compute unit) first copies the
// messages of the first hot_n ranks, which most in-edges name, to LDS; an
// edge from such a source reads its message there (its global gather is
// redirected to snap[0], one line for all such lanes), and the next most
// gathered messages share cache lines.
// Each lane takes the min of its edges per row, a segmented scan over the
// wavefront joins the lanes, and the lane holding a row's last edge applies
// it: with a plain store if the row began in the tile (no other wavefront
// touches it), with an atomic min if it began in an earlier tile; the part
// of a row that goes on past the tile is applied with an atomic min too.
constexpr int64_t kPullTile = 1024;
constexpr int kPullThreads = 1024;
constexpr int kPullWaves = kPullThreads / 64;
constexpr int kPullHotMax = 40960;  // hot messages in LDS (160 KB)
__global__ __launch_bounds__(kPullThreads) void pull_min_tiles(
    const Ctl* __restrict__ ctlp, int64_t n, int64_t m, bool pull_ok, uint32_t pull_div,
    const int32_t* __restrict__ idx, const uint32_t* __restrict__ w,
    const uint32_t* __restrict__ starts, const uint32_t* __restrict__ rows,
    const uint32_t* __restrict__ tile_row, int64_t ntiles, int64_t nrows,
    const uint32_t* __restrict__ snap, int hot_n,
    uint32_t* prop, uint32_t* next) {
  extern __shared__ uint32_t hot[];  // hot_n messages
  if (!use_pull(*ctlp, GM_PROG_SSSP, pull_ok, n, m, pull_div)) return;
  typedef int v4i __attribute__((ext_vector_type(4)));
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  {
    const int n4 = hot_n >> 2;
    for (int i = threadIdx.x; i < n4; i += kPullThreads)
      reinterpret_cast<v4u*>(hot)[i] = reinterpret_cast<const v4u*>(snap)[i];
    for (int i = 4 * n4 + threadIdx.x; i < hot_n; i += kPullThreads) hot[i] = snap[i];
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * kPullWaves;
  const int sh = (lane & 7) * 4;  // this lane's 4 bits in its word of `starts`
  for (int64_t t = __builtin_amdgcn_readfirstlane(blockIdx.x * kPullWaves + (threadIdx.x >> 6));
       t < ntiles; t += stride) {
    const int64_t e0 = t * kPullTile;
    const bool whole = e0 + kPullTile <= m;  // the last tile may be partial
    v4i src[4];
    v4u wt[4];
    uint32_t fa[4], fb[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t ev = e0 + v * 256 + lane * 4;
      src[v] = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(idx + ev));  // padded
      if (whole) {
        wt[v] = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(w + ev));
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) wt[v][q] = ev + q < m ? w[ev + q] : 0u;
      }
      fa[v] = starts[ev >> 5];
      fb[v] = starts[(ev >> 5) + 1];
    }
    uint32_t cand[4][4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t sv = (uint32_t)src[v][q];
        const bool in_lds = sv < (uint32_t)hot_n;
        const uint32_t g = snap[in_lds ? 0u : sv];
        const uint32_t l = hot[in_lds ? sv : 0u];
        cand[v][q] = in_lds ? l : g;
      }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool real = whole || e0 + v * 256 + lane * 4 + q < m;
        cand[v][q] = real ? process<GM_PROG_SSSP>(cand[v][q], wt[v][q]) : 0xFFFFFFFFu;
      }
    const uint32_t r0 = tile_row[t];  // index in `rows` of the row holding edge e0
    // A start at the tile's first edge opens row r0 itself, not the next.
    const int f0 = __builtin_amdgcn_readfirstlane((int)((fa[0] >> sh) & 1u));
    MinSeg carry{0, 0xFFFFFFFFu};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t nib = (fa[v] >> sh) & 0xFu;  // bit q: edge q of the lane starts a row
      const uint32_t nx = sh == 28 ? (fb[v] & 1u) : (fa[v] >> (sh + 4)) & 1u;
      const uint32_t ends = (nib >> 1) | (nx << 3);  // bit q: edge q ends its row
      uint32_t sm[4];
      sm[0] = cand[v][0];
#pragma unroll
      for (int q = 1; q < 4; ++q) sm[q] = (nib >> q) & 1u ? cand[v][q] : min(sm[q - 1], cand[v][q]);
      const MinSeg ex = mseg_scan(MinSeg{(int)__popc(nib), sm[3]}, carry, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!((ends >> q) & 1u)) continue;
        const int lc = (int)__popc(nib & ((2u << q) - 1u));  // starts at or before edge q
        const int c = ex.c + lc;                              // ... since the tile's first edge
        const uint32_t y = lc > 0 ? sm[q] : min(ex.s, sm[q]);
        if (y == 0xFFFFFFFFu) continue;
        if (c > 0) {
          const int64_t ri = (int64_t)r0 + c - f0;
          if (ri < nrows) apply_min<true>(rows[ri], y, prop, next);
        } else {
          apply_min<false>(rows[r0], y, prop, next);  // begun in an earlier tile
        }
      }
      if (v == 3 && lane == 63 && !(ends >> 3)) {  // goes on past the tile
        const int c = ex.c + (int)__popc(nib);
        const uint32_t y = nib ? sm[3] : min(ex.s, sm[3]);
        const int64_t ri = (int64_t)r0 + c - f0;
        if (y != 0xFFFFFFFFu && ri < nrows) apply_min<false>(rows[ri], y, prop, next);
      }
    }
  }
}

// Index array of the pull in ranks: tidx[e] = rank_of[idx[e]]; 0 past m (to
// the end of the last tile).
__global__ void pull_tag(const int32_t* __restrict__ idx, int64_t m, int64_t mpad,
                         const uint32_t* __restrict__ rank_of, int32_t* __restrict__ tidx) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < mpad;
       e += (int64_t)gridDim.x * blockDim.x)
    tidx[e] = e < m ? (int32_t)rank_of[idx[e]] : 0;
}

// Sort key of a vertex for its rank: most out-edges first, ties by id.
__global__ void pull_hot_keys(const uint32_t* __restrict__ push_off, int64_t n,
                              unsigned long long* __restrict__ key) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t d = push_off[v + 1] - push_off[v];
    key[v] = ((unsigned long long)(0xFFFFFFFFu - d) << 32) | (uint32_t)v;
  }
}

__global__ void pull_ranks(const unsigned long long* __restrict__ key, int64_t n,
                           uint32_t* __restrict__ vert_of, uint32_t* __restrict__ rank_of) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t v = (uint32_t)key[i];
    vert_of[i] = v;
    rank_of[v] = (uint32_t)i;
  }
}

// Layout of a pull over the adjacency off/idx/w (n rows, m edges): the
// row-start bitmap (bit off[v] of every row with edges, and bit m), the
// rows with edges in order, and for each tile the index in that list of the
// row holding its first edge.
__global__ void pull_rows(const uint32_t* __restrict__ off, int64_t n,
                          const uint32_t* __restrict__ cidx, uint32_t* __restrict__ rows,
                          uint32_t* __restrict__ starts) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t b = off[v];
    if (off[v + 1] > b) {
      rows[cidx[v]] = (uint32_t)v;
      atomicOr(&starts[b >> 5], 1u << (b & 31));
    }
  }
}

__global__ void pull_flags(const uint32_t* __restrict__ off, int64_t n, uint32_t* __restrict__ f,
                           uint32_t* __restrict__ starts, int64_t m) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n;
       v += (int64_t)gridDim.x * blockDim.x)
    f[v] = v < n && off[v + 1] > off[v] ? 1u : 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&starts[m >> 5], 1u << (m & 31));
}

__global__ void pull_tile_rows(const uint32_t* __restrict__ off, int64_t n,
                               const uint32_t* __restrict__ cidx, int64_t ntiles,
                               uint32_t* __restrict__ tile_row) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntiles;
       t += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t e = (uint32_t)(t * kPullTile);
    int64_t lo = 0, hi = n;  // the last v with off[v] <= e: the row holding edge e
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (off[mid] <= e)
        lo = mid;
      else
        hi = mid;
    }
    tile_row[t] = cidx[lo];
  }
}

__global__ void reset_ctl(Ctl* ctl) {
  ctl->packed = 0;
  ctl->msg_min = 0xFFFFFFFFu;
  ctl->msg_max = 0;
}

__global__ void fill_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// active_out[v] = bit v of the frontier; then clear the frontier.
__global__ void bits_epilogue(uint32_t* bits, int64_t words, int64_t n, int32_t* active_out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t word = bits[i];
    if (active_out)
      for (int k = 0; k < 32 && i * 32 + k < n; ++k) active_out[i * 32 + k] = (word >> k) & 1u;
    if (word) bits[i] = 0;
  }
}

__global__ void id_range(const int32_t* __restrict__ ids, int64_t count, int64_t n,
                         unsigned int* __restrict__ bad) {
  unsigned int b = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    b |= (ids[i] < 0 || (int64_t)ids[i] >= n) ? 1u : 0u;
  for (int o = 32; o > 0; o >>= 1) b |= __shfl_xor(b, o, 64);
  if (b && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

inline unsigned blocks_for(int64_t n, int64_t cap = 8192) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

__global__ void all_offsets(const uint32_t* __restrict__ out_off, const uint32_t* __restrict__ in_off,
                            int64_t n, uint32_t* __restrict__ all_off) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n;
       v += (int64_t)gridDim.x * blockDim.x)
    all_off[v] = out_off[v] + in_off[v];
}

// One wavefront per vertex: its out-list, then its in-list.
__global__ void all_lists(const uint32_t* __restrict__ out_off, const int32_t* __restrict__ out_idx,
                          const uint32_t* __restrict__ out_w, const uint32_t* __restrict__ in_off,
                          const int32_t* __restrict__ in_idx, const uint32_t* __restrict__ in_w,
                          int64_t n, const uint32_t* __restrict__ all_off,
                          int32_t* __restrict__ all_idx, uint32_t* __restrict__ all_w) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t v = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; v < n; v += waves) {
    const uint32_t ob = out_off[v], oe = out_off[v + 1], ib = in_off[v], ie = in_off[v + 1];
    const uint32_t base = all_off[v], mid = base + (oe - ob);
    for (uint32_t j = lane; j < oe - ob; j += 64) {
      all_idx[base + j] = out_idx[ob + j];
      if (all_w) all_w[base + j] = out_w[ob + j];
    }
    for (uint32_t j = lane; j < ie - ib; j += 64) {
      all_idx[mid + j] = in_idx[ib + j];
      if (all_w) all_w[mid + j] = in_w[ib + j];
    }
  }
}

// Sort keys of the relabelling: mask - degree (a stable ascending sort puts
// higher degrees first, ties in label order), the vertex as value.
__global__ void degree_keys(const uint32_t* __restrict__ off, int64_t n, uint32_t mask,
                            uint32_t* __restrict__ key, int32_t* __restrict__ val) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    key[v] = mask - (off[v + 1] - off[v]);
    val[v] = (int32_t)v;
  }
}

__global__ void invert_perm(const int32_t* __restrict__ old_of, int64_t n,
                            int32_t* __restrict__ new_of) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    new_of[old_of[i]] = (int32_t)i;
}

// len[i] = degree of the vertex with new label i; len[n] = 0 (an exclusive
// scan of n + 1 lengths gives the offsets, the last one the edge count).
__global__ void relabel_lengths(const uint32_t* __restrict__ off, const int32_t* __restrict__ old_of,
                                int64_t n, uint32_t* __restrict__ len) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i == n) {
      len[i] = 0;
    } else {
      const int32_t v = old_of[i];
      len[i] = off[v + 1] - off[v];
    }
  }
}

// Row i of the relabelled adjacency, one wavefront per row: the row of
// old_of[i], its targets mapped to new labels, values alike, in the row's
// own order.
__global__ void relabel_rows(const uint32_t* __restrict__ off, const int32_t* __restrict__ idx,
                             const uint32_t* __restrict__ w, const int32_t* __restrict__ old_of,
                             const int32_t* __restrict__ new_of, int64_t n,
                             const uint32_t* __restrict__ noff, int32_t* __restrict__ nidx,
                             uint32_t* __restrict__ nw) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; i < n; i += waves) {
    const int32_t v = old_of[i];
    const uint32_t b = off[v], e = off[v + 1], nb = noff[i];
    for (uint32_t j = lane; j < e - b; j += 64) {
      nidx[nb + j] = new_of[idx[b + j]];
      if (nw) nw[nb + j] = w[b + j];
    }
  }
}

// out[i] = src[index[i]]: values between the caller's labels and the new ones.
__global__ void permute_u32(const uint32_t* __restrict__ src, const int32_t* __restrict__ index,
                            int64_t n, uint32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = src[index[i]];
}

// The caller's frontier bitvector (vertices below n) as bits of the new
// labels, into a cleared bitvector.
__global__ __launch_bounds__(kThreads) void seed_bitmap_mapped(const uint32_t* __restrict__ in,
                                                               int64_t n,
                                                               const int32_t* __restrict__ new_of,
                                                               uint32_t* bits) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    if ((in[v >> 5] >> (v & 31)) & 1u) {
      const int32_t u = new_of[v];
      atomicOr(&bits[u >> 5], 1u << (u & 31));
    }
}

// The caller's frontier ids in new labels (list variant).
__global__ void map_ids(const int32_t* __restrict__ ids, int64_t count,
                        const int32_t* __restrict__ new_of, int32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = new_of[ids[i]];
}

Workspace* ensure_ws(gm_graph g, hipStream_t s) {
  Workspace* ws = static_cast<Workspace*>(g->min_ws);
  if (ws) return ws;
  ws = new Workspace();
  g->min_ws = ws;
  try {
    const int64_t n = g->n;
    const int64_t words = (n + 31) / 32;
    ws->n = n;
    ws->q = dalloc<int32_t>(n);
    ws->qmsg = dalloc<uint32_t>(n);
    ws->qbeg = dalloc<uint32_t>(n);
    ws->qest = dalloc<uint32_t>(n);
    ws->bits[0] = dalloc<uint32_t>(words);
    ws->bits[1] = dalloc<uint32_t>(words);
    ws->ctl = dalloc<Ctl>(kMaxCtl + 1);
    ws->sinfo = dalloc<SendInfo>(kSendBlocksMax);
    void* h = nullptr;
    GM_HIP(hipHostMalloc(&h, kMaxCtl * sizeof(Ctl), hipHostMallocDefault));
    ws->host_ctl = static_cast<Ctl*>(h);
    fill_kernel<<<blocks_for(words), kThreads, 0, s>>>(ws->bits[0], words, 0);
    fill_kernel<<<blocks_for(words), kThreads, 0, s>>>(ws->bits[1], words, 0);
    GM_HIP(hipGetLastError());
  } catch (...) {
    free_min_workspace(g);  // a failed build leaves no workspace behind
    throw;
  }
  return ws;
}

// The adjacency messages travel along for `order` (the in-layout is needed
// for GM_ORDER_IN and GM_ORDER_ALL).
Adj adjacency(gm_graph g, Workspace* ws, int order, hipStream_t s) {
  if (order == GM_ORDER_IN)
    return Adj{g->in_off, g->in_idx, static_cast<const uint32_t*>(g->in_w)};
  if (order != GM_ORDER_ALL)
    return Adj{g->out_off, g->out_idx, static_cast<const uint32_t*>(g->out_w)};
  if (!ws->all_off) {
    const int64_t n = g->n, m = g->m;
    if (2 * m > (int64_t)UINT32_MAX) throw Unsupported{"GM_ORDER_ALL: more than 2^32 - 1 edges"};
    const bool weighted = g->wtype == GM_W_U32;
    uint32_t* off = nullptr;
    int32_t* idx = nullptr;
    uint32_t* w = nullptr;
    try {
      off = dalloc<uint32_t>(n + 1);
      idx = dalloc<int32_t>(2 * m + kIdxPad);
      if (weighted) w = dalloc<uint32_t>(2 * m);
      all_offsets<<<blocks_for(n + 1), kThreads, 0, s>>>(g->out_off, g->in_off, n, off);
      all_lists<<<blocks_for(64 * n), kThreads, 0, s>>>(
          g->out_off, g->out_idx, static_cast<const uint32_t*>(g->out_w), g->in_off, g->in_idx,
          static_cast<const uint32_t*>(g->in_w), n, off, idx, w);
      GM_HIP(hipGetLastError());
      GM_HIP(hipStreamSynchronize(s));
    } catch (...) {
      dfree(off);
      dfree(idx);
      dfree(w);
      throw;
    }
    ws->all_idx = idx;
    ws->all_w = w;
    ws->all_off = off;
  }
  return Adj{ws->all_off, ws->all_idx, ws->all_w};
}

void free_relab(Relab* rl) {
  if (!rl) return;
  dfree(rl->new_of);
  dfree(rl->old_of);
  dfree(rl->prop);
  dfree(rl->ids);
  dfree(rl->active);
  rl->out.release();
  rl->in.release();
  rl->all.release();
  delete rl;
}

// The permutation and per-run buffers of the relabelling (built once per
// graph; a failed build leaves none behind).
Relab* ensure_relab(gm_graph g, Workspace* ws, hipStream_t s) {
  if (ws->rl) return ws->rl;
  const int64_t n = g->n;
  const bool has_in = g->in_off != nullptr;
  const uint32_t* doff = has_in ? g->in_off : g->out_off;
  const int64_t maxd = has_in ? g->max_in : g->max_out;
  int bits = 1;  // 2^bits > every degree
  while (bits < 32 && ((int64_t)1 << bits) <= maxd) ++bits;
  const uint32_t mask = bits >= 32 ? 0xFFFFFFFFu : (1u << bits) - 1u;
  Relab* rl = new Relab();
  uint32_t* k1 = nullptr;
  uint32_t* k2 = nullptr;
  int32_t* v1 = nullptr;
  void* tmp = nullptr;
  auto drop_temps = [&]() {
    dfree(tmp);
    dfree(k1);
    dfree(k2);
    dfree(v1);
  };
  try {
    rl->new_of = dalloc<int32_t>(n);
    rl->old_of = dalloc<int32_t>(n);
    rl->prop = dalloc<uint32_t>(n);
    rl->ids = dalloc<int32_t>(n);
    rl->active = dalloc<int32_t>(n);
    k1 = dalloc<uint32_t>(n);
    k2 = dalloc<uint32_t>(n);
    v1 = dalloc<int32_t>(n);
    degree_keys<<<blocks_for(n), kThreads, 0, s>>>(doff, n, mask, k1, v1);
    GM_HIP(hipGetLastError());
    size_t bytes = 0;
    GM_HIP(rocprim::radix_sort_pairs(nullptr, bytes, k1, k2, v1, rl->old_of, (size_t)n, 0, bits, s));
    tmp = dmalloc(bytes);
    GM_HIP(rocprim::radix_sort_pairs(tmp, bytes, k1, k2, v1, rl->old_of, (size_t)n, 0, bits, s));
    invert_perm<<<blocks_for(n), kThreads, 0, s>>>(rl->old_of, n, rl->new_of);
    GM_HIP(hipGetLastError());
    GM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    drop_temps();
    free_relab(rl);
    throw;
  }
  drop_temps();
  ws->rl = rl;
  return rl;
}

// One adjacency (off, idx, w) rebuilt in the labels of rl.
OwnedAdj relabel_adj(gm_graph g, const Relab* rl, const uint32_t* off, const int32_t* idx,
                     const uint32_t* w, hipStream_t s) {
  const int64_t n = g->n, m = g->m;
  OwnedAdj a;
  uint32_t* len = nullptr;
  void* tmp = nullptr;
  try {
    a.off = dalloc<uint32_t>(n + 1);
    a.idx = dalloc<int32_t>(m + kIdxPad);
    if (w) a.w = dalloc<uint32_t>(m);
    len = dalloc<uint32_t>(n + 1);
    relabel_lengths<<<blocks_for(n + 1), kThreads, 0, s>>>(off, rl->old_of, n, len);
    GM_HIP(hipGetLastError());
    size_t bytes = 0;
    GM_HIP(rocprim::exclusive_scan(nullptr, bytes, len, a.off, 0u, (size_t)(n + 1),
                                   rocprim::plus<uint32_t>(), s));
    tmp = dmalloc(bytes);
    GM_HIP(rocprim::exclusive_scan(tmp, bytes, len, a.off, 0u, (size_t)(n + 1),
                                   rocprim::plus<uint32_t>(), s));
    relabel_rows<<<blocks_for(64 * n), kThreads, 0, s>>>(off, idx, w, rl->old_of, rl->new_of, n,
                                                         a.off, a.idx, a.w);
    fill_kernel<<<1, kThreads, 0, s>>>(reinterpret_cast<uint32_t*>(a.idx) + m, kIdxPad, 0u);
    GM_HIP(hipGetLastError());
    GM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    dfree(tmp);
    dfree(len);
    a.release();
    throw;
  }
  dfree(tmp);
  dfree(len);
  return a;
}

// The relabelled adjacency for `order` (GM_ORDER_ALL: each vertex's
// relabelled out-list followed by its relabelled in-list).
Adj relab_adjacency(gm_graph g, Relab* rl, int order, hipStream_t s) {
  const bool weighted = g->wtype == GM_W_U32;
  const uint32_t* out_w = weighted ? static_cast<const uint32_t*>(g->out_w) : nullptr;
  const uint32_t* in_w = weighted ? static_cast<const uint32_t*>(g->in_w) : nullptr;
  if ((order == GM_ORDER_IN || order == GM_ORDER_ALL) && !rl->in.off)
    rl->in = relabel_adj(g, rl, g->in_off, g->in_idx, in_w, s);
  if (order != GM_ORDER_IN && !rl->out.off)
    rl->out = relabel_adj(g, rl, g->out_off, g->out_idx, out_w, s);
  if (order == GM_ORDER_IN) return rl->in.view();
  if (order != GM_ORDER_ALL) return rl->out.view();
  if (!rl->all.off) {
    const int64_t n = g->n, m = g->m;
    if (2 * m > (int64_t)UINT32_MAX) throw Unsupported{"GM_ORDER_ALL: more than 2^32 - 1 edges"};
    OwnedAdj a;
    try {
      a.off = dalloc<uint32_t>(n + 1);
      a.idx = dalloc<int32_t>(2 * m + kIdxPad);
      if (weighted) a.w = dalloc<uint32_t>(2 * m);
      all_offsets<<<blocks_for(n + 1), kThreads, 0, s>>>(rl->out.off, rl->in.off, n, a.off);
      all_lists<<<blocks_for(64 * n), kThreads, 0, s>>>(rl->out.off, rl->out.idx, rl->out.w,
                                                        rl->in.off, rl->in.idx, rl->in.w, n,
                                                        a.off, a.idx, a.w);
      fill_kernel<<<1, kThreads, 0, s>>>(reinterpret_cast<uint32_t*>(a.idx) + 2 * m, kIdxPad, 0u);
      GM_HIP(hipGetLastError());
      GM_HIP(hipStreamSynchronize(s));
    } catch (...) {
      (void)hipStreamSynchronize(s);
      a.release();
      throw;
    }
    rl->all = a;
  }
  return rl->all.view();
}

// The SSSP pull's tile layout of the adjacency `pl` (g->m edges; push_off:
// the offsets of the pushed adjacency in the same labels, whose degrees
// pick the hot set), kept in the workspace; another adjacency replaces it.
void ensure_pull_tiles(gm_graph g, Workspace* ws, const Adj& pl, const uint32_t* push_off,
                       hipStream_t s) {
  const uint32_t* off = pl.off;
  if (ws->pt && ws->pt->for_off == off) return;
  delete ws->pt;
  ws->pt = nullptr;
  ++g->ws_gen;
  const int64_t n = g->n, m = g->m;
  PullTiles* pt = new PullTiles();
  void* tmp = nullptr;
  try {
    pt->ntiles = (m + kPullTile - 1) / kPullTile;
    const int64_t words = pt->ntiles * (kPullTile / 32) + 1;
    pt->starts = dalloc<uint32_t>(words);
    fill_kernel<<<blocks_for(words), kThreads, 0, s>>>(pt->starts, words, 0u);
    DevBuf<uint32_t> f(n + 1), cidx(n + 1);
    pull_flags<<<blocks_for(n + 1), kThreads, 0, s>>>(off, n, f.p, pt->starts, m);
    GM_HIP(hipGetLastError());
    size_t bytes = 0;
    GM_HIP(rocprim::exclusive_scan(nullptr, bytes, f.p, cidx.p, 0u, (size_t)(n + 1),
                                   rocprim::plus<uint32_t>(), s));
    tmp = dmalloc(bytes);
    GM_HIP(rocprim::exclusive_scan(tmp, bytes, f.p, cidx.p, 0u, (size_t)(n + 1),
                                   rocprim::plus<uint32_t>(), s));
    uint32_t nrows = 0;
    GM_HIP(hipMemcpyAsync(&nrows, cidx.p + n, 4, hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    dfree(tmp);
    tmp = nullptr;
    pt->nrows = nrows;
    pt->rows = dalloc<uint32_t>(std::max<int64_t>(nrows, 1));
    pt->tile_row = dalloc<uint32_t>(std::max<int64_t>(pt->ntiles, 1));
    pull_rows<<<blocks_for(n), kThreads, 0, s>>>(off, n, cidx.p, pt->rows, pt->starts);
    if (pt->ntiles > 0)
      pull_tile_rows<<<blocks_for(pt->ntiles), kThreads, 0, s>>>(off, n, cidx.p, pt->ntiles,
                                                                 pt->tile_row);
    GM_HIP(hipGetLastError());
    // hot set: the sources with the most out-edges, as many as LDS holds
    int dev = 0, lds_max = 0;
    GM_HIP(hipGetDevice(&dev));
    GM_HIP(hipDeviceGetAttribute(&pt->cus, hipDeviceAttributeMultiprocessorCount, dev));
    GM_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    pt->hot_n = (int)std::min<int64_t>({(int64_t)kPullHotMax, n, (int64_t)lds_max / 4});
    pt->vert_of = dalloc<uint32_t>(n);
    DevBuf<uint32_t> rank_of(n);
    {
      DevBuf<unsigned long long> k1(n), k2(n);
      pull_hot_keys<<<blocks_for(n), kThreads, 0, s>>>(push_off, n, k1.p);
      GM_HIP(hipGetLastError());
      rocprim::double_buffer<unsigned long long> kb(k1.p, k2.p);
      size_t sb = 0;
      GM_HIP(rocprim::radix_sort_keys(nullptr, sb, kb, (size_t)n, 0, 64, s));
      tmp = dmalloc(sb);
      GM_HIP(rocprim::radix_sort_keys(tmp, sb, kb, (size_t)n, 0, 64, s));
      pull_ranks<<<blocks_for(n), kThreads, 0, s>>>(kb.current(), n, pt->vert_of, rank_of.p);
      GM_HIP(hipGetLastError());
      GM_HIP(hipStreamSynchronize(s));
      dfree(tmp);
      tmp = nullptr;
    }
    {
      const int64_t mpad = pt->ntiles * kPullTile;
      pt->tidx = dalloc<int32_t>(std::max<int64_t>(mpad, 1));
      pull_tag<<<blocks_for(mpad), kThreads, 0, s>>>(pl.idx, m, mpad, rank_of.p, pt->tidx);
      GM_HIP(hipGetLastError());
      GM_HIP(hipStreamSynchronize(s));
    }
  } catch (...) {
    (void)hipStreamSynchronize(s);
    dfree(tmp);
    delete pt;
    throw;
  }
  pt->for_off = off;
  ws->pt = pt;
}

// The view of a plain run: the caller's labels, or the relabelled copy
// (then rl is set). BFS pulls only when pushing along out-edges, over the
// in-adjacency (the out-adjacency of a symmetrised graph).
View run_view(gm_graph g, Workspace* ws, int kind, int order, Relab* rl, hipStream_t s) {
  const bool sym = (g->prep & (GM_PREP_SYMMETRIZE | GM_PREP_UPPER_DAG)) == GM_PREP_SYMMETRIZE;
  const bool pull = (kind == GM_PROG_BFS || (kind == GM_PROG_SSSP && g->wtype == GM_W_U32 &&
                                              g->m > 0)) &&
                    order == GM_ORDER_OUT && (sym || g->in_off) && g->n > 0;
  View v{Adj{nullptr, nullptr, nullptr}, Adj{nullptr, nullptr, nullptr}, pull};
  if (!rl) {
    v.push = adjacency(g, ws, order, s);
    if (pull)
      v.pull = sym ? v.push
                   : Adj{g->in_off, g->in_idx, static_cast<const uint32_t*>(g->in_w)};
  } else {
    v.push = relab_adjacency(g, rl, order, s);
    if (pull) v.pull = sym ? v.push : relab_adjacency(g, rl, GM_ORDER_IN, s);
  }
  if (pull && kind == GM_PROG_SSSP) {
    if (!ws->snap) ws->snap = dalloc<uint32_t>(g->n);
    ensure_pull_tiles(g, ws, v.pull, v.push.off, s);
  }
  return v;
}

}  // namespace

void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return;
  fill_kernel<<<blocks_for(n), kThreads, 0, s>>>(p, n, v);
  GM_HIP(hipGetLastError());
}

void free_min_workspace(gm_graph g) {
  Workspace* ws = static_cast<Workspace*>(g->min_ws);
  if (!ws) return;
  dfree(ws->q);
  dfree(ws->qmsg);
  dfree(ws->qbeg);
  dfree(ws->qest);
  dfree(ws->bits[0]);
  dfree(ws->bits[1]);
  dfree(ws->ctl);
  dfree(ws->sinfo);
  dfree(ws->all_off);
  dfree(ws->all_idx);
  dfree(ws->all_w);
  free_relab(ws->rl);
  dfree(ws->snap);
  delete ws->pt;
  if (ws->host_ctl) (void)hipHostFree(ws->host_ctl);
  delete ws;
  g->min_ws = nullptr;
  ++g->ws_gen;
}

bool ids_in_range(const int32_t* ids, int64_t count, int64_t n, hipStream_t s) {
  if (count <= 0) return true;
  unsigned int* bad = dalloc<unsigned int>(1);
  unsigned int h = 0;
  try {
    fill_u32(bad, 1, 0u, s);
    id_range<<<blocks_for(count), kThreads, 0, s>>>(ids, count, n, bad);
    GM_HIP(hipGetLastError());
    GM_HIP(hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    dfree(bad);
    throw;
  }
  dfree(bad);
  return h == 0;
}

namespace {

// One superstep on control record c (reset beforehand): SEND from bits[cur]
// (which also clears bits[cur ^ 1] and resets the record c + 1 of the next
// superstep), then the push or the pull product into bits[cur ^ 1]. After
// the last superstep of a run, bits[cur] of that superstep holds a stale
// frontier, which the run's epilogue clears.
void enqueue_superstep(gm_graph g, Workspace* ws, int kind, const View& view, Ctl* c, int cur,
                       uint32_t* prop, hipStream_t s) {
  const int64_t n = g->n;
  const int64_t words = (n + 31) / 32;
  const int64_t m = g->m;
  const Adj& a = view.push;
  const Adj& pl = view.pull;
  const bool pull_ok = view.pull_ok;
  const uint32_t pull_div = g->tune.pull_div;
  const unsigned push_blocks = g->tune.push_blocks;
  // SEND: contiguous ranges of words, at most kSendBlocksMax workgroups
  int64_t nbk = std::min<int64_t>(std::max<int64_t>((words + kThreads - 1) / kThreads, 1),
                                  kSendBlocksMax);
  const int64_t chunk =
      std::max<int64_t>(((words + nbk - 1) / nbk + kThreads - 1) / kThreads * kThreads, kThreads);
  nbk = std::max<int64_t>((words + chunk - 1) / chunk, 1);
  send_count<<<(unsigned)nbk, kThreads, 0, s>>>(ws->bits[cur], ws->bits[cur ^ 1], words, g->n,
                                                chunk, prop, a.off, ws->sinfo);
  const PullTiles* pt = kind == GM_PROG_SSSP && pull_ok ? ws->pt : nullptr;
  send_write<<<(unsigned)nbk, kThreads, 0, s>>>(
      ws->bits[cur], words, g->n, chunk, prop, a.off, ws->sinfo, ws->q, ws->qmsg, ws->qbeg,
      ws->qest, c, kind, m, pull_ok, pull_div, pt ? ws->snap : nullptr,
      pt ? pt->vert_of : nullptr);
  if (kind != GM_PROG_DEGREE && (g->tune.variant & GM_VARIANT_VERTEX_PUSH)) {
    if (kind == GM_PROG_SSSP)
      push_vertex_kernel<GM_PROG_SSSP><<<blocks_for(n), kThreads, 0, s>>>(
          c, n, m, pull_ok, pull_div, ws->qmsg, ws->qbeg, ws->qest, a.idx, a.w, prop,
          ws->bits[cur ^ 1], nullptr, nullptr);
    else
      push_vertex_kernel<GM_PROG_BFS><<<blocks_for(n), kThreads, 0, s>>>(
          c, n, m, pull_ok, pull_div, ws->qmsg, ws->qbeg, ws->qest, a.idx, nullptr, prop,
          ws->bits[cur ^ 1], nullptr, nullptr);
  } else if (kind == GM_PROG_SSSP)
    push_kernel<GM_PROG_SSSP><<<push_blocks, kThreads, 0, s>>>(
        c, n, m, pull_ok, pull_div, ws->qmsg, ws->qbeg, ws->qest, a.idx, a.w, prop,
        ws->bits[cur ^ 1]);
  else if (kind == GM_PROG_DEGREE)
    push_kernel<GM_PROG_DEGREE><<<push_blocks, kThreads, 0, s>>>(
        c, n, m, false, pull_div, ws->qmsg, ws->qbeg, ws->qest, a.idx, nullptr, prop,
        ws->bits[cur ^ 1]);
  else
    push_kernel<GM_PROG_BFS><<<push_blocks, kThreads, 0, s>>>(
        c, n, m, pull_ok, pull_div, ws->qmsg, ws->qbeg, ws->qest, a.idx, nullptr, prop,
        ws->bits[cur ^ 1]);
  if (pull_ok && kind == GM_PROG_BFS)
    pull_kernel<<<blocks_for(n, 8192), kThreads, 0, s>>>(c, n, m, pull_ok, pull_div, pl.off,
                                                         pl.idx, ws->bits[cur], prop,
                                                         ws->bits[cur ^ 1]);
  if (pull_ok && kind == GM_PROG_SSSP) {
    pull_min_tiles<<<(unsigned)std::max(pt->cus, 1), kPullThreads,
                     (size_t)pt->hot_n * sizeof(uint32_t), s>>>(
        c, n, m, pull_ok, pull_div, pt->tidx, pl.w, pt->starts, pt->rows, pt->tile_row,
        pt->ntiles, pt->nrows, ws->snap, pt->hot_n, prop, ws->bits[cur ^ 1]);
  }
  GM_HIP(hipGetLastError());
}

// Zero a control record (the first of a batch of supersteps).
void start_batch(Workspace* ws, hipStream_t s) {
  reset_ctl<<<1, 1, 0, s>>>(ws->ctl);
  GM_HIP(hipGetLastError());
}


// prop[v] = 0 and v active, for every id.
__global__ void seed_sources(const int32_t* __restrict__ ids, int64_t count, uint32_t* prop,
                             uint32_t* bits) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = ids[i];
    prop[v] = 0;
    atomicOr(&bits[v >> 5], 1u << (v & 31));
  }
}

__global__ void set_zero(const int32_t* __restrict__ ids, int64_t count, uint32_t* prop) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    prop[ids[i]] = 0;
}

// Outcome of `steps` recorded supersteps (one thread).
__global__ void min_summary(const Ctl* __restrict__ ctl, int32_t steps, PlanResult* res) {
  int32_t it = 0;
  unsigned long long e = 0;
  for (int32_t b = 0; b < steps; ++b) {
    if ((ctl[b].packed >> 32) == 0) break;
    ++it;
    e += (uint32_t)ctl[b].packed;
  }
  res->iters = it;
  res->converged = 1;
  res->edges = e;
}

// A frontier left after the last recorded superstep means the run did not
// converge; the frontier is cleared either way. Every writer stores 0.
__global__ void bits_finish(uint32_t* bits, int64_t words, int32_t* converged) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (bits[i]) {
      *converged = 0;
      bits[i] = 0;
    }
  }
}

}  // namespace

void prepare_min_program(gm_graph g, hipStream_t s) {
  ensure_ws(g, s);
  GM_HIP(hipStreamSynchronize(s));
}

void prepare_plain_min_program(gm_graph g, int kind, hipStream_t s) {
  Workspace* ws = ensure_ws(g, s);
  if (g->n > 0) {  // the relabelled copy and the SSSP pull layout, where they apply
    Relab* rl = (g->tune.variant & GM_VARIANT_DEGREE_ORDER) ? ensure_relab(g, ws, s) : nullptr;
    (void)run_view(g, ws, kind, GM_ORDER_OUT, rl, s);
  }
  GM_HIP(hipStreamSynchronize(s));
}

void enqueue_min_program(gm_graph g, int kind, const int32_t* ids, int64_t count, int32_t steps,
                         uint32_t* prop, PlanResult* res, hipStream_t s) {
  Workspace* ws = static_cast<Workspace*>(g->min_ws);
  if (!ws || steps < 1 || steps > kMaxCtl) throw Unsupported{"captured run not prepared"};
  const int64_t n = g->n;
  const int64_t words = (n + 31) / 32;
  fill_kernel<<<blocks_for(n), kThreads, 0, s>>>(prop, n,
                                                 kind == GM_PROG_SSSP ? 0xFFFFFFFFu : kInfBfs);
  if (count > 0)
    seed_sources<<<blocks_for(count), kThreads, 0, s>>>(ids, count, prop, ws->bits[0]);
  GM_HIP(hipGetLastError());
  int cur = 0;
  const bool sym = (g->prep & (GM_PREP_SYMMETRIZE | GM_PREP_UPPER_DAG)) == GM_PREP_SYMMETRIZE;
  // captured SSSP runs push only (no snapshot buffer is prepared for them)
  View view{Adj{g->out_off, g->out_idx, static_cast<const uint32_t*>(g->out_w)},
            Adj{sym ? g->out_off : g->in_off, sym ? g->out_idx : g->in_idx, nullptr}, false};
  view.pull_ok = kind == GM_PROG_BFS && view.pull.off != nullptr;
  start_batch(ws, s);
  for (int32_t b = 0; b < steps; ++b) {
    enqueue_superstep(g, ws, kind, view, ws->ctl + b, cur, prop, s);
    cur ^= 1;
  }
  min_summary<<<1, 1, 0, s>>>(ws->ctl, steps, res);
  bits_finish<<<blocks_for(words), kThreads, 0, s>>>(ws->bits[cur], words, &res->converged);
  fill_kernel<<<blocks_for(words), kThreads, 0, s>>>(ws->bits[cur ^ 1], words, 0);  // stale
  GM_HIP(hipGetLastError());
}

// Property array of a fresh run: unreached everywhere, 0 at the ids (their
// frontier bits are set by the run itself).
void init_min_prop(gm_graph g, int kind, const int32_t* ids, int64_t count, uint32_t* prop,
                   hipStream_t s) {
  const int64_t n = g->n;
  fill_kernel<<<blocks_for(n), kThreads, 0, s>>>(prop, n,
                                                 kind == GM_PROG_SSSP ? 0xFFFFFFFFu : kInfBfs);
  if (count > 0) set_zero<<<blocks_for(count), kThreads, 0, s>>>(ids, count, prop);
  GM_HIP(hipGetLastError());
}

namespace {

// Device buffers of the list-frontier variant, freed at scope exit.
struct ListBufs {
  uint32_t* lst = nullptr;       // current frontier: sorted distinct ids (n)
  uint32_t* app[2] = {nullptr, nullptr};  // appended lowered vertices, sort buffers (cap)
  unsigned int* cnt = nullptr;   // [0]: appended count, [1]: distinct count
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  ~ListBufs() {
    dfree(lst);
    dfree(app[0]);
    dfree(app[1]);
    dfree(cnt);
    dfree(tmp);
  }
};

// Sort app[0][0..k) and keep each id once, into lst; returns the number of
// distinct ids (synchronises s).
int64_t sort_unique(ListBufs& b, int64_t k, hipStream_t s) {
  if (k == 0) return 0;
  rocprim::double_buffer<uint32_t> kb(b.app[0], b.app[1]);
  size_t need = 0, need2 = 0;
  GM_HIP(rocprim::radix_sort_keys(nullptr, need, kb, (size_t)k, 0, 32, s));
  GM_HIP(rocprim::unique(nullptr, need2, kb.current(), b.lst, b.cnt + 1, (size_t)k,
                         rocprim::equal_to<uint32_t>(), s));
  need = std::max(need, need2);
  if (need > b.tmp_bytes) {
    dfree(b.tmp);
    b.tmp = nullptr;
    b.tmp = dmalloc(need);
    b.tmp_bytes = need;
  }
  GM_HIP(rocprim::radix_sort_keys(b.tmp, need, kb, (size_t)k, 0, 32, s));
  need = b.tmp_bytes;
  GM_HIP(rocprim::unique(b.tmp, need, kb.current(), b.lst, b.cnt + 1, (size_t)k,
                         rocprim::equal_to<uint32_t>(), s));
  unsigned int h = 0;
  GM_HIP(hipMemcpyAsync(&h, b.cnt + 1, 4, hipMemcpyDeviceToHost, s));
  GM_HIP(hipStreamSynchronize(s));
  return h;
}

}  // namespace

// BFS / SSSP with the frontier as a sorted list of distinct vertex ids (the
// GM_VARIANT_LIST_FRONTIER ablation): each superstep is SEND from the list,
// the push product appending every lowered vertex, and a sort + unique that
// forms the next list (its length read by the host).
static int32_t run_min_program_list(gm_graph g, Workspace* ws, const Adj& adj, int kind,
                                    const int32_t* ids, int64_t count, int32_t max_iters,
                                    uint32_t* prop, int32_t* active_out, hipStream_t s,
                                    RunStats* stats) {
  const int64_t n = g->n;
  uint32_t medges = 0;
  GM_HIP(hipMemcpyAsync(&medges, adj.off + n, 4, hipMemcpyDeviceToHost, s));
  GM_HIP(hipStreamSynchronize(s));
  const int64_t cap = std::max<int64_t>({(int64_t)medges, count, 1});
  ListBufs b;
  b.lst = dalloc<uint32_t>(std::max<int64_t>(n, 1));
  b.app[0] = dalloc<uint32_t>(cap);
  b.app[1] = dalloc<uint32_t>(cap);
  b.cnt = dalloc<unsigned int>(2);
  if (count > 0) {
    ids_to_u32<<<blocks_for(count), kThreads, 0, s>>>(ids, count, b.app[0]);
    GM_HIP(hipGetLastError());
  }
  int64_t c = sort_unique(b, count, s);
  const bool vertex_push = (g->tune.variant & GM_VARIANT_VERTEX_PUSH) != 0;
  int32_t iters = 0;
  RunStats st{};
  while (c > 0 && (max_iters <= 0 || iters < max_iters)) {
    start_batch(ws, s);
    fill_u32(b.cnt, 1, 0u, s);
    send_list_kernel<<<blocks_for(c, 4096), kThreads, 0, s>>>(b.lst, c, prop, adj.off, ws->q,
                                                               ws->qmsg, ws->qbeg, ws->qest,
                                                               ws->ctl);
    if (vertex_push) {
      if (kind == GM_PROG_SSSP)
        push_vertex_kernel<GM_PROG_SSSP><<<blocks_for(c), kThreads, 0, s>>>(
            ws->ctl, n, g->m, false, 1, ws->qmsg, ws->qbeg, ws->qest, adj.idx, adj.w, prop, nullptr,
            b.app[0], b.cnt);
      else
        push_vertex_kernel<GM_PROG_BFS><<<blocks_for(c), kThreads, 0, s>>>(
            ws->ctl, n, g->m, false, 1, ws->qmsg, ws->qbeg, ws->qest, adj.idx, nullptr, prop, nullptr,
            b.app[0], b.cnt);
    } else if (kind == GM_PROG_SSSP) {
      push_kernel<GM_PROG_SSSP><<<g->tune.push_blocks, kThreads, 0, s>>>(
          ws->ctl, n, g->m, false, 1, ws->qmsg, ws->qbeg, ws->qest, adj.idx, adj.w, prop, nullptr,
          b.app[0], b.cnt);
    } else {
      push_kernel<GM_PROG_BFS><<<g->tune.push_blocks, kThreads, 0, s>>>(
          ws->ctl, n, g->m, false, 1, ws->qmsg, ws->qbeg, ws->qest, adj.idx, nullptr, prop, nullptr,
          b.app[0], b.cnt);
    }
    GM_HIP(hipGetLastError());
    unsigned int appended = 0;
    GM_HIP(hipMemcpyAsync(ws->host_ctl, ws->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    GM_HIP(hipMemcpyAsync(&appended, b.cnt, 4, hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    ++iters;
    ++st.push_supersteps;
    st.edges_scanned += (uint32_t)ws->host_ctl[0].packed;
    c = sort_unique(b, appended, s);
  }
  if (active_out) {
    fill_u32(reinterpret_cast<uint32_t*>(active_out), n, 0u, s);
    if (c > 0) {
      list_to_active<<<blocks_for(c), kThreads, 0, s>>>(b.lst, c, active_out);
      GM_HIP(hipGetLastError());
    }
  }
  GM_HIP(hipStreamSynchronize(s));
  st.supersteps = iters;
  if (stats) *stats = st;
  return iters;
}

// The supersteps of a plain run on a view (labels of `view`): prop and the
// first frontier (in bits[0]: the caller's ids or bitmap, already seeded, or
// every vertex for the degree program) in, prop and the final frontier
// (active_out, if set) out.
static int32_t run_supersteps(gm_graph g, Workspace* ws, int kind, const View& view,
                              bool have_frontier, int32_t max_iters, uint32_t* prop,
                              int32_t* active_out, hipStream_t s, RunStats* stats) {
  const int64_t n = g->n;
  const int64_t words = (n + 31) / 32;
  int32_t batch = (int32_t)g->tune.superstep_batch;
  if (batch < 1) batch = 1;
  int cur = 0;
  if (kind == GM_PROG_DEGREE) {  // every vertex sends; the property starts at 0
    fill_kernel<<<blocks_for(n), kThreads, 0, s>>>(prop, n, 0u);
    seed_all<<<blocks_for(words), kThreads, 0, s>>>(words, n, ws->bits[0]);
    GM_HIP(hipGetLastError());
  }
  int32_t iters = 0;
  RunStats st{};
  bool done = !have_frontier && kind != GM_PROG_DEGREE;  // an empty bitmap: one SEND
  uint64_t prev_cnt = 0, last_cnt = 0;  // frontier sizes of the last two supersteps
  bool near = false;  // the next batch may pull (near_pull of its last two supersteps)
  Ctl prev_ctl{0, 0, 0}, last_ctl{0, 0, 0};
  while (!done) {
    int32_t nb = batch;
    if (max_iters > 0 && max_iters - iters < nb) nb = max_iters - iters;
    if (nb > kMaxCtl) nb = kMaxCtl;
    start_batch(ws, s);
    View bv = view;
    bv.pull_ok = view.pull_ok && (iters == 0 || near);
    for (int32_t b = 0; b < nb; ++b) {
      enqueue_superstep(g, ws, kind, bv, ws->ctl + b, cur, prop, s);
      cur ^= 1;
    }
    GM_HIP(hipMemcpyAsync(ws->host_ctl, ws->ctl, nb * sizeof(Ctl), hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    for (int32_t b = 0; b < nb; ++b) {
      const Ctl& c = ws->host_ctl[b];
      const uint64_t cnt = c.packed >> 32;
      if (cnt == 0) {
        done = true;
        break;
      }
      prev_cnt = last_cnt;
      last_cnt = cnt;
      ++iters;
      st.edges_scanned += (uint32_t)c.packed;
      prev_ctl = last_ctl;
      last_ctl = c;
      const bool pulled = use_pull(c, kind, bv.pull_ok, n, g->m, g->tune.pull_div);
      if (pulled)
        ++st.pull_supersteps;
      else
        ++st.push_supersteps;
    }
    if (max_iters > 0 && iters >= max_iters) done = true;
    near = near_pull(last_ctl, prev_ctl, kind, n, g->m, g->tune.pull_div);
    // A run whose frontier holds up is long: each further batch is twice as
    // long, so a run of S supersteps waits for the host about log2(S) times,
    // not S / batch. One whose frontier fell below half from one superstep to
    // the next at the end of the batch is ending: the next batch goes back to
    // the first length, since every superstep enqueued after the frontier
    // empties still costs its launches.
    const int32_t batch0 = std::max<int32_t>(1, (int32_t)g->tune.superstep_batch);
    batch = 2 * last_cnt < prev_cnt ? batch0 : std::min<int32_t>(2 * batch, kMaxCtl);
  }
  // bits[cur] holds the frontier left after the last superstep (empty when
  // the program converged); report it and leave the workspace cleared (the
  // other vector holds a stale frontier).
  bits_epilogue<<<blocks_for(words), kThreads, 0, s>>>(ws->bits[cur], words, n, active_out);
  fill_kernel<<<blocks_for(words), kThreads, 0, s>>>(ws->bits[cur ^ 1], words, 0);
  GM_HIP(hipGetLastError());
  st.supersteps = iters;
  if (stats) *stats = st;
  return iters;
}

int32_t run_min_program(gm_graph g, int kind, int order, const int32_t* ids, int64_t count,
                        const uint32_t* bitmap, int32_t max_iters, uint32_t* prop,
                        int32_t* active_out, hipStream_t s, RunStats* stats) {
  Workspace* ws = ensure_ws(g, s);
  const int64_t n = g->n;
  const int64_t words = (n + 31) / 32;
  const bool list = (g->tune.variant & GM_VARIANT_LIST_FRONTIER) && kind != GM_PROG_DEGREE;
  if (list && bitmap) throw Unsupported{"the list-frontier variant takes frontier ids"};
  Relab* rl = nullptr;
  if (n > 0 && (g->tune.variant & GM_VARIANT_DEGREE_ORDER)) rl = ensure_relab(g, ws, s);
  const View view = run_view(g, ws, kind, order, rl, s);
  const bool have_frontier = bitmap != nullptr || count > 0;
  int32_t iters = 0;
  if (!rl) {
    if (!list && kind != GM_PROG_DEGREE) {
      if (bitmap)
        seed_bitmap<<<blocks_for(words), kThreads, 0, s>>>(bitmap, words, n, ws->bits[0]);
      else if (count > 0)
        seed_bits<<<blocks_for(count), kThreads, 0, s>>>(ids, count, ws->bits[0]);
      GM_HIP(hipGetLastError());
    }
    iters = list ? run_min_program_list(g, ws, view.push, kind, ids, count, max_iters, prop,
                                        active_out, s, stats)
                 : run_supersteps(g, ws, kind, view, have_frontier, max_iters, prop, active_out,
                                  s, stats);
    GM_HIP(hipStreamSynchronize(s));
    return iters;
  }
  // Relabelled run: the caller's values and frontier into the new labels,
  // the supersteps, the results back.
  if (kind != GM_PROG_DEGREE)
    permute_u32<<<blocks_for(n), kThreads, 0, s>>>(prop, rl->old_of, n, rl->prop);
  if (count > 0) map_ids<<<blocks_for(count), kThreads, 0, s>>>(ids, count, rl->new_of, rl->ids);
  if (!list && kind != GM_PROG_DEGREE) {
    if (bitmap)
      seed_bitmap_mapped<<<blocks_for(n), kThreads, 0, s>>>(bitmap, n, rl->new_of, ws->bits[0]);
    else if (count > 0)
      seed_bits<<<blocks_for(count), kThreads, 0, s>>>(rl->ids, count, ws->bits[0]);
  }
  GM_HIP(hipGetLastError());
  int32_t* act = active_out ? rl->active : nullptr;
  iters = list ? run_min_program_list(g, ws, view.push, kind, rl->ids, count, max_iters, rl->prop,
                                      act, s, stats)
               : run_supersteps(g, ws, kind, view, have_frontier, max_iters, rl->prop, act, s,
                                stats);
  permute_u32<<<blocks_for(n), kThreads, 0, s>>>(rl->prop, rl->new_of, n, prop);
  if (active_out)
    permute_u32<<<blocks_for(n), kThreads, 0, s>>>(reinterpret_cast<const uint32_t*>(rl->active),
                                                   rl->new_of, n,
                                                   reinterpret_cast<uint32_t*>(active_out));
  GM_HIP(hipGetLastError());
  GM_HIP(hipStreamSynchronize(s));
  return iters;
}

}  // namespace gm
