// Batched forms of the generalized SpMSpV: k sources (or personalised
// PageRank seeds) run together, so one read of the matrix serves all k
// frontiers (an SpMM with a dense n x k frontier block, semirings as in
// Sec. 3). Column s of every result equals the plain run from source s.
//
//  - BFS (k <= 64): the frontier of vertex v over all sources is one 64-bit
//    mask (REDUCE = or); new bits get level t + 1. Each superstep pushes
//    (small frontier: edges of the active vertices split evenly over
//    wavefronts) or pulls (large frontier: every vertex ORs its neighbours'
//    masks until every source that has not reached it is covered), as
//    decided on the device from the frontier's out-edge count.
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

// ---------------------------------------------------------------- BFS -----
// Superstep t reads the frontier masks fr (bit s: source s reached the
// vertex at level t) and writes the next ones. Direction per superstep, chosen
// on the device from the frontier's size: push (few active vertices: their
// edges are split evenly over wavefronts and each edge ORs the sender's mask
// into the receiver's next mask) or pull (every vertex not yet reached by all
// sources ORs its neighbours' masks, stopping once nothing is left to learn;
// vertices are taken in decreasing degree order, a power-of-two number of
// lanes per vertex as in the PageRank pull). Levels are unique, so both
// directions give the same result.

// Frontier of one superstep (written by the previous one).
struct BfsCtl {
  unsigned long long active;  // vertices with a non-empty mask
  unsigned long long edges;   // their degrees
  uint32_t push;              // 1: push superstep
  uint32_t pad;
};

constexpr int kBfsStatBlocks = 1024;  // grid of the apply and pull kernels
constexpr int kBfsClasses = 12;
constexpr uint32_t kBfsClassMax[kBfsClasses] = {0, 1, 2, 4, 8, 16, 32, 64, 128, 256, 512,
                                                0xFFFFFFFFu};
constexpr int kBfsClassLanes[kBfsClasses] = {1, 1, 1, 1, 1, 2, 4, 8, 16, 32, 64, 64};
constexpr int kBfsClassUnroll[kBfsClasses] = {1, 1, 2, 4, 8, 8, 8, 8, 8, 8, 8, 8};

// Vertices in decreasing degree order cut into wavefront units (class c: 64 /
// kBfsClassLanes[c] vertices per unit), longest class first.
struct BfsBins {
  int64_t class_begin[kBfsClasses];  // position in the order
  int64_t class_rows[kBfsClasses];
  int64_t class_unit0[kBfsClasses];  // decreases with c; class 0 (degree 0) is never pulled
  int64_t nunits;
};

__global__ void bbfs_init(int64_t n, int k, int32_t* level, unsigned long long* vis,
                          unsigned long long* fr0, unsigned long long* fr1, BfsCtl* ctl0) {
  const int64_t total = n * k;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x)
    level[i] = (int32_t)kInfBfs;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    vis[v] = 0;
    fr0[v] = 0;
    fr1[v] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl0->active = (unsigned long long)k;  // at most k source vertices
    ctl0->edges = 0;
    ctl0->push = 1;
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

__device__ inline void set_levels(int32_t* level, int64_t v, int k, unsigned long long bits,
                                  int32_t lev) {
  for (unsigned long long b = bits; b; b &= b - 1) level[v * k + (__ffsll((long long)b) - 1)] = lev;
}

// Block-wide sum of (count, edges) into stat[blockIdx.x] (every block writes).
__device__ inline void block_stat(unsigned long long cnt, unsigned long long edges,
                                  unsigned long long* stat) {
  __shared__ unsigned long long sc[kThreads / 64], se[kThreads / 64];
  for (int o = 32; o > 0; o >>= 1) {
    cnt += __shfl_xor(cnt, o, 64);
    edges += __shfl_xor(edges, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sc[threadIdx.x >> 6] = cnt;
    se[threadIdx.x >> 6] = edges;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long c = 0, e = 0;
    for (int i = 0; i < kThreads / 64; ++i) {
      c += sc[i];
      e += se[i];
    }
    stat[2 * blockIdx.x] = c;
    stat[2 * blockIdx.x + 1] = e;
  }
}

// SEND of a push superstep: queue the active vertices with their first edge
// and the exclusive prefix of their degrees.
__global__ __launch_bounds__(kThreads) void bbfs_send(
    const BfsCtl* __restrict__ ctl, int64_t n, const unsigned long long* __restrict__ fr,
    const uint32_t* __restrict__ off, int32_t* __restrict__ q, uint32_t* __restrict__ qbeg,
    uint32_t* __restrict__ qest, BCtl* __restrict__ qctl) {
  if (!ctl->push || ctl->active == 0) return;
  __shared__ uint32_t sh[2 * kWaves];
  __shared__ unsigned long long base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t v0 = (int64_t)blockIdx.x * kThreads; v0 < n; v0 += (int64_t)gridDim.x * kThreads) {
    const int64_t v = v0 + threadIdx.x;
    const bool a = v < n && fr[v] != 0;
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
    if (threadIdx.x == 0 && ct) base = atomicAdd(&qctl->packed, ((unsigned long long)ct << 32) | et);
    __syncthreads();
    if (ct && a) {
      const unsigned long long bp = base;
      const uint32_t slot = (uint32_t)(bp >> 32) + cb + ci - cnt;
      q[slot] = (int32_t)v;
      qbeg[slot] = off[v];
      qest[slot] = (uint32_t)bp + eb + ei - deg;
    }
    __syncthreads();
  }
}

// PROCESS + REDUCE of a push superstep: one edge per lane, the edges of the
// queued vertices split evenly over the wavefronts.
__global__ __launch_bounds__(kThreads) void bbfs_push(
    const BfsCtl* __restrict__ ctl, const BCtl* __restrict__ qctl, const int32_t* __restrict__ q,
    const uint32_t* __restrict__ qbeg, const uint32_t* __restrict__ qest,
    const int32_t* __restrict__ idx, const unsigned long long* __restrict__ fr,
    const unsigned long long* __restrict__ vis, unsigned long long* fnext) {
  if (!ctl->push || ctl->active == 0) return;
  const uint32_t count = (uint32_t)(qctl->packed >> 32);
  const uint64_t E = (uint32_t)qctl->packed;
  if (count == 0 || E == 0) return;
  const int lane = threadIdx.x & 63;
  const uint64_t nw = (uint64_t)gridDim.x * kWaves;
  const uint64_t wid = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const uint32_t e_begin = (uint32_t)(E * wid / nw), e_end = (uint32_t)(E * (wid + 1) / nw);
  if (e_begin >= e_end) return;
  uint32_t lo = 0, hi = count;  // last slot whose prefix is <= e_begin, in [lo, hi)
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
  uint32_t e = e_begin;
  for (uint32_t s0 = lo; e < e_end; s0 += 64) {
    const uint32_t s = s0 + lane;
    const bool valid = s < count;
    const uint32_t est = valid ? qest[s] : (uint32_t)E;
    const uint32_t beg = valid ? qbeg[s] : 0u;
    const unsigned long long mk = valid ? fr[q[s]] : 0ull;
    const uint32_t win_end = s0 + 64 < count ? qest[s0 + 64] : (uint32_t)E;
    const uint32_t stop = win_end < e_end ? win_end : e_end;
    for (; e < stop; e += 64) {
      const uint32_t ee = e + lane;
      int j = 0;  // owner: the last lane whose prefix is <= ee
#pragma unroll
      for (int step = 32; step > 0; step >>= 1) {
        const uint32_t ex = __shfl(est, j + step, 64);
        if (ex <= ee) j += step;
      }
      const uint32_t ej = __shfl(est, j, 64);
      const uint32_t bj = __shfl(beg, j, 64);
      const unsigned long long m = __shfl(mk, j, 64);
      if (ee < stop) {
        const int32_t v = idx[bj + (ee - ej)];
        const unsigned long long nw_bits = m & ~vis[v];
        if (nw_bits)
          __hip_atomic_fetch_or(&fnext[v], nw_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    e = stop;
  }
}

// APPLY of a push superstep: new bits become visited and get level t + 1.
// Frontier statistics count out-edges (what the next push would walk).
__global__ __launch_bounds__(kThreads) void bbfs_apply(
    const BfsCtl* __restrict__ ctl, int64_t n, int k, int32_t t, const uint32_t* __restrict__ off,
    unsigned long long* vis, unsigned long long* fnext, int32_t* level,
    unsigned long long* stat) {
  if (!ctl->push || ctl->active == 0) return;
  unsigned long long cnt = 0, edges = 0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long m = fnext[v];
    if (m) {
      const unsigned long long seen = vis[v];
      const unsigned long long nw = m & ~seen;
      fnext[v] = nw;
      if (nw) {
        vis[v] = seen | nw;
        set_levels(level, v, k, nw, t + 1);
        ++cnt;
        edges += off[v + 1] - off[v];
      }
    }
  }
  block_stat(cnt, edges, stat);
}

__device__ inline unsigned long long group_or(unsigned long long v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

// OR of the frontier masks of the neighbours [b, e) of one vertex, taken by
// `lanes` lanes with kU loads in flight each; stops once acc | seen == full
// (checked by the whole lane group after each pass).
template <int kU>
__device__ inline unsigned long long pull_or(const int32_t* __restrict__ idx,
                                             const unsigned long long* __restrict__ fr,
                                             uint32_t b, uint32_t e, int sub, int lanes,
                                             unsigned long long seen, unsigned long long full) {
  unsigned long long acc = 0;
  for (uint32_t k0 = b + sub; k0 < e + sub; k0 += kU * lanes) {
    int32_t u[kU];
#pragma unroll
    for (int q = 0; q < kU; ++q) {
      const uint32_t kk = k0 + q * lanes;
      u[q] = idx[kk < e ? kk : e - 1];
    }
    unsigned long long m[kU];
#pragma unroll
    for (int q = 0; q < kU; ++q) m[q] = fr[u[q]];
#pragma unroll
    for (int q = 0; q < kU; ++q) acc |= k0 + q * lanes < e ? m[q] : 0ull;
    if ((group_or(acc, lanes) | seen) == full) break;
  }
  return group_or(acc, lanes);
}

// PROCESS + REDUCE + APPLY of a pull superstep.
__global__ __launch_bounds__(kThreads) void bbfs_pull(
    const BfsCtl* __restrict__ ctl, int k, int32_t t, BfsBins bins,
    const int32_t* __restrict__ order, const uint32_t* __restrict__ off,
    const int32_t* __restrict__ idx, const uint32_t* __restrict__ out_off,
    const unsigned long long* __restrict__ fr, unsigned long long* vis,
    unsigned long long* fnext, int32_t* level, unsigned long long* stat) {
  if (ctl->push || ctl->active == 0) return;
  const unsigned long long full = full_mask(k);
  const int lane = threadIdx.x & 63;
  unsigned long long cnt = 0, edges = 0;
  const int64_t stride = (int64_t)gridDim.x * kWaves;
  for (int64_t u = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); u < bins.nunits;
       u += stride) {
    int cls = 1;
    while (u < bins.class_unit0[cls]) ++cls;
    const int lanes = kBfsClassLanes[cls];
    const int64_t local = (u - bins.class_unit0[cls]) * (64 / lanes) + lane / lanes;
    const bool valid = local < bins.class_rows[cls];
    const int64_t v = valid ? order[bins.class_begin[cls] + local] : 0;
    const int sub = lane % lanes;
    const unsigned long long seen = valid ? vis[v] : full;
    unsigned long long acc = 0;
    uint32_t b = 0, e = 0;
    if (valid) {
      b = off[v];
      e = off[v + 1];
    }
    if (seen != full) {
      switch (kBfsClassUnroll[cls]) {
        case 1: acc = pull_or<1>(idx, fr, b, e, sub, lanes, seen, full); break;
        case 2: acc = pull_or<2>(idx, fr, b, e, sub, lanes, seen, full); break;
        case 4: acc = pull_or<4>(idx, fr, b, e, sub, lanes, seen, full); break;
        default: acc = pull_or<8>(idx, fr, b, e, sub, lanes, seen, full); break;
      }
    }
    const unsigned long long nw = acc & ~seen;
    if (valid && sub == 0 && nw) {
      vis[v] = seen | nw;
      fnext[v] = nw;
      set_levels(level, v, k, nw, t + 1);
      ++cnt;
      edges += out_off[v + 1] - out_off[v];
    }
  }
  block_stat(cnt, edges, stat);
}

// Frontier of the next superstep and its direction (one workgroup).
__global__ void bbfs_decide(const BfsCtl* __restrict__ ctl, const unsigned long long* __restrict__ stat,
                            int nstat, uint64_t m, uint32_t pull_div, BfsCtl* __restrict__ next) {
  __shared__ unsigned long long sc[kWaves], se[kWaves];
  unsigned long long c = 0, e = 0;
  if (ctl->active != 0)
    for (int i = threadIdx.x; i < nstat; i += blockDim.x) {
      c += stat[2 * i];
      e += stat[2 * i + 1];
    }
  for (int o = 32; o > 0; o >>= 1) {
    c += __shfl_xor(c, o, 64);
    e += __shfl_xor(e, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sc[threadIdx.x >> 6] = c;
    se[threadIdx.x >> 6] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    c = e = 0;
    for (int i = 0; i < kWaves; ++i) {
      c += sc[i];
      e += se[i];
    }
    next->active = c;
    next->edges = e;
    next->push = e * pull_div <= m ? 1u : 0u;
  }
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
  BfsCtl* bctl = nullptr;  // kMaxPlanSteps + 1 records: the frontier of each superstep
  BfsCtl* host_bctl = nullptr;
  unsigned long long* bstat = nullptr;  // 2 * kBfsStatBlocks partial counts
  int32_t* border = nullptr;            // vertices by decreasing pull degree
  BfsBins bbins{};
  int32_t* bq = nullptr;                // push queue
  uint32_t* bqbeg = nullptr;
  uint32_t* bqest = nullptr;
  BCtl* bqctl = nullptr;                // kMaxPlanSteps queue records
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
  // b->items marks complete work items: set last (a failure leaves none)
  PprItem* it = nullptr;
  PprSplit* sp = nullptr;
  try {
    it = dalloc<PprItem>(items.size());
    sp = dalloc<PprSplit>(splits.size());
    GM_HIP(hipMemcpyAsync(it, items.data(), items.size() * sizeof(PprItem),
                          hipMemcpyHostToDevice, s));
    if (!splits.empty())
      GM_HIP(hipMemcpyAsync(sp, splits.data(), splits.size() * sizeof(PprSplit),
                            hipMemcpyHostToDevice, s));
    GM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    dfree(it);
    dfree(sp);
    throw;
  }
  b->nitems = (int64_t)items.size();
  b->nsplit = (int64_t)splits.size();
  b->npartial = np;
  b->items_chunk = chunk;
  b->items = it;
  b->splits = sp;
}

// Pull adjacency of batched BFS: the out-lists of a symmetrised graph, else
// the in-lists.
void bfs_adjacency(gm_graph g, const uint32_t** off, const int32_t** idx) {
  const bool sym = (g->prep & (GM_PREP_SYMMETRIZE | GM_PREP_UPPER_DAG)) == GM_PREP_SYMMETRIZE;
  *off = sym ? g->out_off : g->in_off;
  *idx = sym ? g->out_idx : g->in_idx;
}

void ensure_bfs_ws(gm_graph g, Batch* b, hipStream_t s) {
  if (b->vis) return;
  const int64_t n = g->n;
  const uint32_t* doff;
  const int32_t* didx;
  bfs_adjacency(g, &doff, &didx);
  // vertices by decreasing pull degree (counting sort), cut into classes
  std::vector<uint32_t> off(n + 1);
  GM_HIP(hipMemcpyAsync(off.data(), doff, (n + 1) * 4, hipMemcpyDeviceToHost, s));
  GM_HIP(hipStreamSynchronize(s));
  uint32_t maxd = 0;
  for (int64_t v = 0; v < n; ++v) maxd = std::max(maxd, off[v + 1] - off[v]);
  std::vector<int64_t> cnt((size_t)maxd + 2, 0);
  for (int64_t v = 0; v < n; ++v) ++cnt[maxd - (off[v + 1] - off[v])];
  int64_t acc = 0;
  for (size_t i = 0; i < cnt.size(); ++i) {
    const int64_t c = cnt[i];
    cnt[i] = acc;
    acc += c;
  }
  std::vector<int32_t> order(n);
  for (int64_t v = 0; v < n; ++v) order[cnt[maxd - (off[v + 1] - off[v])]++] = (int32_t)v;
  BfsBins& bins = b->bbins;
  int64_t i = 0, unit = 0;
  for (int c = kBfsClasses - 1; c >= 0; --c) {
    const int64_t r0 = i;
    if (c == 0)
      i = n;
    else
      while (i < n && off[order[i] + 1] - off[order[i]] > kBfsClassMax[c - 1]) ++i;
    bins.class_begin[c] = r0;
    bins.class_rows[c] = i - r0;
    bins.class_unit0[c] = unit;
    if (c > 0) {
      const int64_t rpu = 64 / kBfsClassLanes[c];
      unit += (bins.class_rows[c] + rpu - 1) / rpu;
    }
  }
  bins.nunits = unit;
  // b->vis marks a complete workspace: it is set last, and a failed
  // allocation frees what was taken, so the next call starts over
  unsigned long long* vis = nullptr;
  try {
    b->fr[0] = dalloc<unsigned long long>(n);
    b->fr[1] = dalloc<unsigned long long>(n);
    b->bctl = dalloc<BfsCtl>(kMaxPlanSteps + 1);
    b->bstat = dalloc<unsigned long long>(2 * kBfsStatBlocks);
    b->border = dalloc<int32_t>(n);
    b->bq = dalloc<int32_t>(n);
    b->bqbeg = dalloc<uint32_t>(n);
    b->bqest = dalloc<uint32_t>(n);
    b->bqctl = dalloc<BCtl>(kMaxPlanSteps);
    void* h = nullptr;
    GM_HIP(hipHostMalloc(&h, sizeof(BfsCtl), hipHostMallocDefault));
    b->host_bctl = static_cast<BfsCtl*>(h);
    GM_HIP(hipMemcpyAsync(b->border, order.data(), n * 4, hipMemcpyHostToDevice, s));
    GM_HIP(hipStreamSynchronize(s));
    vis = dalloc<unsigned long long>(n);
  } catch (...) {
    for (void** p : {(void**)&b->fr[0], (void**)&b->fr[1], (void**)&b->bctl, (void**)&b->bstat,
                     (void**)&b->border, (void**)&b->bq, (void**)&b->bqbeg, (void**)&b->bqest,
                     (void**)&b->bqctl}) {
      dfree(*p);
      *p = nullptr;
    }
    if (b->host_bctl) (void)hipHostFree(b->host_bctl);
    b->host_bctl = nullptr;
    throw;
  }
  b->vis = vis;
}

void ensure_sssp_ws(gm_graph g, Batch* b, int k) {
  const int64_t n = g->n;
  if (!b->act[0]) {  // act[0] marks a complete workspace: set last
    unsigned long long* act = nullptr;
    try {
      b->q = dalloc<int32_t>(n);
      b->qbeg = dalloc<uint32_t>(n);
      b->qest = dalloc<uint32_t>(n);
      b->ctl = dalloc<BCtl>(kMaxPlanSteps);
      void* h = nullptr;
      GM_HIP(hipHostMalloc(&h, sizeof(BCtl), hipHostMallocDefault));
      b->host_ctl = static_cast<BCtl*>(h);
      act = dalloc<unsigned long long>(2 * n);  // both masks in one buffer
    } catch (...) {
      for (void** p : {(void**)&b->q, (void**)&b->qbeg, (void**)&b->qest, (void**)&b->ctl}) {
        dfree(*p);
        *p = nullptr;
      }
      if (b->host_ctl) (void)hipHostFree(b->host_ctl);
      b->host_ctl = nullptr;
      throw;
    }
    b->act[0] = act;
    b->act[1] = act + n;
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

void bfs_init(gm_graph g, Batch* b, const int32_t* sources, int k, int32_t* level, hipStream_t s) {
  const int64_t n = g->n;
  bbfs_init<<<blocks_for(n * k), kThreads, 0, s>>>(n, k, level, b->vis, b->fr[0], b->fr[1], b->bctl);
  bbfs_seed<<<1, 64, 0, s>>>(k, sources, level, b->vis, b->fr[0]);
  GM_HIP(hipGetLastError());
}

// Superstep t (new vertices get level t + 1): frontier fr[cur] described by
// bctl[rec]; writes fr[cur ^ 1] and bctl[rec + 1]; clears fr[cur]. Does
// nothing if bctl[rec] is empty.
void bfs_superstep(gm_graph g, Batch* b, int k, int32_t t, int32_t rec, int cur, int32_t* level,
                   hipStream_t s) {
  const int64_t n = g->n;
  const uint32_t* off;
  const int32_t* idx;
  bfs_adjacency(g, &off, &idx);
  const BfsCtl* c = b->bctl + rec;
  BCtl* qc = b->bqctl + rec;
  reset_bctl<<<1, 1, 0, s>>>(qc);
  bbfs_send<<<blocks_for(n, 4096), kThreads, 0, s>>>(c, n, b->fr[cur], g->out_off, b->bq, b->bqbeg,
                                                     b->bqest, qc);
  bbfs_push<<<g->tune.push_blocks, kThreads, 0, s>>>(c, qc, b->bq, b->bqbeg, b->bqest, g->out_idx,
                                                     b->fr[cur], b->vis, b->fr[cur ^ 1]);
  bbfs_apply<<<kBfsStatBlocks, kThreads, 0, s>>>(c, n, k, t, g->out_off, b->vis, b->fr[cur ^ 1],
                                                 level, b->bstat);
  bbfs_pull<<<kBfsStatBlocks, kThreads, 0, s>>>(c, k, t, b->bbins, b->border, off, idx, g->out_off,
                                                b->fr[cur], b->vis, b->fr[cur ^ 1], level,
                                                b->bstat);
  bbfs_decide<<<1, kThreads, 0, s>>>(c, b->bstat, kBfsStatBlocks, (uint64_t)g->m, g->tune.pull_div,
                                     b->bctl + rec + 1);
  fill_u32(reinterpret_cast<uint32_t*>(b->fr[cur]), 2 * n, 0u, s);
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
// iff the frontier it leaves (bctl[t + 1]) is empty; that superstep still
// counts, as in the plain run.
__global__ void bbfs_summary(const BfsCtl* __restrict__ bctl, int32_t steps, PlanResult* res) {
  int32_t it = steps, conv = 0;
  unsigned long long e = 0;
  for (int32_t t = 0; t < steps; ++t) {
    e += bctl[t].edges;
    if (bctl[t + 1].active == 0) {
      it = t + 1;
      conv = 1;
      break;
    }
  }
  res->iters = it;
  res->converged = conv;
  res->edges = e;
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
  dfree(b->bctl);
  if (b->host_bctl) (void)hipHostFree(b->host_bctl);
  dfree(b->bstat);
  dfree(b->border);
  dfree(b->bq);
  dfree(b->bqbeg);
  dfree(b->bqest);
  dfree(b->bqctl);
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
  ensure_bfs_ws(g, b, s);
  bfs_init(g, b, sources, k, level, s);
  int cur = 0;
  int32_t t = 0;
  // bctl holds kMaxPlanSteps + 1 records; longer runs restart at record 0
  // with the last frontier record carried over.
  int32_t rec = 0;
  for (;; ++t) {
    if (max_iters > 0 && t >= max_iters) break;
    if (rec == kMaxPlanSteps) {
      GM_HIP(hipMemcpyAsync(b->bctl, b->bctl + rec, sizeof(BfsCtl), hipMemcpyDeviceToDevice, s));
      rec = 0;
    }
    bfs_superstep(g, b, k, t, rec, cur, level, s);
    GM_HIP(hipMemcpyAsync(b->host_bctl, b->bctl + rec + 1, sizeof(BfsCtl), hipMemcpyDeviceToHost,
                          s));
    GM_HIP(hipStreamSynchronize(s));
    cur ^= 1;
    ++rec;
    if (b->host_bctl->active == 0) {
      ++t;  // this superstep scanned the deepest frontier and found nothing new
      break;
    }
  }
  // leave both frontiers cleared for the next run
  fill_u32(reinterpret_cast<uint32_t*>(b->fr[cur]), 2 * g->n, 0u, s);
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
    ensure_bfs_ws(g, b, s);
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
    int cur = 0;
    for (int32_t t = 0; t < steps; ++t) {
      bfs_superstep(g, b, k, t, t, cur, level, s);
      cur ^= 1;
    }
    bbfs_summary<<<1, 1, 0, s>>>(b->bctl, steps, res);
    fill_u32(reinterpret_cast<uint32_t*>(b->fr[cur]), 2 * g->n, 0u, s);
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
