// PageRank (Sec. 3 I, Eq. (1)) and personalised PageRank as a pull-direction
// generalized SpMV over the in-adjacency, with APPLY and the next SEND fused
// into the same kernel.
//
// One superstep = one launch of pr_pull:
//   y_v   = sum_{u -> v} x_u (* w_uv)          PROCESS = msg (* w), REDUCE = +
//   PR_v  = r * tele(v) + (1 - r) * y_v        APPLY, for every vertex
//   x'_v  = PR_v / outdeg(v)                   SEND for the next superstep
// where x_u = PR_u / outdeg(u) is the message (0 for dangling vertices, which
// send nothing). Row sums are accumulated in double, in a fixed order, so the
// result does not depend on scheduling.
//
// Work decomposition (static, built once per graph): consecutive destination
// rows are grouped into tasks of at most kBlockEdges in-edges and kMaxRows
// rows; a row with more in-edges is split into chunks of kBlockEdges edges
// whose partial sums are combined, in chunk order, by a small second kernel
// (pr_finish) after the launch. A task's edges are streamed once, coalesced, and their
// messages gathered into LDS; rows are then reduced from LDS by one thread
// (short rows) or one wavefront (rows longer than kLaneRow).
#include <vector>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxRows = 1024;
constexpr int kBlockEdges = 2048;          // in-edges per work item
constexpr int kPer = kBlockEdges / kThreads;  // edges per thread, loaded together
constexpr uint32_t kLaneRow = 32;
constexpr uint32_t kNoLong = 0xFFFFFFFFu;

struct Task {
  uint32_t row_begin, row_end, edge_begin, edge_end;
  uint32_t long_id;  // split row id, or kNoLong
  uint32_t chunk;    // partial-sum slot of this chunk
};

struct LongRow {
  uint32_t row;
  uint32_t first_chunk;
  uint32_t nchunks;
  uint32_t pad;
};

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Messages of the in-edges [e0 + tid + k * kThreads] for k < kPer: all index
// loads are issued before any gather so each thread keeps kPer loads in flight.
template <bool kWeighted>
__device__ inline void gather_edges(const int32_t* __restrict__ idx, const float* __restrict__ w,
                                    const float* __restrict__ x, uint32_t e0, uint32_t ne,
                                    float (&val)[kPer]) {
  int32_t src[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t i = threadIdx.x + k * kThreads;
    src[k] = i < ne ? idx[e0 + i] : -1;
  }
  float wv[kPer];
  if constexpr (kWeighted) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t i = threadIdx.x + k * kThreads;
      wv[k] = i < ne ? w[e0 + i] : 0.0f;
    }
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) val[k] = src[k] >= 0 ? x[src[k]] : 0.0f;
  if constexpr (kWeighted) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) val[k] *= wv[k];
  }
}

template <bool kPersonal>
__device__ inline void apply_row(uint32_t v, double y, float r, int32_t seed,
                                 const float* __restrict__ inv_outdeg, float* __restrict__ x_out,
                                 float* __restrict__ rank_out) {
  double tele = 1.0;
  if constexpr (kPersonal) tele = (int32_t)v == seed ? 1.0 : 0.0;
  const float pr = (float)((double)r * tele + (1.0 - (double)r) * y);
  x_out[v] = pr * inv_outdeg[v];
  if (rank_out) rank_out[v] = pr;
}

template <bool kWeighted, bool kPersonal>
__global__ __launch_bounds__(kThreads) void pr_pull(
    const Task* __restrict__ tasks, const LongRow* __restrict__ longs,
    const uint32_t* __restrict__ in_off, const int32_t* __restrict__ in_idx,
    const float* __restrict__ in_w, const float* __restrict__ x_in,
    const float* __restrict__ inv_outdeg, float r, int32_t seed, float* __restrict__ x_out,
    float* __restrict__ rank_out, double* __restrict__ partial) {
  __shared__ float vals[kBlockEdges];
  __shared__ uint32_t offs[kMaxRows + 1];
  __shared__ double wsum[kWaves];

  const Task t = tasks[blockIdx.x];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  if (t.long_id != kNoLong) {
    // One chunk of a split row.
    float val[kPer];
    gather_edges<kWeighted>(in_idx, in_w, x_in, t.edge_begin, t.edge_end - t.edge_begin, val);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) acc += (double)val[k];
    acc = wave_sum(acc);
    if (lane == 0) wsum[wave] = acc;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int i = 0; i < kWaves; ++i) s += wsum[i];
      partial[t.chunk] = s;  // combined by pr_finish after this launch
    }
    return;
  }

  const uint32_t nrows = t.row_end - t.row_begin;
  const uint32_t e0 = t.edge_begin;
  for (uint32_t i = tid; i <= nrows; i += kThreads) offs[i] = in_off[t.row_begin + i] - e0;
  const uint32_t ne = t.edge_end - e0;
  {
    float val[kPer];
    gather_edges<kWeighted>(in_idx, in_w, x_in, e0, ne, val);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t i = tid + k * kThreads;
      if (i < ne) vals[i] = val[k];
    }
  }
  __syncthreads();

  // Short rows: one thread each, sequential sum from LDS.
  for (uint32_t i = tid; i < nrows; i += kThreads) {
    const uint32_t b = offs[i], e = offs[i + 1];
    if (e - b > kLaneRow) continue;
    double y = 0.0;
    for (uint32_t j = b; j < e; ++j) y += (double)vals[j];
    apply_row<kPersonal>(t.row_begin + i, y, r, seed, inv_outdeg, x_out, rank_out);
  }
  // Longer rows: one wavefront each.
  for (uint32_t base = wave * 64; base < nrows; base += kThreads) {
    const uint32_t i = base + lane;
    const bool longrow = i < nrows && offs[i + 1] - offs[i] > kLaneRow;
    unsigned long long mask = __ballot(longrow);
    while (mask) {
      const int j = __ffsll((long long)mask) - 1;
      mask &= mask - 1;
      const uint32_t row = base + j;
      const uint32_t b = offs[row], e = offs[row + 1];
      double y = 0.0;
      for (uint32_t k = b + lane; k < e; k += 64) y += (double)vals[k];
      y = wave_sum(y);
      if (lane == 0) apply_row<kPersonal>(t.row_begin + row, y, r, seed, inv_outdeg, x_out, rank_out);
    }
  }
}

// Rows split into chunks: sum the chunk partials in chunk order, then APPLY.
template <bool kPersonal>
__global__ void pr_finish(const LongRow* __restrict__ longs, int64_t nlong,
                          const double* __restrict__ partial, const float* __restrict__ inv_outdeg,
                          float r, int32_t seed, float* __restrict__ x_out,
                          float* __restrict__ rank_out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nlong;
       i += (int64_t)gridDim.x * blockDim.x) {
    const LongRow lr = longs[i];
    double y = 0.0;
    for (uint32_t c = 0; c < lr.nchunks; ++c) y += partial[lr.first_chunk + c];
    apply_row<kPersonal>(lr.row, y, r, seed, inv_outdeg, x_out, rank_out);
  }
}

// x_v = PR_v / outdeg(v): the first SEND of a run.
__global__ void pr_send(const float* __restrict__ rank, const float* __restrict__ inv_outdeg,
                        int64_t n, float* __restrict__ x) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    x[v] = rank[v] * inv_outdeg[v];
}

struct Schedule {
  Task* tasks = nullptr;
  LongRow* longs = nullptr;
  double* partial = nullptr;
  int64_t ntasks = 0, nlong = 0;
  float* x[2] = {nullptr, nullptr};
  int block_edges = 0;
};

Schedule* sched(gm_graph g) { return static_cast<Schedule*>(g->pr_sched); }

}  // namespace

void free_pull_schedule(gm_graph g) {
  Schedule* s = sched(g);
  if (!s) return;
  dfree(s->tasks);
  dfree(s->longs);
  dfree(s->partial);
  dfree(s->x[0]);
  dfree(s->x[1]);
  delete s;
  g->pr_sched = nullptr;
}

void ensure_pull_schedule(gm_graph g, hipStream_t st) {
  const int block_edges = kBlockEdges;
  if (sched(g)) return;
  free_pull_schedule(g);
  const int64_t n = g->n;
  std::vector<uint32_t> off(n + 1);
  GM_HIP(hipMemcpyAsync(off.data(), g->in_off, (n + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost,
                        st));
  GM_HIP(hipStreamSynchronize(st));
  std::vector<Task> tasks;
  std::vector<LongRow> longs;
  uint32_t nchunk_total = 0;
  const uint32_t B = (uint32_t)block_edges;
  int64_t r = 0;
  while (r < n) {
    const uint32_t deg = off[r + 1] - off[r];
    if (deg > B) {
      const uint32_t nch = (deg + B - 1) / B;
      const uint32_t id = (uint32_t)longs.size();
      longs.push_back({(uint32_t)r, nchunk_total, nch, 0});
      for (uint32_t c = 0; c < nch; ++c) {
        const uint32_t eb = off[r] + c * B;
        const uint32_t ee = eb + B < off[r + 1] ? eb + B : off[r + 1];
        tasks.push_back({(uint32_t)r, (uint32_t)r + 1, eb, ee, id, nchunk_total + c});
      }
      nchunk_total += nch;
      ++r;
      continue;
    }
    const int64_t r0 = r;
    uint32_t edges = 0;
    while (r < n && r - r0 < kMaxRows) {
      const uint32_t d = off[r + 1] - off[r];
      if (d > B || edges + d > B) break;
      edges += d;
      ++r;
    }
    tasks.push_back({(uint32_t)r0, (uint32_t)r, off[r0], off[r], kNoLong, 0});
  }
  Schedule* s = new Schedule();
  try {
    s->block_edges = block_edges;
    s->ntasks = (int64_t)tasks.size();
    s->nlong = (int64_t)longs.size();
    s->tasks = dalloc<Task>(tasks.size());
    s->longs = dalloc<LongRow>(longs.size());
    s->partial = dalloc<double>(nchunk_total);
    s->x[0] = dalloc<float>(n);
    s->x[1] = dalloc<float>(n);
    GM_HIP(hipMemcpyAsync(s->tasks, tasks.data(), tasks.size() * sizeof(Task),
                          hipMemcpyHostToDevice, st));
    if (!longs.empty())
      GM_HIP(hipMemcpyAsync(s->longs, longs.data(), longs.size() * sizeof(LongRow),
                            hipMemcpyHostToDevice, st));
    GM_HIP(hipStreamSynchronize(st));
  } catch (...) {
    g->pr_sched = s;
    free_pull_schedule(g);
    throw;
  }
  g->pr_sched = s;
}

void run_pagerank(gm_graph g, float r, int32_t iters, float* rank, int32_t seed, hipStream_t st) {
  ensure_pull_schedule(g, st);
  Schedule* s = sched(g);
  const int64_t n = g->n;
  {
    int64_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 65536) blocks = 65536;
    pr_send<<<(unsigned)(blocks < 1 ? 1 : blocks), kThreads, 0, st>>>(rank, g->inv_outdeg, n,
                                                                        s->x[0]);
    GM_HIP(hipGetLastError());
  }
  const bool weighted = g->wtype == GM_W_F32;
  const bool personal = seed >= 0;
  const float* w = static_cast<const float*>(g->in_w);
  for (int32_t it = 0; it < iters; ++it) {
    const float* xin = s->x[it & 1];
    float* xout = s->x[(it + 1) & 1];
    float* rout = it == iters - 1 ? rank : nullptr;
    auto launch = [&](auto kern) {
      kern<<<(unsigned)s->ntasks, kThreads, 0, st>>>(s->tasks, s->longs, g->in_off, g->in_idx, w,
                                                     xin, g->inv_outdeg, r, seed, xout, rout,
                                                     s->partial);
    };
    if (weighted && personal)
      launch(pr_pull<true, true>);
    else if (weighted)
      launch(pr_pull<true, false>);
    else if (personal)
      launch(pr_pull<false, true>);
    else
      launch(pr_pull<false, false>);
    if (s->nlong > 0) {
      const unsigned fb = (unsigned)((s->nlong + kThreads - 1) / kThreads);
      if (personal)
        pr_finish<true><<<fb, kThreads, 0, st>>>(s->longs, s->nlong, s->partial, g->inv_outdeg, r,
                                                  seed, xout, rout);
      else
        pr_finish<false><<<fb, kThreads, 0, st>>>(s->longs, s->nlong, s->partial, g->inv_outdeg,
                                                   r, seed, xout, rout);
    }
    GM_HIP(hipGetLastError());
  }
}

}  // namespace gm
