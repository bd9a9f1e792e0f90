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
// kernel per step, one pass over the CSR in canonical edge order, so the
// gradient lands in the caller's edge order with one read-modify-write per
// edge and step.
//
// Rows are scheduled like the forward pull: sorted by out-degree into
// classes with a power-of-two number of lanes per row (at most eight edges
// per lane, loads unconditional), rows longer than kChunk split into chunks
// whose partial sums a second kernel adds in chunk order. Sums in double.
#include <algorithm>
#include <vector>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kUnroll = 8;
constexpr uint32_t kChunk = kThreads * kUnroll;
constexpr int kClasses = 13;
constexpr uint32_t kClassMax[kClasses] = {0, 1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048};
constexpr int kClassLanes[kClasses] = {1, 1, 1, 1, 1, 2, 4, 8, 16, 32, 64, 256, 256};
constexpr int kClassUnroll[kClasses] = {1, 1, 2, 4, 8, 8, 8, 8, 8, 8, 8, 4, 8};

struct Chunk {
  uint32_t row;
  uint32_t edge_begin;
  uint32_t edge_end;
  uint32_t pad;
};

struct Split {
  uint32_t row;
  uint32_t first;
  uint32_t count;
  uint32_t pad;
};

struct Bins {
  int64_t nchunks;
  int64_t class_begin[kClasses];   // first position in the sorted row list
  int64_t class_rows[kClasses];
  int64_t class_block0[kClasses];  // decreases with c
};

struct VjpPlan {
  int32_t* rows = nullptr;  // rows by decreasing out-degree
  Chunk* chunks = nullptr;
  Split* splits = nullptr;
  int64_t nsplit = 0;
  double* partial = nullptr;
  float* abar[2] = {nullptr, nullptr};
  int64_t nblocks = 0;
  Bins bins{};
};

__device__ inline double group_sum(double v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Edges [b, e) of row u with `lanes` lanes (this lane starts at b + sub):
// gradient update and the sum of w * abar_next. Loads unconditional.
template <int kU>
__device__ inline double row_step(const int32_t* __restrict__ idx, const float* __restrict__ w,
                                  const float* __restrict__ abar_next, float cu,
                                  float* __restrict__ grad_w, uint32_t b, uint32_t e, int sub,
                                  int lanes) {
  double acc = 0.0;
  for (uint32_t k0 = b + sub; k0 < e; k0 += kU * lanes) {
    uint32_t k[kU];
#pragma unroll
    for (int q = 0; q < kU; ++q) {
      const uint32_t kk = k0 + q * lanes;
      k[q] = kk < e ? kk : e - 1;
    }
    int32_t v[kU];
    float wv[kU], g[kU];
#pragma unroll
    for (int q = 0; q < kU; ++q) {
      v[q] = idx[k[q]];
      wv[q] = w[k[q]];
      g[q] = grad_w[k[q]];
    }
    float a[kU];
#pragma unroll
    for (int q = 0; q < kU; ++q) a[q] = abar_next[v[q]];
#pragma unroll
    for (int q = 0; q < kU; ++q) {
      if (k0 + q * lanes < e) {
        acc += (double)wv[q] * (double)a[q];
        grad_w[k[q]] = g[q] + cu * a[q];
      }
    }
  }
  return acc;
}

template <int kU>
__device__ inline double row_step_u(int unroll, const int32_t* idx, const float* w,
                                    const float* abar_next, float cu, float* grad_w, uint32_t b,
                                    uint32_t e, int sub, int lanes) {
  switch (unroll) {
    case 1:
      return row_step<1>(idx, w, abar_next, cu, grad_w, b, e, sub, lanes);
    case 2:
      return row_step<2>(idx, w, abar_next, cu, grad_w, b, e, sub, lanes);
    case 4:
      return row_step<4>(idx, w, abar_next, cu, grad_w, b, e, sub, lanes);
    default:
      return row_step<8>(idx, w, abar_next, cu, grad_w, b, e, sub, lanes);
  }
}

__global__ __launch_bounds__(kThreads) void vjp_step(
    const int32_t* __restrict__ rows, const uint32_t* __restrict__ off,
    const int32_t* __restrict__ idx, const float* __restrict__ w, const float* __restrict__ pr_t,
    const float* __restrict__ inv_outdeg, float r, const float* __restrict__ abar_next,
    float* __restrict__ abar_cur, float* __restrict__ grad_w, const Chunk* __restrict__ chunks,
    double* __restrict__ partial, Bins bins) {
  __shared__ double wsum[kWaves];
  const int64_t blk = blockIdx.x;
  const int tid = threadIdx.x;
  const float one_r = 1.0f - r;
  if (blk < bins.nchunks) {
    const Chunk c = chunks[blk];
    const float cu = one_r * pr_t[c.row] * inv_outdeg[c.row];
    double acc = row_step<kUnroll>(idx, w, abar_next, cu, grad_w, c.edge_begin, c.edge_end, tid,
                                   kThreads);
    acc = group_sum(acc, 64);
    if ((tid & 63) == 0) wsum[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) partial[blk] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    return;
  }
  int cls = 0;
  while (blk < bins.class_block0[cls]) ++cls;
  const int lanes = kClassLanes[cls];
  if (lanes == kThreads) {
    const uint32_t u = (uint32_t)rows[bins.class_begin[cls] + (blk - bins.class_block0[cls])];
    const float cu = one_r * pr_t[u] * inv_outdeg[u];
    double acc = row_step_u<kUnroll>(kClassUnroll[cls], idx, w, abar_next, cu, grad_w, off[u],
                                     off[u + 1], tid, kThreads);
    acc = group_sum(acc, 64);
    if ((tid & 63) == 0) wsum[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0)
      abar_cur[u] = (float)((double)one_r * (double)inv_outdeg[u] *
                            ((wsum[0] + wsum[1]) + (wsum[2] + wsum[3])));
    return;
  }
  const int64_t local = (blk - bins.class_block0[cls]) * (kThreads / lanes) + tid / lanes;
  const bool valid = local < bins.class_rows[cls];
  const uint32_t u = valid ? (uint32_t)rows[bins.class_begin[cls] + local] : 0u;
  const int sub = tid % lanes;
  double acc = 0.0;
  if (valid && cls > 0) {
    const float cu = one_r * pr_t[u] * inv_outdeg[u];
    acc = row_step_u<kUnroll>(kClassUnroll[cls], idx, w, abar_next, cu, grad_w, off[u], off[u + 1],
                              sub, lanes);
  }
  acc = group_sum(acc, lanes);
  if (valid && sub == 0) abar_cur[u] = (float)((double)one_r * (double)inv_outdeg[u] * acc);
}

__global__ void vjp_finish(const Split* __restrict__ splits, int64_t nsplit,
                           const double* __restrict__ partial, const float* __restrict__ inv_outdeg,
                           float r, float* __restrict__ abar_cur) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nsplit;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Split sp = splits[i];
    double acc = 0.0;
    for (uint32_t c = 0; c < sp.count; ++c) acc += partial[sp.first + c];
    abar_cur[sp.row] = (float)((1.0 - (double)r) * (double)inv_outdeg[sp.row] * acc);
  }
}

__global__ void copy_f32(const float* __restrict__ a, int64_t n, float* __restrict__ b) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
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
  const int64_t n = g->n;
  std::vector<uint32_t> off(n + 1);
  GM_HIP(hipMemcpyAsync(off.data(), g->out_off, (n + 1) * 4, hipMemcpyDeviceToHost, st));
  GM_HIP(hipStreamSynchronize(st));
  const uint32_t maxd = (uint32_t)g->max_out;
  std::vector<int64_t> cnt((size_t)maxd + 2, 0);
  for (int64_t v = 0; v < n; ++v) ++cnt[maxd - (off[v + 1] - off[v])];
  int64_t acc = 0;
  for (auto& c : cnt) {
    const int64_t t = c;
    c = acc;
    acc += t;
  }
  std::vector<int32_t> rows(n);
  for (int64_t v = 0; v < n; ++v) rows[cnt[maxd - (off[v + 1] - off[v])]++] = (int32_t)v;
  auto deg = [&](int64_t i) { return off[rows[i] + 1] - off[rows[i]]; };
  VjpPlan* p = new VjpPlan();
  g->vjp_plan = p;
  try {
    std::vector<Chunk> chunks;
    std::vector<Split> splits;
    int64_t i = 0;
    while (i < n && deg(i) > kChunk) {
      const uint32_t u = (uint32_t)rows[i];
      const uint32_t nch = (deg(i) + kChunk - 1) / kChunk;
      splits.push_back({u, (uint32_t)chunks.size(), nch, 0});
      for (uint32_t c = 0; c < nch; ++c) {
        const uint32_t eb = off[u] + c * kChunk;
        chunks.push_back({u, eb, std::min(eb + kChunk, off[u + 1]), 0});
      }
      ++i;
    }
    p->bins.nchunks = (int64_t)chunks.size();
    p->nsplit = (int64_t)splits.size();
    int64_t block = p->bins.nchunks;
    for (int c = kClasses - 1; c >= 0; --c) {
      const int64_t r0 = i;
      if (c == 0)
        i = n;
      else
        while (i < n && deg(i) > kClassMax[c - 1]) ++i;
      p->bins.class_begin[c] = r0;
      p->bins.class_rows[c] = i - r0;
      p->bins.class_block0[c] = block;
      const int64_t rpb = kThreads / kClassLanes[c];
      block += (p->bins.class_rows[c] + rpb - 1) / rpb;
    }
    p->nblocks = block;
    p->rows = dalloc<int32_t>(n);
    p->chunks = dalloc<Chunk>(chunks.size());
    p->splits = dalloc<Split>(splits.size());
    p->partial = dalloc<double>(chunks.size());
    p->abar[0] = dalloc<float>(n);
    p->abar[1] = dalloc<float>(n);
    GM_HIP(hipMemcpyAsync(p->rows, rows.data(), n * 4, hipMemcpyHostToDevice, st));
    if (!chunks.empty())
      GM_HIP(hipMemcpyAsync(p->chunks, chunks.data(), chunks.size() * sizeof(Chunk),
                            hipMemcpyHostToDevice, st));
    if (!splits.empty())
      GM_HIP(hipMemcpyAsync(p->splits, splits.data(), splits.size() * sizeof(Split),
                            hipMemcpyHostToDevice, st));
    GM_HIP(hipStreamSynchronize(st));
  } catch (...) {
    free_vjp_plan(g);
    throw;
  }
  return p;
}

}  // namespace

void free_vjp_plan(gm_graph g) {
  VjpPlan* p = plan(g);
  if (!p) return;
  dfree(p->rows);
  dfree(p->chunks);
  dfree(p->splits);
  dfree(p->partial);
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
  fill_u32(reinterpret_cast<uint32_t*>(grad_w), m, 0u, st);
  copy_f32<<<blocks_for(n), kThreads, 0, st>>>(grad_out, n, p->abar[0]);  // abar^T = c
  GM_HIP(hipGetLastError());
  int cur = 0;
  for (int32_t t = T - 1; t >= 0; --t) {
    const float* an = p->abar[cur];
    float* ac = p->abar[cur ^ 1];
    if (p->nblocks > 0)
      vjp_step<<<(unsigned)p->nblocks, kThreads, 0, st>>>(p->rows, g->out_off, g->out_idx, w,
                                                          hist + (int64_t)t * n, g->inv_outdeg, r,
                                                          an, ac, grad_w, p->chunks, p->partial,
                                                          p->bins);
    if (p->nsplit > 0)
      vjp_finish<<<(unsigned)((p->nsplit + kThreads - 1) / kThreads), kThreads, 0, st>>>(
          p->splits, p->nsplit, p->partial, g->inv_outdeg, r, ac);
    GM_HIP(hipGetLastError());
    cur ^= 1;
  }
}

}  // namespace gm
