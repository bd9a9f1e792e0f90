// PageRank (Sec. 3 I, Eq. (1)) and personalised PageRank as a pull-direction
// generalized SpMV over the in-adjacency, with APPLY and the next SEND fused
// into the same kernel.
//
// One superstep = one launch of pr_pull (+ pr_finish for split rows):
//   y_v   = sum_{u -> v} x_u (* w_uv)          PROCESS = msg (* w), REDUCE = +
//   PR_v  = r * tele(v) + (1 - r) * y_v        APPLY, for every vertex
//   x'_v  = PR_v / outdeg(v)                   SEND for the next superstep
// where x_u = PR_u / outdeg(u) is the message (0 for dangling vertices, which
// send nothing). Row sums are accumulated in double in a fixed order, so the
// result does not depend on scheduling.
//
// Dense layout (built once per graph, on first use): vertices are relabelled
// in decreasing in-degree order and the in-adjacency is rebuilt in the new
// labels. Rows of similar length are then contiguous, so each degree class
// gets its own number of lanes per row (from 1 up to a wavefront, so that a
// lane gathers up to eight messages at once; the longest rows are cut into
// chunks reduced by separate wavefronts), every access to per-row data is a
// coalesced stream, and the most frequently gathered messages (high-degree
// vertices, which in RMAT graphs have high in- and out-degree alike) sit
// together at low labels: the first of them (a tuning parameter, up to
// kHotMax) are copied to LDS by every workgroup and read from there, the next
// ones stay cache resident. The
// caller's rank vector is mapped into the new labels by the first SEND and
// back after the last APPLY.
#include <algorithm>
#include <cstring>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;
constexpr int kPullThreads = 1024;  // one workgroup per CU: its LDS holds the hot messages
constexpr int kPullWaves = kPullThreads / 64;
constexpr int kUnroll = 8;  // most edges per lane; all of a lane's loads are in flight at once
constexpr int kHotMax = 32768;  // at most this many hot messages in LDS (128 KB)
constexpr uint32_t kChunk = 4096;  // rows longer than this are cut into chunks of kChunk edges

// Degree classes c = 0..kClasses-1: in-degree in (kClassMax[c-1],
// kClassMax[c]] (class 0: in-degree 0), each row taken by kClassLanes[c]
// lanes with kClassUnroll[c] edges per lane and pass. Degree ranges double
// from class to class up to 512, so at most half of a lane's load slots are
// padding; the last class (a wavefront per row, looping) reaches kChunk.
constexpr int kClasses = 12;
constexpr uint32_t kClassMax[kClasses] = {0, 1, 2, 4, 8, 16, 32, 64, 128, 256, 512, kChunk};
constexpr int kClassLanes[kClasses] = {1, 1, 1, 1, 1, 2, 4, 8, 16, 32, 64, 64};
constexpr int kClassUnroll[kClasses] = {1, 1, 2, 4, 8, 8, 8, 8, 8, 8, 8, 8};

struct SplitChunk {
  uint32_t row;  // new label
  uint32_t edge_begin;
  uint32_t edge_end;
  uint32_t pad;
};

struct SplitRow {
  uint32_t row;
  uint32_t first_chunk;
  uint32_t nchunks;
  uint32_t pad;
};

// Work units of one superstep, one wavefront each: the chunks of split rows
// first, then the classes from the longest rows (c = kClasses - 1) down to
// in-degree 1 (c = 1); a unit of class c is 64 / kClassLanes[c] consecutive
// rows. Rows with in-degree 0 are written once per run (pr_const_rows).
struct Bins {
  int64_t nchunks;
  int64_t class_begin[kClasses];  // first row (new label)
  int64_t class_rows[kClasses];
  int64_t class_unit0[kClasses];  // first unit; decreases with c (class 0: end)
  int64_t nunits;
};

struct Dense {
  int64_t n = 0, m = 0;
  int32_t* new_of = nullptr;    // old label -> new label
  int32_t* old_of = nullptr;    // new label -> old label
  uint32_t* off = nullptr;      // relabelled in-adjacency
  int32_t* idx = nullptr;
  float* w = nullptr;           // edge values in the relabelled order (weighted graphs)
  uint32_t* ceid = nullptr;     // canonical (CSR) edge id of each relabelled in-edge
  float* wdyn = nullptr;        // caller-supplied edge values, relabelled per call
  float* inv_outdeg = nullptr;  // new labels
  float* x[2] = {nullptr, nullptr};
  float* pr = nullptr;          // PR in new labels (last superstep)
  SplitChunk* chunks = nullptr;
  SplitRow* splits = nullptr;
  double* partial = nullptr;
  int64_t nsplit = 0;
  int cus = 0;                  // compute units of the device
  Bins bins{};
};

__device__ inline double group_sum(double v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <bool kPersonal>
__device__ inline void apply_row(uint32_t v, double y, float r, int32_t seed,
                                 const float* __restrict__ inv_outdeg, float* __restrict__ x_out,
                                 float* __restrict__ pr_out) {
  double tele = 1.0;
  if constexpr (kPersonal) tele = (int32_t)v == seed ? 1.0 : 0.0;
  const float pr = (float)((double)r * tele + (1.0 - (double)r) * y);
  x_out[v] = pr * inv_outdeg[v];
  if (pr_out) pr_out[v] = pr;
}

// Sum of the messages of in-edges [b, e) taken by `lanes` lanes with stride
// `lanes` (this lane starts at b + sub), kU loads in flight per lane.
// Positions past the end are clamped to the last edge and their values
// dropped by a select, so every load is unconditional and all of a lane's
// index loads, then all of its gathers, are issued back to back. Index and
// edge-value streams are read once per superstep and loaded non-temporally,
// which keeps the gathered messages in the caches. A message of a label
// below hot_n comes from the LDS copy (the lane's global gather then reads
// x[0], one line shared by all such lanes); the others from x.
template <int kU, bool kWeighted>
__device__ inline double row_partial(const int32_t* __restrict__ idx, const float* __restrict__ w,
                                     const float* __restrict__ x, const float* hot, int hot_n,
                                     uint32_t b, uint32_t e, int sub, int lanes) {
  double acc = 0.0;
  for (uint32_t k0 = b + sub; k0 < e; k0 += kU * lanes) {
    uint32_t k[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t kk = k0 + u * lanes;
      k[u] = kk < e ? kk : e - 1;
    }
    int32_t src[kU];
    float wv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      src[u] = __builtin_nontemporal_load(idx + k[u]);
      if constexpr (kWeighted) wv[u] = __builtin_nontemporal_load(w + k[u]);
    }
    float val[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const bool in_lds = src[u] < hot_n;
      const float g = x[in_lds ? 0 : src[u]];
      const float l = hot[in_lds ? src[u] : 0];
      val[u] = in_lds ? l : g;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if constexpr (kWeighted) val[u] *= wv[u];
      acc += k0 + u * lanes < e ? (double)val[u] : 0.0;
    }
  }
  return acc;
}

template <bool kWeighted>
__device__ inline double row_partial_u(int unroll, const int32_t* __restrict__ idx,
                                       const float* __restrict__ w, const float* __restrict__ x,
                                       const float* hot, int hot_n, uint32_t b, uint32_t e,
                                       int sub, int lanes) {
  switch (unroll) {
    case 1:
      return row_partial<1, kWeighted>(idx, w, x, hot, hot_n, b, e, sub, lanes);
    case 2:
      return row_partial<2, kWeighted>(idx, w, x, hot, hot_n, b, e, sub, lanes);
    case 4:
      return row_partial<4, kWeighted>(idx, w, x, hot, hot_n, b, e, sub, lanes);
    default:
      return row_partial<8, kWeighted>(idx, w, x, hot, hot_n, b, e, sub, lanes);
  }
}

// One superstep: y = A^T x (pull over in-edges), APPLY, next SEND. Each
// workgroup first copies the messages of the hottest labels to LDS, then its
// wavefronts take work units with a stride of all wavefronts of the grid.
template <bool kWeighted, bool kPersonal>
__global__ __launch_bounds__(kPullThreads) void pr_pull(
    const uint32_t* __restrict__ off, const int32_t* __restrict__ idx,
    const float* __restrict__ w, const float* __restrict__ x_in,
    const float* __restrict__ inv_outdeg, float r, int32_t seed, float* __restrict__ x_out,
    float* __restrict__ pr_out, const SplitChunk* __restrict__ chunks,
    double* __restrict__ partial, Bins bins, int hot_n) {
  extern __shared__ float hot[];  // hot_n floats
  for (int i = threadIdx.x; i < hot_n; i += kPullThreads) hot[i] = x_in[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * kPullWaves;
  for (int64_t u = (int64_t)blockIdx.x * kPullWaves + (threadIdx.x >> 6); u < bins.nunits;
       u += stride) {
    if (u < bins.nchunks) {
      // One chunk of a split row: partial sum, combined by pr_finish.
      const SplitChunk c = chunks[u];
      double acc = row_partial<kUnroll, kWeighted>(idx, w, x_in, hot, hot_n, c.edge_begin,
                                                   c.edge_end, lane, 64);
      acc = group_sum(acc, 64);
      if (lane == 0) partial[u] = acc;
      continue;
    }
    // Class of this unit: the class with the largest first unit <= u.
    int cls = 1;
    while (u < bins.class_unit0[cls]) ++cls;
    const int lanes = kClassLanes[cls];
    const int64_t local = (u - bins.class_unit0[cls]) * (64 / lanes) + lane / lanes;
    const bool valid = local < bins.class_rows[cls];
    const uint32_t row = (uint32_t)(bins.class_begin[cls] + (valid ? local : 0));
    const int sub = lane % lanes;
    double y = 0.0;
    if (valid)
      y = row_partial_u<kWeighted>(kClassUnroll[cls], idx, w, x_in, hot, hot_n, off[row],
                                   off[row + 1], sub, lanes);
    y = group_sum(y, lanes);
    if (valid && sub == 0) apply_row<kPersonal>(row, y, r, seed, inv_outdeg, x_out, pr_out);
  }
}

template <bool kPersonal>
__global__ void pr_finish(const SplitRow* __restrict__ splits, int64_t nsplit,
                          const double* __restrict__ partial, const float* __restrict__ inv_outdeg,
                          float r, int32_t seed, float* __restrict__ x_out,
                          float* __restrict__ pr_out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nsplit;
       i += (int64_t)gridDim.x * blockDim.x) {
    const SplitRow sr = splits[i];
    double y = 0.0;
    for (uint32_t c = 0; c < sr.nchunks; ++c) y += partial[sr.first_chunk + c];
    apply_row<kPersonal>(sr.row, y, r, seed, inv_outdeg, x_out, pr_out);
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

// Relabelled in-adjacency keys: (new row << b | new source), value = in-edge id.
__global__ void relabel_keys(const uint32_t* __restrict__ in_off, const int32_t* __restrict__ in_idx,
                             const int32_t* __restrict__ new_of, int64_t n, int b,
                             unsigned long long* __restrict__ keys, uint32_t* __restrict__ eid) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long row = (unsigned long long)(uint32_t)new_of[v] << b;
    for (uint32_t e = in_off[v]; e < in_off[v + 1]; ++e) {
      keys[e] = row | (uint32_t)new_of[in_idx[e]];
      eid[e] = e;
    }
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
  dfree(d->off);
  dfree(d->idx);
  dfree(d->w);
  dfree(d->ceid);
  dfree(d->wdyn);
  dfree(d->inv_outdeg);
  dfree(d->x[0]);
  dfree(d->x[1]);
  dfree(d->pr);
  dfree(d->chunks);
  dfree(d->splits);
  dfree(d->partial);
  delete d;
  g->pr_sched = nullptr;
  ++g->ws_gen;
}

void ensure_pull_schedule(gm_graph g, hipStream_t st) {
  if (dense(g)) return;
  const int64_t n = g->n, m = g->m;
  // Counting sort of the vertices by decreasing in-degree (ties by label).
  std::vector<uint32_t> off(n + 1);
  GM_HIP(hipMemcpyAsync(off.data(), g->in_off, (n + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost,
                        st));
  GM_HIP(hipStreamSynchronize(st));
  const uint32_t maxd = (uint32_t)g->max_in;
  std::vector<int64_t> cnt((size_t)maxd + 2, 0);
  for (int64_t v = 0; v < n; ++v) ++cnt[maxd - (off[v + 1] - off[v])];
  int64_t acc = 0;
  for (size_t i = 0; i < cnt.size(); ++i) {
    const int64_t c = cnt[i];
    cnt[i] = acc;
    acc += c;
  }
  std::vector<int32_t> old_of(n), new_of(n);
  for (int64_t v = 0; v < n; ++v) {
    const int64_t pos = cnt[maxd - (off[v + 1] - off[v])]++;
    old_of[pos] = (int32_t)v;
    new_of[v] = (int32_t)pos;
  }
  std::vector<uint32_t> noff(n + 1);
  noff[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t v = old_of[i];
    noff[i + 1] = noff[i] + (off[v + 1] - off[v]);
  }
  Dense* d = new Dense();
  g->pr_sched = d;
  try {
    d->n = n;
    d->m = m;
    // Split rows first, then the degree classes from long to empty rows.
    std::vector<SplitChunk> chunks;
    std::vector<SplitRow> splits;
    int64_t i = 0;
    while (i < n && noff[i + 1] - noff[i] > kChunk) {
      const uint32_t deg = noff[i + 1] - noff[i];
      const uint32_t nch = (deg + kChunk - 1) / kChunk;
      splits.push_back({(uint32_t)i, (uint32_t)chunks.size(), nch, 0});
      for (uint32_t c = 0; c < nch; ++c) {
        const uint32_t eb = noff[i] + c * kChunk;
        chunks.push_back({(uint32_t)i, eb, std::min(eb + kChunk, noff[i + 1]), 0});
      }
      ++i;
    }
    Bins& bins = d->bins;
    bins.nchunks = (int64_t)chunks.size();
    d->nsplit = (int64_t)splits.size();
    int64_t unit = bins.nchunks;
    for (int c = kClasses - 1; c >= 0; --c) {
      const int64_t r0 = i;
      if (c == 0)
        i = n;  // the rest has in-degree 0
      else
        while (i < n && noff[i + 1] - noff[i] > kClassMax[c - 1]) ++i;
      bins.class_begin[c] = r0;
      bins.class_rows[c] = i - r0;
      bins.class_unit0[c] = unit;
      if (c > 0) {
        const int64_t rpu = 64 / kClassLanes[c];
        unit += (bins.class_rows[c] + rpu - 1) / rpu;
      }
    }
    bins.nunits = unit;
    int dev = 0;
    GM_HIP(hipGetDevice(&dev));
    GM_HIP(hipDeviceGetAttribute(&d->cus, hipDeviceAttributeMultiprocessorCount, dev));
    d->new_of = dalloc<int32_t>(n);
    d->old_of = dalloc<int32_t>(n);
    d->off = dalloc<uint32_t>(n + 1);
    d->idx = dalloc<int32_t>(m);
    d->inv_outdeg = dalloc<float>(n);
    d->x[0] = dalloc<float>(n);
    d->x[1] = dalloc<float>(n);
    d->pr = dalloc<float>(n);
    d->chunks = dalloc<SplitChunk>(chunks.size());
    d->splits = dalloc<SplitRow>(splits.size());
    d->partial = dalloc<double>(chunks.size());
    GM_HIP(hipMemcpyAsync(d->new_of, new_of.data(), n * 4, hipMemcpyHostToDevice, st));
    GM_HIP(hipMemcpyAsync(d->old_of, old_of.data(), n * 4, hipMemcpyHostToDevice, st));
    GM_HIP(hipMemcpyAsync(d->off, noff.data(), (n + 1) * 4, hipMemcpyHostToDevice, st));
    if (!chunks.empty())
      GM_HIP(hipMemcpyAsync(d->chunks, chunks.data(), chunks.size() * sizeof(SplitChunk),
                            hipMemcpyHostToDevice, st));
    if (!splits.empty())
      GM_HIP(hipMemcpyAsync(d->splits, splits.data(), splits.size() * sizeof(SplitRow),
                            hipMemcpyHostToDevice, st));
    gather_f32<<<blocks_for(n), kThreads, 0, st>>>(g->inv_outdeg, d->old_of, n, d->inv_outdeg);
    GM_HIP(hipGetLastError());
    if (m > 0) {
      int b = 1;
      while ((1ll << b) < n) ++b;
      DevBuf<unsigned long long> k1(m), k2(m);
      DevBuf<uint32_t> e1(m), e2(m);
      relabel_keys<<<blocks_for(n), kThreads, 0, st>>>(g->in_off, g->in_idx, d->new_of, n, b, k1.p,
                                                       e1.p);
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
      if (g->wtype == GM_W_F32) d->w = dalloc<float>(m);
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
// with `lds` bytes of LDS each (the kernel strides over its work units), no
// more than there are units.
static unsigned pull_grid(Dense* d, size_t lds, bool weighted, bool personal) {
  const void* k = weighted ? (personal ? (const void*)pr_pull<true, true> : (const void*)pr_pull<true, false>)
                           : (personal ? (const void*)pr_pull<false, true> : (const void*)pr_pull<false, false>);
  int per_cu = 0;
  GM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kPullThreads, lds));
  const int64_t fit = (int64_t)std::max(per_cu, 1) * std::max(d->cus, 1);
  const int64_t want = (d->bins.nunits + kPullWaves - 1) / kPullWaves;
  return (unsigned)std::max<int64_t>(1, std::min(fit, want));
}

// Supersteps of (personalised, optionally weighted) PageRank from the rank
// vector `rank0` (caller labels). w: relabelled edge values or NULL. After
// the last superstep the ranks go to `rank_out`; with `hist` (T + 1 rows),
// PR^t is also written to row t for t = 1..iters.
static void pagerank_driver(gm_graph g, Dense* d, float r, int32_t iters, const float* rank0,
                            int32_t seed_new, const float* w, float* hist, float* rank_out,
                            hipStream_t st) {
  const int64_t n = g->n;
  const bool weighted = w != nullptr;
  const bool personal = seed_new >= 0;
  pr_send0<<<blocks_for(n), kThreads, 0, st>>>(rank0, d->old_of, d->inv_outdeg, n, d->x[0]);
  GM_HIP(hipGetLastError());
  const int64_t c0 = d->bins.class_begin[0], n0 = d->bins.class_rows[0];
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
  const int hot_n = (int)std::min<int64_t>(std::min<int64_t>(g->tune.pr_hot, kHotMax), n);
  const size_t lds = (size_t)hot_n * sizeof(float);
  const unsigned grid = pull_grid(d, lds, weighted, personal);
  const_rows(d->x[1], d->pr);
  for (int32_t it = 0; it < iters; ++it) {
    const float* xin = d->x[it & 1];
    float* xout = d->x[(it + 1) & 1];
    float* pout = (hist || it == iters - 1) ? d->pr : nullptr;
    auto launch = [&](auto kern) {
      if (d->bins.nunits > 0)
        kern<<<grid, kPullThreads, lds, st>>>(d->off, d->idx, w, xin, d->inv_outdeg, r, seed_new,
                                              xout, pout, d->chunks, d->partial, d->bins, hot_n);
    };
    if (weighted && personal)
      launch(pr_pull<true, true>);
    else if (weighted)
      launch(pr_pull<true, false>);
    else if (personal)
      launch(pr_pull<false, true>);
    else
      launch(pr_pull<false, false>);
    if (d->nsplit > 0) {
      const unsigned fb = (unsigned)((d->nsplit + kThreads - 1) / kThreads);
      if (personal)
        pr_finish<true><<<fb, kThreads, 0, st>>>(d->splits, d->nsplit, d->partial, d->inv_outdeg,
                                                  r, seed_new, xout, pout);
      else
        pr_finish<false><<<fb, kThreads, 0, st>>>(d->splits, d->nsplit, d->partial, d->inv_outdeg,
                                                   r, seed_new, xout, pout);
    }
    GM_HIP(hipGetLastError());
    if (it == 0) const_rows(d->x[0], nullptr);  // x[0] held PR^0 messages until now
    if (hist) {
      pr_unpermute<<<blocks_for(n), kThreads, 0, st>>>(d->pr, d->new_of, n, hist + (it + 1) * n);
      GM_HIP(hipGetLastError());
    }
  }
  if (rank_out) {
    pr_unpermute<<<blocks_for(n), kThreads, 0, st>>>(d->pr, d->new_of, n, rank_out);
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
  pagerank_driver(g, d, r, iters, rank, seed_new, g->wtype == GM_W_F32 ? d->w : nullptr, nullptr,
                  rank, st);
}

// PR^0 = 1 for every vertex, then `iters` supersteps (no allocation and no
// host synchronisation once the pull schedule exists).
void enqueue_pagerank(gm_graph g, float r, int32_t iters, float* rank, hipStream_t st) {
  Dense* d = dense(g);
  if (!d) throw Unsupported{"captured run not prepared"};
  fill_f32(rank, g->n, 1.0f, st);
  pagerank_driver(g, d, r, iters, rank, -1, g->wtype == GM_W_F32 ? d->w : nullptr, nullptr, rank,
                  st);
}

void run_pagerank_history(gm_graph g, const float* w, float r, int32_t T, float* hist,
                          hipStream_t st) {
  ensure_pull_schedule(g, st);
  Dense* d = dense(g);
  if (!d->wdyn) d->wdyn = dalloc<float>(g->m);
  if (g->m > 0) {
    gather_w<<<blocks_for(g->m), kThreads, 0, st>>>(w, d->ceid, g->m, d->wdyn);
    GM_HIP(hipGetLastError());
  }
  pagerank_driver(g, d, r, T, hist, -1, d->wdyn, hist, nullptr, st);
}

}  // namespace gm
