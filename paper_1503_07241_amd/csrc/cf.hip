// Collaborative filtering (Sec. 3 III): loss of Eq. (3) and its gradients
// with respect to the user and item factors, as generalized SpMV passes over
// the rating matrix G (users x items, uint8 ratings).
//
//   e_uv   = G_uv - p_u . p_v                          (Eq. (4), PROCESS)
//   L      = sum e_uv^2 + lambda sum |p_u|^2 + lambda sum |p_v|^2   (Eq. (3))
//   dL/dp_u = -2 sum_v e_uv p_v + 2 lambda p_u          (row pass, REDUCE +)
//   dL/dp_v = -2 sum_u e_uv p_u + 2 lambda p_v          (column pass: the
//                                                        transpose-direction
//                                                        adjoint product)
// so that the GD updates of Eqs. (5)-(6) are p <- p - (gamma / 2) dL/dp.
//
// Both passes run the same kernel over a compressed layout (rows: CSR by user;
// columns: CSC by item). A wavefront owns one work item - a segment (user or
// item) or a chunk of at most kChunk of its ratings - split into groups of G
// lanes, each lane holding four coordinates of the segment's factor in
// registers; a group takes one rating at a time, gathers the other side's
// factor row (coalesced), forms e with a shuffle-reduced FP32 dot product and
// accumulates e * p_other in double. Chunked segments write partial sums
// that a second kernel adds in chunk order. The loss is reduced per
// workgroup and then in a fixed order, so results are deterministic.
#include <algorithm>
#include <cstring>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;
constexpr uint32_t kChunk = 2048;  // ratings per work item
constexpr int kUnroll = 4;         // ratings in flight per lane group

struct CfItem {
  uint32_t seg;
  uint32_t begin;
  uint32_t end;
  int32_t partial;  // partial slot for chunked segments, -1 otherwise
};

struct CfSplit {
  uint32_t seg;
  uint32_t first;
  uint32_t count;
  uint32_t pad;
};

struct CfSide {
  CfItem* items = nullptr;
  int64_t nitems = 0;
  CfSplit* splits = nullptr;
  int64_t nsplit = 0;
  int64_t npartial = 0;
};

struct CfPlan {
  CfSide side[2];  // 0: rows (users), 1: columns (items)
  double* partial = nullptr;  // largest npartial * K of the two sides
  int64_t partial_k = 0;
  double* loss_part = nullptr;
  int64_t nloss = 0;
};

__device__ inline float group_sum_f(float v, int lanes) {
  for (int o = lanes >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wavefront per work item (a segment, or a chunk of a long one). The
// wavefront is cut into 64 / G groups of G lanes; a group takes one rating
// at a time, each of its lanes holding four coordinates of the two factor
// rows (G = K / 4 rounded up to a power of two), so one rating costs four
// multiply-adds per lane and log2(G) shuffles for the dot product. Groups
// take the item's ratings in turn, kUnroll at once; their partial gradient
// sums are combined over the groups at the end of the item.
template <bool kGrad, bool kLoss>
__global__ __launch_bounds__(kThreads) void cf_pass(
    int K, int G, const CfItem* __restrict__ items, int64_t nitems,
    const int32_t* __restrict__ other_idx, const uint8_t* __restrict__ val,
    const float* __restrict__ P_own, const float* __restrict__ P_other, float lambda,
    float scale, float* __restrict__ grad, double* __restrict__ partial,
    double* __restrict__ loss_part) {
  __shared__ double lsum[kThreads / 64];
  const int lane = threadIdx.x & 63;
  const int grp = lane / G, sub = lane % G, ngrp = 64 / G;
  const int k0 = 4 * sub;
  const int64_t it = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  double loss = 0.0;
  if (it < nitems) {  // wavefront-uniform
    const CfItem item = items[it];
    float own[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      own[c] = k0 + c < K ? P_own[(int64_t)item.seg * K + k0 + c] : 0.0f;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const uint32_t step = (uint32_t)ngrp * kUnroll;
    for (uint32_t e0 = item.begin + grp; e0 < item.end + grp; e0 += step) {
      int32_t j[kUnroll];
      float g[kUnroll];
      bool ok[kUnroll];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const uint32_t e = e0 + q * ngrp;
        ok[q] = e < item.end;
        const uint32_t ec = ok[q] ? e : item.end - 1;
        j[q] = other_idx[ec];
        g[q] = (float)val[ec];
      }
      float o[kUnroll][4];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          o[q][c] = k0 + c < K ? P_other[(int64_t)j[q] * K + k0 + c] : 0.0f;
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        float d = own[0] * o[q][0];
        d = fmaf(own[1], o[q][1], d);
        d = fmaf(own[2], o[q][2], d);
        d = fmaf(own[3], o[q][3], d);
        const double err = (double)g[q] - (double)group_sum_f(d, G);
        if (ok[q]) {
          if (kGrad) {
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += err * (double)o[q][c];
          }
          if (kLoss && sub == 0) loss += err * err;
        }
      }
    }
    if (kGrad) {
      // combine the groups: lanes with the same sub hold the same coordinates
#pragma unroll
      for (int c = 0; c < 4; ++c)
        for (int off = G; off < 64; off <<= 1) acc[c] += __shfl_xor(acc[c], off, 64);
      if (grp == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (k0 + c >= K) continue;
          if (item.partial >= 0)
            partial[(int64_t)item.partial * K + k0 + c] = acc[c];
          else
            grad[(int64_t)item.seg * K + k0 + c] = (float)((double)scale *
                (-2.0 * acc[c] + 2.0 * (double)lambda * (double)own[c]));
        }
      }
    }
  }
  if (kLoss) {
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
    if ((threadIdx.x & 63) == 0) lsum[threadIdx.x >> 6] = loss;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = (lsum[0] + lsum[1]) + (lsum[2] + lsum[3]);
  }
}

__global__ void cf_finish(int K, const CfSplit* __restrict__ splits, int64_t nsplit,
                          const double* __restrict__ partial, const float* __restrict__ P_own,
                          float lambda, float scale, float* __restrict__ grad) {
  const int64_t total = nsplit * K;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sidx = i / K;
    const int k = (int)(i - sidx * K);
    const CfSplit sp = splits[sidx];
    double acc = 0.0;
    for (uint32_t c = 0; c < sp.count; ++c) acc += partial[(int64_t)(sp.first + c) * K + k];
    const double own = P_own[(int64_t)sp.seg * K + k];
    grad[(int64_t)sp.seg * K + k] = (float)((double)scale * (-2.0 * acc + 2.0 * (double)lambda * own));
  }
}

// lambda * |P|^2 partial sums, one per block (fixed order).
__global__ void sq_norm(const float* __restrict__ P, int64_t count, double* __restrict__ part) {
  __shared__ double ws[kThreads / 64];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x = P[i];
    s += x * x;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// Sum of a double array by one workgroup in a fixed order; out[0] =
// sum(a) + lambda * (sum(b) + sum(c)) where b, c are the norm partials.
__global__ void finish_loss(const double* __restrict__ a, int64_t na, const double* __restrict__ b,
                            int64_t nb, const double* __restrict__ c, int64_t nc, double lambda,
                            double* __restrict__ out) {
  __shared__ double ws[3][kThreads];
  double sa = 0.0, sb = 0.0, sc = 0.0;
  for (int64_t i = threadIdx.x; i < na; i += kThreads) sa += a[i];
  for (int64_t i = threadIdx.x; i < nb; i += kThreads) sb += b[i];
  for (int64_t i = threadIdx.x; i < nc; i += kThreads) sc += c[i];
  ws[0][threadIdx.x] = sa;
  ws[1][threadIdx.x] = sb;
  ws[2][threadIdx.x] = sc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0, tc = 0.0;
    for (int i = 0; i < kThreads; ++i) {
      ta += ws[0][i];
      tb += ws[1][i];
      tc += ws[2][i];
    }
    *out = ta + lambda * (tb + tc);
  }
}

// Bipartite build: packed (row << bc | col) keys with ratings as values.
__global__ void bip_keys(const int32_t* __restrict__ row, const int32_t* __restrict__ col,
                         const uint8_t* __restrict__ v, int64_t m, int bc,
                         unsigned long long* __restrict__ keys, uint32_t* __restrict__ vals) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    keys[e] = ((unsigned long long)(uint32_t)row[e] << bc) | (uint32_t)col[e];
    vals[e] = v[e];
  }
}

// flag[i] = 1 if key i repeats key i-1 (duplicate rating).
__global__ void dup_flags(const unsigned long long* __restrict__ keys, int64_t m,
                          unsigned int* __restrict__ dup) {
  unsigned int d = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    d |= (i > 0 && keys[i] == keys[i - 1]) ? 1u : 0u;
  if (__syncthreads_or(d) && threadIdx.x == 0) *dup = 1u;
}

__global__ void split_keys(const unsigned long long* __restrict__ keys,
                           const uint32_t* __restrict__ vals, int64_t m, int bc,
                           int32_t* __restrict__ idx, uint8_t* __restrict__ v) {
  const unsigned long long mask = (1ull << bc) - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    idx[i] = (int32_t)(keys[i] & mask);
    v[i] = (uint8_t)vals[i];
  }
}

__global__ void swap_keys(const unsigned long long* __restrict__ keys, int64_t m, int br, int bc,
                          unsigned long long* __restrict__ out) {
  const unsigned long long cmask = (1ull << bc) - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = ((keys[i] & cmask) << br) | (keys[i] >> bc);
}

__global__ void seg_offsets(const unsigned long long* __restrict__ keys, int64_t m, int shift,
                            int64_t nseg, uint32_t* __restrict__ off) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r <= nseg;
       r += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long target = (unsigned long long)r << shift;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < target)
        lo = mid + 1;
      else
        hi = mid;
    }
    off[r] = (uint32_t)lo;
  }
}

inline unsigned blocks_for(int64_t n, int64_t cap = 65536) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

inline int bits_for(int64_t n) {
  int b = 1;
  while ((1ll << b) < n) ++b;
  return b;
}

template <class T>
struct DevBuf {
  T* p = nullptr;
  explicit DevBuf(size_t n) : p(dalloc<T>(n)) {}
  ~DevBuf() { dfree(p); }
};

void sort_pairs(unsigned long long*& k1, unsigned long long*& k2, uint32_t*& v1, uint32_t*& v2,
                int64_t m, int end_bit, hipStream_t s) {
  rocprim::double_buffer<unsigned long long> kb(k1, k2);
  rocprim::double_buffer<uint32_t> vb(v1, v2);
  size_t bytes = 0;
  GM_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kb, vb, (size_t)m, 0, end_bit, s));
  void* tmp = dmalloc(bytes);
  const hipError_t err = rocprim::radix_sort_pairs(tmp, bytes, kb, vb, (size_t)m, 0, end_bit, s);
  if (err == hipSuccess) (void)hipStreamSynchronize(s);
  dfree(tmp);
  GM_HIP(err);
  if (kb.current() != k1) std::swap(k1, k2);
  if (vb.current() != v1) std::swap(v1, v2);
}

CfSide make_side(const std::vector<uint32_t>& off, int64_t nseg, hipStream_t s) {
  std::vector<CfItem> items;
  std::vector<CfSplit> splits;
  int32_t np = 0;
  std::vector<int64_t> longs;
  for (int64_t i = 0; i < nseg; ++i)
    if (off[i + 1] - off[i] > kChunk) longs.push_back(i);
  std::sort(longs.begin(), longs.end(),
            [&](int64_t a, int64_t b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
  std::vector<uint8_t> is_long(nseg, 0);
  for (int64_t i : longs) {
    is_long[i] = 1;
    const uint32_t nch = (off[i + 1] - off[i] + kChunk - 1) / kChunk;
    splits.push_back({(uint32_t)i, (uint32_t)np, nch, 0});
    for (uint32_t c = 0; c < nch; ++c) {
      const uint32_t b = off[i] + c * kChunk;
      items.push_back({(uint32_t)i, b, std::min(b + kChunk, off[i + 1]), np++});
    }
  }
  for (int64_t i = 0; i < nseg; ++i)
    if (!is_long[i]) items.push_back({(uint32_t)i, off[i], off[i + 1], -1});
  CfSide side;
  side.nitems = (int64_t)items.size();
  side.nsplit = (int64_t)splits.size();
  side.npartial = np;
  side.items = dalloc<CfItem>(items.size());
  side.splits = dalloc<CfSplit>(splits.size());
  GM_HIP(hipMemcpyAsync(side.items, items.data(), items.size() * sizeof(CfItem),
                        hipMemcpyHostToDevice, s));
  if (!splits.empty())
    GM_HIP(hipMemcpyAsync(side.splits, splits.data(), splits.size() * sizeof(CfSplit),
                          hipMemcpyHostToDevice, s));
  GM_HIP(hipStreamSynchronize(s));  // the copies read items and splits, which end here
  return side;
}

CfPlan* plan(gm_graph g) { return static_cast<CfPlan*>(g->cf_plan); }

}  // namespace

void free_cf_plan(gm_graph g) {
  CfPlan* p = plan(g);
  if (!p) return;
  for (int i = 0; i < 2; ++i) {
    dfree(p->side[i].items);
    dfree(p->side[i].splits);
  }
  dfree(p->partial);
  dfree(p->loss_part);
  delete p;
  g->cf_plan = nullptr;
  ++g->ws_gen;
}

void build_bipartite(gm_graph g, const int32_t* row, const int32_t* col, const uint8_t* val,
                     int64_t m, hipStream_t s) {
  const int64_t nr = g->n_rows, nc = g->n_cols;
  const int br = bits_for(nr), bc = bits_for(nc);
  DevBuf<unsigned long long> k1(m), k2(m);
  DevBuf<uint32_t> v1(m), v2(m);
  {
    DevBuf<int32_t> dr(m), dc(m);
    DevBuf<uint8_t> dv(m);
    if (m > 0) {
      GM_HIP(hipMemcpyAsync(dr.p, row, m * 4, hipMemcpyHostToDevice, s));
      GM_HIP(hipMemcpyAsync(dc.p, col, m * 4, hipMemcpyHostToDevice, s));
      GM_HIP(hipMemcpyAsync(dv.p, val, m, hipMemcpyHostToDevice, s));
      bip_keys<<<blocks_for(m), kThreads, 0, s>>>(dr.p, dc.p, dv.p, m, bc, k1.p, v1.p);
      GM_HIP(hipGetLastError());
      GM_HIP(hipStreamSynchronize(s));
    }
  }
  if (m > 0) sort_pairs(k1.p, k2.p, v1.p, v2.p, m, br + bc, s);
  {
    DevBuf<unsigned int> dup(1);
    unsigned int h = 0;
    fill_u32(dup.p, 1, 0u, s);
    if (m > 0) dup_flags<<<blocks_for(m), kThreads, 0, s>>>(k1.p, m, dup.p);
    GM_HIP(hipMemcpyAsync(&h, dup.p, 4, hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    if (h) throw Unsupported{"duplicate (row, column) ratings"};
  }
  g->m = m;
  g->out_off = dalloc<uint32_t>(nr + 1);
  g->out_idx = dalloc<int32_t>(m);
  g->out_val = dalloc<uint8_t>(m);
  seg_offsets<<<blocks_for(nr + 1), kThreads, 0, s>>>(k1.p, m, bc, nr, g->out_off);
  if (m > 0) split_keys<<<blocks_for(m), kThreads, 0, s>>>(k1.p, v1.p, m, bc, g->out_idx, g->out_val);
  GM_HIP(hipGetLastError());
  if (m > 0) {
    swap_keys<<<blocks_for(m), kThreads, 0, s>>>(k1.p, m, br, bc, k2.p);
    GM_HIP(hipGetLastError());
    std::swap(k1.p, k2.p);
    sort_pairs(k1.p, k2.p, v1.p, v2.p, m, br + bc, s);
  }
  g->in_off = dalloc<uint32_t>(nc + 1);
  g->in_idx = dalloc<int32_t>(m);
  g->in_val = dalloc<uint8_t>(m);
  seg_offsets<<<blocks_for(nc + 1), kThreads, 0, s>>>(k1.p, m, br, nc, g->in_off);
  if (m > 0) split_keys<<<blocks_for(m), kThreads, 0, s>>>(k1.p, v1.p, m, br, g->in_idx, g->in_val);
  GM_HIP(hipGetLastError());
  GM_HIP(hipStreamSynchronize(s));
  g->device_bytes = (nr + 1 + nc + 1) * 4 + 2 * m * 5;
}

static CfPlan* ensure_plan(gm_graph g, int K, hipStream_t s) {
  CfPlan* p = plan(g);
  if (!p) {
    p = new CfPlan();
    g->cf_plan = p;
    try {
      for (int side = 0; side < 2; ++side) {
        const int64_t nseg = side == 0 ? g->n_rows : g->n_cols;
        std::vector<uint32_t> off(nseg + 1);
        GM_HIP(hipMemcpyAsync(off.data(), side == 0 ? g->out_off : g->in_off, (nseg + 1) * 4,
                              hipMemcpyDeviceToHost, s));
        GM_HIP(hipStreamSynchronize(s));
        p->side[side] = make_side(off, nseg, s);
      }
      GM_HIP(hipStreamSynchronize(s));
    } catch (...) {
      free_cf_plan(g);
      throw;
    }
  }
  if (p->partial_k < K) {
    dfree(p->partial);
    p->partial = nullptr;
    const int64_t np = std::max(p->side[0].npartial, p->side[1].npartial);
    p->partial = dalloc<double>((size_t)np * K);
    p->partial_k = K;
  }
  return p;
}

// Lanes per rating: four coordinates per lane, a power of two.
static int group_for(int K) {
  int G = 1;
  while (4 * G < K) G <<= 1;
  return G;
}

void run_cf_forward(gm_graph g, int K, const float* PU, const float* PV, float lambda,
                    double* loss_dev, hipStream_t s) {
  CfPlan* p = ensure_plan(g, K, s);
  const int G = group_for(K);
  const CfSide& rows = p->side[0];
  const unsigned blocks = (unsigned)((rows.nitems + kThreads / 64 - 1) / (kThreads / 64));
  const int64_t nu = g->n_rows * K, nv = g->n_cols * K;
  const unsigned bu = blocks_for(nu, 1024), bv = blocks_for(nv, 1024);
  const int64_t need = (int64_t)blocks + bu + bv;
  if (p->nloss < need) {
    dfree(p->loss_part);
    p->loss_part = nullptr;
    p->loss_part = dalloc<double>(need);
    p->nloss = need;
  }
  if (rows.nitems > 0)
    cf_pass<false, true><<<blocks, kThreads, 0, s>>>(K, G, rows.items, rows.nitems, g->out_idx,
                                                     g->out_val, PU, PV, lambda, 1.0f, nullptr,
                                                     nullptr, p->loss_part);
  sq_norm<<<bu, kThreads, 0, s>>>(PU, nu, p->loss_part + blocks);
  sq_norm<<<bv, kThreads, 0, s>>>(PV, nv, p->loss_part + blocks + bu);
  finish_loss<<<1, kThreads, 0, s>>>(p->loss_part, rows.nitems > 0 ? blocks : 0,
                                     p->loss_part + blocks, bu, p->loss_part + blocks + bu, bv,
                                     (double)lambda, loss_dev);
  GM_HIP(hipGetLastError());
}

void run_cf_backward(gm_graph g, int K, const float* PU, const float* PV, float lambda, float scale,
                     float* gPU, float* gPV, hipStream_t s) {
  CfPlan* p = ensure_plan(g, K, s);
  const int G = group_for(K);
  for (int side = 0; side < 2; ++side) {
    float* grad = side == 0 ? gPU : gPV;
    if (!grad) continue;
    const CfSide& sd = p->side[side];
    const float* own = side == 0 ? PU : PV;
    const float* other = side == 0 ? PV : PU;
    if (sd.nitems > 0) {
      const unsigned blocks = (unsigned)((sd.nitems + kThreads / 64 - 1) / (kThreads / 64));
      cf_pass<true, false><<<blocks, kThreads, 0, s>>>(
          K, G, sd.items, sd.nitems, side == 0 ? g->out_idx : g->in_idx,
          side == 0 ? g->out_val : g->in_val, own, other, lambda, scale, grad, p->partial,
          nullptr);
      GM_HIP(hipGetLastError());
    }
    if (sd.nsplit > 0) {
      cf_finish<<<blocks_for(sd.nsplit * K), kThreads, 0, s>>>(K, sd.splits, sd.nsplit, p->partial,
                                                               own, lambda, scale, grad);
      GM_HIP(hipGetLastError());
    }
  }
}

}  // namespace gm
