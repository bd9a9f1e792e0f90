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
// Both passes run one kernel over a compressed layout (rows: CSR by user;
// columns: CSC by item). A group of G lanes (G = K / 4 rounded up to a power
// of two) holds four coordinates each of one segment's factor row; a
// wavefront's 64 / G groups each work on a work item of their own (a
// segment, or a piece of one): a group takes its item's ratings 8 (or G) at
// a time, their indices and values loaded one step ahead by the group's
// lanes together and passed around the group, gathers the other side's
// factor rows (one 16-byte load per lane: a whole cache line per rating when
// K = 4 G), forms e with a DPP sum across the group and accumulates
// e * p_other: the terms of one step in float, the steps in double. Items
// are ordered by decreasing length, so the groups of a wavefront finish
// together. The loss adds every e^2 in double per lane, then per workgroup,
// then over the workgroups in a fixed order.
//
// The column pass gathers user rows (61 MB at the Netflix shape), more than
// an XCD's 4 MB L2: its items are cut at user-block boundaries (kUserBlock
// users) and the items of block b go to the workgroups of XCD b % 8
// (workgroups are dispatched to the eight XCDs round robin), which take them
// in block order, so each XCD gathers from about one L2-resident block at a
// time. Column items write partial sums in double; a second kernel adds an
// item's partials in a fixed order. Every sum is double and in a fixed order,
// so results do not depend on scheduling.
#include <algorithm>
#include <cstring>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
// Ratings per step of a group of G lanes: 8, or G when G is larger.
template <int G>
constexpr int ratings_per_step() {
  return G > 8 ? G : 8;
}
constexpr uint32_t kRowPiece = 1024;    // longer user segments are cut into pieces
constexpr uint32_t kColPiece = 1024;    // longest column item within a user block
constexpr uint32_t kUserBlock = 16384;  // users per block of the column pass
constexpr int kXcds = 8;                // XCDs of the device, fed round robin
constexpr unsigned kGridMax = 2048;     // at most this many workgroups per pass

// A piece of work: ratings [begin, end) of segment seg (a row or a column);
// slot >= 0: write the partial sum to partial[slot], else the gradient.
struct GroupItem {
  uint32_t seg;
  uint32_t begin;
  uint32_t end;
  int32_t slot;
};

// Segments whose gradient is the sum of partial slots [first, first + count).
struct CfSplit {
  uint32_t seg;
  uint32_t first;
  uint32_t count;
  uint32_t pad;
};

struct CfSide {
  GroupItem* items = nullptr;
  int64_t nitems = 0;
  int64_t xcd_first[kXcds + 1] = {};  // column side: items of XCD x are [first[x], first[x+1])
  CfSplit* splits = nullptr;
  int64_t nsplit = 0;
  int64_t npartial = 0;
};

struct CfPlan {
  CfSide side[2];  // 0: rows (users), 1: columns (items)
  double* partial = nullptr;  // largest npartial * K of the two sides
  int64_t partial_k = 0;
  float* grad[2] = {nullptr, nullptr};  // gradients of a descent step (grad_k columns)
  int64_t grad_k = 0;
  double* loss_part = nullptr;  // kGridMax workgroup sums, then 2 x 1024 norm sums
};

// Sum over a group of G lanes (G a power of two, at most 16) by DPP moves
// within rows of 16 lanes: swaps of neighbours and of pairs, then the mirror
// of each half row and of the row; every lane ends with the group's sum.
template <int kCtrl>
__device__ inline float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xF, 0xF, false));
}

template <int G>
__device__ inline float group_sum(float v) {
  if constexpr (G >= 2) v += dpp_move<0xB1>(v);   // quad_perm 1,0,3,2
  if constexpr (G >= 4) v += dpp_move<0x4E>(v);   // quad_perm 2,3,0,1
  if constexpr (G >= 8) v += dpp_move<0x141>(v);  // row_half_mirror
  if constexpr (G >= 16) v += dpp_move<0x140>(v); // row_mirror
  return v;
}

// Four coordinates k0..k0+3 of row r (kVec: K == 4 G, rows 16-byte aligned).
template <bool kVec>
__device__ inline float4 load4(const float* __restrict__ P, uint32_t r, int K, int k0) {
  if constexpr (kVec) {
    return *reinterpret_cast<const float4*>(P + (size_t)r * K + k0);
  } else {
    const float* p = P + (size_t)r * K;
    return make_float4(k0 < K ? p[k0] : 0.0f, k0 + 1 < K ? p[k0 + 1] : 0.0f,
                       k0 + 2 < K ? p[k0 + 2] : 0.0f, k0 + 3 < K ? p[k0 + 3] : 0.0f);
  }
}

// One pass. kGrad: accumulate sum e * p_other per item; kLoss: sum e^2;
// kXcd: items grouped by XCD (column pass), workgroup w takes the items of
// XCD w % kXcds.
template <int G, bool kVec, bool kGrad, bool kLoss, bool kXcd>
__global__ __launch_bounds__(kThreads) void cf_groups(
    int K, const GroupItem* __restrict__ items, int64_t nitems, CfSide side,
    const int32_t* __restrict__ other_idx, const uint8_t* __restrict__ val,
    const float* __restrict__ P_own, const float* __restrict__ P_other, float lambda,
    float scale, float* __restrict__ grad, double* __restrict__ partial,
    double* __restrict__ loss_part) {
  constexpr int kGroups = 64 / G;
  constexpr int kU = ratings_per_step<G>();
  __shared__ double lsum[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane % G, grp = lane / G;
  const int k0 = 4 * sub;
  int64_t first = 0, last = nitems, slot, stride;
  if constexpr (kXcd) {
    const int x = blockIdx.x % kXcds;
    first = side.xcd_first[x];
    last = side.xcd_first[x + 1];
    slot = ((int64_t)(blockIdx.x / kXcds) * kWaves + wave) * kGroups + grp;
    stride = (int64_t)(gridDim.x / kXcds) * kWaves * kGroups;
  } else {
    slot = ((int64_t)blockIdx.x * kWaves + wave) * kGroups + grp;
    stride = (int64_t)gridDim.x * kWaves * kGroups;
  }
  double loss = 0.0;
  // A step's kU indices and values are loaded by the group's lanes together
  // (lane sub holds ratings sub, sub + G, ...: one coalesced load per
  // register for the whole group) and handed to every lane of the group by
  // LDS-crossbar permutes; the next step's are loaded before this step's sums.
  constexpr int kR = kU / G;  // ratings per lane and step
  const int base = grp * G;
  for (int64_t i = first + slot; i < last; i += stride) {
    const GroupItem it = items[i];
    const float4 own = load4<kVec>(P_own, it.seg, K, k0);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int32_t jl[kR] = {};
    int32_t gl[kR] = {};
    if (it.begin < it.end) {  // a segment without ratings reads nothing
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const uint32_t e = it.begin + sub + r * G;
        const uint32_t ec = e < it.end ? e : it.begin;
        jl[r] = other_idx[ec];
        gl[r] = val[ec];
      }
    }
    for (uint32_t e0 = it.begin; e0 < it.end; e0 += kU) {
      int32_t j[kU];
      float g[kU];
#pragma unroll
      for (int q = 0; q < kU; ++q) {
        j[q] = __shfl(jl[q / G], base + q % G, 64);
        g[q] = (float)__shfl(gl[q / G], base + q % G, 64);
      }
      float4 o[kU];
#pragma unroll
      for (int q = 0; q < kU; ++q) o[q] = load4<kVec>(P_other, (uint32_t)j[q], K, k0);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const uint32_t e = e0 + kU + sub + r * G;
        const uint32_t ec = e < it.end ? e : it.begin;
        jl[r] = other_idx[ec];
        gl[r] = val[ec];
      }
      // gradient terms: a step's (at most kU) in float, the steps in double;
      // the loss: every e^2 in double (e = G_uv - d exactly)
      float st[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q = 0; q < kU; ++q) {
        float d = own.x * o[q].x;
        d = fmaf(own.y, o[q].y, d);
        d = fmaf(own.z, o[q].z, d);
        d = fmaf(own.w, o[q].w, d);
        d = group_sum<G>(d);
        const bool live = e0 + q < it.end;
        if constexpr (kGrad) {
          const float err = live ? g[q] - d : 0.0f;
          st[0] = fmaf(err, o[q].x, st[0]);
          st[1] = fmaf(err, o[q].y, st[1]);
          st[2] = fmaf(err, o[q].z, st[2]);
          st[3] = fmaf(err, o[q].w, st[3]);
        }
        if constexpr (kLoss) {
          const double err = (double)g[q] - (double)d;
          if (live && sub == 0) loss += err * err;
        }
      }
      if constexpr (kGrad) {
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += (double)st[c];
      }
    }
    if constexpr (kGrad) {
      const float ow[4] = {own.x, own.y, own.z, own.w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (k0 + c >= K) continue;
        if (it.slot >= 0)
          partial[(int64_t)it.slot * K + k0 + c] = acc[c];
        else
          grad[(int64_t)it.seg * K + k0 + c] =
              (float)((double)scale * (-2.0 * acc[c] + 2.0 * (double)lambda * (double)ow[c]));
      }
    }
  }
  if constexpr (kLoss) {
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
    if (lane == 0) lsum[wave] = loss;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kWaves; ++w) t += lsum[w];
      loss_part[blockIdx.x] = t;
    }
  }
}

// Gradient of a segment whose sum is split over partial slots (fixed order).
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

// |P|^2 partial sums, one per block (fixed order).
__global__ void sq_norm(const float* __restrict__ P, int64_t count, double* __restrict__ part) {
  __shared__ double ws[kWaves];
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

// out[0] = sum(a) + lambda * (sum(b) + sum(c)), each sum by one workgroup's
// lanes in a fixed order.
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
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      ws[0][threadIdx.x] += ws[0][threadIdx.x + h];
      ws[1][threadIdx.x] += ws[1][threadIdx.x + h];
      ws[2][threadIdx.x] += ws[2][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = ws[0][0] + lambda * (ws[1][0] + ws[2][0]);
}

// One descent step of Eqs. (5)-(6): P <- P - (gamma / 2) dL/dP.
__global__ void cf_step(float* __restrict__ P, const float* __restrict__ grad, int64_t count,
                        float half_gamma) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    P[i] = fmaf(-half_gamma, grad[i], P[i]);
}

// bounds[v * (nb + 1) + b] = first rating of column v whose user is in block
// b or later (b = 0..nb).
__global__ void col_block_bounds(const uint32_t* __restrict__ off, const int32_t* __restrict__ idx,
                                 int64_t ncols, int64_t nb, uint32_t* __restrict__ bounds) {
  const int64_t total = ncols * (nb + 1);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = i / (nb + 1), b = i - v * (nb + 1);
    const int64_t target = b * (int64_t)kUserBlock;
    uint32_t lo = off[v], hi = off[v + 1];
    while (lo < hi) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if ((int64_t)idx[mid] < target)
        lo = mid + 1;
      else
        hi = mid;
    }
    bounds[i] = lo;
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

// Row-side work items: segments of at most kRowPiece ratings are one item
// (a segment without ratings too: its gradient is the L2 term alone), longer
// ones are cut into pieces with partial slots; items ordered by decreasing
// length.
CfSide make_row_side(const std::vector<uint32_t>& off, int64_t nseg, hipStream_t s) {
  std::vector<GroupItem> items;
  std::vector<CfSplit> splits;
  int32_t np = 0;
  for (int64_t i = 0; i < nseg; ++i) {
    const uint32_t b = off[i], e = off[i + 1];
    if (e - b <= kRowPiece) {
      items.push_back({(uint32_t)i, b, e, -1});
      continue;
    }
    const uint32_t cnt = (e - b + kRowPiece - 1) / kRowPiece;
    splits.push_back({(uint32_t)i, (uint32_t)np, cnt, 0});
    for (uint32_t c = 0; c < cnt; ++c)
      items.push_back({(uint32_t)i, b + c * kRowPiece, std::min(e, b + (c + 1) * kRowPiece), np++});
  }
  std::stable_sort(items.begin(), items.end(), [](const GroupItem& a, const GroupItem& b) {
    return a.end - a.begin > b.end - b.begin;
  });
  CfSide side;
  side.nitems = (int64_t)items.size();
  side.nsplit = (int64_t)splits.size();
  side.npartial = np;
  side.xcd_first[kXcds] = side.nitems;
  side.items = dalloc<GroupItem>(items.size());
  side.splits = dalloc<CfSplit>(splits.size());
  if (!items.empty())
    GM_HIP(hipMemcpyAsync(side.items, items.data(), items.size() * sizeof(GroupItem),
                          hipMemcpyHostToDevice, s));
  if (!splits.empty())
    GM_HIP(hipMemcpyAsync(side.splits, splits.data(), splits.size() * sizeof(CfSplit),
                          hipMemcpyHostToDevice, s));
  GM_HIP(hipStreamSynchronize(s));  // the copies read the host vectors
  return side;
}

// Column-side work items: each column's ratings cut at user-block
// boundaries (and into pieces of at most kColPiece), every item with a slot
// of its own (a column's slots are consecutive, in block order); items of
// block b go to XCD b % kXcds, in block order, longest first within a block.
CfSide make_col_side(const std::vector<uint32_t>& bounds, int64_t ncols, int64_t nb,
                     hipStream_t s) {
  struct Tagged {
    GroupItem it;
    uint32_t block;
  };
  std::vector<Tagged> all;
  std::vector<CfSplit> splits;
  uint32_t np = 0;
  for (int64_t v = 0; v < ncols; ++v) {
    const uint32_t first = np;
    for (int64_t b = 0; b < nb; ++b) {
      const uint32_t lo = bounds[v * (nb + 1) + b], hi = bounds[v * (nb + 1) + b + 1];
      for (uint32_t p = lo; p < hi; p += kColPiece)
        all.push_back({{(uint32_t)v, p, std::min(hi, p + kColPiece), (int32_t)np++}, (uint32_t)b});
    }
    splits.push_back({(uint32_t)v, first, np - first, 0});
  }
  std::stable_sort(all.begin(), all.end(), [](const Tagged& a, const Tagged& b) {
    const uint32_t xa = a.block % kXcds, xb = b.block % kXcds;
    if (xa != xb) return xa < xb;
    if (a.block != b.block) return a.block < b.block;
    return a.it.end - a.it.begin > b.it.end - b.it.begin;
  });
  CfSide side;
  std::vector<GroupItem> items(all.size());
  for (size_t i = 0; i < all.size(); ++i) items[i] = all[i].it;
  for (int x = 0; x <= kXcds; ++x) {
    int64_t i = 0;
    while (i < (int64_t)all.size() && (int64_t)(all[i].block % kXcds) < x) ++i;
    side.xcd_first[x] = x == kXcds ? (int64_t)all.size() : i;
  }
  side.nitems = (int64_t)items.size();
  side.nsplit = (int64_t)splits.size();
  side.npartial = np;
  side.items = dalloc<GroupItem>(items.size());
  side.splits = dalloc<CfSplit>(splits.size());
  if (!items.empty())
    GM_HIP(hipMemcpyAsync(side.items, items.data(), items.size() * sizeof(GroupItem),
                          hipMemcpyHostToDevice, s));
  if (!splits.empty())
    GM_HIP(hipMemcpyAsync(side.splits, splits.data(), splits.size() * sizeof(CfSplit),
                          hipMemcpyHostToDevice, s));
  GM_HIP(hipStreamSynchronize(s));
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
  dfree(p->grad[0]);
  dfree(p->grad[1]);
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
      const int64_t nr = g->n_rows, nc = g->n_cols;
      std::vector<uint32_t> off(nr + 1);
      GM_HIP(hipMemcpyAsync(off.data(), g->out_off, (nr + 1) * 4, hipMemcpyDeviceToHost, s));
      GM_HIP(hipStreamSynchronize(s));
      p->side[0] = make_row_side(off, nr, s);
      const int64_t nb = (nr + kUserBlock - 1) / kUserBlock;
      std::vector<uint32_t> bounds(nc * (nb + 1));
      DevBuf<uint32_t> db(bounds.size());
      col_block_bounds<<<blocks_for((int64_t)bounds.size()), kThreads, 0, s>>>(
          g->in_off, g->in_idx, nc, nb, db.p);
      GM_HIP(hipGetLastError());
      GM_HIP(hipMemcpyAsync(bounds.data(), db.p, bounds.size() * 4, hipMemcpyDeviceToHost, s));
      GM_HIP(hipStreamSynchronize(s));
      p->side[1] = make_col_side(bounds, nc, nb, s);
      p->loss_part = dalloc<double>(kGridMax + 2 * 1024);
    } catch (...) {
      free_cf_plan(g);
      throw;
    }
  }
  if (p->partial_k < K) {
    dfree(p->partial);
    p->partial = nullptr;
    p->partial_k = 0;
    const int64_t np = std::max(p->side[0].npartial, p->side[1].npartial);
    p->partial = dalloc<double>((size_t)np * K);
    p->partial_k = K;
  }
  return p;
}

// Lanes per rating: four coordinates per lane, a power of two (K <= 64).
static int group_for(int K) {
  int G = 1;
  while (4 * G < K) G <<= 1;
  return G;
}

// Launch cf_groups for the group size and load width K needs.
template <bool kGrad, bool kLoss, bool kXcd>
static unsigned launch_pass(int K, const CfSide& sd, const int32_t* idx, const uint8_t* val,
                        const float* own, const float* other, float lambda, float scale,
                        float* grad, double* partial, double* loss_part, hipStream_t s) {
  const int G = group_for(K);
  const bool vec = K == 4 * G;
  auto go = [&](auto kern) {
    // as many workgroups as are resident at once (a multiple of kXcds): each
    // takes every grid-th item of its list
    int dev = 0, cus = 0, per_cu = 0;
    GM_HIP(hipGetDevice(&dev));
    GM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    GM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, 0));
    unsigned grid = (unsigned)std::max(1, per_cu) * (unsigned)std::max(1, cus);
    grid = std::min(kGridMax, std::max((unsigned)kXcds, grid / kXcds * kXcds));
    kern<<<grid, kThreads, 0, s>>>(K, sd.items, sd.nitems, sd, idx, val, own, other, lambda, scale,
                                   grad, partial, loss_part);
    return grid;
  };
  unsigned grid = 0;
#define GM_CF_CASE(g)                                                        \
  case g:                                                                    \
    if (vec)                                                                 \
      grid = go(cf_groups<g, true, kGrad, kLoss, kXcd>);                     \
    else                                                                     \
      grid = go(cf_groups<g, false, kGrad, kLoss, kXcd>);                    \
    break;
  switch (G) {
    GM_CF_CASE(1)
    GM_CF_CASE(2)
    GM_CF_CASE(4)
    GM_CF_CASE(8)
    GM_CF_CASE(16)
    default:
      throw Unsupported{"K above 64"};
  }
#undef GM_CF_CASE
  GM_HIP(hipGetLastError());
  return grid;
}

void run_cf_forward(gm_graph g, int K, const float* PU, const float* PV, float lambda,
                    double* loss_dev, hipStream_t s) {
  CfPlan* p = ensure_plan(g, K, s);
  const CfSide& rows = p->side[0];
  const unsigned grid = launch_pass<false, true, false>(K, rows, g->out_idx, g->out_val, PU, PV,
                                                        lambda, 1.0f, nullptr, nullptr,
                                                        p->loss_part, s);
  const int64_t nu = g->n_rows * K, nv = g->n_cols * K;
  const unsigned bu = blocks_for(nu, 1024), bv = blocks_for(nv, 1024);
  sq_norm<<<bu, kThreads, 0, s>>>(PU, nu, p->loss_part + kGridMax);
  sq_norm<<<bv, kThreads, 0, s>>>(PV, nv, p->loss_part + kGridMax + 1024);
  finish_loss<<<1, kThreads, 0, s>>>(p->loss_part, grid, p->loss_part + kGridMax, bu,
                                     p->loss_part + kGridMax + 1024, bv, (double)lambda, loss_dev);
  GM_HIP(hipGetLastError());
}

void run_cf_backward(gm_graph g, int K, const float* PU, const float* PV, float lambda, float scale,
                     float* gPU, float* gPV, hipStream_t s) {
  CfPlan* p = ensure_plan(g, K, s);
  if (gPU) {
    const CfSide& sd = p->side[0];
    launch_pass<true, false, false>(K, sd, g->out_idx, g->out_val, PU, PV, lambda, scale, gPU,
                                    p->partial, nullptr, s);
    if (sd.nsplit > 0) {
      cf_finish<<<blocks_for(sd.nsplit * K), kThreads, 0, s>>>(K, sd.splits, sd.nsplit, p->partial,
                                                               PU, lambda, scale, gPU);
      GM_HIP(hipGetLastError());
    }
  }
  if (gPV) {
    const CfSide& sd = p->side[1];
    launch_pass<true, false, true>(K, sd, g->in_idx, g->in_val, PV, PU, lambda, scale, gPV,
                                   p->partial, nullptr, s);
    if (sd.nsplit > 0) {
      cf_finish<<<blocks_for(sd.nsplit * K), kThreads, 0, s>>>(K, sd.splits, sd.nsplit, p->partial,
                                                               PV, lambda, scale, gPV);
      GM_HIP(hipGetLastError());
    }
  }
}

void run_cf_gd(gm_graph g, int K, float* PU, float* PV, float lambda, float gamma, int32_t iters,
               double* loss_hist, hipStream_t s) {
  CfPlan* p = ensure_plan(g, K, s);
  const int64_t nu = g->n_rows * K, nv = g->n_cols * K;
  if (p->grad_k < K) {
    dfree(p->grad[0]);
    dfree(p->grad[1]);
    p->grad[0] = p->grad[1] = nullptr;
    p->grad_k = 0;
    p->grad[0] = dalloc<float>(nu);
    p->grad[1] = dalloc<float>(nv);
    p->grad_k = K;
  }
  for (int32_t t = 0; t < iters; ++t) {
    if (loss_hist) run_cf_forward(g, K, PU, PV, lambda, loss_hist + t, s);
    run_cf_backward(g, K, PU, PV, lambda, 1.0f, p->grad[0], p->grad[1], s);
    cf_step<<<blocks_for(nu), kThreads, 0, s>>>(PU, p->grad[0], nu, 0.5f * gamma);
    cf_step<<<blocks_for(nv), kThreads, 0, s>>>(PV, p->grad[1], nv, 0.5f * gamma);
    GM_HIP(hipGetLastError());
  }
  if (loss_hist) run_cf_forward(g, K, PU, PV, lambda, loss_hist + iters, s);
}

}  // namespace gm
