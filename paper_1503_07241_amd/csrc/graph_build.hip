// Device-side graph construction: raw edge list -> sorted, deduplicated
// out-adjacency (CSR of G, i.e. the columns of G^T that Alg. 1 walks) and
// in-adjacency (CSC of G), with the preprocessing of Sec. 5.1.
//
// Loading is not part of the measured path (the paper excludes it, Sec. 5.2).
// The two global key sorts use rocPRIM's radix sort; every other step is a
// kernel of this file.
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n, int threads = kThreads) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > (1ll << 30)) b = 1ll << 30;
  return (unsigned)b;
}

// Number of bits that hold a vertex id in [0, n).
inline int id_bits(int64_t n) {
  int b = 1;
  while ((1ll << b) < n) ++b;
  return b;
}

// Edge e of the raw list -> packed (row << b | col) key(s); keys of dropped
// edges get bit 2b set so they sort after every kept key.
__global__ void make_keys(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                          const uint32_t* __restrict__ wbits, int64_t m, int b, uint32_t prep,
                          unsigned long long* __restrict__ keys, uint32_t* __restrict__ vals,
                          unsigned long long* __restrict__ dropped) {
  const unsigned long long invalid = 1ull << (2 * b);
  unsigned long long local_drop = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t s = (uint32_t)src[e], d = (uint32_t)dst[e];
    const bool loop = s == d;
    const bool drop_loop = loop && (prep & (GM_PREP_DROP_SELF_LOOPS | GM_PREP_UPPER_DAG));
    if (prep & GM_PREP_UPPER_DAG) {
      const uint64_t lo = s < d ? s : d, hi = s < d ? d : s;
      keys[e] = drop_loop ? invalid : ((lo << b) | hi);
      if (vals) vals[e] = wbits[e];
      local_drop += drop_loop;
    } else if (prep & GM_PREP_SYMMETRIZE) {
      keys[e] = drop_loop ? invalid : ((s << b) | d);
      keys[m + e] = (drop_loop || loop) ? invalid : ((d << b) | s);
      if (vals) {
        vals[e] = wbits[e];
        vals[m + e] = wbits[e];
      }
      local_drop += drop_loop + (drop_loop || loop);
    } else {
      keys[e] = drop_loop ? invalid : ((s << b) | d);
      if (vals) vals[e] = wbits[e];
      local_drop += drop_loop;
    }
  }
  for (int o = 32; o > 0; o >>= 1) local_drop += __shfl_xor(local_drop, o, 64);
  if ((threadIdx.x & 63) == 0 && local_drop) atomicAdd(dropped, local_drop);
}

__global__ void head_flags(const unsigned long long* __restrict__ keys, int64_t k,
                           uint32_t* __restrict__ flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k;
       i += (int64_t)gridDim.x * blockDim.x)
    flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// Compact the heads: unique key, smallest value of its run.
template <bool kFloat>
__global__ void compact_unique(const unsigned long long* __restrict__ keys,
                               const uint32_t* __restrict__ vals, const uint32_t* __restrict__ flag,
                               const unsigned long long* __restrict__ pos, int64_t k,
                               unsigned long long* __restrict__ ukeys, uint32_t* __restrict__ uvals) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[i]) continue;
    const unsigned long long key = keys[i];
    const uint64_t p = pos[i];
    ukeys[p] = key;
    if (vals) {
      uint32_t best = vals[i];
      for (int64_t j = i + 1; j < k && keys[j] == key; ++j) {
        const uint32_t v = vals[j];
        if (kFloat) {
          if (__uint_as_float(v) < __uint_as_float(best)) best = v;
        } else if (v < best) {
          best = v;
        }
      }
      uvals[p] = best;
    }
  }
}

// off[r] = first index i with (key[i] >> b) >= r, for r in [0, n].
__global__ void row_offsets(const unsigned long long* __restrict__ keys, int64_t k, int b,
                            int64_t n, uint32_t* __restrict__ off) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r <= n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long target = (unsigned long long)r << b;
    int64_t lo = 0, hi = k;
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

__global__ void low_ids(const unsigned long long* __restrict__ keys, int64_t k, int b,
                        int32_t* __restrict__ out) {
  const unsigned long long mask = (1ull << b) - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int32_t)(keys[i] & mask);
}

// Transposed keys (col << b | row) of the canonical edges, value = edge id.
__global__ void transpose_keys(const unsigned long long* __restrict__ keys, int64_t k, int b,
                               unsigned long long* __restrict__ tkeys, uint32_t* __restrict__ eid) {
  const unsigned long long mask = (1ull << b) - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k;
       i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long key = keys[i];
    tkeys[i] = ((key & mask) << b) | (key >> b);
    eid[i] = (uint32_t)i;
  }
}

__global__ void gather_u32(const uint32_t* __restrict__ src, const uint32_t* __restrict__ idx,
                           int64_t k, uint32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = src[idx[i]];
}

// Per-vertex 1/degree, plus the largest degree (stats[0]) and the number of
// vertices with nonzero degree (stats[1]).
__global__ void degree_stats(const uint32_t* __restrict__ off, int64_t n,
                             float* __restrict__ inv_deg, unsigned int* __restrict__ stats) {
  unsigned int local = 0, nz = 0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t d = off[v + 1] - off[v];
    if (inv_deg) inv_deg[v] = d ? 1.0f / (float)d : 0.0f;
    local = d > local ? d : local;
    nz += d != 0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned int t = __shfl_xor(local, o, 64);
    local = t > local ? t : local;
    nz += __shfl_xor(nz, o, 64);
  }
  if ((threadIdx.x & 63) == 0 && local) {
    atomicMax(&stats[0], local);
    atomicAdd(&stats[1], nz);
  }
}

struct Scratch {
  void* p = nullptr;
  ~Scratch() { dfree(p); }
};

void radix_sort(unsigned long long*& keys, unsigned long long*& alt, uint32_t*& vals,
                uint32_t*& valt, int64_t k, int end_bit, hipStream_t s) {
  rocprim::double_buffer<unsigned long long> kb(keys, alt);
  size_t bytes = 0;
  Scratch tmp;
  if (vals) {
    rocprim::double_buffer<uint32_t> vb(vals, valt);
    GM_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kb, vb, (size_t)k, 0, end_bit, s));
    tmp.p = dmalloc(bytes);
    GM_HIP(rocprim::radix_sort_pairs(tmp.p, bytes, kb, vb, (size_t)k, 0, end_bit, s));
    if (vb.current() != vals) std::swap(vals, valt);
  } else {
    GM_HIP(rocprim::radix_sort_keys(nullptr, bytes, kb, (size_t)k, 0, end_bit, s));
    tmp.p = dmalloc(bytes);
    GM_HIP(rocprim::radix_sort_keys(tmp.p, bytes, kb, (size_t)k, 0, end_bit, s));
  }
  if (kb.current() != keys) std::swap(keys, alt);
  GM_HIP(hipStreamSynchronize(s));
}

template <class T>
struct DevBuf {
  T* p = nullptr;
  explicit DevBuf(size_t n) : p(dalloc<T>(n)) {}
  ~DevBuf() { dfree(p); }
  T* release() {
    T* q = p;
    p = nullptr;
    return q;
  }
};

}  // namespace

void build_graph(gm_graph g, const int32_t* src, const int32_t* dst, const void* w, int64_t m_in,
                 hipStream_t s) {
  const int64_t n = g->n;
  const int b = id_bits(n);
  const bool sym = (g->prep & GM_PREP_SYMMETRIZE) && !(g->prep & GM_PREP_UPPER_DAG);
  const int64_t k = sym ? 2 * m_in : m_in;
  const bool weighted = g->wtype != GM_W_NONE;

  DevBuf<unsigned long long> keys(k), alt(k);
  DevBuf<uint32_t> vals(weighted ? k : 0), valt(weighted ? k : 0);
  uint32_t* vp = weighted ? vals.p : nullptr;
  uint32_t* vq = weighted ? valt.p : nullptr;
  DevBuf<unsigned long long> counter(1);
  GM_HIP(hipMemsetAsync(counter.p, 0, sizeof(unsigned long long), s));
  {
    // Raw list upload; the temporaries live only for the key pass.
    DevBuf<int32_t> dsrc(m_in), ddst(m_in);
    DevBuf<uint32_t> dw(weighted ? m_in : 0);
    if (m_in > 0) {
      GM_HIP(hipMemcpyAsync(dsrc.p, src, m_in * sizeof(int32_t), hipMemcpyHostToDevice, s));
      GM_HIP(hipMemcpyAsync(ddst.p, dst, m_in * sizeof(int32_t), hipMemcpyHostToDevice, s));
      if (weighted)
        GM_HIP(hipMemcpyAsync(dw.p, w, m_in * sizeof(uint32_t), hipMemcpyHostToDevice, s));
      make_keys<<<grid_for(m_in), kThreads, 0, s>>>(dsrc.p, ddst.p, weighted ? dw.p : nullptr, m_in,
                                                    b, g->prep, keys.p, vp, counter.p);
      GM_HIP(hipGetLastError());
    }
    GM_HIP(hipStreamSynchronize(s));
  }
  unsigned long long dropped = 0;
  GM_HIP(hipMemcpy(&dropped, counter.p, sizeof(dropped), hipMemcpyDeviceToHost));
  const int64_t kv = k - (int64_t)dropped;  // kept keys (still with duplicates)

  if (k > 0) radix_sort(keys.p, alt.p, vp, vq, k, 2 * b + 1, s);

  // Unique (row, col) pairs; a duplicate keeps its smallest value.
  int64_t m = 0;
  DevBuf<unsigned long long> ukeys(kv);
  DevBuf<uint32_t> uvals(weighted ? kv : 0);
  if (kv > 0) {
    DevBuf<uint32_t> flag(kv);
    DevBuf<unsigned long long> pos(kv);
    head_flags<<<grid_for(kv), kThreads, 0, s>>>(keys.p, kv, flag.p);
    GM_HIP(hipGetLastError());
    size_t bytes = 0;
    GM_HIP(rocprim::exclusive_scan(nullptr, bytes, flag.p, pos.p, 0ull, (size_t)kv,
                                   rocprim::plus<unsigned long long>(), s));
    Scratch tmp;
    tmp.p = dmalloc(bytes);
    GM_HIP(rocprim::exclusive_scan(tmp.p, bytes, flag.p, pos.p, 0ull, (size_t)kv,
                                   rocprim::plus<unsigned long long>(), s));
    if (g->wtype == GM_W_F32)
      compact_unique<true><<<grid_for(kv), kThreads, 0, s>>>(keys.p, vp, flag.p, pos.p, kv, ukeys.p,
                                                             uvals.p);
    else
      compact_unique<false><<<grid_for(kv), kThreads, 0, s>>>(keys.p, vp, flag.p, pos.p, kv,
                                                              ukeys.p, weighted ? uvals.p : nullptr);
    GM_HIP(hipGetLastError());
    unsigned long long last_pos = 0;
    uint32_t last_flag = 0;
    GM_HIP(hipMemcpyAsync(&last_pos, pos.p + kv - 1, sizeof(last_pos), hipMemcpyDeviceToHost, s));
    GM_HIP(hipMemcpyAsync(&last_flag, flag.p + kv - 1, sizeof(last_flag), hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    m = (int64_t)last_pos + last_flag;
  }
  if (m > (int64_t)UINT32_MAX) throw Unsupported{"more than 2^32-1 edges after preprocessing"};
  g->m = m;
  // Release the sort buffers before allocating the adjacency.
  {
    DevBuf<unsigned long long> k1(0), k2(0);
    std::swap(k1.p, keys.p);
    std::swap(k2.p, alt.p);
    DevBuf<uint32_t> v1(0), v2(0);
    std::swap(v1.p, vals.p);
    std::swap(v2.p, valt.p);
  }

  DevBuf<unsigned int> maxdeg(2);
  // Out-adjacency (always built: it fixes the canonical edge order).
  {
    DevBuf<uint32_t> off(n + 1);
    DevBuf<int32_t> idx(m + kIdxPad);
    row_offsets<<<grid_for(n + 1), kThreads, 0, s>>>(ukeys.p, m, b, n, off.p);
    if (m > 0) low_ids<<<grid_for(m), kThreads, 0, s>>>(ukeys.p, m, b, idx.p);
    GM_HIP(hipGetLastError());
    DevBuf<float> inv(n);
    GM_HIP(hipMemsetAsync(maxdeg.p, 0, 2 * sizeof(unsigned int), s));
    degree_stats<<<grid_for(n), kThreads, 0, s>>>(off.p, n, inv.p, maxdeg.p);
    GM_HIP(hipGetLastError());
    unsigned int mx[2] = {0, 0};
    GM_HIP(hipMemcpyAsync(mx, maxdeg.p, sizeof(mx), hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    g->max_out = mx[0];
    g->n_src = mx[1];
    g->out_off = off.release();
    g->out_idx = idx.release();
    g->inv_outdeg = inv.release();
    g->device_bytes += (n + 1) * 4 + m * 4 + n * 4;
    if (weighted) {
      g->out_w = uvals.release();
      g->device_bytes += m * 4;
    }
  }
  // In-adjacency.
  if (g->layouts & GM_LAYOUT_IN) {
    DevBuf<unsigned long long> tk(m), tk2(m);
    DevBuf<uint32_t> eid(m), eid2(m);
    if (m > 0) {
      transpose_keys<<<grid_for(m), kThreads, 0, s>>>(ukeys.p, m, b, tk.p, eid.p);
      GM_HIP(hipGetLastError());
      uint32_t* ep = eid.p;
      uint32_t* eq = eid2.p;
      radix_sort(tk.p, tk2.p, ep, eq, m, 2 * b, s);
      eid.p = ep;
      eid2.p = eq;
    }
    DevBuf<uint32_t> off(n + 1);
    DevBuf<int32_t> idx(m + kIdxPad);
    row_offsets<<<grid_for(n + 1), kThreads, 0, s>>>(tk.p, m, b, n, off.p);
    if (m > 0) low_ids<<<grid_for(m), kThreads, 0, s>>>(tk.p, m, b, idx.p);
    GM_HIP(hipGetLastError());
    if (weighted && m > 0) {
      DevBuf<uint32_t> iw(m);
      gather_u32<<<grid_for(m), kThreads, 0, s>>>(static_cast<const uint32_t*>(g->out_w), eid.p, m,
                                                  iw.p);
      GM_HIP(hipGetLastError());
      g->in_w = iw.release();
      g->device_bytes += m * 4;
    }
    GM_HIP(hipMemsetAsync(maxdeg.p, 0, 2 * sizeof(unsigned int), s));
    degree_stats<<<grid_for(n), kThreads, 0, s>>>(off.p, n, nullptr, maxdeg.p);
    GM_HIP(hipGetLastError());
    unsigned int mx[2] = {0, 0};
    GM_HIP(hipMemcpyAsync(mx, maxdeg.p, sizeof(mx), hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    g->max_in = mx[0];
    g->n_dst = mx[1];
    g->in_off = off.release();
    g->in_idx = idx.release();
    g->in_eid = eid.release();
    g->device_bytes += (n + 1) * 4 + 2 * m * 4;
  }
}

void free_graph_memory(gm_graph g) {
  dfree(g->out_off);
  dfree(g->out_idx);
  dfree(g->out_w);
  dfree(g->in_off);
  dfree(g->in_idx);
  dfree(g->in_w);
  dfree(g->in_eid);
  dfree(g->inv_outdeg);
  dfree(g->out_val);
  dfree(g->in_val);
  g->out_val = g->in_val = nullptr;
  g->out_off = g->in_off = g->in_eid = nullptr;
  g->out_idx = g->in_idx = nullptr;
  g->out_w = g->in_w = nullptr;
  g->inv_outdeg = nullptr;
}

}  // namespace gm
