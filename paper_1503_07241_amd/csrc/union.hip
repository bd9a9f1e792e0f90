// Block-diagonal union of graphs: the graphs of a mixed batch become one
// graph whose adjacency matrix has them as diagonal blocks, so that one
// generalized SpMV serves all of them (the product of a block-diagonal
// matrix is the products of its blocks). Part i keeps its vertices at
// [base_i, base_i + n_i) with base_i = n_0 + ... + n_{i-1}; its edges follow
// those of the parts before it, which keeps the union's edge list sorted by
// (src, dst), i.e. in canonical order.
#include <algorithm>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

// dst[i] = src[i] + add (32-bit words: offsets, vertex ids and edge ids).
__global__ void shift_copy(const uint32_t* __restrict__ src, int64_t count, uint32_t add,
                           uint32_t* __restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i] + add;
}

void shifted(const void* src, int64_t count, uint32_t add, void* dst, hipStream_t s) {
  if (count <= 0) return;
  shift_copy<<<grid_for(count), kThreads, 0, s>>>(static_cast<const uint32_t*>(src), count, add,
                                                  static_cast<uint32_t*>(dst));
  GM_HIP(hipGetLastError());
}

void copied(const void* src, int64_t bytes, void* dst, hipStream_t s) {
  if (bytes > 0) GM_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
}

}  // namespace

void build_union(gm_graph u, const gm_graph* parts, int32_t count, hipStream_t s) {
  const int64_t n = u->n, m = u->m;
  const bool weighted = u->wtype != GM_W_NONE;
  const bool in = (u->layouts & GM_LAYOUT_IN) != 0;
  u->out_off = dalloc<uint32_t>(n + 1);
  u->out_idx = dalloc<int32_t>(m + kIdxPad);
  u->inv_outdeg = dalloc<float>(n);
  u->device_bytes = (n + 1) * 4 + m * 4 + n * 4;
  if (weighted) {
    u->out_w = dalloc<uint32_t>(m);
    u->device_bytes += m * 4;
  }
  if (in) {
    u->in_off = dalloc<uint32_t>(n + 1);
    u->in_idx = dalloc<int32_t>(m + kIdxPad);
    u->in_eid = dalloc<uint32_t>(m);
    u->device_bytes += (n + 1) * 4 + 2 * m * 4;
    if (weighted) {
      u->in_w = dalloc<uint32_t>(m);
      u->device_bytes += m * 4;
    }
  }
  int64_t vb = 0, eb = 0;
  for (int32_t i = 0; i < count; ++i) {
    const gm_graph p = parts[i];
    const int64_t pn = p->n, pm = p->m;
    // offsets: rows [vb, vb + pn); the last part also writes offset n
    const int64_t noff = i + 1 == count ? pn + 1 : pn;
    shifted(p->out_off, noff, (uint32_t)eb, u->out_off + vb, s);
    shifted(p->out_idx, pm, (uint32_t)vb, u->out_idx + eb, s);
    copied(p->inv_outdeg, pn * 4, u->inv_outdeg + vb, s);
    if (weighted) copied(p->out_w, pm * 4, static_cast<uint32_t*>(u->out_w) + eb, s);
    if (in) {
      shifted(p->in_off, noff, (uint32_t)eb, u->in_off + vb, s);
      shifted(p->in_idx, pm, (uint32_t)vb, u->in_idx + eb, s);
      shifted(p->in_eid, pm, (uint32_t)eb, u->in_eid + eb, s);
      if (weighted) copied(p->in_w, pm * 4, static_cast<uint32_t*>(u->in_w) + eb, s);
    }
    vb += pn;
    eb += pm;
  }
  GM_HIP(hipStreamSynchronize(s));
}

}  // namespace gm
