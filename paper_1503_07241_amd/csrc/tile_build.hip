// Device build of the edge-tile layout that PageRank's pull superstep and
// the transpose pass of its reverse mode share: the vertices relabelled by
// decreasing degree (ties by label, so that rows with edges are the labels
// [0, rows)), the row offsets in the new labels, the row-start bitmap, the
// row of each tile's first edge and the rows that span tiles. Everything is
// computed by kernels and rocPRIM calls; the host reads back two counts.
#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "gm_internal.h"
#include "tiles.h"

namespace gm {
namespace tiles {
namespace {

constexpr int kThr = 256;

unsigned grid(int64_t n) {
  int64_t b = (n + kThr - 1) / kThr;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

#define GRID_LOOP(i, n)                                                     \
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); \
       i += (int64_t)gridDim.x * blockDim.x)

// Sort keys: maxd - degree, so an ascending stable sort orders the vertices
// by decreasing degree, equal degrees by label.
__global__ void degree_keys(const uint32_t* __restrict__ off, int64_t n, uint32_t maxd,
                            uint32_t* __restrict__ key, int32_t* __restrict__ val) {
  GRID_LOOP(v, n) {
    key[v] = maxd - (off[v + 1] - off[v]);
    val[v] = (int32_t)v;
  }
}

// new_of from old_of, and the degree of each new label (entry n: 0, so an
// exclusive scan over n + 1 entries ends with m).
__global__ void invert_and_degrees(const uint32_t* __restrict__ off,
                                   const int32_t* __restrict__ old_of, int64_t n,
                                   int32_t* __restrict__ new_of, uint32_t* __restrict__ deg) {
  GRID_LOOP(i, n + 1) {
    if (i == n) {
      deg[n] = 0;
    } else {
      const int32_t v = old_of[i];
      new_of[v] = (int32_t)i;
      deg[i] = off[v + 1] - off[v];
    }
  }
}

__global__ void fill_words(uint32_t* __restrict__ a, int64_t n, uint32_t value) {
  GRID_LOOP(i, n) a[i] = value;
}

// Per new label u: its bit in the row-start bitmap, whether it spans tiles
// (flag, entry n: 0) and, for the last row with edges, rows = u + 1; bit m
// of the bitmap marks the end of the last row.
__global__ void row_marks(const uint32_t* __restrict__ noff, int64_t n, int64_t m,
                          uint32_t* __restrict__ starts, uint32_t* __restrict__ flag,
                          unsigned long long* __restrict__ rows_out) {
  GRID_LOOP(u, n + 1) {
    uint32_t f = 0;
    if (u < n) {
      const uint32_t a = noff[u], b = noff[u + 1];
      if (b > a) {
        atomicOr(&starts[a >> 5], 1u << (a & 31));
        f = (int64_t)a / kTile != (int64_t)(b - 1) / kTile ? 1u : 0u;
        if (u + 1 == n || noff[u + 2] == b) *rows_out = (unsigned long long)(u + 1);
      }
    } else {
      atomicOr(&starts[m >> 5], 1u << (m & 31));
    }
    flag[u] = f;
  }
}

// Row of the first edge of each tile: the last row with edges whose first
// edge is at or before it.
__global__ void first_rows(const uint32_t* __restrict__ noff, int64_t rows, int64_t ntiles,
                           uint32_t* __restrict__ tile_row) {
  GRID_LOOP(t, ntiles) {
    const uint32_t e = (uint32_t)(t * kTile);
    int64_t lo = 0, hi = rows - 1;  // noff[lo] <= e always (noff[0] = 0)
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (noff[mid] <= e)
        lo = mid;
      else
        hi = mid - 1;
    }
    tile_row[t] = (uint32_t)lo;
  }
}

__global__ void cross_rows(const uint32_t* __restrict__ noff, const uint32_t* __restrict__ flag,
                           const uint32_t* __restrict__ pos, int64_t n,
                           Cross* __restrict__ cross) {
  GRID_LOOP(u, n) {
    if (flag[u]) {
      const uint32_t a = noff[u], b = noff[u + 1];
      cross[pos[u]] = Cross{(uint32_t)u, (uint32_t)((int64_t)a / kTile),
                            (uint32_t)((int64_t)(b - 1) / kTile), 0u};
    }
  }
}

template <class T>
struct Tmp {
  T* p = nullptr;
  explicit Tmp(size_t count) : p(dalloc<T>(count)) {}
  ~Tmp() { dfree(p); }
  Tmp(const Tmp&) = delete;
  Tmp& operator=(const Tmp&) = delete;
};

}  // namespace

void free_device_layout(DeviceLayout* L) {
  dfree(L->old_of);
  dfree(L->new_of);
  dfree(L->noff);
  dfree(L->starts);
  dfree(L->tile_row);
  dfree(L->cross);
  *L = DeviceLayout{};
}

DeviceLayout build_device_layout(const uint32_t* off, int64_t n, int64_t m, uint32_t maxd,
                                 hipStream_t st) {
  DeviceLayout L;
  L.ntiles = (m + kTile - 1) / kTile;
  L.mpad = L.ntiles * kTile;
  const int64_t words = L.mpad / 32 + 1;
  try {
    L.old_of = dalloc<int32_t>(n);
    L.new_of = dalloc<int32_t>(n);
    L.noff = dalloc<uint32_t>(n + 1);
    L.starts = dalloc<uint32_t>(words);
    L.tile_row = dalloc<uint32_t>(L.ntiles);
    Tmp<uint32_t> deg(n + 1), flag(n + 1), pos(n + 1);
    Tmp<unsigned long long> counts(2);
    {
      int bits = 1;
      while (bits < 32 && ((int64_t)1 << bits) <= (int64_t)maxd) ++bits;
      Tmp<uint32_t> k1(n), k2(n);
      Tmp<int32_t> v1(n);
      degree_keys<<<grid(n), kThr, 0, st>>>(off, n, maxd, k1.p, v1.p);
      GM_HIP(hipGetLastError());
      size_t bytes = 0;
      GM_HIP(rocprim::radix_sort_pairs(nullptr, bytes, k1.p, k2.p, v1.p, L.old_of, (size_t)n, 0,
                                       bits, st));
      Tmp<unsigned char> tmp(bytes);
      GM_HIP(rocprim::radix_sort_pairs(tmp.p, bytes, k1.p, k2.p, v1.p, L.old_of, (size_t)n, 0,
                                       bits, st));
      invert_and_degrees<<<grid(n + 1), kThr, 0, st>>>(off, L.old_of, n, L.new_of, deg.p);
      GM_HIP(hipGetLastError());
      GM_HIP(hipStreamSynchronize(st));  // the temporaries go out of scope
    }
    {
      size_t bytes = 0;
      GM_HIP(rocprim::exclusive_scan(nullptr, bytes, deg.p, L.noff, 0u, (size_t)(n + 1),
                                     rocprim::plus<uint32_t>(), st));
      Tmp<unsigned char> tmp(bytes);
      GM_HIP(rocprim::exclusive_scan(tmp.p, bytes, deg.p, L.noff, 0u, (size_t)(n + 1),
                                     rocprim::plus<uint32_t>(), st));
      fill_words<<<grid(words), kThr, 0, st>>>(L.starts, words, 0u);
      fill_words<<<1, kThr, 0, st>>>(reinterpret_cast<uint32_t*>(counts.p), 4, 0u);
      row_marks<<<grid(n + 1), kThr, 0, st>>>(L.noff, n, m, L.starts, flag.p, counts.p);
      GM_HIP(hipGetLastError());
      size_t sbytes = 0;
      GM_HIP(rocprim::exclusive_scan(nullptr, sbytes, flag.p, pos.p, 0u, (size_t)(n + 1),
                                     rocprim::plus<uint32_t>(), st));
      Tmp<unsigned char> stmp(sbytes);
      GM_HIP(rocprim::exclusive_scan(stmp.p, sbytes, flag.p, pos.p, 0u, (size_t)(n + 1),
                                     rocprim::plus<uint32_t>(), st));
      uint32_t ncross = 0;
      unsigned long long rows = 0;
      GM_HIP(hipMemcpyAsync(&ncross, pos.p + n, 4, hipMemcpyDeviceToHost, st));
      GM_HIP(hipMemcpyAsync(&rows, counts.p, 8, hipMemcpyDeviceToHost, st));
      GM_HIP(hipStreamSynchronize(st));
      L.rows = (int64_t)rows;
      L.ncross = ncross;
    }
    L.cross = dalloc<Cross>(L.ncross);
    if (L.ntiles > 0)
      first_rows<<<grid(L.ntiles), kThr, 0, st>>>(L.noff, L.rows, L.ntiles, L.tile_row);
    if (L.ncross > 0) cross_rows<<<grid(n), kThr, 0, st>>>(L.noff, flag.p, pos.p, n, L.cross);
    GM_HIP(hipGetLastError());
    GM_HIP(hipStreamSynchronize(st));
  } catch (...) {
    (void)hipStreamSynchronize(st);
    free_device_layout(&L);
    throw;
  }
  return L;
}

}  // namespace tiles
}  // namespace gm
