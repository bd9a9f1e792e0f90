// Shared pieces of the edge-tile SpMV kernels (PageRank's pull superstep
// and the transpose pass of its reverse mode): the relabelled adjacency is
// cut into tiles of kTile consecutive edges regardless of rows; a wavefront
// reduces a tile with a segmented scan whose segments are the rows (a bitmap
// marks each row's first edge). Rows with edges are the labels [0, rows).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace gm {
namespace tiles {

constexpr int kTileThreads = 1024;  // one workgroup per CU: its LDS holds the hot vector entries
constexpr int kTileWaves = kTileThreads / 64;
constexpr int kRounds = 4;                // rounds of 256 edges per tile
constexpr int64_t kTile = kRounds * 256;  // edges per tile: 4 consecutive per lane and round
constexpr int kTileHotMax = 40960;        // at most this many hot entries in LDS (160 KB)
constexpr int kCrossLanes = 16;           // lanes per row that spans tiles

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// A row whose edges lie in more than one tile: tiles ta (where it starts)
// to tb (where it ends).
struct Cross {
  uint32_t row;
  uint32_t ta;
  uint32_t tb;
  uint32_t pad;
};

// A tile layout built on the device from the row offsets off (n + 1
// entries) of an adjacency whose degrees are at most maxd: the vertices
// relabelled by decreasing degree (ties by label), so that rows with edges
// are the new labels [0, rows); their offsets noff (n + 1); the row-start
// bitmap starts (bit noff[u] for every row with edges, and bit m; mpad / 32
// + 1 words); the row holding each tile's first edge; the rows that span
// tiles, in increasing order. The caller owns the arrays:
// free_device_layout releases those still set.
struct DeviceLayout {
  int64_t rows = 0, ntiles = 0, mpad = 0, ncross = 0;
  int32_t* old_of = nullptr;     // new label -> old label
  int32_t* new_of = nullptr;     // old label -> new label
  uint32_t* noff = nullptr;
  uint32_t* starts = nullptr;
  uint32_t* tile_row = nullptr;  // ntiles entries
  Cross* cross = nullptr;        // ncross entries
};

DeviceLayout build_device_layout(const uint32_t* off, int64_t n, int64_t m, uint32_t maxd,
                                 hipStream_t st);
void free_device_layout(DeviceLayout* L);

// Copy of the first hot_n messages to LDS: all of a thread's 16-byte loads
// are issued before the first store.
__device__ inline void load_hot(const float* __restrict__ x_in, float* hot, int hot_n) {
  constexpr int kPer = kTileHotMax / 4 / kTileThreads;
  const int n4 = hot_n >> 2;
  v4f tmp[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * kTileThreads;
    if (i < n4) tmp[k] = reinterpret_cast<const v4f*>(x_in)[i];
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * kTileThreads;
    if (i < n4) reinterpret_cast<v4f*>(hot)[i] = tmp[k];
  }
  for (int i = 4 * n4 + threadIdx.x; i < hot_n; i += kTileThreads) hot[i] = x_in[i];
  __syncthreads();
}

// Segmented-sum state of a run of edges: c = number of row starts in it, s =
// sum of the messages after the last of them (of all, if c = 0). Combining
// an earlier run a with a later run b is associative, which makes the
// segmented sum a scan.
struct Seg {
  int c;
  double s;
};

__device__ inline Seg seg_join(Seg a, Seg b) { return {a.c + b.c, b.c > 0 ? b.s : a.s + b.s}; }

// Data-parallel move of a Seg between lanes (DPP control kCtrl); a lane
// whose source is outside its row of 16 lanes keeps `old`.
template <int kCtrl>
__device__ inline Seg seg_dpp(Seg old, Seg v) {
  const unsigned long long ob = (unsigned long long)__double_as_longlong(old.s);
  const unsigned long long vb = (unsigned long long)__double_as_longlong(v.s);
  const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)ob, (int)(uint32_t)vb, kCtrl, 0xF, 0xF,
                                             false);
  const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(ob >> 32), (int)(uint32_t)(vb >> 32),
                                             kCtrl, 0xF, 0xF, false);
  const int c = __builtin_amdgcn_update_dpp(old.c, v.c, kCtrl, 0xF, 0xF, false);
  return {c, __longlong_as_double((long long)(((unsigned long long)(uint32_t)hi << 32) |
                                              (uint32_t)lo))};
}

__device__ inline Seg seg_lane(Seg v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v.s);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return {__builtin_amdgcn_readlane(v.c, lane),
          __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo))};
}

// Wavefront scan of one round: from each lane's own run `own` and the run
// `carry` of everything before the round, the lane's exclusive prefix (all
// earlier lanes, carry included); `carry` moves on to the end of the round.
__device__ inline Seg seg_scan(Seg own, Seg& carry, int lane) {
  constexpr Seg id{0, 0.0};
  Seg x = own;  // inclusive scan within each row of 16 lanes (row_shr 1, 2, 4, 8)
  x = seg_join(seg_dpp<0x111>(id, x), x);
  x = seg_join(seg_dpp<0x112>(id, x), x);
  x = seg_join(seg_dpp<0x114>(id, x), x);
  x = seg_join(seg_dpp<0x118>(id, x), x);
  const Seg p1 = seg_join(carry, seg_lane(x, 15));
  const Seg p2 = seg_join(p1, seg_lane(x, 31));
  const Seg p3 = seg_join(p2, seg_lane(x, 47));
  const int row = lane >> 4;
  const Seg before = row == 0 ? carry : row == 1 ? p1 : row == 2 ? p2 : p3;
  const Seg incl = seg_join(before, x);
  carry = seg_lane(incl, 63);
  return seg_dpp<0x111>(before, incl);  // the row's first lane takes `before`
}

// Wavefront exclusive prefix of the lanes' integers `own` (row starts), with
// `carry` the count before the round; `carry` moves on to the end of the
// round.
__device__ inline int count_scan(int own, int& carry, int lane) {
  int x = own;  // inclusive within each row of 16 lanes
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);
  const int t0 = __builtin_amdgcn_readlane(x, 15);
  const int t1 = __builtin_amdgcn_readlane(x, 31);
  const int t2 = __builtin_amdgcn_readlane(x, 47);
  const int row = lane >> 4;
  const int incl = carry + (row > 0 ? t0 : 0) + (row > 1 ? t1 : 0) + (row > 2 ? t2 : 0) + x;
  carry = __builtin_amdgcn_readlane(incl, 63);
  return incl - own;
}

}  // namespace tiles
}  // namespace gm
