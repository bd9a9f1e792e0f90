// Triangle counting as the two vertex programs of Sec. 4.2 on the
// upper-triangle DAG (edges u -> v with u < v, Sec. 5.1 preprocessing).
// Program 1 (every vertex collects its sorted list of in-neighbours) is the
// in-adjacency built at load time. Program 2 is this file: every vertex u
// sends in(u) along its out-edges (SEND), each receiver v counts
// |in(u) ∩ in(v)| per message (PROCESS), sums them (REDUCE +) and adds the
// sum to its count (APPLY). A triangle a < b < c is counted exactly once,
// at c, through the message from b (common in-neighbour a); the total is the
// N_triangles of Eq. (7).
//
// Work organisation: the intersection for DAG edge (u -> v) is computed by
// one endpoint (its "owner"): an owner x puts in(x) in a hash table in LDS
// (very long lists in LDS-sized pieces) once, then streams the in-list of
// every partner through it, one probe per element, up to the last element
// below x (in(x) holds only smaller ids; the stream lengths are computed
// with the plan). The endpoint whose partner stream is shorter owns the
// edge. The match count of edge (u -> v) is credited to the
// receiver v, as APPLY prescribes. Owner/partner lists are built once per
// graph and cut into work items of bounded size, one wavefront or workgroup
// each. The lanes of a wavefront split a window of 64 partners' streams
// into equal runs of 32-byte units, one bucket read per element in most
// cases.
// All counts are exact integers, independent of scheduling.
#include <algorithm>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kWaveMax = 512;          // owners with |in(x)| <= this: LDS table per wavefront
constexpr uint32_t kCreditPartner = 0x80000000u;  // partner entry flag: credit goes to it
constexpr int32_t kEmpty = -1;

// Table classes by the owner's in-list length d: LDS tables per wavefront,
// LDS tables per workgroup of growing size (small tables leave room for
// more resident wavefronts); longer in-lists are cut into pieces of the
// largest table size, each piece an owner of its own whose partners stream
// only their elements in the piece's id range. A table has at least 4 d
// slots.
enum TcKind { kWaveTable, kBlockTable, kSplitTable };
struct TcClass {
  uint32_t max_d;
  uint32_t slots;  // LDS slots per table
  int threads;     // workgroup size
  TcKind kind;
};
constexpr int kClassesTc = 7;
constexpr TcClass kTcClass[kClassesTc] = {{128, 512, 256, kWaveTable},          // 2 KB per wavefront
                                          {kWaveMax, 2048, 256, kWaveTable},    // 8 KB per wavefront
                                          {1024, 4096, 512, kBlockTable},       // 16 KB
                                          {2048, 8192, 512, kBlockTable},       // 32 KB
                                          {4096, 16384, 512, kBlockTable},      // 64 KB
                                          {8192, 32768, 1024, kBlockTable},     // 128 KB
                                          {UINT32_MAX, 32768, 1024, kSplitTable}};
constexpr uint32_t kPieceMax = 8192;  // in-list entries per piece of a split owner

// A work item: owner x and a range of its partner list.
struct Item {
  int32_t owner;
  uint32_t p_begin;
  uint32_t p_end;
  uint32_t pad;
};

// A work item of one piece of a split owner: the piece is in(x) positions
// [tb, te) (ids [lo, hi)); partner j starts at element pstart[sbase + j -
// p_begin] of its in-list and stops at hi.
struct PieceItem {
  int32_t owner;
  uint32_t p_begin;
  uint32_t p_end;
  uint32_t tb;
  uint32_t te;
  int32_t hi;
  uint32_t sbase;
  uint32_t pad;
};

struct TcPlan {
  Item* items[kClassesTc] = {};  // per table class
  int64_t nitems[kClassesTc] = {};
  int32_t* keys = nullptr;         // key of every in-list entry (in_idx order), padded
  uint32_t* work = nullptr;        // partner id | kCreditPartner, grouped by owner
  uint32_t* wlen = nullptr;        // per partner entry: elements streamed
  PieceItem* pieces = nullptr;     // work items of split owners
  int64_t npieces = 0;
  uint32_t* pstart = nullptr;      // per piece item and partner: first element >= the piece's low id
  uint32_t* plen = nullptr;        // ... and the number of its elements in the piece's range
  unsigned long long* total = nullptr;
  // tuning the plan was built with
  uint32_t wave_max = 0, wave_work = 0, block_work = 0;
  // one stream per table-class launch (forked from and joined to the
  // caller's stream), so that the launches overlap instead of each ending in
  // a tail of idle compute units
  hipStream_t lanes[kClassesTc] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t done[kClassesTc] = {};
};

// Tables and partner streams hold keys, not ids: key = id times an odd
// constant mod 2^32 (a bijection, so equal keys mean equal ids), computed
// once per graph. A key's home bucket in a table of 2^(32 - shift) buckets
// is its top bits (multiplicative hashing, which spreads the skewed low bits
// of RMAT ids over the whole table). No id below 2^31 has the key -1, the
// empty-slot mark.
constexpr uint32_t kKeyMul = 0x9E3779B1u;

__device__ inline uint32_t home_bucket(int32_t key, uint32_t shift) { return (uint32_t)key >> shift; }

__global__ void make_keys(const int32_t* __restrict__ idx, int64_t m, int32_t* __restrict__ keys) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = (int32_t)((uint32_t)idx[i] * kKeyMul);
}

// Shift for a table with bmask + 1 buckets (a power of two, at least 16).
__device__ inline uint32_t bucket_shift(uint32_t bmask) { return 32u - (uint32_t)__popc(bmask); }

// Tables are buckets of 4 slots (one 16-byte LDS read); a key lives in its
// home bucket or, when that is full, in the next buckets (linear probing
// over buckets). At most a quarter of the slots are used, so that a home
// bucket is full in about 2% of lookups (in up to 16% at half the slots
// used, where the overflow walk cost a quarter of all vector instructions).
__device__ inline void table_insert(int32_t* T, uint32_t bmask, int32_t key) {
  uint32_t b = home_bucket(key, bucket_shift(bmask));
  for (;;) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (atomicCAS(&T[4 * b + i], kEmpty, key) == kEmpty) return;
    b = (b + 1) & bmask;
  }
}

// 1 if key is one of the bucket's slots.
__device__ inline uint32_t in_bucket(int4 q, int32_t key) {
  const uint32_t a = min((uint32_t)(q.x ^ key), (uint32_t)(q.y ^ key));
  const uint32_t b = min((uint32_t)(q.z ^ key), (uint32_t)(q.w ^ key));
  return min(a, b) == 0u ? 1u : 0u;
}

// True if no slot of the bucket is free: inserts fill slots in order, so
// the last one is taken only in a full bucket.
__device__ inline bool bucket_full(int4 q) { return q.w != kEmpty; }

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline uint32_t wave_incl_scan(uint32_t x, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  return x;
}

// Elements per unit of a partner stream: an aligned 32-byte half line of
// the key array, loaded whole, so that a line is requested from L2 about
// twice (a lane that took a line a quad at a time would mostly find it
// evicted from L1 before its next quad; whole 64-byte lines cost more
// registers than the saved requests are worth).
constexpr uint32_t kLine = 8;

struct Line {
  int4 q[kLine / 4];
};

__device__ __forceinline__ Line load_line(const int32_t* __restrict__ keys, uint32_t l) {
  const int4* p = reinterpret_cast<const int4*>(keys + (size_t)kLine * l);
  Line L;
#pragma unroll
  for (int k = 0; k < (int)kLine / 4; ++k) L.q[k] = p[k];
  return L;
}

// Matches of unit l of the key array (elements kLine l .. kLine l + kLine - 1,
// those in [s, e) counted) in the table. Every element reads its home
// bucket; those whose home bucket is full without holding them go on to the
// next buckets in one loop that follows a single key per lane at a time (an
// unrolled pass per element would run for every element position whenever
// any lane of the wavefront needed it).
__device__ __forceinline__ uint32_t probe_line(const int4* T4, uint32_t bmask, uint32_t shift,
                                               const Line& L, uint32_t l, uint32_t s, uint32_t e) {
  const int32_t base = (int32_t)(kLine * l);
  const int32_t lo = (int32_t)s - base, hi = (int32_t)e - base;
  constexpr uint32_t kAll = (1u << kLine) - 1u;
  const uint32_t ok =
      (hi >= (int32_t)kLine ? kAll : (1u << hi) - 1u) & (lo <= 0 ? kAll : ~((1u << lo) - 1u));
  int32_t key[kLine];
#pragma unroll
  for (int k = 0; k < (int)kLine / 4; ++k) {
    key[4 * k] = L.q[k].x;
    key[4 * k + 1] = L.q[k].y;
    key[4 * k + 2] = L.q[k].z;
    key[4 * k + 3] = L.q[k].w;
  }
  uint32_t hits = 0, more = 0;  // bit i: element i found / home bucket full without it
#pragma unroll
  for (int i = 0; i < (int)kLine; ++i) {
    const int4 b = T4[home_bucket(key[i], shift)];
    const uint32_t h = in_bucket(b, key[i]);
    hits |= h << i;
    more |= (h == 0u && bucket_full(b)) ? 1u << i : 0u;
  }
  more &= ok;
  // Keys whose home bucket is full without them go on to the next buckets,
  // one bucket read per pass for one pending key of each lane (the passes
  // of a wavefront are the most any of its lanes needs).
  uint32_t cur = 0, bk = 0;  // bit of the key being followed (0: none), its bucket
  int32_t ck = 0;
  while (more | cur) {
    if (!cur) {
      const int i = __builtin_ctz(more);
      cur = 1u << i;
      more &= more - 1u;
      ck = key[0];
#pragma unroll
      for (int k = 1; k < (int)kLine; ++k) ck = i == k ? key[k] : ck;
      bk = home_bucket(ck, shift);
    }
    bk = (bk + 1) & bmask;
    const int4 b = T4[bk];
    if (in_bucket(b, ck)) {
      hits |= cur;
      cur = 0;
    } else if (!bucket_full(b)) {
      cur = 0;
    }
  }
  return (uint32_t)__popc(hits & ok);
}

// Per-wavefront LDS scratch of a partner window.
struct Window {
  uint32_t excl[65];  // first unit of each lane's partner in the window's unit sequence; [64] = total
  uint32_t la[64];    // the partner's first aligned unit in the index array
  uint32_t s[64];     // its stream [s, e)
  uint32_t e[64];
  uint32_t cnt[64];   // its matches
};

// Partners [p_begin, p_end) of one owner in windows of 64 (lane l of a
// window holds partner j0 + l; windows step by j_step). A partner streams
// the elements [s, s + len) of the index array: s = in_off[y] and len =
// lens[j], or, for the pieces of a split owner, s = pstart[j + shift] and
// len = lens[j + shift]. The window's streams are cut into aligned units of
// kLine elements and the unit sequence into 64 equal contiguous ranges, one
// per lane: a lane finds the partner of its first unit by binary search over
// the window's prefix sums (in LDS), then walks its range, moving to the next
// partner at each boundary, the next unit's loads issued before the current
// unit is probed. Matches credited to the owner are returned; those credited
// to a partner are added to counts[partner].
__device__ __forceinline__ unsigned long long walk_partners(const int4* T4, uint32_t bmask,
                                                   const uint32_t* __restrict__ work,
                                                   uint32_t p_begin, uint32_t p_end,
                                                   uint32_t j_step,
                                                   const uint32_t* __restrict__ in_off,
                                                   const int32_t* __restrict__ keys,
                                                   unsigned long long* counts, Window* W,
                                                   const uint32_t* __restrict__ lens,
                                                   const uint32_t* __restrict__ pstart = nullptr,
                                                   int64_t shift = 0) {
  const int lane = threadIdx.x & 63;
  const uint32_t hshift = bucket_shift(bmask);
  unsigned long long own = 0;
  for (uint32_t j0 = p_begin; j0 < p_end; j0 += j_step) {
    const uint32_t j = j0 + lane;
    uint32_t entry = 0, s = 0, e = 0;
    if (j < p_end) {
      entry = work[j];
      const uint32_t y = entry & ~kCreditPartner;
      s = pstart ? pstart[j + shift] : in_off[y];
      e = s + lens[j + shift];
    }
    const uint32_t la = s / kLine;
    const uint32_t nl = e > s ? (e + kLine - 1) / kLine - la : 0u;
    const uint32_t incl = wave_incl_scan(nl, lane);
    const uint32_t total = __shfl(incl, 63, 64);
    W->excl[lane] = incl - nl;
    if (lane == 63) W->excl[64] = total;
    W->la[lane] = la;
    W->s[lane] = s;
    W->e[lane] = e;
    W->cnt[lane] = 0;
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    const uint32_t per = (total + 63) / 64;
    uint32_t idx = min(total, per * lane);
    const uint32_t iend = min(total, idx + per);
    if (idx < iend) {
      int o = 0;  // the last lane whose first unit is <= idx
      for (int step = 32; step > 0; step >>= 1)
        if (W->excl[o + step] <= idx) o += step;
      uint32_t bound = W->excl[o + 1];
      uint32_t l = W->la[o] + (idx - W->excl[o]);
      uint32_t so = W->s[o], eo = W->e[o];
      Line v = load_line(keys, l);
      while (idx < iend) {
        const Line cv = v;
        const uint32_t cl = l, cs = so, ce = eo;
        const int co = o;
        ++idx;
        ++l;
        if (idx < iend) {
          if (idx == bound) {  // next partner with units
            do {
              ++o;
              bound = W->excl[o + 1];
            } while (bound <= idx);
            l = W->la[o];
            so = W->s[o];
            eo = W->e[o];
          }
          v = load_line(keys, l);
        }
        const uint32_t c = probe_line(T4, bmask, hshift, cv, cl, cs, ce);
        if (c) atomicAdd(&W->cnt[co], c);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    const uint32_t mine = W->cnt[lane];
    if (j < p_end && mine) {
      if (entry & kCreditPartner)
        atomicAdd(&counts[entry & ~kCreditPartner], (unsigned long long)mine);
      else
        own += mine;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  return own;
}

// Bucket mask of the table of an owner with d in-neighbours: at least four
// times as many slots as keys, at least 16 buckets.
__device__ __host__ inline uint32_t table_buckets(uint32_t d) {
  uint32_t slots = 64;
  while (slots < 4 * d) slots <<= 1;
  return slots / 4;
}

// One wavefront per work item of an owner whose table fits kSlots slots.
template <uint32_t kSlots>
__global__ __launch_bounds__(kThreads) void tc_wave(const Item* __restrict__ items, int64_t nitems,
                                                    const uint32_t* __restrict__ in_off,
                                                    const int32_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ work,
                                                    const uint32_t* __restrict__ wlen,
                                                    unsigned long long* counts) {
  __shared__ int4 tables[kWaves][kSlots / 4];
  __shared__ Window wins[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * kWaves + wave;
  if (r >= nitems) return;  // the whole wavefront leaves together
  const Item it = items[r];
  const int32_t x = it.owner;
  const uint32_t b = in_off[x], d = in_off[x + 1] - b;
  const uint32_t nb = table_buckets(d);
  int4* T4 = tables[wave];
  for (uint32_t k = lane; k < nb; k += 64) T4[k] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  int32_t* T = reinterpret_cast<int32_t*>(T4);
  for (uint32_t k = lane; k < d; k += 64) table_insert(T, nb - 1, keys[b + k]);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  const unsigned long long c = wave_sum_u64(walk_partners(
      T4, nb - 1, work, it.p_begin, it.p_end, 64, in_off, keys, counts, &wins[wave], wlen));
  if (lane == 0 && c) atomicAdd(&counts[x], c);
}

// One workgroup of kThr threads per work item, the owner's table (kSlots
// slots) in LDS. Wavefront w takes partners p_begin + 64 w + lane, then
// steps of one workgroup.
template <uint32_t kSlots, int kThr>
__global__ __launch_bounds__(kThr) void tc_block(const Item* __restrict__ items,
                                                 const uint32_t* __restrict__ in_off,
                                                 const int32_t* __restrict__ keys,
                                                 const uint32_t* __restrict__ work,
                                                 const uint32_t* __restrict__ wlen,
                                                 unsigned long long* counts) {
  constexpr int kW = kThr / 64;
  __shared__ int4 ltable[kSlots / 4];
  __shared__ Window wins[kW];
  __shared__ unsigned long long part[kW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const Item it = items[blockIdx.x];
  const int32_t x = it.owner;
  const uint32_t b = in_off[x], d = in_off[x + 1] - b;
  const uint32_t nb = table_buckets(d);
  const uint32_t bmask = nb - 1;
  for (uint32_t k = threadIdx.x; k < nb; k += kThr)
    ltable[k] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
  __syncthreads();
  int32_t* T = reinterpret_cast<int32_t*>(ltable);
  for (uint32_t k = threadIdx.x; k < d; k += kThr) table_insert(T, bmask, keys[b + k]);
  __syncthreads();
  const unsigned long long c = wave_sum_u64(walk_partners(
      ltable, bmask, work, it.p_begin + wave * 64, it.p_end, kThr, in_off, keys, counts,
      &wins[wave], wlen));
  if (lane == 0) part[wave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int i = 0; i < kW; ++i) t += part[i];
    if (t) atomicAdd(&counts[x], t);
  }
}

// One workgroup per work item of a piece of a split owner.
template <uint32_t kSlots, int kThr>
__global__ __launch_bounds__(kThr) void tc_piece(const PieceItem* __restrict__ items,
                                                 const uint32_t* __restrict__ in_off,
                                                 const int32_t* __restrict__ keys,
                                                 const uint32_t* __restrict__ work,
                                                 const uint32_t* __restrict__ pstart,
                                                 const uint32_t* __restrict__ plen,
                                                 unsigned long long* counts) {
  constexpr int kW = kThr / 64;
  __shared__ int4 ltable[kSlots / 4];
  __shared__ Window wins[kW];
  __shared__ unsigned long long part[kW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const PieceItem it = items[blockIdx.x];
  const uint32_t d = it.te - it.tb;
  const uint32_t nb = table_buckets(d);
  const uint32_t bmask = nb - 1;
  for (uint32_t k = threadIdx.x; k < nb; k += kThr)
    ltable[k] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
  __syncthreads();
  int32_t* T = reinterpret_cast<int32_t*>(ltable);
  for (uint32_t k = threadIdx.x; k < d; k += kThr) table_insert(T, bmask, keys[it.tb + k]);
  __syncthreads();
  const unsigned long long c = wave_sum_u64(walk_partners(
      ltable, bmask, work, it.p_begin + wave * 64, it.p_end, kThr, in_off, keys, counts,
      &wins[wave], plen, pstart, (int64_t)it.sbase - (int64_t)it.p_begin));
  if (lane == 0) part[wave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int i = 0; i < kW; ++i) t += part[i];
    if (t) atomicAdd(&counts[it.owner], t);
  }
}

__global__ void sum_u64(const unsigned long long* __restrict__ a, int64_t n,
                        unsigned long long* __restrict__ total) {
  __shared__ unsigned long long part[kWaves];
  unsigned long long s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += a[i];
  s = wave_sum_u64(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(total, (part[0] + part[1]) + (part[2] + part[3]));
}

__global__ void zero_u64(unsigned long long* __restrict__ a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

// ---------------------------------------------------------------------------
// Work plan, built on the device from the DAG's in-adjacency (rocPRIM's
// radix sort, scan and select as library primitives; every step of the plan
// is one of the kernels below).
//
// For DAG edge (u -> v), u < v: in(u) ∩ in(v) = in(u) ∩ (in(v) ∩ [0, u)).
// Either v owns it (its table holds in(v); lanes stream in(u), |in(u)|
// elements, credit to v = the owner) or u owns it (table in(u); lanes stream
// the prefix of in(v) below u, credit to the partner v). The cheaper stream
// decides; an edge with nothing to stream closes no triangle. Streams stop
// at the owner's id in both cases, since in(x) holds only ids below x.
// Each owner's partners are ordered by decreasing stream length (ties in
// in-edge order), so that the lanes of a window walk lists of similar length.
// ---------------------------------------------------------------------------
constexpr int kPlanThreads = 256;

inline unsigned plan_grid(int64_t n) {
  int64_t b = (n + kPlanThreads - 1) / kPlanThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

inline int bits_for(uint64_t x) {  // smallest b with 2^b >= x
  int b = 0;
  while (b < 63 && (1ull << b) < x) ++b;
  return b;
}

// Table class of an owner with d in-neighbours (wave_max: the longest in-list
// that gets a per-wavefront table).
__device__ __host__ inline int tc_class(uint32_t d, uint32_t wave_max) {
  if (d <= wave_max) return d <= kTcClass[0].max_d ? 0 : 1;
  int c = 2;
  while (d > kTcClass[c].max_d) ++c;
  return c;
}

// First position in [b, e) of a sorted id array holding a value >= x.
__device__ inline uint32_t lower_pos(const int32_t* __restrict__ a, uint32_t b, uint32_t e,
                                     int32_t x) {
  while (b < e) {
    const uint32_t mid = b + ((e - b) >> 1);
    if (a[mid] < x)
      b = mid + 1;
    else
      e = mid;
  }
  return b;
}

// rowid[j] = v for every in-edge j of row v: one wavefront per row, its
// lanes storing consecutive entries.
__global__ void plan_row_ids(const uint32_t* __restrict__ in_off, int64_t n,
                             uint32_t* __restrict__ rowid) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t v = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; v < n; v += waves) {
    const uint32_t b = in_off[v], e = in_off[v + 1];
    for (uint32_t j = b + lane; j < e; j += 64) rowid[j] = (uint32_t)v;
  }
}

// One thread per in-edge j (u = in_idx[j] -> v = row of j): the sort key
// (owner, decreasing stream length) and the work entry (partner, with the
// credit flag when the partner receives the count). Edges with nothing to
// stream get a key past every owner.
__global__ void plan_edges(const uint32_t* __restrict__ in_off, const int32_t* __restrict__ in_idx,
                           const uint32_t* __restrict__ rowid, int64_t n, int64_t m, int cb,
                           unsigned long long* __restrict__ key, uint32_t* __restrict__ val) {
  const unsigned long long cmask = (1ull << cb) - 1;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t v = rowid[j];
    const int32_t u = in_idx[j];
    const uint32_t a = in_off[u + 1] - in_off[u];  // |in(u)|
    const uint32_t b = (uint32_t)j - in_off[v];    // |in(v) ∩ [0, u)|
    if (a == 0 || b == 0) {
      key[j] = ((unsigned long long)n << cb) | cmask;
      val[j] = 0;
      continue;
    }
    const bool by_u = b < a;
    const uint32_t owner = by_u ? (uint32_t)u : v;
    const uint32_t cost = by_u ? b : a;
    key[j] = ((unsigned long long)owner << cb) | (cmask - cost);
    val[j] = by_u ? (v | kCreditPartner) : (uint32_t)u;
  }
}

// work_off[x] = first sorted entry of owner x (x = n: the number of entries).
__global__ void plan_owner_offsets(const unsigned long long* __restrict__ key, int64_t m, int cb,
                                   int64_t n, uint32_t* __restrict__ work_off) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x <= n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long t = (unsigned long long)x << cb;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (key[mid] < t)
        lo = mid + 1;
      else
        hi = mid;
    }
    work_off[x] = (uint32_t)lo;
  }
}

// Sorted entries -> work entries and stream lengths.
__global__ void plan_work(const unsigned long long* __restrict__ key,
                          const uint32_t* __restrict__ val, int64_t w, int cb,
                          uint32_t* __restrict__ work, uint32_t* __restrict__ wlen) {
  const unsigned long long cmask = (1ull << cb) - 1;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < w;
       j += (int64_t)gridDim.x * blockDim.x) {
    work[j] = val[j];
    wlen[j] = (uint32_t)(cmask - (key[j] & cmask));
  }
}


// Work items of the owners with a table in LDS: an owner's partners are cut
// where the streamed elements before a partner cross a multiple of the
// class's budget (so an item streams at most budget + its last partner's
// length). flag[j] = 1 where an item starts.
__global__ void plan_item_flags(const unsigned long long* __restrict__ key, int cb,
                                const uint32_t* __restrict__ work_off, int64_t w,
                                const uint32_t* __restrict__ in_off,
                                const unsigned long long* __restrict__ pre, uint32_t wave_max,
                                uint32_t wave_work, uint32_t block_work,
                                uint8_t* __restrict__ flag) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < w;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t x = (uint32_t)(key[j] >> cb);
    const int c = tc_class(in_off[x + 1] - in_off[x], wave_max);
    uint8_t f = 0;
    if (kTcClass[c].kind != kSplitTable) {
      const unsigned long long budget = kTcClass[c].kind == kWaveTable ? wave_work : block_work;
      const uint32_t p0 = work_off[x];
      f = (uint32_t)j == p0 ||
          (pre[j] - pre[p0]) / budget != (pre[j - 1] - pre[p0]) / budget;
    }
    flag[j] = f;
  }
}

// Items from their first entries: owner, partner range, the sort key (class,
// decreasing partner count: the largest items of a class start first), and
// the per-class item counts.
__global__ void plan_items(const uint32_t* __restrict__ start, int64_t nitems,
                           const unsigned long long* __restrict__ key, int cb,
                           const uint32_t* __restrict__ work_off,
                           const uint32_t* __restrict__ in_off, uint32_t wave_max,
                           Item* __restrict__ items, unsigned long long* __restrict__ skey,
                           uint32_t* __restrict__ sidx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nitems;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t j = start[i];
    const uint32_t x = (uint32_t)(key[j] >> cb);
    uint32_t end = work_off[x + 1];
    if (i + 1 < nitems && start[i + 1] < end) end = start[i + 1];
    const int c = tc_class(in_off[x + 1] - in_off[x], wave_max);
    items[i] = Item{(int32_t)x, j, end, 0};
    skey[i] = ((unsigned long long)c << 32) | (0xFFFFFFFFu - (end - j));
    sidx[i] = (uint32_t)i;
  }
}

// first[c] = the first item of class c in the items sorted by class
// (c = 0..kClassesTc; first[kClassesTc] = nitems).
__global__ void plan_class_bounds(const unsigned long long* __restrict__ skey, int64_t nitems,
                                  uint32_t* __restrict__ first) {
  const int c = threadIdx.x;
  if (c > kClassesTc) return;
  const unsigned long long t = (unsigned long long)c << 32;
  int64_t lo = 0, hi = nitems;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (skey[mid] < t)
      lo = mid + 1;
    else
      hi = mid;
  }
  first[c] = (uint32_t)lo;
}

template <class T>
__global__ void plan_gather(const T* __restrict__ src, const uint32_t* __restrict__ idx, int64_t n,
                            T* __restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[idx[i]];
}

// Owners whose in-list is cut into pieces (class kSplitTable) and have partners.
__global__ void plan_split_flags(const uint32_t* __restrict__ in_off,
                                 const uint32_t* __restrict__ work_off, int64_t n,
                                 uint32_t wave_max, uint8_t* __restrict__ flag) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x)
    flag[x] = kTcClass[tc_class(in_off[x + 1] - in_off[x], wave_max)].kind == kSplitTable &&
              work_off[x + 1] > work_off[x];
}

// In-list and partner-list bounds of each split owner: in_off[x], in_off[x +
// 1], work_off[x], work_off[x + 1] for owner x = owners[i], at out[4 i].
__global__ void plan_split_bounds(const uint32_t* __restrict__ owners, int64_t nsplit,
                                  const uint32_t* __restrict__ in_off,
                                  const uint32_t* __restrict__ work_off,
                                  uint32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nsplit;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t x = owners[i];
    out[4 * i] = in_off[x];
    out[4 * i + 1] = in_off[x + 1];
    out[4 * i + 2] = work_off[x];
    out[4 * i + 3] = work_off[x + 1];
  }
}

// One piece of a split owner: in(x) positions [tb, te) (absolute), ids
// [lo, hi), partners [p0, p0 + np); its (partner, piece) pairs start at base.
struct PieceSeg {
  int32_t owner;
  uint32_t tb, te;
  int32_t lo, hi;
  uint32_t p0, np;
  uint32_t base;
};

__global__ void plan_seg_bounds(PieceSeg* __restrict__ seg, int64_t nseg,
                                const uint32_t* __restrict__ in_off,
                                const int32_t* __restrict__ in_idx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nseg;
       i += (int64_t)gridDim.x * blockDim.x) {
    PieceSeg s = seg[i];
    s.lo = in_idx[s.tb];
    s.hi = s.te < in_off[s.owner + 1] ? in_idx[s.te] : s.owner;
    seg[i] = s;
  }
}

__device__ inline uint32_t seg_of(const PieceSeg* __restrict__ seg, int64_t nseg, uint32_t p) {
  int64_t lo = 0, hi = nseg;  // the last segment with base <= p
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (seg[mid].base <= p)
      lo = mid;
    else
      hi = mid;
  }
  return (uint32_t)lo;
}

// One thread per (piece, partner) pair: where the partner's in-list enters
// the piece's id range [lo, hi) and how many of its elements lie in it.
__global__ void plan_pairs(const PieceSeg* __restrict__ seg, int64_t nseg, int64_t npairs,
                           const uint32_t* __restrict__ work, const uint32_t* __restrict__ in_off,
                           const int32_t* __restrict__ in_idx, uint32_t* __restrict__ pstart,
                           uint32_t* __restrict__ plen) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const PieceSeg s = seg[seg_of(seg, nseg, (uint32_t)p)];
    const uint32_t y = work[s.p0 + ((uint32_t)p - s.base)] & ~kCreditPartner;
    const uint32_t b = in_off[y], e = in_off[y + 1];
    const uint32_t f = lower_pos(in_idx, b, e, s.lo);
    pstart[p] = f;
    plen[p] = lower_pos(in_idx, f, e, s.hi) - f;
  }
}

__global__ void plan_piece_flags(const PieceSeg* __restrict__ seg, int64_t nseg, int64_t npairs,
                                 const unsigned long long* __restrict__ pre, uint32_t budget,
                                 uint8_t* __restrict__ flag) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t b = seg[seg_of(seg, nseg, (uint32_t)p)].base;
    flag[p] = (uint32_t)p == b || (pre[p] - pre[b]) / budget != (pre[p - 1] - pre[b]) / budget;
  }
}

__global__ void plan_piece_items(const uint32_t* __restrict__ start, int64_t nitems,
                                 const PieceSeg* __restrict__ seg, int64_t nseg,
                                 PieceItem* __restrict__ items,
                                 unsigned long long* __restrict__ skey,
                                 uint32_t* __restrict__ sidx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nitems;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = start[i];
    const PieceSeg s = seg[seg_of(seg, nseg, p)];
    uint32_t end = s.base + s.np;
    if (i + 1 < nitems && start[i + 1] < end) end = start[i + 1];
    items[i] = PieceItem{s.owner, s.p0 + (p - s.base), s.p0 + (end - s.base), s.tb, s.te, s.hi,
                         p, 0};
    skey[i] = 0xFFFFFFFFu - (end - p);
    sidx[i] = (uint32_t)i;
  }
}

TcPlan* plan(gm_graph g) { return static_cast<TcPlan*>(g->tc_plan); }

// Device memory for the temporaries of one plan build: taken in order from
// a few large chunks and released together when the build ends (after the
// stream has drained), so that the build makes a handful of allocations
// rather than one per temporary.
struct Pool {
  hipStream_t s;
  std::vector<void*> chunks;
  char* cur = nullptr;
  size_t left = 0;
  explicit Pool(hipStream_t st) : s(st) {}
  Pool(const Pool&) = delete;
  Pool& operator=(const Pool&) = delete;
  ~Pool() {
    (void)hipStreamSynchronize(s);
    for (void* c : chunks) dfree(c);
  }
  void* take(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    if (bytes > left) {
      const size_t cb = std::max(bytes, (size_t)256 << 20);
      void* c = dmalloc(cb);
      chunks.push_back(c);
      cur = static_cast<char*>(c);
      left = cb;
    }
    void* p = cur;
    cur += bytes;
    left -= bytes;
    return p;
  }
};

// A temporary of the plan build.
struct Scratch {
  void* p = nullptr;
  Scratch(Pool& pool, size_t bytes) : p(pool.take(bytes)) {}
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// rocPRIM calls: query the temporary storage, take it from the pool, run.
template <class F>
void with_temp(Pool& pool, F&& f) {
  size_t bytes = 0;
  GM_HIP(f(nullptr, bytes));
  void* tmp = pool.take(bytes);
  GM_HIP(f(tmp, bytes));
}

// Stable sort of (key, index) pairs on the low `bits` bits; returns the
// buffers holding the result.
void sort_pairs(Pool& pool, Scratch& k1, Scratch& k2, Scratch& v1, Scratch& v2, int64_t n,
                int bits, hipStream_t s, unsigned long long** kout, uint32_t** vout) {
  rocprim::double_buffer<unsigned long long> kb(k1.as<unsigned long long>(),
                                                k2.as<unsigned long long>());
  rocprim::double_buffer<uint32_t> vb(v1.as<uint32_t>(), v2.as<uint32_t>());
  if (n > 0)
    with_temp(pool, [&](void* t, size_t& b) {
      return rocprim::radix_sort_pairs(t, b, kb, vb, (size_t)n, 0, bits, s);
    });
  *kout = kb.current();
  *vout = vb.current();
}

// Exclusive prefix sums of n uint32 values into uint64.
void exclusive_u64(Pool& pool, const uint32_t* in, unsigned long long* out, int64_t n,
                   hipStream_t s) {
  if (n == 0) return;
  with_temp(pool, [&](void* t, size_t& b) {
    return rocprim::exclusive_scan(t, b, in, out, 0ull, (size_t)n,
                                   rocprim::plus<unsigned long long>(), s);
  });
}

// Positions i < n with flag[i] != 0, in order, into out; returns their count
// (synchronises s).
int64_t select_flagged(Pool& pool, const uint8_t* flag, int64_t n, uint32_t* out,
                       hipStream_t s) {
  if (n == 0) return 0;
  Scratch cnt(pool, sizeof(unsigned long long));
  with_temp(pool, [&](void* t, size_t& b) {
    return rocprim::select(t, b, rocprim::counting_iterator<uint32_t>(0u), flag, out,
                           cnt.as<unsigned long long>(), (size_t)n, s);
  });
  unsigned long long h = 0;
  GM_HIP(hipMemcpyAsync(&h, cnt.p, sizeof(h), hipMemcpyDeviceToHost, s));
  GM_HIP(hipStreamSynchronize(s));
  return (int64_t)h;
}

}  // namespace

static TcPlan* ensure_plan(gm_graph g, hipStream_t s);

void free_tc_plan(gm_graph g) {
  TcPlan* p = plan(g);
  if (!p) return;
  for (int c = 0; c < kClassesTc; ++c) dfree(p->items[c]);
  dfree(p->keys);
  dfree(p->work);
  dfree(p->pieces);
  dfree(p->pstart);
  dfree(p->plen);
  dfree(p->wlen);
  for (int c = 0; c < kClassesTc; ++c) {
    if (p->lanes[c]) (void)hipStreamDestroy(p->lanes[c]);
    if (p->done[c]) (void)hipEventDestroy(p->done[c]);
  }
  if (p->fork) (void)hipEventDestroy(p->fork);
  dfree(p->total);
  delete p;
  g->tc_plan = nullptr;
  ++g->ws_gen;
}

void prepare_triangle_count(gm_graph g, hipStream_t s) {
  ensure_plan(g, s);
  GM_HIP(hipStreamSynchronize(s));
}

static TcPlan* ensure_plan(gm_graph g, hipStream_t s) {
  const uint32_t wave_max = std::min(g->tune.tc_wave_max, kWaveMax);
  const uint32_t wave_work = g->tune.tc_wave_work, block_work = g->tune.tc_block_work;
  if (TcPlan* p = plan(g)) {
    if (p->wave_max == wave_max && p->wave_work == wave_work && p->block_work == block_work)
      return p;
    free_tc_plan(g);
  }
  const int64_t n = g->n, m = g->m;
  TcPlan* p = new TcPlan();
  g->tc_plan = p;
  p->wave_max = wave_max;
  p->wave_work = wave_work;
  p->block_work = block_work;
  try {
    p->keys = dalloc<int32_t>(m + kIdxPad);
    p->total = dalloc<unsigned long long>(1);
    GM_HIP(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
    for (int c = 0; c < kClassesTc; ++c) {
      GM_HIP(hipStreamCreateWithFlags(&p->lanes[c], hipStreamNonBlocking));
      GM_HIP(hipEventCreateWithFlags(&p->done[c], hipEventDisableTiming));
    }
    if (m > 0) {
      Pool pool(s);
      make_keys<<<plan_grid(m), kPlanThreads, 0, s>>>(g->in_idx, m, p->keys);
      GM_HIP(hipGetLastError());
      // owners, partners and stream lengths, sorted by (owner, decreasing length)
      const int cb = bits_for((uint64_t)g->max_in + 1);
      const int ob = bits_for((uint64_t)n + 1);
      Scratch k1(pool, m * 8), k2(pool, m * 8), v1(pool, m * 4), v2(pool, m * 4);
      plan_row_ids<<<plan_grid(n), kPlanThreads, 0, s>>>(g->in_off, n, v2.as<uint32_t>());
      plan_edges<<<plan_grid(m), kPlanThreads, 0, s>>>(g->in_off, g->in_idx, v2.as<uint32_t>(),
                                                       n, m, cb, k1.as<unsigned long long>(),
                                                       v1.as<uint32_t>());
      GM_HIP(hipGetLastError());
      unsigned long long* key = nullptr;
      uint32_t* val = nullptr;
      sort_pairs(pool, k1, k2, v1, v2, m, ob + cb, s, &key, &val);
      Scratch woff(pool, (n + 1) * 4);
      uint32_t* work_off = woff.as<uint32_t>();
      plan_owner_offsets<<<plan_grid(n + 1), kPlanThreads, 0, s>>>(key, m, cb, n, work_off);
      GM_HIP(hipGetLastError());
      uint32_t wh = 0;
      GM_HIP(hipMemcpyAsync(&wh, work_off + n, 4, hipMemcpyDeviceToHost, s));
      GM_HIP(hipStreamSynchronize(s));
      const int64_t w = wh;
      p->work = dalloc<uint32_t>(w);
      p->wlen = dalloc<uint32_t>(w);
      if (w > 0) {
        plan_work<<<plan_grid(w), kPlanThreads, 0, s>>>(key, val, w, cb, p->work, p->wlen);
        GM_HIP(hipGetLastError());
        // work items of owners with a table in LDS, grouped by class, largest first
        Scratch pre(pool, w * 8), flag(pool, w), start(pool, w * 4);
        exclusive_u64(pool, p->wlen, pre.as<unsigned long long>(), w, s);
        plan_item_flags<<<plan_grid(w), kPlanThreads, 0, s>>>(
            key, cb, work_off, w, g->in_off, pre.as<unsigned long long>(), wave_max, wave_work,
            block_work, flag.as<uint8_t>());
        GM_HIP(hipGetLastError());
        const int64_t ni =
            select_flagged(pool, flag.as<uint8_t>(), w, start.as<uint32_t>(), s);
        if (ni > 0) {
          Scratch it(pool, ni * sizeof(Item)), sk1(pool, ni * 8), sk2(pool, ni * 8),
              si1(pool, ni * 4), si2(pool, ni * 4), cfirst(pool, (kClassesTc + 1) * 4);
          plan_items<<<plan_grid(ni), kPlanThreads, 0, s>>>(
              start.as<uint32_t>(), ni, key, cb, work_off, g->in_off, wave_max, it.as<Item>(),
              sk1.as<unsigned long long>(), si1.as<uint32_t>());
          GM_HIP(hipGetLastError());
          unsigned long long* sk = nullptr;
          uint32_t* si = nullptr;
          sort_pairs(pool, sk1, sk2, si1, si2, ni, 35, s, &sk, &si);
          plan_class_bounds<<<1, 64, 0, s>>>(sk, ni, cfirst.as<uint32_t>());
          GM_HIP(hipGetLastError());
          uint32_t first[kClassesTc + 1] = {};
          GM_HIP(hipMemcpyAsync(first, cfirst.p, sizeof(first), hipMemcpyDeviceToHost, s));
          GM_HIP(hipStreamSynchronize(s));
          for (int c = 0; c < kClassesTc; ++c) {
            const uint32_t cnt = first[c + 1] - first[c];
            p->nitems[c] = cnt;
            p->items[c] = dalloc<Item>(cnt);
            if (cnt > 0) {
              plan_gather<Item><<<plan_grid(cnt), kPlanThreads, 0, s>>>(it.as<Item>(),
                                                                        si + first[c], cnt,
                                                                        p->items[c]);
              GM_HIP(hipGetLastError());
            }
          }
          GM_HIP(hipStreamSynchronize(s));
        }
        // owners cut into pieces: one segment per piece, one pair per (piece, partner)
        Scratch sflag(pool, n), sown(pool, n * 4);
        plan_split_flags<<<plan_grid(n), kPlanThreads, 0, s>>>(g->in_off, work_off, n, wave_max,
                                                               sflag.as<uint8_t>());
        GM_HIP(hipGetLastError());
        const int64_t nsplit =
            select_flagged(pool, sflag.as<uint8_t>(), n, sown.as<uint32_t>(), s);
        if (nsplit > 0) {
          std::vector<uint32_t> owners(nsplit), bnd(4 * nsplit);
          Scratch sbnd(pool, nsplit * 16);
          plan_split_bounds<<<plan_grid(nsplit), kPlanThreads, 0, s>>>(
              sown.as<uint32_t>(), nsplit, g->in_off, work_off, sbnd.as<uint32_t>());
          GM_HIP(hipGetLastError());
          GM_HIP(hipMemcpyAsync(owners.data(), sown.p, nsplit * 4, hipMemcpyDeviceToHost, s));
          GM_HIP(hipMemcpyAsync(bnd.data(), sbnd.p, nsplit * 16, hipMemcpyDeviceToHost, s));
          GM_HIP(hipStreamSynchronize(s));
          std::vector<PieceSeg> segs;
          uint32_t base = 0;
          for (int64_t i = 0; i < nsplit; ++i) {
            const uint32_t xb = bnd[4 * i], d = bnd[4 * i + 1] - xb;
            const uint32_t p0 = bnd[4 * i + 2], np = bnd[4 * i + 3] - p0;
            for (uint32_t tb = 0; tb < d; tb += kPieceMax) {
              const uint32_t te = std::min(d, tb + kPieceMax);
              if ((uint64_t)base + np > UINT32_MAX)
                throw Unsupported{"triangle count: too many (piece, partner) pairs"};
              segs.push_back(PieceSeg{(int32_t)owners[i], xb + tb, xb + te, 0, 0, p0, np, base});
              base += np;
            }
          }
          const int64_t nseg = (int64_t)segs.size(), npairs = base;
          Scratch dseg(pool, nseg * sizeof(PieceSeg));
          GM_HIP(hipMemcpyAsync(dseg.p, segs.data(), nseg * sizeof(PieceSeg),
                                hipMemcpyHostToDevice, s));
          plan_seg_bounds<<<plan_grid(nseg), kPlanThreads, 0, s>>>(dseg.as<PieceSeg>(), nseg,
                                                                   g->in_off, g->in_idx);
          p->pstart = dalloc<uint32_t>(npairs);
          p->plen = dalloc<uint32_t>(npairs);
          plan_pairs<<<plan_grid(npairs), kPlanThreads, 0, s>>>(
              dseg.as<PieceSeg>(), nseg, npairs, p->work, g->in_off, g->in_idx, p->pstart,
              p->plen);
          GM_HIP(hipGetLastError());
          Scratch ppre(pool, npairs * 8), pflag(pool, npairs), pstarts(pool, npairs * 4);
          exclusive_u64(pool, p->plen, ppre.as<unsigned long long>(), npairs, s);
          plan_piece_flags<<<plan_grid(npairs), kPlanThreads, 0, s>>>(
              dseg.as<PieceSeg>(), nseg, npairs, ppre.as<unsigned long long>(), block_work,
              pflag.as<uint8_t>());
          GM_HIP(hipGetLastError());
          const int64_t np = select_flagged(pool, pflag.as<uint8_t>(), npairs,
                                            pstarts.as<uint32_t>(), s);
          Scratch pit(pool, np * sizeof(PieceItem)), pk1(pool, np * 8), pk2(pool, np * 8),
              pi1(pool, np * 4), pi2(pool, np * 4);
          plan_piece_items<<<plan_grid(np), kPlanThreads, 0, s>>>(
              pstarts.as<uint32_t>(), np, dseg.as<PieceSeg>(), nseg, pit.as<PieceItem>(),
              pk1.as<unsigned long long>(), pi1.as<uint32_t>());
          GM_HIP(hipGetLastError());
          unsigned long long* pk = nullptr;
          uint32_t* pi = nullptr;
          sort_pairs(pool, pk1, pk2, pi1, pi2, np, 32, s, &pk, &pi);
          p->npieces = np;
          p->pieces = dalloc<PieceItem>(np);
          plan_gather<PieceItem><<<plan_grid(np), kPlanThreads, 0, s>>>(pit.as<PieceItem>(), pi,
                                                                        np, p->pieces);
          GM_HIP(hipGetLastError());
          GM_HIP(hipStreamSynchronize(s));
        }
      }
    }
    for (int c = 0; c < kClassesTc; ++c)
      if (!p->items[c]) p->items[c] = dalloc<Item>(0);
    GM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    free_tc_plan(g);
    throw;
  }
  return p;
}

void run_triangle_count(gm_graph g, unsigned long long* counts, unsigned long long* total_host,
                        hipStream_t s) {
  TcPlan* p = ensure_plan(g, s);
  static_assert(kTcClass[0].slots == 512 && kTcClass[1].slots == 2048 &&
                    kTcClass[2].slots == 4096 && kTcClass[3].slots == 8192 &&
                    kTcClass[4].slots == 16384 && kTcClass[5].slots == 32768 &&
                    kTcClass[5].threads == 1024 && kTcClass[6].kind == kSplitTable &&
                    kTcClass[6].slots == 32768 && kTcClass[6].threads == 1024 &&
                    4 * kPieceMax <= kTcClass[6].slots,
                "kernel instances below follow the class table");
  // Each class on its own stream, forked from s and joined back: the
  // launches run side by side (counts are only added to, atomically).
  GM_HIP(hipEventRecord(p->fork, s));
  const auto on = [&](int c) {
    GM_HIP(hipStreamWaitEvent(p->lanes[c], p->fork, 0));
    return p->lanes[c];
  };
  const auto join = [&](int c) {
    GM_HIP(hipGetLastError());
    GM_HIP(hipEventRecord(p->done[c], p->lanes[c]));
    GM_HIP(hipStreamWaitEvent(s, p->done[c], 0));
  };
  if (p->npieces > 0) {
    tc_piece<32768, 1024><<<(unsigned)p->npieces, 1024, 0, on(6)>>>(
        p->pieces, g->in_off, p->keys, p->work, p->pstart, p->plen, counts);
    join(6);
  }
  const auto block = [&](int c, auto kern) {
    if (p->nitems[c] > 0) {
      kern<<<(unsigned)p->nitems[c], kTcClass[c].threads, 0, on(c)>>>(
          p->items[c], g->in_off, p->keys, p->work, p->wlen, counts);
      join(c);
    }
  };
  block(5, tc_block<32768, 1024>);
  block(4, tc_block<16384, 512>);
  block(3, tc_block<8192, 512>);
  block(2, tc_block<4096, 512>);
  const auto wave = [&](int c, auto kern) {
    if (p->nitems[c] > 0) {
      const int64_t blocks = (p->nitems[c] + kWaves - 1) / kWaves;
      kern<<<(unsigned)blocks, kThreads, 0, on(c)>>>(p->items[c], p->nitems[c], g->in_off,
                                                     p->keys, p->work, p->wlen, counts);
      join(c);
    }
  };
  wave(1, tc_wave<2048>);
  wave(0, tc_wave<512>);
  if (total_host) {
    zero_u64<<<1, 64, 0, s>>>(p->total, 1);
    int64_t blocks = (g->n + kThreads - 1) / kThreads;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    sum_u64<<<(unsigned)blocks, kThreads, 0, s>>>(counts, g->n, p->total);
    GM_HIP(hipGetLastError());
    GM_HIP(hipMemcpyAsync(total_host, p->total, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          s));
    GM_HIP(hipStreamSynchronize(s));
  }
}

void zero_counts(unsigned long long* a, int64_t n, hipStream_t s) {
  int64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  zero_u64<<<(unsigned)blocks, kThreads, 0, s>>>(a, n);
  GM_HIP(hipGetLastError());
}

}  // namespace gm
