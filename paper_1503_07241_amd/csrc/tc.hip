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
// the endpoint whose in-list is longer (its "owner"; ties go to v). An owner
// x puts in(x) in a hash table (LDS, or global memory for very long lists)
// once, then streams the shorter in-list of every partner through it, one
// probe per element. The match count of edge (u -> v) is credited to the
// receiver v, as APPLY prescribes. Owner/partner lists are built once per
// graph and cut into work items of bounded size, one wavefront or workgroup
// each. Partner lists are walked in windows of 64 per wavefront with their
// elements spread evenly over the lanes (prefix sum + 6-step owner search).
// All counts are exact integers, independent of scheduling.
#include <algorithm>
#include <vector>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kWaveMax = 1024;          // owners with |in(x)| <= this: LDS table per wavefront
constexpr uint32_t kBlockMax = 8192;         // owners up to this: LDS table per workgroup
constexpr uint32_t kWaveSlots = 2048;
constexpr uint32_t kBlockSlots = 16384;      // 64 KB
constexpr uint32_t kCreditPartner = 0x80000000u;  // partner entry flag: credit goes to it
constexpr int32_t kEmpty = -1;
constexpr int kRounds = 4;                   // element loads in flight per lane
constexpr int kBlockThreads = 512;           // workgroup size of the LDS-table class
constexpr int kBlockWaves = kBlockThreads / 64;

// A work item: owner x and a range of its partner list.
struct Item {
  int32_t owner;
  uint32_t p_begin;
  uint32_t p_end;
  uint32_t table;  // global-table index (largest owners), else unused
};

struct TcPlan {
  Item* items[3] = {nullptr, nullptr, nullptr};  // wave / block / global-table classes
  int64_t nitems[3] = {0, 0, 0};
  uint32_t* work = nullptr;        // partner id | kCreditPartner, grouped by owner
  int32_t* gtable = nullptr;       // hash tables of the largest owners
  uint64_t* gtable_off = nullptr;  // per table: first slot
  uint32_t* gtable_mask = nullptr;
  int32_t* gtable_owner = nullptr;
  int64_t ntables = 0;
  unsigned long long* total = nullptr;
  // tuning the plan was built with
  uint32_t wave_max = 0, wave_work = 0, block_work = 0;
};

// 32-bit integer mixer (xor-shift-multiply rounds); every output bit depends
// on every input bit, which matters because RMAT ids have very skewed bits.
__device__ inline uint32_t hash_id(int32_t id) {
  uint32_t x = (uint32_t)id;
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ inline void table_insert(int32_t* T, uint32_t mask, int32_t id) {
  uint32_t s = hash_id(id) & mask;
  while (atomicCAS(&T[s], kEmpty, id) != kEmpty) s = (s + 1) & mask;
}

// The table holds at most half as many ids as slots, so a probe ends.
__device__ inline bool table_has(const int32_t* T, uint32_t mask, int32_t id) {
  uint32_t s = hash_id(id) & mask;
  for (;;) {
    const int32_t t = T[s];
    if (t == id) return true;
    if (t == kEmpty) return false;
    s = (s + 1) & mask;
  }
}

__device__ inline uint32_t wave_incl_scan(uint32_t x, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  return x;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline unsigned long long lanes_below(int lane) {
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Walk partners [p_begin, p_end) with stride j_step (windows of 64 partners,
// one per lane) through table T. Matches credited to the owner are returned;
// matches credited to a partner are added to counts[partner]. wcnt is this
// wavefront's 64-entry LDS scratch.
__device__ inline unsigned long long walk_partners(const int32_t* T, uint32_t mask,
                                                   const uint32_t* __restrict__ work,
                                                   uint32_t p_begin, uint32_t p_end,
                                                   uint32_t j_step,
                                                   const uint32_t* __restrict__ in_off,
                                                   const int32_t* __restrict__ in_idx,
                                                   unsigned long long* counts, uint32_t* wcnt) {
  const int lane = threadIdx.x & 63;
  unsigned long long own_cnt = 0;
  for (uint32_t j0 = p_begin; j0 < p_end; j0 += j_step) {
    const uint32_t j = j0 + lane;
    uint32_t pb = 0, pd = 0, entry = 0;
    if (j < p_end) {
      entry = work[j];
      const int32_t y = (int32_t)(entry & ~kCreditPartner);
      pb = in_off[y];
      pd = in_off[y + 1] - pb;
    }
    wcnt[lane] = 0;
    const uint32_t incl = wave_incl_scan(pd, lane);
    const uint32_t excl = incl - pd;
    const uint32_t tot = __shfl(incl, 63, 64);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    for (uint32_t i0 = 0; i0 < tot; i0 += 64 * kRounds) {
      // kRounds rounds of 64 elements: all element loads first, then probes.
      int own[kRounds];
      int32_t elem[kRounds];
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        const uint32_t i = i0 + r * 64 + lane;
        int o = 0;  // partner owning element i: the last lane with excl <= i
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
          const uint32_t ex = __shfl(excl, o + step, 64);
          if (ex <= i) o += step;
        }
        const uint32_t oex = __shfl(excl, o, 64);
        const uint32_t opb = __shfl(pb, o, 64);
        own[r] = o;
        elem[r] = in_idx[i < tot ? opb + (i - oex) : 0u];
      }
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        const uint32_t i = i0 + r * 64 + lane;
        const int o = own[r];
        const bool hit = i < tot && table_has(T, mask, elem[r]);
        // Lanes of one partner are contiguous: the first lane of each run
        // adds the run's hits to the partner's counter (one adder each).
        const int prev = __shfl_up(o, 1, 64);
        const bool head = i < tot && (lane == 0 || prev != o);
        const unsigned long long heads = __ballot(head);
        const unsigned long long hits = __ballot(hit);
        const unsigned long long after = heads & ~lanes_below(lane + 1);
        const int end = after ? __ffsll((long long)after) - 1 : 64;
        const unsigned long long run = (end == 64 ? ~0ull : lanes_below(end)) & ~lanes_below(lane);
        if (head) {
          const uint32_t cnt = (uint32_t)__popcll(hits & run);
          if (cnt) atomicAdd(&wcnt[o], cnt);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    const uint32_t mine = wcnt[lane];
    if (j < p_end && mine) {
      if (entry & kCreditPartner)
        atomicAdd(&counts[entry & ~kCreditPartner], (unsigned long long)mine);
      else
        own_cnt += mine;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  return own_cnt;
}

// One wavefront per work item of an owner with |in(x)| <= kWaveMax.
__global__ __launch_bounds__(kThreads) void tc_wave(const Item* __restrict__ items, int64_t nitems,
                                                    const uint32_t* __restrict__ in_off,
                                                    const int32_t* __restrict__ in_idx,
                                                    const uint32_t* __restrict__ work,
                                                    unsigned long long* counts) {
  __shared__ int32_t tables[kWaves][kWaveSlots];
  __shared__ uint32_t wcnt[kWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * kWaves + wave;
  if (r >= nitems) return;  // the whole wavefront leaves together
  const Item it = items[r];
  const int32_t x = it.owner;
  const uint32_t b = in_off[x], d = in_off[x + 1] - b;
  uint32_t slots = 64;
  while (slots < 2 * d) slots <<= 1;
  int32_t* T = tables[wave];
  for (uint32_t k = lane; k < slots; k += 64) T[k] = kEmpty;
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  for (uint32_t k = lane; k < d; k += 64) table_insert(T, slots - 1, in_idx[b + k]);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  const unsigned long long c = wave_sum_u64(
      walk_partners(T, slots - 1, work, it.p_begin, it.p_end, 64, in_off, in_idx, counts,
                    wcnt[wave]));
  if (lane == 0 && c) atomicAdd(&counts[x], c);
}

// One workgroup per work item; the owner's table in LDS (kGlobal = false) or
// one of the precomputed global tables.
template <bool kGlobal>
__global__ __launch_bounds__(kBlockThreads) void tc_block(const Item* __restrict__ items,
                                                     const uint32_t* __restrict__ in_off,
                                                     const int32_t* __restrict__ in_idx,
                                                     const uint32_t* __restrict__ work,
                                                     const int32_t* __restrict__ gtable,
                                                     const uint64_t* __restrict__ gtable_off,
                                                     const uint32_t* __restrict__ gtable_mask,
                                                     unsigned long long* counts) {
  __shared__ int32_t ltable[kGlobal ? 1 : kBlockSlots];
  __shared__ uint32_t wcnt[kBlockWaves][64];
  __shared__ unsigned long long part[kBlockWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const Item it = items[blockIdx.x];
  const int32_t x = it.owner;
  const int32_t* T;
  uint32_t mask;
  if constexpr (kGlobal) {
    T = gtable + gtable_off[it.table];
    mask = gtable_mask[it.table];
  } else {
    const uint32_t b = in_off[x], d = in_off[x + 1] - b;
    uint32_t slots = 64;
    while (slots < 2 * d) slots <<= 1;
    mask = slots - 1;
    for (uint32_t k = threadIdx.x; k < slots; k += kBlockThreads) ltable[k] = kEmpty;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < d; k += kBlockThreads)
      table_insert(ltable, mask, in_idx[b + k]);
    __syncthreads();
    T = ltable;
  }
  const unsigned long long c =
      wave_sum_u64(walk_partners(T, mask, work, it.p_begin + wave * 64, it.p_end,
                                 kBlockWaves * 64, in_off, in_idx, counts, wcnt[wave]));
  if (lane == 0) part[wave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int i = 0; i < kBlockWaves; ++i) t += part[i];
    if (t) atomicAdd(&counts[x], t);
  }
}

// Global tables of the largest owners, built once per graph.
__global__ __launch_bounds__(kThreads) void build_tables(const int32_t* __restrict__ owner,
                                                         const uint64_t* __restrict__ toff,
                                                         const uint32_t* __restrict__ tmask,
                                                         const uint32_t* __restrict__ in_off,
                                                         const int32_t* __restrict__ in_idx,
                                                         int32_t* __restrict__ gtable) {
  const int32_t x = owner[blockIdx.x];
  int32_t* T = gtable + toff[blockIdx.x];
  const uint32_t mask = tmask[blockIdx.x];
  const uint32_t b = in_off[x], d = in_off[x + 1] - b;
  for (uint32_t k = threadIdx.x; k <= mask; k += kThreads) T[k] = kEmpty;
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < d; k += kThreads) table_insert(T, mask, in_idx[b + k]);
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

TcPlan* plan(gm_graph g) { return static_cast<TcPlan*>(g->tc_plan); }

}  // namespace

static TcPlan* ensure_plan(gm_graph g, hipStream_t s);

void free_tc_plan(gm_graph g) {
  TcPlan* p = plan(g);
  if (!p) return;
  for (int c = 0; c < 3; ++c) dfree(p->items[c]);
  dfree(p->work);
  dfree(p->gtable);
  dfree(p->gtable_off);
  dfree(p->gtable_mask);
  dfree(p->gtable_owner);
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
  std::vector<uint32_t> in_off(n + 1), out_off(n + 1);
  std::vector<int32_t> out_idx(m);
  GM_HIP(hipMemcpyAsync(in_off.data(), g->in_off, (n + 1) * 4, hipMemcpyDeviceToHost, s));
  GM_HIP(hipMemcpyAsync(out_off.data(), g->out_off, (n + 1) * 4, hipMemcpyDeviceToHost, s));
  if (m > 0)
    GM_HIP(hipMemcpyAsync(out_idx.data(), g->out_idx, m * 4, hipMemcpyDeviceToHost, s));
  GM_HIP(hipStreamSynchronize(s));
  auto din = [&](int64_t v) { return in_off[v + 1] - in_off[v]; };
  // Owner of DAG edge (u -> v): the endpoint with the longer in-list (ties: v).
  // Edges with an empty in-list at either end close no triangle and are skipped.
  std::vector<uint32_t> work_off(n + 1, 0);
  for (int64_t u = 0; u < n; ++u)
    for (uint32_t e = out_off[u]; e < out_off[u + 1]; ++e) {
      const int32_t v = out_idx[e];
      if (din(u) == 0 || din(v) == 0) continue;
      ++work_off[(din(u) > din(v) ? u : v) + 1];
    }
  for (int64_t v = 0; v < n; ++v) work_off[v + 1] += work_off[v];
  std::vector<uint32_t> work(work_off[n]), cur(work_off.begin(), work_off.end() - 1);
  for (int64_t u = 0; u < n; ++u)
    for (uint32_t e = out_off[u]; e < out_off[u + 1]; ++e) {
      const int32_t v = out_idx[e];
      if (din(u) == 0 || din(v) == 0) continue;
      if (din(u) > din(v))
        work[cur[u]++] = (uint32_t)v | kCreditPartner;  // owner u scans in(v), credits v
      else
        work[cur[v]++] = (uint32_t)u;  // owner v scans in(u), credits itself
    }
  // Work items: each owner's partners cut where the scanned elements reach
  // the class's budget (a partner longer than the budget is an item alone);
  // workgroup items also hold at most one 64-partner window per wavefront so
  // that all of their wavefronts have partners to walk.
  std::vector<Item> items[3];
  std::vector<uint64_t> goff;
  std::vector<uint32_t> gmask;
  std::vector<int32_t> gowner;
  uint64_t gslots = 0;
  for (int64_t x = 0; x < n; ++x) {
    const uint32_t p0 = work_off[x], p1 = work_off[x + 1];
    if (p0 == p1) continue;
    const uint32_t d = din(x);
    const int cls = d <= wave_max ? 0 : d <= kBlockMax ? 1 : 2;
    const uint32_t budget = cls == 0 ? wave_work : block_work;
    const uint32_t max_partners = cls == 0 ? UINT32_MAX : (uint32_t)kBlockWaves * 64;
    uint32_t table = 0;
    if (cls == 2) {
      uint64_t slots = 64;
      while (slots < 2ull * d) slots <<= 1;
      table = (uint32_t)goff.size();
      goff.push_back(gslots);
      gmask.push_back((uint32_t)(slots - 1));
      gowner.push_back((int32_t)x);
      gslots += slots;
    }
    uint32_t start = p0;
    uint64_t acc = 0;
    for (uint32_t j = p0; j < p1; ++j) {
      const uint32_t y = work[j] & ~kCreditPartner;
      const uint64_t len = din(y);
      if (acc > 0 && (acc + len > budget || j - start >= max_partners)) {
        items[cls].push_back({(int32_t)x, start, j, table});
        start = j;
        acc = 0;
      }
      acc += len;
    }
    items[cls].push_back({(int32_t)x, start, p1, table});
  }
  // Largest items first so the long ones start early.
  for (int c = 0; c < 3; ++c)
    std::stable_sort(items[c].begin(), items[c].end(), [&](const Item& a, const Item& b) {
      return a.p_end - a.p_begin > b.p_end - b.p_begin;
    });
  TcPlan* p = new TcPlan();
  g->tc_plan = p;
  p->wave_max = wave_max;
  p->wave_work = wave_work;
  p->block_work = block_work;
  try {
    for (int c = 0; c < 3; ++c) {
      p->nitems[c] = (int64_t)items[c].size();
      p->items[c] = dalloc<Item>(items[c].size());
      if (!items[c].empty())
        GM_HIP(hipMemcpyAsync(p->items[c], items[c].data(), items[c].size() * sizeof(Item),
                              hipMemcpyHostToDevice, s));
    }
    p->work = dalloc<uint32_t>(work.size());
    if (!work.empty())
      GM_HIP(hipMemcpyAsync(p->work, work.data(), work.size() * 4, hipMemcpyHostToDevice, s));
    p->ntables = (int64_t)goff.size();
    p->gtable = dalloc<int32_t>(gslots);
    p->gtable_off = dalloc<uint64_t>(goff.size());
    p->gtable_mask = dalloc<uint32_t>(gmask.size());
    p->gtable_owner = dalloc<int32_t>(gowner.size());
    if (p->ntables > 0) {
      GM_HIP(hipMemcpyAsync(p->gtable_off, goff.data(), goff.size() * 8, hipMemcpyHostToDevice, s));
      GM_HIP(hipMemcpyAsync(p->gtable_mask, gmask.data(), gmask.size() * 4, hipMemcpyHostToDevice,
                            s));
      GM_HIP(hipMemcpyAsync(p->gtable_owner, gowner.data(), gowner.size() * 4,
                            hipMemcpyHostToDevice, s));
      build_tables<<<(unsigned)p->ntables, kThreads, 0, s>>>(
          p->gtable_owner, p->gtable_off, p->gtable_mask, g->in_off, g->in_idx, p->gtable);
      GM_HIP(hipGetLastError());
    }
    p->total = dalloc<unsigned long long>(1);
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
  if (p->nitems[2] > 0)
    tc_block<true><<<(unsigned)p->nitems[2], kBlockThreads, 0, s>>>(
        p->items[2], g->in_off, g->in_idx, p->work, p->gtable, p->gtable_off, p->gtable_mask,
        counts);
  if (p->nitems[1] > 0)
    tc_block<false><<<(unsigned)p->nitems[1], kBlockThreads, 0, s>>>(
        p->items[1], g->in_off, g->in_idx, p->work, nullptr, nullptr, nullptr, counts);
  if (p->nitems[0] > 0) {
    const int64_t blocks = (p->nitems[0] + kWaves - 1) / kWaves;
    tc_wave<<<(unsigned)blocks, kThreads, 0, s>>>(p->items[0], p->nitems[0], g->in_off, g->in_idx,
                                                  p->work, counts);
  }
  GM_HIP(hipGetLastError());
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
