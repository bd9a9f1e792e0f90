/*
 * Seeded synthetic inputs for the GraphMat workloads (RMAT graphs, edge
 * weights, source sets, a bipartite rating graph, dense factors).
 *
 * This module is shared by the GPU path's tests/bench and by the CPU oracle.
 * It holds no part of the method's arithmetic: it only draws random numbers
 * and shapes them into raw inputs (a raw COO edge list with self-loops and
 * duplicates still present, weights, vertex ids, ratings).
 *
 * Randomness is counter-based: value i of stream (seed, stream) is the i-th
 * output of a SplitMix64 generator (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) whose state starts at a
 * value derived from (seed, stream). Every output therefore depends only on
 * its (seed, stream, index) and never on thread count or call order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

/* SplitMix64 output function. */
static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Starting state of stream (seed, stream). */
static inline uint64_t stream_state(uint64_t seed, uint64_t stream) {
  return mix64(mix64(seed + GOLDEN) ^ (stream * 0xD1B54A32D192ED03ULL));
}

/* i-th output of the SplitMix64 sequence that starts at state s0. */
static inline uint64_t rng_at(uint64_t s0, uint64_t i) { return mix64(s0 + (i + 1) * GOLDEN); }

/* Uniform double in [0, 1) with 53 random bits. */
static inline double unit53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* Stream ids, one per kind of draw. */
enum {
  ST_RMAT = 1,
  ST_WEIGHT_U32 = 2,
  ST_WEIGHT_F32 = 3,
  ST_SOURCES = 4,
  ST_UNIFORM = 5,
  ST_NORMAL = 6,
  ST_CF_DEGREE = 7,
  ST_CF_ITEMPERM = 8,
  ST_CF_PICK = 9,
  ST_CF_TRUE = 10,
  ST_CF_NOISE = 11,
  ST_CF_ADJUST = 12,
};

uint64_t gg_rng_u64(uint64_t seed, uint64_t stream, uint64_t i) {
  return rng_at(stream_state(seed, stream), i);
}

/*
 * Recursive-matrix (RMAT) edge generator, Graph500 style without noise or
 * label permutation: for each of m edges and each of `scale` levels, one
 * uniform draw picks a quadrant (a: top-left, b: top-right = dst bit set,
 * c: bottom-left = src bit set, d: both bits set), most significant bit
 * first. Self-loops and duplicate edges are kept.
 */
void gg_rmat(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed,
             int32_t* src, int32_t* dst) {
  const uint64_t s0 = stream_state(seed, ST_RMAT);
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint32_t s = 0, d = 0;
    for (int32_t l = 0; l < scale; ++l) {
      const double u = unit53(rng_at(s0, (uint64_t)e * (uint64_t)scale + (uint64_t)l));
      const uint32_t bit = 1u << (scale - 1 - l);
      if (u < a) {
      } else if (u < ab) {
        d |= bit;
      } else if (u < abc) {
        s |= bit;
      } else {
        s |= bit;
        d |= bit;
      }
    }
    src[e] = (int32_t)s;
    dst[e] = (int32_t)d;
  }
}

/* Key that names an ordered vertex pair; duplicates of an edge share it. */
static inline uint64_t pair_key(int32_t u, int32_t v) {
  return ((uint64_t)(uint32_t)u << 32) | (uint64_t)(uint32_t)v;
}

/*
 * Integer edge weights in [lo, hi], uniform, drawn per ordered vertex pair
 * (so duplicate copies of an edge carry the same weight).
 */
void gg_weights_u32(int64_t m, const int32_t* src, const int32_t* dst, uint64_t seed,
                    uint32_t lo, uint32_t hi, uint32_t* w) {
  const uint64_t s0 = stream_state(seed, ST_WEIGHT_U32);
  const double span = (double)hi - (double)lo + 1.0;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    const double u = unit53(rng_at(s0, pair_key(src[e], dst[e])));
    uint64_t v = (uint64_t)lo + (uint64_t)floor(span * u);
    if (v > hi) v = hi;
    w[e] = (uint32_t)v;
  }
}

/* Real edge weights uniform in [lo, hi), drawn per ordered vertex pair. */
void gg_weights_f32(int64_t m, const int32_t* src, const int32_t* dst, uint64_t seed, double lo,
                    double hi, float* w) {
  const uint64_t s0 = stream_state(seed, ST_WEIGHT_F32);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    const double u = unit53(rng_at(s0, pair_key(src[e], dst[e])));
    w[e] = (float)(lo + (hi - lo) * u);
  }
}

/* n floats uniform in [lo, hi). */
void gg_uniform_f32(int64_t n, uint64_t seed, double lo, double hi, float* out) {
  const uint64_t s0 = stream_state(seed, ST_UNIFORM);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = (float)(lo + (hi - lo) * unit53(rng_at(s0, (uint64_t)i)));
}

/* Standard normal from draws (2i, 2i+1) of a stream, by Box-Muller. */
static inline double normal_at(uint64_t s0, uint64_t i) {
  const double u1 = 1.0 - unit53(rng_at(s0, 2 * i)); /* (0, 1] */
  const double u2 = unit53(rng_at(s0, 2 * i + 1));
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* n floats from N(0, std^2). */
void gg_normal_f32(int64_t n, uint64_t seed, double stddev, float* out) {
  const uint64_t s0 = stream_state(seed, ST_NORMAL);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = (float)(stddev * normal_at(s0, (uint64_t)i));
}

/*
 * k distinct source vertices among those that have at least one out-edge
 * that is not a self-loop in the raw edge list. Vertex `first` (if it
 * qualifies) is always entry 0; the rest are drawn uniformly in order.
 * Returns the number of sources written (< k only if too few qualify).
 */
int64_t gg_sources(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, int64_t k,
                   uint64_t seed, int32_t first, int32_t* out) {
  uint8_t* ok = (uint8_t*)calloc((size_t)n, 1);
  uint8_t* taken = (uint8_t*)calloc((size_t)n, 1);
  if (!ok || !taken) {
    free(ok);
    free(taken);
    return -1;
  }
  int64_t navail = 0;
  for (int64_t e = 0; e < m; ++e)
    if (src[e] != dst[e] && !ok[src[e]]) {
      ok[src[e]] = 1;
      ++navail;
    }
  int64_t cnt = 0;
  if (first >= 0 && first < n && ok[first] && k > 0) {
    out[cnt++] = first;
    taken[first] = 1;
  }
  const uint64_t s0 = stream_state(seed, ST_SOURCES);
  const int64_t want = k < navail ? k : navail;
  for (uint64_t i = 0; cnt < want; ++i) {
    int64_t v = (int64_t)(unit53(rng_at(s0, i)) * (double)n);
    if (v >= n) v = n - 1;
    if (ok[v] && !taken[v]) {
      taken[v] = 1;
      out[cnt++] = (int32_t)v;
    }
  }
  free(ok);
  free(taken);
  return cnt;
}

/* ---------------------------------------------------------------------- */
/* Bipartite rating graph shaped like the Netflix prize matrix.            */
/* ---------------------------------------------------------------------- */

/*
 * Per-user rating counts: a continuous power law p(d) ~ d^-gamma on
 * [dmin, dmax + 1), floored, then adjusted by single steps (users picked in
 * a seeded order) so the counts sum to exactly `total` and stay in
 * [dmin, dmax].
 */
int gg_cf_degrees(int64_t n_users, int64_t dmin, int64_t dmax, double gamma, int64_t total,
                  uint64_t seed, int64_t* deg) {
  const uint64_t s0 = stream_state(seed, ST_CF_DEGREE);
  const double e1 = 1.0 - gamma;
  const double lo = pow((double)dmin, e1), hi = pow((double)(dmax + 1), e1);
  int64_t sum = 0;
  for (int64_t u = 0; u < n_users; ++u) {
    const double x = pow(lo + unit53(rng_at(s0, (uint64_t)u)) * (hi - lo), 1.0 / e1);
    int64_t d = (int64_t)floor(x);
    if (d < dmin) d = dmin;
    if (d > dmax) d = dmax;
    deg[u] = d;
    sum += d;
  }
  if (total < n_users * dmin || total > n_users * dmax) return -1;
  const uint64_t s1 = stream_state(seed, ST_CF_ADJUST);
  /* Scale toward the target first, then fix the residue one step at a time. */
  if (sum != total) {
    const double f = (double)total / (double)sum;
    sum = 0;
    for (int64_t u = 0; u < n_users; ++u) {
      int64_t d = (int64_t)floor((double)deg[u] * f);
      if (d < dmin) d = dmin;
      if (d > dmax) d = dmax;
      deg[u] = d;
      sum += d;
    }
  }
  for (uint64_t i = 0; sum != total; ++i) {
    int64_t u = (int64_t)(unit53(rng_at(s1, i)) * (double)n_users);
    if (u >= n_users) u = n_users - 1;
    if (sum < total && deg[u] < dmax) {
      ++deg[u];
      ++sum;
    } else if (sum > total && deg[u] > dmin) {
      --deg[u];
      --sum;
    }
  }
  return 0;
}

typedef struct {
  double key;
  int32_t idx;
} keyed_t;

/* descending by key, ties by index */
static int cmp_key_desc(const void* a, const void* b) {
  const keyed_t* x = (const keyed_t*)a;
  const keyed_t* y = (const keyed_t*)b;
  if (x->key != y->key) return x->key < y->key ? 1 : -1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

static int cmp_i32(const void* a, const void* b) {
  const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/*
 * Ratings. Users are rows; `off` (n_users + 1) is the prefix sum of the
 * per-user counts and fixes where each user's ratings go. Each user draws
 * its items without replacement with probability proportional to
 * (rank + 1)^-alpha, where rank is the item's place in a seeded random
 * permutation of the items; draws with replacement are rejected when the
 * item is already taken, which is the same distribution as successive
 * weighted sampling. A user that takes more than a quarter of the items
 * instead keeps the top keys u^(1/w) (Efraimidis and Spirakis, 2006).
 * Each user's items are sorted. Ratings are
 * clip(round(3 + u*.v* + N(0, sigma^2)), 1, 5) with true factors u*, v*
 * (rows of k floats) supplied by the caller.
 */
int gg_cf_ratings(int64_t n_users, int64_t n_items, const int64_t* off, double alpha,
                  uint64_t seed, int32_t k, const float* ustar, const float* vstar,
                  double sigma, int32_t* item_out, uint8_t* rating_out) {
  /* Seeded permutation of the items (Fisher-Yates). */
  int32_t* perm = (int32_t*)malloc((size_t)n_items * sizeof(int32_t));
  double* cum = (double*)malloc((size_t)n_items * sizeof(double));
  double* wgt = (double*)malloc((size_t)n_items * sizeof(double));
  if (!perm || !cum || !wgt) {
    free(perm);
    free(cum);
    free(wgt);
    return -1;
  }
  const uint64_t sp = stream_state(seed, ST_CF_ITEMPERM);
  for (int64_t i = 0; i < n_items; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n_items - 1; i > 0; --i) {
    int64_t j = (int64_t)(unit53(rng_at(sp, (uint64_t)i)) * (double)(i + 1));
    if (j > i) j = i;
    const int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
  /* weight of the item at rank r is (r+1)^-alpha */
  double acc = 0.0;
  for (int64_t r = 0; r < n_items; ++r) {
    wgt[perm[r]] = pow((double)(r + 1), -alpha);
  }
  for (int64_t r = 0; r < n_items; ++r) {
    acc += pow((double)(r + 1), -alpha);
    cum[r] = acc;
  }
  const double wsum = acc;
  const uint64_t spick = stream_state(seed, ST_CF_PICK);
  const uint64_t snoise = stream_state(seed, ST_CF_NOISE);
  int fail = 0;
#pragma omp parallel
  {
    uint8_t* taken = (uint8_t*)calloc((size_t)n_items, 1);
    keyed_t* kv = (keyed_t*)malloc((size_t)n_items * sizeof(keyed_t));
    if (!taken || !kv) fail = 1;
#pragma omp for schedule(dynamic, 256)
    for (int64_t u = 0; u < n_users; ++u) {
      if (!taken || !kv) continue;
      const int64_t d = off[u + 1] - off[u];
      int32_t* items = item_out + off[u];
      /* per-user draws live at indices [u * 2^24, (u+1) * 2^24) of the stream */
      const uint64_t base = (uint64_t)u << 24;
      if (d * 4 > n_items) {
        for (int64_t i = 0; i < n_items; ++i) {
          const double uu = 1.0 - unit53(rng_at(spick, base + (uint64_t)i)); /* (0,1] */
          kv[i].key = log(uu) / wgt[i];                                     /* log(u^(1/w)) */
          kv[i].idx = (int32_t)i;
        }
        qsort(kv, (size_t)n_items, sizeof(keyed_t), cmp_key_desc);
        for (int64_t i = 0; i < d; ++i) items[i] = kv[i].idx;
      } else {
        int64_t got = 0;
        for (uint64_t t = 0; got < d; ++t) {
          const double x = unit53(rng_at(spick, base + t)) * wsum;
          int64_t lo = 0, hi = n_items - 1; /* first rank with cum > x */
          while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (cum[mid] > x)
              hi = mid;
            else
              lo = mid + 1;
          }
          const int32_t it = perm[lo];
          if (!taken[it]) {
            taken[it] = 1;
            items[got++] = it;
          }
        }
        for (int64_t i = 0; i < d; ++i) taken[items[i]] = 0;
      }
      qsort(items, (size_t)d, sizeof(int32_t), cmp_i32);
      for (int64_t i = 0; i < d; ++i) {
        const int32_t it = items[i];
        double dot = 0.0;
        for (int32_t q = 0; q < k; ++q) dot += (double)ustar[u * k + q] * (double)vstar[(int64_t)it * k + q];
        const double r = 3.0 + dot + sigma * normal_at(snoise, (uint64_t)(off[u] + i));
        long v = lround(r);
        if (v < 1) v = 1;
        if (v > 5) v = 5;
        rating_out[off[u] + i] = (uint8_t)v;
      }
    }
    free(taken);
    free(kv);
  }
  free(perm);
  free(cum);
  free(wgt);
  return fail ? -1 : 0;
}
