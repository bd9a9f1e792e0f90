/*
 * Host-only driver for the sanitizer build of the oracle (test
 * infrastructure): built with AddressSanitizer and UndefinedBehaviorSanitizer
 * together with oracle/oracle.c, it runs every oracle entry point on small
 * seeded graphs (a random graph with isolated vertices, a single vertex,
 * a graph without edges) and checks a few identities between them, so that
 * an out-of-bounds access, a use of freed memory, a leak or undefined
 * arithmetic anywhere in the oracle stops the run. Prints "ok" on success.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int32_t orc_bfs(int64_t n, const int64_t* off, const int32_t* idx, int64_t nroots,
                const int32_t* roots, int32_t* level);
int orc_dijkstra(int64_t n, const int64_t* off, const int32_t* idx, const uint32_t* w,
                 int64_t nsrc, const int32_t* srcs, uint32_t* dist);
int32_t orc_run_min_program(int64_t n, const int64_t* off, const int32_t* idx,
                            const uint32_t* w, uint32_t* prop, uint8_t* active,
                            int32_t max_iters);
int orc_pagerank(int64_t n, const int64_t* in_off, const int32_t* in_src, const double* in_w,
                 const int64_t* outdeg, double r, int32_t T, const double* tele, double* hist);
int orc_pagerank_vjp_w(int64_t n, const int64_t* out_off, const int32_t* out_dst,
                       const double* out_w, double r, int32_t T, const double* hist,
                       const double* c, double* grad_w);
int orc_tc_per_vertex(int64_t n, const int64_t* in_off, const int32_t* in_src, int64_t nv,
                      const int32_t* verts, uint64_t* counts);
uint64_t orc_tc_total(int64_t n, const int64_t* in_off, const int32_t* in_src);
int orc_cf(int64_t n_users, int64_t n_items, int64_t m, const int32_t* user, const int32_t* item,
           const uint8_t* rating, int32_t K, const float* PU, const float* PV, double lambda,
           double* loss, double* gU, double* gV);
int orc_bfs_certificate(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        const int32_t* lv, int32_t root, int32_t inf);

static uint64_t rng = 88172645463325252ull;  // xorshift64, fixed seed
static uint32_t next_u32(void) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (uint32_t)(rng >> 11);
}

#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      exit(1);                                                \
    }                                                         \
  } while (0)

/* A directed graph as sorted, duplicate-free CSR (out-lists by source). */
typedef struct {
  int64_t n, m;
  int64_t* off;
  int32_t* idx;
  uint32_t* w;
} Csr;

static int cmp_pair(const void* a, const void* b) {
  const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return x < y ? -1 : x > y;
}

/* Build CSR from m0 random pairs (self-loops and duplicates dropped); keep
 * only pairs with src < dst when dag != 0. Vertices >= n_active stay isolated. */
static Csr make_graph(int64_t n, int64_t n_active, int64_t m0, int dag) {
  Csr g;
  int64_t* key = (int64_t*)malloc((size_t)(m0 > 0 ? m0 : 1) * sizeof(int64_t));
  int64_t m = 0;
  for (int64_t i = 0; i < m0 && n_active > 0; ++i) {
    int64_t s = next_u32() % n_active, d = next_u32() % n_active;
    if (s == d) continue;
    if (dag && s > d) {
      const int64_t t = s;
      s = d;
      d = t;
    }
    key[m++] = s * n + d;
  }
  qsort(key, (size_t)m, sizeof(int64_t), cmp_pair);
  int64_t u = 0;
  for (int64_t i = 0; i < m; ++i)
    if (i == 0 || key[i] != key[i - 1]) key[u++] = key[i];
  g.n = n;
  g.m = u;
  g.off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  g.idx = (int32_t*)malloc((size_t)(u > 0 ? u : 1) * sizeof(int32_t));
  g.w = (uint32_t*)malloc((size_t)(u > 0 ? u : 1) * sizeof(uint32_t));
  for (int64_t i = 0; i < u; ++i) {
    ++g.off[key[i] / n + 1];
    g.idx[i] = (int32_t)(key[i] % n);
    g.w[i] = 1 + next_u32() % 1000;
  }
  for (int64_t v = 0; v < n; ++v) g.off[v + 1] += g.off[v];
  free(key);
  return g;
}

static Csr transpose(const Csr* g) {
  Csr t;
  t.n = g->n;
  t.m = g->m;
  t.off = (int64_t*)calloc((size_t)g->n + 1, sizeof(int64_t));
  t.idx = (int32_t*)malloc((size_t)(g->m > 0 ? g->m : 1) * sizeof(int32_t));
  t.w = (uint32_t*)malloc((size_t)(g->m > 0 ? g->m : 1) * sizeof(uint32_t));
  for (int64_t e = 0; e < g->m; ++e) ++t.off[g->idx[e] + 1];
  for (int64_t v = 0; v < g->n; ++v) t.off[v + 1] += t.off[v];
  int64_t* pos = (int64_t*)malloc((size_t)(g->n > 0 ? g->n : 1) * sizeof(int64_t));
  memcpy(pos, t.off, (size_t)g->n * sizeof(int64_t));
  for (int64_t u = 0; u < g->n; ++u)
    for (int64_t e = g->off[u]; e < g->off[u + 1]; ++e) {
      const int64_t p = pos[g->idx[e]]++;
      t.idx[p] = (int32_t)u;  /* sources in increasing order: sorted in-lists */
      t.w[p] = g->w[e];
    }
  free(pos);
  return t;
}

static void free_graph(Csr* g) {
  free(g->off);
  free(g->idx);
  free(g->w);
}

static void run_all(int64_t n, int64_t n_active, int64_t m0) {
  Csr g = make_graph(n, n_active, m0, 0);
  Csr gin = transpose(&g);
  const int32_t root = 0;
  /* BFS, its certificate, and Alg. 2 with BFS messages */
  int32_t* lv = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  CHECK(orc_bfs(n, g.off, g.idx, 1, &root, lv) >= 0);
  int32_t* src = (int32_t*)malloc((size_t)(g.m > 0 ? g.m : 1) * sizeof(int32_t));
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = g.off[u]; e < g.off[u + 1]; ++e) src[e] = (int32_t)u;
  CHECK(orc_bfs_certificate(n, g.m, src, g.idx, lv, root, INT32_MAX) == 0);
  uint32_t* prop = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
  uint8_t* act = (uint8_t*)calloc((size_t)n, 1);
  for (int64_t v = 0; v < n; ++v) prop[v] = UINT32_MAX;
  prop[root] = 0;
  act[root] = 1;
  CHECK(orc_run_min_program(n, g.off, g.idx, NULL, prop, act, -1) >= 0);
  for (int64_t v = 0; v < n; ++v)
    CHECK(lv[v] == INT32_MAX ? prop[v] == UINT32_MAX : prop[v] == (uint32_t)lv[v]);
  /* SSSP: Dijkstra and Alg. 2 with weights agree */
  uint32_t* dist = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
  CHECK(orc_dijkstra(n, g.off, g.idx, g.w, 1, &root, dist) == 0);
  for (int64_t v = 0; v < n; ++v) prop[v] = UINT32_MAX;
  memset(act, 0, (size_t)n);
  prop[root] = 0;
  act[root] = 1;
  CHECK(orc_run_min_program(n, g.off, g.idx, g.w, prop, act, -1) >= 0);
  for (int64_t v = 0; v < n; ++v) CHECK(prop[v] == dist[v]);
  /* PageRank (T = 5) and its weight gradient */
  const int32_t T = 5;
  double* in_w = (double*)malloc((size_t)(g.m > 0 ? g.m : 1) * sizeof(double));
  double* out_w = (double*)malloc((size_t)(g.m > 0 ? g.m : 1) * sizeof(double));
  for (int64_t e = 0; e < g.m; ++e) in_w[e] = out_w[e] = 1.0;
  int64_t* outdeg = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  double* tele = (double*)malloc((size_t)n * sizeof(double));
  double* hist = (double*)malloc((size_t)(T + 1) * (size_t)n * sizeof(double));
  double* c = (double*)malloc((size_t)n * sizeof(double));
  double* gw = (double*)malloc((size_t)(g.m > 0 ? g.m : 1) * sizeof(double));
  for (int64_t v = 0; v < n; ++v) {
    outdeg[v] = g.off[v + 1] - g.off[v];
    tele[v] = 1.0;
    hist[v] = 1.0;
    c[v] = (double)(next_u32() % 100) / 100.0;
  }
  CHECK(orc_pagerank(n, gin.off, gin.idx, in_w, outdeg, 0.15, T, tele, hist) == 0);
  CHECK(orc_pagerank_vjp_w(n, g.off, g.idx, out_w, 0.15, T, hist, c, gw) == 0);
  /* TC on the upper-triangle DAG: total = sum of per-vertex counts */
  Csr dag = make_graph(n, n_active, m0, 1);
  Csr din = transpose(&dag);
  int32_t* verts = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  uint64_t* counts = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
  for (int64_t v = 0; v < n; ++v) verts[v] = (int32_t)v;
  CHECK(orc_tc_per_vertex(n, din.off, din.idx, n, verts, counts) == 0);
  uint64_t sum = 0;
  for (int64_t v = 0; v < n; ++v) sum += counts[v];
  CHECK(orc_tc_total(n, din.off, din.idx) == sum);
  /* CF on the edges as ratings (users = sources, items = targets) */
  const int32_t K = 3;
  uint8_t* rating = (uint8_t*)malloc((size_t)(g.m > 0 ? g.m : 1));
  for (int64_t e = 0; e < g.m; ++e) rating[e] = (uint8_t)(1 + next_u32() % 5);
  float* PU = (float*)malloc((size_t)n * K * sizeof(float));
  float* PV = (float*)malloc((size_t)n * K * sizeof(float));
  for (int64_t i = 0; i < n * K; ++i) {
    PU[i] = (float)(next_u32() % 1000) / 1000.0f;
    PV[i] = (float)(next_u32() % 1000) / 1000.0f;
  }
  double loss = 0.0;
  double* gU = (double*)malloc((size_t)n * K * sizeof(double));
  double* gV = (double*)malloc((size_t)n * K * sizeof(double));
  CHECK(orc_cf(n, n, g.m, src, g.idx, rating, K, PU, PV, 0.05, &loss, gU, gV) == 0);
  CHECK(loss >= 0.0);
  free(lv);
  free(src);
  free(prop);
  free(act);
  free(dist);
  free(in_w);
  free(out_w);
  free(outdeg);
  free(tele);
  free(hist);
  free(c);
  free(gw);
  free(verts);
  free(counts);
  free(rating);
  free(PU);
  free(PV);
  free(gU);
  free(gV);
  free_graph(&g);
  free_graph(&gin);
  free_graph(&dag);
  free_graph(&din);
}

int main(void) {
  run_all(300, 250, 3000); /* random graph, 50 isolated vertices */
  run_all(1, 1, 0);        /* a single vertex */
  run_all(40, 40, 0);      /* no edges */
  run_all(64, 64, 4000);   /* dense: many duplicates dropped */
  printf("ok\n");
  return 0;
}
