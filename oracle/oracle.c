/*
 * CPU oracle for the GraphMat generalized-SpMSpV path.
 *
 * TEST INFRASTRUCTURE ONLY. This file is compiled into liboracle.so and is
 * called by the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark. The GPU library never includes, links or calls it, and it
 * shares no code with the GPU kernels.
 *
 * Everything here is plain, single-threaded and written for obvious
 * correctness, in double precision where the method uses real numbers.
 * Graphs arrive as compressed adjacency (offsets int64[n+1], neighbour
 * ids int32) built by the Python side of the oracle.
 *
 * Paper: Sundaram et al., "GraphMat: High performance graph analytics made
 * productive", VLDB 2015 (arXiv 1503.07241).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define INF_I32 INT32_MAX
#define INF_U32 UINT32_MAX

/* ---------------------------------------------------------------------- */
/* BFS: hop distance from the root set (Sec. 3 II, Eq. (2)).               */
/* Definition: level(v) = min number of edges on a path from a root to v;  */
/* roots have level 0; unreachable vertices keep INT32_MAX. A FIFO queue   */
/* visits vertices in nondecreasing distance, so the first visit fixes it. */
/* Returns the largest finite level.                                       */
/* ---------------------------------------------------------------------- */
int32_t orc_bfs(int64_t n, const int64_t* off, const int32_t* idx, int64_t nroots,
                const int32_t* roots, int32_t* level) {
  int32_t* queue = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!queue) return -1;
  for (int64_t v = 0; v < n; ++v) level[v] = INF_I32;
  int64_t head = 0, tail = 0;
  for (int64_t i = 0; i < nroots; ++i) {
    if (level[roots[i]] != 0) {
      level[roots[i]] = 0;
      queue[tail++] = roots[i];
    }
  }
  int32_t maxlev = 0;
  while (head < tail) {
    const int32_t u = queue[head++];
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      const int32_t v = idx[e];
      if (level[v] == INF_I32) {
        level[v] = level[u] + 1;
        if (level[v] > maxlev) maxlev = level[v];
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return maxlev;
}

/* ---------------------------------------------------------------------- */
/* SSSP: shortest-path distance (Sec. 3 V, Eq. (8)) with unsigned integer   */
/* weights, by Dijkstra's algorithm on a binary heap with lazy deletion.   */
/* dist(v) = min over paths source->v of the weight sum; unreachable       */
/* vertices keep UINT32_MAX. Sums are formed in 64 bits; a path whose sum  */
/* reaches UINT32_MAX is reported as UINT32_MAX (saturation).              */
/* ---------------------------------------------------------------------- */
typedef struct {
  uint64_t d;
  int32_t v;
} heap_item;

static void heap_push(heap_item* h, int64_t* size, heap_item it) {
  int64_t i = (*size)++;
  h[i] = it;
  while (i > 0) {
    const int64_t p = (i - 1) / 2;
    if (h[p].d <= h[i].d) break;
    const heap_item t = h[p];
    h[p] = h[i];
    h[i] = t;
    i = p;
  }
}

static heap_item heap_pop(heap_item* h, int64_t* size) {
  const heap_item top = h[0];
  h[0] = h[--(*size)];
  int64_t i = 0;
  for (;;) {
    const int64_t l = 2 * i + 1, r = l + 1;
    int64_t s = i;
    if (l < *size && h[l].d < h[s].d) s = l;
    if (r < *size && h[r].d < h[s].d) s = r;
    if (s == i) break;
    const heap_item t = h[s];
    h[s] = h[i];
    h[i] = t;
    i = s;
  }
  return top;
}

int orc_dijkstra(int64_t n, const int64_t* off, const int32_t* idx, const uint32_t* w,
                 int64_t nsrc, const int32_t* srcs, uint32_t* dist) {
  const int64_t m = off[n];
  uint64_t* d = (uint64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
  heap_item* h = (heap_item*)malloc((size_t)(m + nsrc + 1) * sizeof(heap_item));
  if (!d || !h) {
    free(d);
    free(h);
    return -1;
  }
  for (int64_t v = 0; v < n; ++v) d[v] = UINT64_MAX;
  int64_t size = 0;
  for (int64_t i = 0; i < nsrc; ++i) {
    d[srcs[i]] = 0;
    heap_item it = {0, srcs[i]};
    heap_push(h, &size, it);
  }
  while (size > 0) {
    const heap_item it = heap_pop(h, &size);
    if (it.d != d[it.v]) continue; /* stale entry */
    const int32_t u = it.v;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      const uint64_t nd = d[u] + (uint64_t)w[e];
      if (nd < d[idx[e]]) {
        d[idx[e]] = nd;
        heap_item jt = {nd, idx[e]};
        heap_push(h, &size, jt);
      }
    }
  }
  for (int64_t v = 0; v < n; ++v) dist[v] = d[v] >= (uint64_t)INF_U32 ? INF_U32 : (uint32_t)d[v];
  free(d);
  free(h);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* The superstep loop of Alg. 2 for the two min-programs of Sec. 3         */
/* (BFS, Eq. (2); SSSP, Eq. (8)), taken step by step:                      */
/*   1. every active vertex u sends the message x_u = prop(u);            */
/*   2. the generalized SpMV of Alg. 1 walks the columns j of G^T (the     */
/*      out-edges of j) whose message is present and folds                 */
/*      PROCESS(x_j, w_jk) into y_k with REDUCE = min;                    */
/*   3. every vertex k that received a message applies                    */
/*      prop(k) = min(prop(k), y_k) and is active next iff prop changed;   */
/*   4. stop when no vertex is active or after max_iters supersteps.       */
/* PROCESS is msg + 1 when w == NULL (BFS) and msg + w_jk otherwise       */
/* (SSSP), both saturating at UINT32_MAX; prop is unsigned here (BFS       */
/* callers map INT32_MAX <-> UINT32_MAX themselves).                       */
/* Returns the number of supersteps that started with an active vertex.   */
/* ---------------------------------------------------------------------- */
int32_t orc_run_min_program(int64_t n, const int64_t* off, const int32_t* idx,
                            const uint32_t* w, uint32_t* prop, uint8_t* active,
                            int32_t max_iters) {
  uint32_t* x = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
  uint8_t* xvalid = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  uint32_t* y = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
  uint8_t* yvalid = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  if (!x || !xvalid || !y || !yvalid) {
    free(x);
    free(xvalid);
    free(y);
    free(yvalid);
    return -1;
  }
  int32_t done = 0;
  for (int32_t it = 0; max_iters <= 0 || it < max_iters; ++it) {
    int64_t nactive = 0;
    for (int64_t v = 0; v < n; ++v) nactive += active[v] != 0;
    if (nactive == 0) break;
    /* 1. SEND_MESSAGE */
    for (int64_t v = 0; v < n; ++v) {
      xvalid[v] = active[v] != 0;
      if (xvalid[v]) x[v] = prop[v];
    }
    /* 2. SPMV: y = G^T x with (PROCESS, REDUCE=min) */
    memset(yvalid, 0, (size_t)n);
    for (int64_t j = 0; j < n; ++j) {
      if (!xvalid[j]) continue;
      for (int64_t e = off[j]; e < off[j + 1]; ++e) {
        const int32_t k = idx[e];
        const uint64_t add = w ? (uint64_t)w[e] : 1u;
        uint64_t r = (uint64_t)x[j] + add;
        if (r > INF_U32) r = INF_U32;
        if (!yvalid[k] || (uint32_t)r < y[k]) y[k] = (uint32_t)r;
        yvalid[k] = 1;
      }
    }
    /* 3. reset active; APPLY to every vertex that received a message */
    memset(active, 0, (size_t)n);
    for (int64_t k = 0; k < n; ++k) {
      if (!yvalid[k]) continue;
      const uint32_t old = prop[k];
      const uint32_t nw = y[k] < old ? y[k] : old;
      prop[k] = nw;
      if (nw != old) active[k] = 1;
    }
    ++done;
  }
  free(x);
  free(xvalid);
  free(y);
  free(yvalid);
  return done;
}

/* ---------------------------------------------------------------------- */
/* PageRank, Eq. (1), generalised with edge weights and a teleport vector: */
/*   PR^{t+1}(v) = r * tele(v) + (1 - r) * sum_{u -> v} w_uv PR^t(u)/deg(u) */
/* deg(u) is the (unweighted) out-degree. tele = 1 everywhere and w = 1    */
/* give Eq. (1) exactly; tele = e_s gives personalised PageRank for seed   */
/* s. Computed in the pull direction over in-edges (CSC), for every vertex */
/* each step (Jacobi iteration). hist holds PR^0..PR^T, (T+1) x n.         */
/* ---------------------------------------------------------------------- */
int orc_pagerank(int64_t n, const int64_t* in_off, const int32_t* in_src, const double* in_w,
                 const int64_t* outdeg, double r, int32_t T, const double* tele,
                 double* hist) {
  for (int32_t t = 0; t < T; ++t) {
    const double* cur = hist + (int64_t)t * n;
    double* nxt = hist + (int64_t)(t + 1) * n;
    for (int64_t v = 0; v < n; ++v) {
      double s = 0.0;
      for (int64_t e = in_off[v]; e < in_off[v + 1]; ++e) {
        const int32_t u = in_src[e];
        const double wv = in_w ? in_w[e] : 1.0;
        s += wv * cur[u] / (double)outdeg[u];
      }
      nxt[v] = r * tele[v] + (1.0 - r) * s;
    }
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Reverse-mode derivative of the weighted PageRank above with respect to  */
/* the edge weights. With upstream c = dL/dPR^T, abar^T = c, and for       */
/* t = T-1 .. 0 (chain rule through one step):                             */
/*   dL/dw_uv += (1 - r) * PR^t(u) / deg(u) * abar^{t+1}(v)                */
/*   abar^t(u)  = (1 - r) / deg(u) * sum_{v: u -> v} w_uv abar^{t+1}(v)    */
/* The second line is the transpose-direction product, over out-edges      */
/* (CSR). grad_w is in CSR edge order.                                     */
/* ---------------------------------------------------------------------- */
int orc_pagerank_vjp_w(int64_t n, const int64_t* out_off, const int32_t* out_dst,
                       const double* out_w, double r, int32_t T, const double* hist,
                       const double* c, double* grad_w) {
  const int64_t m = out_off[n];
  double* a_next = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double* a_cur = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  if (!a_next || !a_cur) {
    free(a_next);
    free(a_cur);
    return -1;
  }
  for (int64_t e = 0; e < m; ++e) grad_w[e] = 0.0;
  for (int64_t v = 0; v < n; ++v) a_next[v] = c[v];
  for (int32_t t = T - 1; t >= 0; --t) {
    const double* pr = hist + (int64_t)t * n;
    for (int64_t u = 0; u < n; ++u) {
      const int64_t deg = out_off[u + 1] - out_off[u];
      double s = 0.0;
      for (int64_t e = out_off[u]; e < out_off[u + 1]; ++e) {
        const int32_t v = out_dst[e];
        grad_w[e] += (1.0 - r) * pr[u] / (double)deg * a_next[v];
        s += out_w[e] * a_next[v];
      }
      a_cur[u] = deg > 0 ? (1.0 - r) / (double)deg * s : 0.0;
    }
    double* tmp = a_next;
    a_next = a_cur;
    a_cur = tmp;
  }
  free(a_next);
  free(a_cur);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Triangle counting, the two-program form of Sec. 4.2 on the upper-      */
/* triangle DAG (edges u -> v with u < v, Sec. 5.1 preprocessing):         */
/* program 1 gives every vertex its sorted list in(v) of in-neighbours;    */
/* program 2 sends in(u) along every edge u -> v and the receiver adds     */
/* |in(u) ∩ in(v)|. Each triangle a < b < c is counted once, at edge      */
/* (b, c) with common in-neighbour a. in_off/in_src is the CSC of the DAG  */
/* with sorted lists.                                                      */
/* ---------------------------------------------------------------------- */
static uint64_t merge_count(const int32_t* a, int64_t na, const int32_t* b, int64_t nb) {
  uint64_t c = 0;
  int64_t i = 0, j = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j])
      ++i;
    else if (a[i] > b[j])
      ++j;
    else {
      ++c;
      ++i;
      ++j;
    }
  }
  return c;
}

/* Per-receiver counts for the listed vertices: count(v) = sum over u in  */
/* in(v) of |in(u) ∩ in(v)|.                                              */
int orc_tc_per_vertex(int64_t n, const int64_t* in_off, const int32_t* in_src, int64_t nv,
                      const int32_t* verts, uint64_t* counts) {
  (void)n;
  for (int64_t i = 0; i < nv; ++i) {
    const int32_t v = verts[i];
    uint64_t c = 0;
    for (int64_t e = in_off[v]; e < in_off[v + 1]; ++e) {
      const int32_t u = in_src[e];
      c += merge_count(in_src + in_off[u], in_off[u + 1] - in_off[u], in_src + in_off[v],
                       in_off[v + 1] - in_off[v]);
    }
    counts[i] = c;
  }
  return 0;
}

uint64_t orc_tc_total(int64_t n, const int64_t* in_off, const int32_t* in_src) {
  uint64_t total = 0;
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t e = in_off[v]; e < in_off[v + 1]; ++e) {
      const int32_t u = in_src[e];
      total += merge_count(in_src + in_off[u], in_off[u + 1] - in_off[u], in_src + in_off[v],
                           in_off[v + 1] - in_off[v]);
    }
  }
  return total;
}

/* ---------------------------------------------------------------------- */
/* Collaborative filtering, Sec. 3 III: objective Eq. (3)                 */
/*   L = sum_{(u,v) in G} e_uv^2 + lambda sum_u |p_u|^2 + lambda sum_v |p_v|^2 */
/* with e_uv = G_uv - p_u . p_v (Eq. (4)), and its gradients               */
/*   dL/dp_u = -2 sum_v e_uv p_v + 2 lambda p_u,                           */
/*   dL/dp_v = -2 sum_u e_uv p_u + 2 lambda p_v,                           */
/* so that the GD updates Eqs. (5)-(6) are p <- p - (gamma/2) dL/dp. The   */
/* regulariser is counted once per vertex, as Eqs. (5)-(6) place it.       */
/* One pass over the ratings in the given order, double accumulators.      */
/* ---------------------------------------------------------------------- */
int orc_cf(int64_t n_users, int64_t n_items, int64_t m, const int32_t* user, const int32_t* item,
           const uint8_t* rating, int32_t K, const float* PU, const float* PV, double lambda,
           double* loss, double* gU, double* gV) {
  double L = 0.0;
  for (int64_t i = 0; i < n_users * K; ++i) gU[i] = 0.0;
  for (int64_t i = 0; i < n_items * K; ++i) gV[i] = 0.0;
  for (int64_t e = 0; e < m; ++e) {
    const float* pu = PU + (int64_t)user[e] * K;
    const float* pv = PV + (int64_t)item[e] * K;
    double dot = 0.0;
    for (int32_t k = 0; k < K; ++k) dot += (double)pu[k] * (double)pv[k];
    const double err = (double)rating[e] - dot;
    L += err * err;
    double* gu = gU + (int64_t)user[e] * K;
    double* gv = gV + (int64_t)item[e] * K;
    for (int32_t k = 0; k < K; ++k) {
      gu[k] += -2.0 * err * (double)pv[k];
      gv[k] += -2.0 * err * (double)pu[k];
    }
  }
  for (int64_t u = 0; u < n_users; ++u)
    for (int32_t k = 0; k < K; ++k) {
      const double p = PU[u * K + k];
      L += lambda * p * p;
      gU[u * K + k] += 2.0 * lambda * p;
    }
  for (int64_t v = 0; v < n_items; ++v)
    for (int32_t k = 0; k < K; ++k) {
      const double p = PV[v * K + k];
      L += lambda * p * p;
      gV[v * K + k] += 2.0 * lambda * p;
    }
  *loss = L;
  return 0;
}

/*
 * BFS certificate (Sec. 3 II, Eq. (2)): levels lv of an undirected graph given
 * as a list of directed entries (both directions of every edge present) are
 * the hop distances from root iff lv[root] = 0, every entry (u, v) with u
 * reached has v reached with lv[v] <= lv[u] + 1, an entry never joins a
 * reached and an unreached vertex, and every reached v != root has an entry
 * (u, v) with lv[u] = lv[v] - 1. The first two give lv <= distance along
 * any path; the parent entries give a path of length lv[v]. Returns 0 if
 * certified, else a code naming the first failed condition (1 root, 2 edge
 * step, 3 reached/unreached mix, 4 missing parent, 5 negative level).
 */
int orc_bfs_certificate(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        const int32_t* lv, int32_t root, int32_t inf) {
  if (lv[root] != 0) return 1;
  uint8_t* parent = (uint8_t*)calloc((size_t)n, 1);
  if (!parent) return -1;
  int rc = 0;
  for (int64_t e = 0; e < m && rc == 0; ++e) {
    const int32_t a = lv[src[e]], b = lv[dst[e]];
    if (a == inf || b == inf) {
      if (a != b) rc = 3;
      continue;
    }
    if (b > a + 1) rc = 2;
    if (b == a + 1) parent[dst[e]] = 1;
  }
  for (int64_t v = 0; v < n && rc == 0; ++v) {
    if (lv[v] < 0) rc = 5;
    else if (lv[v] != inf && v != root && !parent[v]) rc = 4;
  }
  free(parent);
  return rc;
}
