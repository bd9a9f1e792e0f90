/*
 * gm.h -- C ABI of the GraphMat generalized-SpMSpV library for AMD MI355X
 * (gfx950).
 *
 * The library runs GraphMat vertex programs (Sundaram et al., "GraphMat:
 * High performance graph analytics made productive", VLDB 2015) as
 * generalized sparse-matrix x sparse-vector products on one GPU. Every
 * superstep of a program is Alg. 2 of the paper: active vertices send a
 * message (SEND_MESSAGE), every edge out of an active vertex processes it
 * (PROCESS_MESSAGE), the processed messages arriving at a vertex are
 * combined (REDUCE) and the vertex updates its property (APPLY); vertices
 * whose property changed are active in the next superstep (Sec. 4.1,
 * Sec. 4.3). The product itself is Alg. 1 (Sec. 4.2).
 *
 * Conventions for every call:
 *  - Every call returns a gm_status. Nothing throws or aborts across the
 *    ABI. On failure gm_last_error() returns a message for the calling
 *    thread, output buffers are unspecified and the graph stays valid.
 *  - Arguments are validated before any device work is enqueued.
 *  - "device" pointers are GPU memory owned by the caller, who keeps them
 *    alive until the enqueued work has finished. "host" pointers are read
 *    or written before the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; calls documented as synchronising wait for it.
 *  - A gm_graph is used by one stream and one host thread at a time (its
 *    workspace and cached schedules are shared); distinct graphs are
 *    independent and may be used from different threads.
 *  - Vertex ids are int32 in [0, n). Edge counts are limited to 2^32 - 1
 *    stored edges per graph (32-bit offsets); larger graphs give
 *    GM_EUNSUPPORTED.
 */
#ifndef GM_H_
#define GM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gm_status {
  GM_OK = 0,
  GM_EINVAL = 1,       /* bad argument: null pointer, size, id, enum, dtype */
  GM_ENOMEM = 2,       /* device or host allocation failed */
  GM_EHIP = 3,         /* a HIP runtime call failed */
  GM_EUNSUPPORTED = 4, /* valid but unsupported combination */
  GM_ESTATE = 5        /* handle not live (destroyed or never created) */
} gm_status;

/* Message describing the last failure on the calling thread ("" if none). */
const char* gm_last_error(void);

/* Library version string. */
const char* gm_version(void);

/* ------------------------------------------------------------------------ */
/* Graphs                                                                   */
/* ------------------------------------------------------------------------ */

/* Opaque handle; owns device memory from creation until gm_graph_destroy. */
typedef struct gm_graph_s* gm_graph;

/* Preprocessing applied while loading (Sec. 5.1: self-loops are removed;
 * PageRank and SSSP use the directed graph; BFS replicates edges to make
 * the graph symmetric; triangle counting symmetrises and keeps only the
 * upper triangle, i.e. edges u -> v with u < v). Duplicate edges are
 * always merged; a merged edge keeps the smallest weight. */
enum {
  GM_PREP_DROP_SELF_LOOPS = 1,
  GM_PREP_SYMMETRIZE = 2,
  GM_PREP_UPPER_DAG = 4 /* implies symmetrise, then keep u < v */
};

/* Edge value types (the edge value of Alg. 1). */
enum { GM_W_NONE = 0, GM_W_U32 = 1, GM_W_F32 = 2 };

/* Device layouts to build. The paper stores G^T column-compressed (DCSC,
 * Sec. 4.4.1); its columns are the out-edge lists of the vertices, i.e. a
 * row-compressed out-adjacency (CSR) of G, used by the push direction.
 * The in-adjacency (CSC of G) serves the pull direction. Both keep the
 * neighbour lists sorted. */
enum { GM_LAYOUT_OUT = 1, GM_LAYOUT_IN = 2 };

/*
 * Build a graph on the current HIP device from a host edge list
 * (src[e] -> dst[e], e < m), with optional per-edge values w (host,
 * wtype GM_W_U32 or GM_W_F32; NULL with GM_W_NONE). Mirrors the paper's
 * graph loading (App. A, ReadMTX) followed by the preprocessing of
 * Sec. 5.1 selected by `prep`. Canonical edge order is sorted by
 * (src, dst); every per-edge array exchanged with the library (weights,
 * edge gradients) uses it.
 * Errors: GM_EINVAL if n <= 0 or n > 2^31-1, m < 0, src/dst/out NULL
 * (m > 0), an id is outside [0, n), wtype unknown or w NULL/non-NULL
 * against wtype, layouts == 0 or unknown bits; GM_EUNSUPPORTED if more
 * than 2^32 - 1 edges remain; GM_ENOMEM, GM_EHIP.
 * Synchronises `stream`.
 */
gm_status gm_graph_from_coo(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                            const void* w, int32_t wtype, uint32_t prep, uint32_t layouts,
                            void* stream, gm_graph* out);

/*
 * Read a Matrix Market file, the graph format of the paper's API (App. A,
 * ReadMTX): a "coordinate" matrix with field pattern, integer or real and
 * symmetry general or symmetric. Entry (i, j) is the edge i-1 -> j-1 (the
 * off-diagonal entries of a symmetric file also give j-1 -> i-1) and its
 * value the edge value: integer -> GM_W_U32 (values in [0, 2^32 - 1]),
 * real -> GM_W_F32, pattern -> GM_W_NONE. n = max(rows, cols).
 * Two-call use: with src, dst and w all NULL, *n, *m and *wtype receive the
 * sizes; then host arrays of *m entries (src, dst int32; w uint32 or float
 * per *wtype; any of them may be NULL) are filled, *m on input being their
 * length. Host only: no device work.
 * Errors: GM_EINVAL (path/n/m/wtype NULL, file unreadable or malformed, an
 * entry outside the matrix, arrays shorter than the edge count);
 * GM_EUNSUPPORTED (another field or symmetry, an integer outside uint32).
 */
gm_status gm_mtx_read(const char* path, int64_t* n, int64_t* m, int32_t* src, int32_t* dst,
                      void* w, int32_t* wtype);

/* gm_mtx_read, then gm_graph_from_coo with the file's edges and values
 * (App. A's ReadMTX followed by the preprocessing `prep`). Errors: as those
 * two calls. Synchronises `stream`. */
gm_status gm_graph_from_mtx(const char* path, uint32_t prep, uint32_t layouts, void* stream,
                            gm_graph* out);

typedef struct gm_graph_info {
  int64_t n;          /* vertices */
  int64_t m;          /* stored directed edges after preprocessing */
  int64_t max_out;    /* largest out-degree */
  int64_t max_in;     /* largest in-degree (0 if the in-layout is absent) */
  int32_t wtype;      /* GM_W_* */
  uint32_t prep;      /* GM_PREP_* used */
  uint32_t layouts;   /* GM_LAYOUT_* built */
  int32_t device;     /* HIP device ordinal */
  int64_t device_bytes; /* device memory held by the graph (not the workspace) */
  int64_t n_src;      /* vertices with out-degree > 0 */
  int64_t n_dst;      /* vertices with in-degree > 0 (0 if the in-layout is absent) */
} gm_graph_info;

/* Fill *info (host). Errors: GM_ESTATE, GM_EINVAL (info NULL). */
gm_status gm_graph_get_info(gm_graph g, gm_graph_info* info);

/*
 * Copy the canonical edge list to host arrays of length m: src, dst
 * (either may be NULL) and values w (NULL, or uint32/float per wtype).
 * For a rating graph (gm_bipartite_from_coo) src is the row and dst the
 * column of each rating, by row, and w must be NULL. Errors: GM_ESTATE,
 * GM_EINVAL (w non-NULL on an unweighted graph), GM_EHIP. Synchronous.
 */
gm_status gm_graph_edges(gm_graph g, int32_t* src, int32_t* dst, void* w);

/* Free the graph and its workspace. Errors: GM_ESTATE if not live. */
gm_status gm_graph_destroy(gm_graph g);

/* ------------------------------------------------------------------------ */
/* Vertex programs                                                          */
/* ------------------------------------------------------------------------ */

/* Programs of Sec. 3, each a (SEND, PROCESS, REDUCE, APPLY) tuple. */
enum {
  /* Sec. 3 II, Eq. (2). Property int32 level, INT32_MAX = unreached.
   * SEND level(u); PROCESS msg + 1; REDUCE min; APPLY min.
   * Needs GM_LAYOUT_OUT; uses GM_LAYOUT_IN too (pull supersteps) when
   * built. */
  GM_PROG_BFS = 1,
  /* Sec. 3 V, Eq. (8) and App. A. Property uint32 distance,
   * UINT32_MAX = unreached. SEND dist(u); PROCESS msg + w_uv saturating
   * at UINT32_MAX; REDUCE min; APPLY min. Needs GM_W_U32 and
   * GM_LAYOUT_OUT. */
  GM_PROG_SSSP = 2,
  /* Sec. 3 I, Eq. (1). Property float rank. Every vertex is active in
   * every superstep; SEND rank(u)/outdeg(u) (none if outdeg = 0);
   * PROCESS msg (times w_uv for GM_W_F32 graphs); REDUCE +;
   * APPLY r + (1 - r) * y for every vertex. Runs exactly max_iters
   * supersteps. Needs GM_LAYOUT_IN. */
  GM_PROG_PAGERANK = 3,
  /* Personalised PageRank with one seed s (the first frontier id):
   * APPLY r * [v == s] + (1 - r) * y. Otherwise as GM_PROG_PAGERANK. */
  GM_PROG_PPR = 4,
  /* Triangle counting, program 2 of Sec. 4.2 (Eq. (7)). Needs a graph
   * loaded with GM_PREP_UPPER_DAG and GM_LAYOUT_IN, whose in-lists are
   * program 1's output. Property uint64 count; every vertex u sends its
   * in-neighbour list along its out-edges; PROCESS |in(u) ∩ in(v)|;
   * REDUCE +; APPLY count(v) += y. One superstep; frontier must be NULL. */
  GM_PROG_TC = 5,
  /* Vertex degree as a generalized SpMV with a ones vector (Fig. 1 of the
   * paper): every vertex sends; PROCESS gives 1 per edge; REDUCE +; APPLY
   * sets the property (uint32, written from 0 by the call) to the sum. With
   * GM_ORDER_OUT a vertex counts its in-edges, with GM_ORDER_IN its
   * out-edges (needs GM_LAYOUT_IN), with GM_ORDER_ALL both. One superstep;
   * frontier must be NULL. */
  GM_PROG_DEGREE = 6
};

/* Edges messages travel along (App. A, `order`; Sec. 4.1): out-edges (the
 * receivers of u are its out-neighbours), in-edges (its in-neighbours, i.e.
 * the transposed graph), or both. BFS, SSSP and the degree program take all
 * three (IN and ALL need GM_LAYOUT_IN, SSSP's weights then come with either
 * direction's edge); the other programs and the batched, captured and
 * multi-graph forms take GM_ORDER_OUT. */
enum { GM_ORDER_OUT = 1, GM_ORDER_IN = 2, GM_ORDER_ALL = 3 };

typedef struct gm_program {
  int32_t kind;   /* GM_PROG_* */
  int32_t order;  /* GM_ORDER_* */
  float r;        /* PageRank random-surf probability (Eq. (1)); 0.15 */
  uint32_t flags; /* reserved, must be 0 */
} gm_program;

/* Initially active vertices: the sparse input vector x of Alg. 1. Either
 * `count` distinct ids (device int32, `ids`), or the bitvector form of
 * Sec. 4.4.2 (`bitmap`: device uint32 words, ceil(n / 32) of them, bit
 * v % 32 of word v / 32 set for an active v; bits at or past n are
 * ignored). Exactly one of the two forms names the vertices: a non-NULL
 * bitmap needs ids == NULL and count == 0. */
typedef struct gm_frontier {
  const int32_t* ids;
  int64_t count;
  const uint32_t* bitmap;
} gm_frontier;

/*
 * Build, now, the per-graph schedules a program run needs, which a first
 * run would otherwise build: the frontier workspace of BFS and SSSP (and,
 * with GM_VARIANT_DEGREE_ORDER set, their degree-ordered copy of the
 * out-adjacency; runs along in-edges or both directions build theirs on
 * first use), the tiled pull layout of weighted SSSP (row-start bitmap, row
 * list, hot set), the relabelled pull layout of PageRank and PPR (Sec. 4.4.1 stores the matrix
 * once in the layout its SpMV reads; this is that step), the owner/partner
 * work plan of triangle counting (Sec. 4.2, program 2). Lets a caller time
 * preprocessing and runs apart. prog->kind selects the program; the other
 * fields are ignored. Errors: GM_ESTATE; GM_EINVAL (prog NULL, unknown
 * kind); GM_EUNSUPPORTED (as the run would report); GM_ENOMEM; GM_EHIP.
 * Synchronises `stream`.
 */
gm_status gm_graph_prepare(gm_graph g, const gm_program* prog, void* stream);

/*
 * Free every per-graph schedule and workspace built by runs or
 * gm_graph_prepare (the graph's own adjacency layouts stay); later runs
 * build them again. Captured plans that use g become stale. Errors:
 * GM_ESTATE. Waits for the device.
 */
gm_status gm_graph_release(gm_graph g);

/*
 * Run a vertex program (Alg. 2) on graph g. The caller initialises the
 * property array `vprop` (device, n entries of the program's type) and
 * names the initially active vertices, as App. A does
 * (setAllVertexproperty, then vertexproperty[s] = 0, active[s] = true).
 * BFS and SSSP run until no vertex is active when max_iters <= 0, else at
 * most max_iters supersteps; PageRank runs exactly max_iters (> 0)
 * supersteps with every vertex active (frontier may be NULL); PPR takes
 * its seed from frontier->ids[0].
 * On return *iters_done (host, may be NULL) holds the number of
 * supersteps that started with at least one active vertex, and
 * active_out (device int32 of n entries, may be NULL) marks, with 1, the
 * vertices still active afterwards, so a later call can resume from
 * (vprop, active) exactly.
 * BFS and SSSP accept either frontier form (ids or bitmap); PPR takes its
 * seed from ids only.
 * Errors: GM_ESTATE; GM_EINVAL (prog/vprop NULL, unknown kind or order,
 * flags != 0, frontier missing or count < 0 or ids NULL with
 * count > 0, both ids and bitmap given, a bitmap for PPR, an id out of
 * range, PageRank with max_iters <= 0, r outside [0, 1], a frontier for
 * the degree program); GM_EUNSUPPORTED (program needs a layout or weight
 * type the graph lacks, an order the program does not take, GM_ORDER_ALL
 * beyond 2^32 - 1 edges in both directions); GM_ENOMEM; GM_EHIP.
 * BFS and SSSP synchronise `stream` after batches of supersteps (the
 * first of superstep_batch; each later one twice as long, at most 64, while
 * the frontier holds up, back to superstep_batch once it fell below half
 * of its size from one superstep to the next at the end of a batch; the
 * supersteps after the frontier empties do nothing); PageRank is
 * asynchronous.
 */
gm_status gm_run_vertex_program(gm_graph g, const gm_program* prog, const gm_frontier* frontier,
                                int32_t max_iters, void* vprop, int32_t* active_out,
                                int32_t* iters_done, void* stream);

/*
 * Batched run: k sources (BFS, SSSP) or personalised-PageRank seeds (PPR)
 * processed together, one matrix pass serving all k frontiers (the
 * generalized SpMV of Alg. 1 with a dense n x k frontier block). Column s
 * of the result equals gm_run_vertex_program from sources[s] alone.
 * sources: device int32[k], ids in [0, n). vprop_block: device, n x k,
 * vertex-major (entry (v, s) at v * k + s), initialised by the call:
 *   BFS  (k <= 64)  int32 levels, INT32_MAX unreached; needs a symmetrised
 *                   graph or GM_LAYOUT_IN (pull supersteps over in-edges);
 *   SSSP (k <= 64)  uint32 distances, UINT32_MAX unreached; GM_W_U32;
 *   PPR  (k <= 256) float ranks after exactly max_iters (> 0) supersteps,
 *                   PPR_s^0 = e_s, teleport r to the seed only; GM_LAYOUT_IN.
 * max_iters <= 0 runs BFS/SSSP to convergence. *iters_done (host, may be
 * NULL): supersteps run (for BFS/SSSP the largest count of any source's
 * plain run; SSSP supersteps may end earlier than the slowest plain run
 * because a source reads distances other sources lowered in the same
 * superstep only through its own column - the final values are exact).
 * Errors: GM_ESTATE; GM_EINVAL (NULL pointers, k out of range, order or
 * flags, r, max_iters for PPR, a source out of range, unknown kind);
 * GM_EUNSUPPORTED (layout or weight type missing, n * k > 2^40); GM_ENOMEM;
 * GM_EHIP. Synchronises `stream`.
 */
gm_status gm_run_batched(gm_graph g, const gm_program* prog, const int32_t* sources, int32_t k,
                         int32_t max_iters, void* vprop_block, int32_t* iters_done, void* stream);

/*
 * Triangle count of Eq. (7) (Sec. 3 IV) via the two-program form of
 * Sec. 4.2 on g, which must be loaded with GM_PREP_UPPER_DAG and
 * GM_LAYOUT_IN. counts (device, n uint64, may be NULL) receives, per
 * vertex v, the triangles whose largest vertex is v; *total (host, may be
 * NULL) their sum, exact. Errors: GM_ESTATE; GM_EUNSUPPORTED (graph not an
 * upper-triangle DAG with in-lists); GM_ENOMEM; GM_EHIP. Synchronises
 * `stream`.
 */
gm_status gm_triangle_count(gm_graph g, uint64_t* counts, uint64_t* total, void* stream);

/* ------------------------------------------------------------------------ */
/* Differentiation: adjoint (transpose-direction) products                  */
/* ------------------------------------------------------------------------ */

/*
 * Build a rating graph for collaborative filtering (Sec. 3 III): an
 * n_rows x n_cols matrix G (rows = users, columns = items) with m ratings
 * G[row[e]][col[e]] = val[e] (host arrays; uint8 ratings). Pairs must be
 * distinct. The library keeps it compressed by row and by column. Only the
 * gm_cf_* calls (and gm_graph_get_info / gm_graph_destroy) accept it.
 * Errors: GM_EINVAL (sizes, NULL arrays, ids outside the matrix);
 * GM_EUNSUPPORTED (repeated (row, col) pair, m > 2^32 - 1); GM_ENOMEM;
 * GM_EHIP. Synchronises `stream`.
 */
gm_status gm_bipartite_from_coo(int64_t n_rows, int64_t n_cols, int64_t m, const int32_t* row,
                                const int32_t* col, const uint8_t* val, void* stream,
                                gm_graph* out);

/*
 * CF loss of Eq. (3): L = sum_(u,v) e_uv^2 + lambda sum_u |p_u|^2
 * + lambda sum_v |p_v|^2 with e_uv = G_uv - p_u . p_v (Eq. (4)).
 * PU (n_rows x K) and PV (n_cols x K) are row-major float factors (device);
 * *loss is a device double written on `stream` (asynchronous).
 * Errors: GM_ESTATE; GM_EUNSUPPORTED (not a rating graph); GM_EINVAL
 * (K outside [1, 64], NULL pointers, lambda < 0); GM_ENOMEM; GM_EHIP.
 */
gm_status gm_cf_forward(gm_graph g, int32_t K, const float* PU, const float* PV, float lambda,
                        double* loss, void* stream);

/*
 * Gradients of the CF loss, scaled by `scale` (the upstream gradient):
 *   gPU[u] = scale * (-2 sum_v e_uv p_v + 2 lambda p_u)   (row pass)
 *   gPV[v] = scale * (-2 sum_u e_uv p_u + 2 lambda p_v)   (transpose pass)
 * so a GD step of Eqs. (5)-(6) is p -= (gamma / 2) * g with scale = 1.
 * gPU / gPV are device arrays shaped like PU / PV; either may be NULL (not
 * both). Deterministic. Errors as gm_cf_forward, plus GM_EINVAL if both
 * outputs are NULL or scale is not finite. Asynchronous.
 */
gm_status gm_cf_backward(gm_graph g, int32_t K, const float* PU, const float* PV, float lambda,
                         float scale, float* gPU, float* gPV, void* stream);

/*
 * Collaborative filtering by gradient descent (Sec. 3 III, Eqs. (5)-(6)):
 * `iters` steps, each computing both gradients at the current point (the
 * row and transpose passes of gm_cf_backward) and then updating both factor
 * matrices in place, P <- P - (gamma / 2) dL/dP, i.e. the paper's
 * p <- p + gamma (sum_other e p_other - lambda p). PU, PV: device float
 * factors as for gm_cf_forward, updated in place. loss_hist (device double,
 * iters + 1 entries, may be NULL): the loss of Eq. (3) at the point of each
 * step and after the last. The gradient buffers are kept with the graph.
 * Errors: as gm_cf_forward; GM_EINVAL (iters < 0, gamma negative or not
 * finite). Asynchronous.
 */
gm_status gm_cf_gd(gm_graph g, int32_t K, float* PU, float* PV, float lambda, float gamma,
                   int32_t iters, double* loss_hist, void* stream);

/*
 * Weighted PageRank with history: PR^{t+1}(v) = r + (1 - r) *
 * sum_{u -> v} w_uv PR^t(u) / outdeg(u) (Eq. (1) with edge weights w in
 * canonical edge order, device float[m]; outdeg is the unweighted count).
 * hist is a device float (T + 1) x n array whose row 0 the caller fills
 * with PR^0; the call writes rows 1..T. Needs GM_LAYOUT_IN. w may be NULL
 * only when the graph has no edges (an empty tensor's address).
 * Errors: GM_ESTATE; GM_EINVAL (NULL pointers, T < 1, r outside [0, 1]);
 * GM_EUNSUPPORTED (no in-layout, rating graph); GM_ENOMEM; GM_EHIP.
 * Asynchronous.
 */
gm_status gm_pagerank_forward_w(gm_graph g, const float* w, float r, int32_t T, float* hist,
                                void* stream);

/*
 * Vector-Jacobian product of PR^T with respect to the edge weights: given
 * grad_out = dL/dPR^T (device float[n]) and the history from
 * gm_pagerank_forward_w, writes grad_w = dL/dw (device float[m], canonical
 * edge order) by T reverse steps, each one pass over the out-edges (the
 * product with the transposed matrix); grad_w, like w, may be NULL only
 * when the graph has no edges. Errors as gm_pagerank_forward_w.
 * Asynchronous.
 */
gm_status gm_pagerank_vjp_w(gm_graph g, const float* w, float r, int32_t T, const float* hist,
                            const float* grad_out, float* grad_w, void* stream);

/* ------------------------------------------------------------------------ */
/* Mixed batches and captured runs                                          */
/* ------------------------------------------------------------------------ */

/*
 * Block-diagonal union of `count` graphs (host array of live handles with
 * equal prep, wtype and layouts; no rating graphs): vertex v of parts[i]
 * becomes base_i + v with base_i = n_0 + ... + n_{i-1}, and the edges keep
 * their order part by part, so the union's canonical edge order is the
 * parts' canonical orders one after another. No edge joins two parts, so the
 * adjacency matrix is block diagonal and every program run on the union
 * gives, on part i's vertex range, exactly the run on part i alone: graphs of
 * uneven sizes then share each generalized SpMV of Alg. 1. The parts stay
 * valid and independent of the union.
 * Errors: GM_EINVAL (parts/out NULL, count < 1, differing prep, wtype or
 * layouts); GM_ESTATE (a handle not live); GM_EUNSUPPORTED (a rating graph,
 * more than 2^31 - 1 vertices or 2^32 - 1 edges in total); GM_ENOMEM;
 * GM_EHIP. Synchronises `stream`.
 */
gm_status gm_graph_union(const gm_graph* parts, int32_t count, void* stream, gm_graph* out);

/*
 * One program run over several graphs at once (the mixed batch): the graphs
 * (host array of `count` live handles with equal prep, wtype and layouts)
 * are joined into their block-diagonal union (as gm_graph_union), the
 * program runs once on the union - every generalized SpMV of Alg. 1 serves
 * all graphs - and each graph's part of the result is written to its own
 * property array. Graph i's result equals gm_run_vertex_program on graph i
 * alone. vprops: host array of `count` device pointers, vprops[i] holding
 * n_i entries of the program's type, initialised by the caller as for
 * gm_run_vertex_program (BFS, SSSP, PageRank, TC; PPR is not supported).
 * sources: host array of `count` ids, sources[i] in [0, n_i) the initially
 * active vertex of graph i or -1 for none (BFS, SSSP); NULL for PageRank and
 * TC. max_iters as for gm_run_vertex_program. *iters_done (host, may be
 * NULL): supersteps run, the largest count of any graph. The union and a
 * property array for it are built by the call (device allocations and
 * copies proportional to the graphs' sizes); callers that repeat the same
 * batch keep a union (gm_graph_union) and record its runs in a plan.
 * Errors: GM_EINVAL (NULL arrays, count < 1, differing prep/wtype/layouts, a
 * source out of range, the run's own argument errors); GM_ESTATE (a handle
 * not live); GM_EUNSUPPORTED (rating graphs, PPR, a layout or weight type
 * missing, union too large); GM_ENOMEM; GM_EHIP. Synchronises `stream`.
 */
gm_status gm_run_multi_graph(const gm_graph* graphs, int32_t count, const gm_program* prog,
                             const int32_t* sources, void* const* vprops, int32_t max_iters,
                             int32_t* iters_done, void* stream);

/* One run recorded in a plan. */
typedef struct gm_plan_run {
  gm_graph g;
  gm_program prog;
  int32_t batched;     /* 0: a run as gm_run_vertex_program; 1: as gm_run_batched */
  int32_t max_iters;   /* supersteps recorded. PageRank and PPR run exactly this
                          many; BFS and SSSP at most this many (1..64): the
                          supersteps after the frontier empties do nothing */
  const int32_t* ids;  /* device: frontier ids (BFS, SSSP) or the k sources /
                          seeds of a batched run; NULL for PageRank and TC */
  int64_t count;       /* number of ids (k of a batched run) */
  void* vprop;         /* device output: n entries, or n x k for a batched run */
} gm_plan_run;

/* Outcome of one recorded run after a launch. */
typedef struct gm_plan_result {
  int32_t iters_done;    /* as *iters_done of the corresponding call */
  int32_t converged;     /* 0 if vertices were still active after max_iters
                            supersteps (BFS, SSSP); 1 otherwise */
  int64_t edges_scanned; /* out-edges of the vertices that sent (0 for batched BFS) */
} gm_plan_result;

typedef struct gm_plan_s* gm_plan;

/*
 * Record `nruns` runs, in order, as one HIP graph (supersteps of Alg. 2
 * with the frontier test on the device, so nothing returns to the host
 * between supersteps); gm_plan_launch replays it with one launch. Each run
 * initialises its own output: BFS levels INT32_MAX with 0 at the ids, SSSP
 * distances UINT32_MAX with 0 at the ids, PageRank PR^0 = 1, TC counts 0,
 * batched runs as gm_run_batched. The ids and outputs must stay allocated
 * while the plan lives; ids are read at every launch, so new sources may be
 * written between launches. Plain PPR is not recorded (use a batched run
 * with k = 1).
 * A plan holds device addresses of its graphs' workspaces: destroying a
 * graph, gm_graph_set_tuning, gm_autotune or a call that needs a larger
 * workspace (a batched run with a larger k) makes it stale, and
 * gm_plan_launch then fails with GM_ESTATE.
 * Errors: as the corresponding calls for each run; GM_EINVAL (runs/out
 * NULL, nruns < 1, max_iters outside [1, 64] for BFS or SSSP, ids NULL
 * where needed, an id out of range); GM_EUNSUPPORTED (plain PPR); GM_ENOMEM;
 * GM_EHIP. Synchronises `stream` (capture runs on a library stream).
 */
gm_status gm_plan_create(const gm_plan_run* runs, int32_t nruns, void* stream, gm_plan* out);

/* Replay every recorded run on `stream` (one graph launch, asynchronous).
 * Errors: GM_ESTATE (plan not live, a graph destroyed or its workspace
 * changed since the plan was created); GM_EHIP. */
gm_status gm_plan_launch(gm_plan p, void* stream);

/* Copy the outcome of the last launch, one entry per run, to out (host).
 * Errors: GM_ESTATE, GM_EINVAL (out NULL), GM_EHIP. Synchronises `stream`. */
gm_status gm_plan_results(gm_plan p, gm_plan_result* out, void* stream);

/* Free the plan. Errors: GM_ESTATE if not live. */
gm_status gm_plan_destroy(gm_plan p);

/* ------------------------------------------------------------------------ */
/* Tuning                                                                   */
/* ------------------------------------------------------------------------ */

/* Per-graph schedule parameters. None changes any result, only time. */
typedef struct gm_tuning {
  uint32_t pull_div;        /* pull superstep (in-edges of every vertex) instead
                               of push: BFS when more than n / pull_div
                               vertices are active, SSSP (weighted, along
                               out-edges) when the frontier's out-edges
                               exceed 64 m / pull_div; 1 = push only
                               (1..65536; 128) */
  uint32_t superstep_batch; /* BFS/SSSP: supersteps enqueued before the first
                               host check of the frontier; each later batch is
                               twice as long, up to 64, unless the frontier
                               fell below half at the end of the last
                               (1..64; 4) */
  uint32_t push_blocks;     /* workgroups of the push kernels, plain and batched
                               SSSP (64..65536; 2048) */
  uint32_t ppr_chunk;       /* batched PPR: in-edges per work item (64..65536; 128) */
  uint32_t tc_wave_max;     /* TC: owners with at most this many in-neighbours
                               use a per-wavefront table (64..512; 512) */
  uint32_t tc_wave_work;    /* TC: partner elements per wavefront work item
                               (256..2^24; 2^14) */
  uint32_t tc_block_work;   /* TC: partner elements per workgroup work item
                               (256..2^26; 2^23) */
  uint32_t pr_hot;          /* PageRank/PPR pull and the PageRank reverse
                               pass: the vector entries of the pr_hot
                               highest-degree vertices are staged in LDS by
                               every workgroup (0..40960; 40960, capped by the
                               device's LDS per workgroup) */
  uint32_t variant;         /* alternative schedules of the paper's design
                               choices, for ablation (Sec. 5.4, Fig. 7); each
                               bit swaps one in, results are identical:
                               GM_VARIANT_LIST_FRONTIER, _VERTEX_PUSH,
                               _ROW_PULL, _DEGREE_ORDER (0..15; 0) */
} gm_tuning;

/* Bits of gm_tuning.variant (BFS/SSSP supersteps and the PageRank pull):
 *  GM_VARIANT_LIST_FRONTIER: the next frontier as a sorted, deduplicated
 *    list of vertex ids (the (index, value) sparse vector the paper's
 *    bitvector replaces, Sec. 4.4.2) instead of a bitvector: the product
 *    appends every lowered vertex and the list is sorted and made unique
 *    between supersteps (the host reads its length each superstep);
 *  GM_VARIANT_VERTEX_PUSH: one thread per active vertex walks its out-edges
 *    (no load balancing, Sec. 4.4.3) instead of equal edge ranges;
 *  GM_VARIANT_ROW_PULL: PageRank pulls one row per thread (no edge tiles,
 *    no LDS copy of the hottest messages) instead of the tiled kernel;
 *  GM_VARIANT_DEGREE_ORDER: BFS/SSSP/degree supersteps of
 *    gm_run_vertex_program run on a copy of the adjacency relabelled by
 *    decreasing in-degree (built on first use, one per order; each run maps
 *    its values and frontier in and out) instead of the caller's labels, so
 *    that the values read at random cluster in few cache lines whatever the
 *    caller's vertex order (the locality Sec. 4.4.1's partitioning seeks). */
enum {
  GM_VARIANT_LIST_FRONTIER = 1,
  GM_VARIANT_VERTEX_PUSH = 2,
  GM_VARIANT_ROW_PULL = 4,
  GM_VARIANT_DEGREE_ORDER = 8
};

/* Read g's parameters. Errors: GM_ESTATE, GM_EINVAL (out NULL). */
gm_status gm_graph_get_tuning(gm_graph g, gm_tuning* out);

/* Set g's parameters; workspaces built with other values are rebuilt on
 * next use. Errors: GM_ESTATE, GM_EINVAL (NULL, a value out of range). */
gm_status gm_graph_set_tuning(gm_graph g, const gm_tuning* t);

/*
 * Autotuner: times `prog` on g for candidate values of the parameters that
 * schedule it and keeps the fastest, one parameter at a time (coordinate
 * descent; median of `trials` timed runs per candidate after a warm-up run):
 *   BFS: pull_div, superstep_batch, push_blocks; SSSP: pull_div,
 *   push_blocks, superstep_batch; batched SSSP: push_blocks; batched PPR: ppr_chunk;
 *   TC: tc_wave_max, tc_wave_work, tc_block_work; PageRank: pr_hot;
 *   batched BFS has no parameters (the current values are returned).
 * batched selects gm_run_batched semantics with `count` = k sources; ids are
 * device sources / frontier ids as for the corresponding call (NULL for
 * PageRank and TC); max_iters as for that call (> 0 for PageRank and PPR).
 * The paper's only tunables are its thread and partition counts (Sec. 5.1,
 * 8x threads partitions); these are the GPU equivalents.
 * The library allocates the outputs of the trial runs. chosen (host, may be
 * NULL) receives the parameters kept, which stay set on g.
 * cache_path (host string, may be NULL): a JSON file of earlier choices,
 * keyed by the device architecture, the program (kind, batched, k) and the
 * graph's shape (log2 of n, log2 of the average degree, rounded). If it
 * holds the key, those values are set without timing anything; otherwise
 * the tuner runs and the file is rewritten with the new entry added (a
 * missing file is created). The file is an object of entries
 * "key": {"field": value, ...}, one per line.
 * Errors: as the corresponding call; GM_EINVAL (trials outside [1, 100], a
 * cache file that cannot be parsed or written, stored values out of range);
 * GM_ENOMEM; GM_EHIP. Synchronises `stream`.
 */
gm_status gm_autotune(gm_graph g, const gm_program* prog, int32_t batched, const int32_t* ids,
                      int64_t count, int32_t max_iters, int32_t trials, const char* cache_path,
                      gm_tuning* chosen, void* stream);

/* ------------------------------------------------------------------------ */
/* Allocation-free entry point                                              */
/* ------------------------------------------------------------------------ */

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): PageRank
 * exactly as gm_run_vertex_program with GM_PROG_PAGERANK (rank: device float
 * n, PR^0 in, PR^iters out; iters > 0 supersteps; r as there), but the
 * per-run vectors (two message buffers and PR in the layout's labels, n
 * floats each) and the per-tile partial sums live in a fixed device array of
 * the library, GM_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, allocated with the
 * code object and held until the process ends. A run on g needs
 * 3 * align256(4 n) + 2 * align256(8 * ceil(m / 1024)) bytes of it (n up to
 * about 5.5 million vertices). The call allocates nothing: the graph's pull
 * layout must have been built (gm_graph_prepare with GM_PROG_PAGERANK, or an
 * earlier PageRank run). All calls on one GPU share its array, so calls that
 * overlap on one GPU (on different streams or threads) race; calls on one
 * stream are ordered and safe. Asynchronous.
 * Errors: GM_ESTATE (graph not live, or its pull layout not built);
 * GM_EINVAL (rank NULL, iters <= 0, r outside [0, 1]); GM_EUNSUPPORTED
 * (rating graph, no GM_LAYOUT_IN, more scratch needed than the array holds);
 * GM_EHIP.
 */
#define GM_NOALLOC_SCRATCH_BYTES (64u << 20)
gm_status gm_pagerank_noalloc(gm_graph g, float r, int32_t iters, float* rank, void* stream);

/* Counters of the last gm_run_vertex_program call on a graph. */
typedef struct gm_run_stats {
  int32_t supersteps;      /* supersteps run (as *iters_done) */
  int32_t push_supersteps; /* supersteps that walked out-edges of active vertices */
  int32_t pull_supersteps; /* supersteps that scanned in-edges of all vertices */
  int64_t edges_scanned;   /* sum over supersteps of the out-degrees of the
                              vertices that sent a message (the edges Alg. 1
                              traverses) */
} gm_run_stats;

/* Copy the counters of g's last run to *out (host).
 * Errors: GM_ESTATE, GM_EINVAL (out NULL). */
gm_status gm_last_run_stats(gm_graph g, gm_run_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* GM_H_ */
