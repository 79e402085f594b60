/*
 * sg2v -- colour-coding tree-template counting on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library libsg2v.so.  It implements the decoupled dynamic
 * programme of SubGraph2Vec (Zhang et al., arXiv 2009.11665): for every
 * colouring of the graph and every split of the template into an active and
 * a passive sub-template, a neighbour aggregation B = A_G M_p (Sec. 5.1,
 * Alg. 4, Eq. 1) followed by an element-wise multiply-add of B with the
 * active table through colour-set split tables (Sec. 5.3, Alg. 5).  The
 * colourful count of each colouring is scaled by 1/(P alpha) (Alg. 1).
 *
 * Conventions
 *  - Every function returns an sg2v_status; 0 is success.  On failure the
 *    thread-local message of sg2v_last_error() says why.  No C++ exception
 *    crosses this interface.
 *  - Handles are opaque.  A handle is used from one host thread at a time.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Device work is enqueued on it; functions returning host results
 *    synchronise that stream before returning.
 *  - The caller owns every buffer it passes.  Host buffers are read during
 *    the call only; device buffers borrowed by a handle (see
 *    SG2V_GRAPH_DEVICE_PTRS) must outlive the handle.
 *  - Colours are 0..k-1 (Sec. 2.2.2).  A colour set C of size m has column
 *    index I_C = sum_i binom(c_i, i) over its sorted elements c_1 < ... < c_m
 *    (colexicographic rank; Table 1 leaves the index map open).
 */
#ifndef SG2V_H
#define SG2V_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sg2v_status;
#define SG2V_OK 0
#define SG2V_EINVAL (-1)   /* null pointer, bad size, bad flag */
#define SG2V_ENOTTREE (-2) /* parent array is not one rooted tree */
#define SG2V_ERANGE (-3)   /* k < t, k > SG2V_KMAX, n or nnz out of range */
#define SG2V_ENOMEM (-4)   /* device or host allocation failed, or budget too small */
#define SG2V_EGRAPH (-5)   /* CSR malformed: unsorted row, duplicate, loop, asymmetric */
#define SG2V_EDEVICE (-6)  /* a HIP call failed */

#define SG2V_KMAX 20

/* Arithmetic of the count tables. */
typedef int32_t sg2v_mode;
#define SG2V_FP64 0  /* IEEE double tables */
#define SG2V_FP32S 1 /* float mantissas with a power-of-two exponent per column;
                        final vertex reduction in double */
#define SG2V_U64 2   /* unsigned 64-bit, exact modulo 2^64; overflow is flagged */

typedef struct sg2v_plan sg2v_plan;
typedef struct sg2v_graph sg2v_graph;
typedef struct sg2v_colorings sg2v_colorings;

/* Last error message of the calling thread ("" if none). */
const char *sg2v_last_error(void);

/* Library version string. */
const char *sg2v_version(void);

/* ------------------------------------------------------------------------ */
/* Template plan (Sec. 2.3.2: template partitioning; Table 1: colour-set     */
/* column index).                                                            */

/* Build the partition of a tree template T with t = |V_T| vertices for k
 * colours.  parent[v] is the parent of v and exactly one entry is -1 (the root
 * rho).  Each sub-template T_s is split by cutting the edge from its root to
 * its last child (children in increasing vertex order): the active child
 * keeps the root, the passive child is the cut-off subtree.  Rooted
 * sub-templates that are isomorphic share one table.  Split index tables
 * (for every output colour set, its (active set, passive set) pairs), the
 * automorphism count alpha and the colourful probability P are computed here.
 *   parent : host, t entries, copied.
 *   t      : 1 <= t <= k.
 *   k      : t <= k <= SG2V_KMAX.
 * Errors: EINVAL (null), ENOTTREE (not one tree), ERANGE (t, k). */
sg2v_status sg2v_plan_create(const int32_t *parent, int32_t t, int32_t k, sg2v_plan **out);
void sg2v_plan_destroy(sg2v_plan *plan);

/* Several templates over the same k colours in one plan, for one count of
 * all of them (a treelet distribution, Sec. 2.1).  Rooted sub-templates that
 * are isomorphic are shared across the templates, keyed by their canonical
 * form, so each is aggregated and combined once per colouring.
 *   parents     : host, the parent arrays of the templates one after another
 *                 (sum of sizes entries), each as for sg2v_plan_create.
 *   sizes       : host, n_templates vertex counts, 1 <= sizes[r] <= k.
 * No template may be the same rooted tree as another or a rooted
 * sub-template of another (EINVAL); templates of equal size never are unless
 * they repeat.  Such a plan is counted with sg2v_count_multi; sg2v_count,
 * sg2v_count_batch, sg2v_count_grad and sg2v_autotune reject it.
 * sg2v_plan_info describes its first template (n_templates gives the number).
 * Errors: EINVAL, ENOTTREE, ERANGE. */
sg2v_status sg2v_plan_create_multi(const int32_t *parents, const int32_t *sizes,
                                   int32_t n_templates, int32_t k, sg2v_plan **out);

/* The non-isomorphic (free, unlabelled) trees with t vertices, the template
 * set of a treelet distribution (Sec. 2.1: 47 trees of nine vertices).  Host
 * only; grown one vertex at a time, duplicates removed by the centre-rooted
 * canonical form.  Trees come in increasing order of that form; each parent
 * array has root 0 at a centre and vertices numbered breadth first.
 *   t          : 1 <= t <= SG2V_KMAX (t = 20 has 823,065 trees and takes
 *                seconds).
 *   max_trees  : parent arrays to write (0: count only).
 *   parents_out: host, max_trees * t int32 (nullable when max_trees = 0).
 *   n_trees    : the number of trees.
 * Errors: EINVAL, ERANGE. */
sg2v_status sg2v_trees(int32_t t, int64_t max_trees, int32_t *parents_out, int64_t *n_trees);

/* An isomorphic copy of T whose decomposition (Sec. 2.3.2) costs less; host
 * only.  The colourful count sums rooted counts over every image of the root,
 * so it is the number of colourful injective maps of T: it depends neither on
 * the root nor on the order in which a vertex's children are cut, and alpha is
 * |Aut| of the unrooted tree.  Every vertex is tried as the root; for each, every
 * vertex's children are ordered to minimise that vertex's multiply-add work
 * (all distinct orders of isomorphic-child classes up to 8! of them, else by
 * increasing subtree size).  The root minimising
 *   spmm_weight * sum over distinct passive subtrees (>= 2 vertices) of C(k, |T_p|)
 *   + sum over distinct splits of C(k, |T_s|) C(|T_s|, |T_a|)
 *     (the root split: C(k, |T_a|), its root reduction)
 * is kept, the given root winning ties.  spmm_weight is the cost of one
 * aggregated column per vertex relative to one multiply-add pair per vertex:
 * about 0.5 on graphs of mean degree 200, less on sparser graphs.
 *   parent     : host, t entries (as sg2v_plan_create).
 *   parent_out : host, t entries: the relabelled tree (root 0, children of a
 *                vertex numbered in their chosen cut order, breadth first).
 *   perm_out   : host, t entries or NULL: perm_out[v] = new label of vertex v.
 * Errors: EINVAL (null, negative weight), ENOTTREE, ERANGE (t, k). */
sg2v_status sg2v_template_reroot(const int32_t *parent, int32_t t, int32_t k, double spmm_weight,
                                 int32_t *parent_out, int32_t *perm_out);

typedef struct {
  int32_t t;              /* template vertices */
  int32_t k;              /* colours */
  int32_t n_nodes;        /* distinct rooted sub-templates, single vertex included */
  int32_t n_splits;       /* distinct sub-templates with more than one vertex */
  int32_t n_passive;      /* distinct passive children (one neighbour aggregation each) */
  int32_t root_node;      /* node id of T itself */
  int64_t alpha;          /* |Aut(T)| */
  double colorful_prob;   /* P = k!/((k-t)! k^t) */
  int64_t spmm_columns;   /* sum over distinct passives of C(k, |T_p|) */
  int64_t pairs_per_vertex; /* sum over splits of C(k,|T_s|) C(|T_s|,|T_a|) */
  int64_t widest_table;   /* max over nodes of C(k, |T_s|) */
  int32_t n_templates;    /* templates of the plan (sg2v_plan_create_multi), else 1 */
  int32_t reserved;
  int64_t bytes_per_vertex_fp32; /* device memory of one colouring's pass per graph vertex,
                                    FP32S tables (liveness-packed), with automatic settings */
  int64_t bytes_per_vertex_fp64; /* the same with FP64 or U64 tables */
} sg2v_plan_info_t;

sg2v_status sg2v_plan_info(const sg2v_plan *plan, sg2v_plan_info_t *out);

typedef struct {
  int32_t size;       /* |T_s| */
  int32_t active;     /* node id of T_{s,a}, -1 for a single vertex */
  int32_t passive;    /* node id of T_{s,p}, -1 for a single vertex */
  int32_t vertex;     /* template vertex that roots the first occurrence */
  int32_t n_kept;     /* number of that vertex's first children it keeps */
  int32_t is_passive; /* 1 if some split uses this node as passive child */
  int64_t columns;    /* C(k, size) */
} sg2v_node_info_t;

sg2v_status sg2v_plan_node(const sg2v_plan *plan, int32_t node, sg2v_node_info_t *out);

/* Split index table of a node with more than one vertex (Alg. 5: every way of
 * dividing C_s into an active and a passive colour set): out receives, for every output
 * column I_s in increasing order, C(|T_s|, |T_a|) pairs (I_a, I_p) as int32,
 * i.e. C(k,|T_s|) * C(|T_s|,|T_a|) * 2 values, host memory owned by the caller. */
sg2v_status sg2v_plan_pairs(const sg2v_plan *plan, int32_t node, int32_t *out);

/* ------------------------------------------------------------------------ */
/* Graph (Table 1: A_G as a 0/1 -- or weighted -- sparse matrix in CSR).      */

#define SG2V_GRAPH_DEVICE_PTRS 1u /* row_ptr/col_idx/w are device pointers, borrowed */
#define SG2V_GRAPH_VALIDATE 2u    /* check sorted rows, no loops/duplicates, symmetry */
#define SG2V_GRAPH_RELABEL 4u     /* store the vertices renumbered by decreasing degree (ties in
                                     the caller's order) and dealt round-robin to the eight
                                     neighbour ranges of the SpMM's XCD split, so that each range
                                     holds an equal mix of hubs and low-degree vertices with its
                                     hubs first and together.  Invisible
                                     to the caller: a vertex is coloured by its caller id, so
                                     counts are identical (exact in U64) with and without it;
                                     sg2v_colorings_download and sg2v_debug_table return rows in
                                     the caller's vertex order and sg2v_count_grad writes
                                     gradients in the caller's entry order.  The arrays are
                                     copied (also with DEVICE_PTRS). */

/* Register an undirected graph as symmetric CSR with n vertices and nnz
 * directed entries (each undirected edge appears as (i,j) and (j,i)).
 *   row_ptr : n+1 int64, row_ptr[0] = 0, row_ptr[n] = nnz.
 *   col_idx : nnz int32 in [0, n).
 *   w       : nullable; nnz float edge weights A_G(i,j) (equal on both
 *             directed entries of an edge).  NULL means A_G is 0/1.
 * Host arrays are copied to the device on `stream`.  With DEVICE_PTRS the
 * handle borrows the caller's device arrays.  Rows are grouped by degree for
 * load balance on the device.
 * Errors: EINVAL, ERANGE (n >= 2^31 or nnz < 0), EGRAPH (VALIDATE), EDEVICE. */
sg2v_status sg2v_graph_create(int64_t n, int64_t nnz, const int64_t *row_ptr,
                              const int32_t *col_idx, const float *w, uint32_t flags,
                              void *stream, sg2v_graph **out);
void sg2v_graph_destroy(sg2v_graph *g);

/* ------------------------------------------------------------------------ */
/* Random colourings (Sec. 2.3.1; Alg. 5: colour every vertex per iteration). */

/* Colour all n vertices for colourings first .. first+n_colorings-1 on the
 * device.  Colour of vertex v in colouring j:
 *   h = F(seed ^ F((j << 40) | v)),  colour = (hi32(h) * k) >> 32,
 * F = SplitMix64's output finaliser (Steele, Lea & Flood 2014).  The paper
 * leaves the generator open.  Requires n < 2^40, first + n_colorings < 2^24.
 * Storage: n_colorings x n bytes on the device, colouring-major. */
sg2v_status sg2v_color(const sg2v_graph *g, int32_t k, uint64_t seed, int32_t first,
                       int32_t n_colorings, void *stream, sg2v_colorings **out);
void sg2v_colorings_destroy(sg2v_colorings *c);

/* Copy colourings to the host: out has n_colorings * n bytes. */
sg2v_status sg2v_colorings_download(const sg2v_colorings *c, uint8_t *out, void *stream);

/* ------------------------------------------------------------------------ */
/* Counting (Alg. 1 / Alg. 5).                                                */

/* For every colouring j of `c`, run the dynamic programme for `plan` on `g`
 * and return
 *   colorful[j] = sum_i sum_{|C| = t} M_0(i, I_C)   (colourful labelled maps)
 *   estimate[j] = colorful[j] / (P alpha)           (finalCount of Alg. 1)
 *   *mean_estimate = average of estimate over j.
 * colorful_u64 (nullable): the exact count modulo 2^64, SG2V_U64 mode only.
 * overflow (nullable): set to 1 if a U64 intermediate exceeded 2^64 - 1.
 * All output pointers are host pointers with n_colorings entries (nullable).
 * Colourings are processed in passes of b colourings that sit side by side
 * as extra columns of the same tables (column j * C(k, m) + I_C), so that one
 * SpMM launch over A_G serves all b of them; b = 1024 / (columns of the
 * widest aggregated table), at least 1 (the tuning's batch overrides it) and
 * halved until the pass fits the device memory.  Tables of 1024 or more
 * columns run one colouring per pass: their column chunks each hold one
 * colouring's columns.
 * Errors: EINVAL (k of c differs from the plan's, U64 with weights, a plan
 *         of several templates: see sg2v_count_multi), ENOMEM, EDEVICE. */
sg2v_status sg2v_count(const sg2v_plan *plan, const sg2v_graph *g, const sg2v_colorings *c,
                       sg2v_mode mode, void *stream, double *colorful, uint64_t *colorful_u64,
                       double *estimate, double *mean_estimate, int32_t *overflow);

/* sg2v_count for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as sg2v_count, with the same kernels; it
 * calls no hipMalloc, hipFree or other allocating routine.  Every buffer of
 * the count (tables, partial sums, colour-skip masks, results) is taken from
 * one scratch area of SG2V_NOALLOC_SCRATCH_BYTES in the library's device
 * memory, one area per device, held from the first call on that device until
 * the process ends.  Colourings per pass are halved until a pass fits; a
 * count whose single-colouring pass does not fit returns SG2V_ENOMEM with the
 * size it needed.
 * Set-up: the plan's split tables must already be on the device (one
 * sg2v_count call with the plan on that device uploads them; SG2V_ENOMEM
 * otherwise).  The graph's task tables are made by sg2v_graph_create (for the
 * default split threshold; other thresholds, and the row panels of
 * SG2V_TUNE_SPMM_PANEL, must have been used by an sg2v_count on the graph, or
 * the call returns SG2V_ENOMEM, respectively runs the default SpMM).
 * Every call on one device shares its area, which keeps the last call's
 * contents: calls that overlap on one device (other threads, other streams)
 * race.  The call synchronises `stream` before it returns. */
#define SG2V_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sg2v_status sg2v_count_noalloc(const sg2v_plan *plan, const sg2v_graph *g,
                               const sg2v_colorings *c, sg2v_mode mode, void *stream,
                               double *colorful, uint64_t *colorful_u64, double *estimate,
                               double *mean_estimate, int32_t *overflow);

/* Counts of every template of a plan (sg2v_plan_create_multi, or any plan)
 * over the colourings of c, in one dynamic programme whose shared
 * sub-template tables are computed once per colouring.
 *   colorful, colorful_u64, estimate : n_templates x n_colorings, template-major.
 *   mean_estimate : n_templates, the average estimate of each template.
 *   frequency     : n_templates, mean_estimate normalised to sum 1 (the
 *                   treelet distribution; all zero if every mean is zero).
 * All host pointers are nullable.  Errors as sg2v_count. */
sg2v_status sg2v_count_multi(const sg2v_plan *plan, const sg2v_graph *g, const sg2v_colorings *c,
                             sg2v_mode mode, void *stream, double *colorful,
                             uint64_t *colorful_u64, double *estimate, double *mean_estimate,
                             double *frequency, int32_t *overflow);

/* (eps, delta) driver of the estimator (Alg. 1; Sec. 2.2.2 on the error
 * guarantee): runs N colourings, N fixed by the median-of-means form of the
 * bound N = O(e^k log(1/delta) / eps^2) that Alg. 1 states without constant:
 * r = ceil(8 ln(1/delta)) groups of m = ceil(4 (1/P - 1) / eps^2) colourings
 * (a per-colouring estimate lies in [0, emb/P], so its variance is at most
 * emb^2 (1/P - 1)); the median of the group means is within eps * emb with
 * probability at least 1 - delta.  Colourings are j = 0 .. N-1 of `seed`
 * (sg2v_color), counted with sg2v_count in `mode` on a graph with
 * non-negative weights.
 *   max_colorings : cap on N (0: 2^24 - 1); a smaller cap keeps r groups.
 *   flags         : SG2V_ESTIMATE_ADAPTIVE stops after a group once the
 *                   normal-approximation interval of the mean at level
 *                   1 - delta is within eps of the mean (at least 2 groups).
 *   out           : results (below).
 *   trace         : nullable, host, r doubles: the running mean after each
 *                   group (convergence report).
 * Errors: EINVAL (bad eps, delta or flags), ERANGE (cap >= 2^24), those of
 * sg2v_color and sg2v_count. */
#define SG2V_ESTIMATE_ADAPTIVE 1u
typedef struct {
  int64_t n_colorings;   /* colourings counted */
  int64_t n_bound;       /* r * m from (eps, delta) */
  int64_t group_size;    /* colourings per group */
  int32_t groups;        /* groups counted */
  int32_t stopped_early; /* adaptive stop */
  int32_t capped;        /* max_colorings was below n_bound */
  int32_t reserved;
  double mean;           /* average estimate (Alg. 1's output) */
  double median_of_means;
  double variance;       /* sample variance of the per-colouring estimates */
  double std_error;      /* sqrt(variance / n_colorings) */
  double ci_low, ci_high;   /* mean -+ z std_error, z the two-sided normal quantile of delta */
  double rel_half_width;    /* z std_error / mean */
} sg2v_estimate_t;

sg2v_status sg2v_estimate(const sg2v_plan *plan, const sg2v_graph *g, uint64_t seed, double eps,
                          double delta, sg2v_mode mode, int64_t max_colorings, uint32_t flags,
                          void *stream, sg2v_estimate_t *out, double *trace);

/* Several templates over n_colorings colourings each (colourings
 * seed-derived per plan: sg2v_color(g, k_p, seed, 0, n_colorings)), run as
 * one captured device graph (the templates as parallel branches when their
 * workspaces fit half of the free device memory), or, with the tuning flag
 * SG2V_TUNE_BATCH_PERSISTENT, as one persistent kernel over every template's
 * recorded launches.  The graph or schedule is cached and replayed by later
 * calls with the same arguments.  colorful/estimate: n_plans x n_colorings,
 * plan-major, host.  Errors as sg2v_count; EDEVICE also when a dependency
 * wait of the persistent schedule times out. */
sg2v_status sg2v_count_batch(const sg2v_plan *const *plans, int32_t n_plans,
                             const sg2v_graph *g, uint64_t seed, int32_t n_colorings,
                             sg2v_mode mode, void *stream, double *colorful, double *estimate);

/* Reverse-mode derivative of f = sum_j grad_colorful[j] * colorful[j] with
 * respect to every directed CSR weight A_G(i,j) (entry e of col_idx):
 *   grad_w[e] = df / dA_G(i,j).
 * The derivative with respect to the weight of an undirected edge is the sum
 * over its two directed entries.  The forward tables the backward sweep reads
 * are kept from one forward pass per colouring when they fit (half of the free
 * device memory, or the tuning's budget); otherwise each split recomputes a
 * forward pass up to itself instead of storing them (SG2V_TUNE_GRAD_RECOMPUTE
 * forces that).  Both give the same gradients.
 *   grad_colorful : host, n_colorings doubles.
 *   grad_w        : device, nnz doubles, written.
 * mode: SG2V_FP64, or SG2V_FP32S (FP32 tables, forward and adjoint, each
 * adjoint table with a power-of-two exponent per colouring; the per-entry
 * gradient accumulates in FP64).  U64 is rejected with EINVAL.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
sg2v_status sg2v_count_grad(const sg2v_plan *plan, const sg2v_graph *g, const sg2v_colorings *c,
                            sg2v_mode mode, const double *grad_colorful, void *grad_w,
                            void *stream);

/* ------------------------------------------------------------------------ */
/* Inspection (tests).                                                         */

/* Compute the table of `node` (kind 0: M_s; kind 1: B = A_G M_s, node must be
 * a passive child) for colouring `which` of `c` and copy it to the host as
 * doubles (FP64, FP32S with the column exponent applied) or uint64 (U64),
 * row-major n x C(k, |T_s|). */
sg2v_status sg2v_debug_table(const sg2v_plan *plan, const sg2v_graph *g,
                             const sg2v_colorings *c, sg2v_mode mode, int32_t which,
                             int32_t node, int32_t kind, void *host_out, void *stream);

/* Kernel timing.  Between sg2v_profile_start and sg2v_profile_stop, every
 * kernel launch of the library is bracketed by HIP events on the stream it is
 * launched on.  sg2v_profile_stop synchronises the device and fills out[kind]
 * for kind = 0 .. SG2V_K_COUNT-1 with the launch count, the summed event time,
 * and the summed model figures of those launches:
 *   bytes : compulsory HBM bytes (every table read once and written once,
 *           the adjacency streamed once per SpMM column chunk);
 *   work  : SpMM: edge x colour-set updates (nnz x columns);
 *           eMA/root: multiply-adds (vertices x pairs). */
#define SG2V_K_COLOR 0
#define SG2V_K_HIST 1
#define SG2V_K_SPMM 2
#define SG2V_K_SPMM_COMBINE 3
#define SG2V_K_EMA_GENERAL 4
#define SG2V_K_EMA_SINGLE 5
#define SG2V_K_ROOT 6
#define SG2V_K_COUNT 7

typedef struct {
  int32_t kind;
  int32_t launches;
  double ms;
  double bytes;
  double work;
} sg2v_prof_entry_t;

sg2v_status sg2v_profile_start(void);
sg2v_status sg2v_profile_stop(sg2v_prof_entry_t *out);

/* Tuning knobs (0 = automatic).  spmm_width: columns per SpMM chunk (row
 * segments of 2 to 32 lanes of 16 bytes: up to 128 FP32 or 64 FP64 columns);
 * ema_rows: rows per eMA tile; batch: colourings per pass; flags:
 * SG2V_TUNE_NO_COLOR_SKIP disables the colour-based skipping of SpMM row
 * segments, SG2V_TUNE_NO_COLOR_EMA the colour-restricted multiply-add
 * (vertices grouped by colour); budget_bytes: device memory the count may use;
 * xsplit_group and launch_chunks bound the column chunks one SpMM launch
 * covers (a table wider than that takes several launches, each starting at a
 * later chunk). */
#define SG2V_TUNE_NO_COLOR_SKIP 1
#define SG2V_TUNE_NO_COLOR_EMA 2
#define SG2V_TUNE_SPMM_UNROLL4 4 /* 4 row gathers in flight per SpMM stream (default below a mean
                                    degree of 64) */
#define SG2V_TUNE_SPMM_UNROLL8 128 /* 8 row gathers in flight per SpMM stream (default from a mean
                                      degree of 64) */
#define SG2V_TUNE_NO_XSPLIT 8    /* never split long SpMM tasks over the XCDs, and keep 128-byte
                                    chunks (overrides the two below) */
#define SG2V_TUNE_FORCE_XSPLIT 16 /* split even when a chunk fits the caches (tests) */
#define SG2V_TUNE_XSPLIT 32      /* split long SpMM tasks over the XCDs' neighbour ranges when one
                                    column chunk of the gathered table exceeds 32 MB, also with an
                                    explicit spmm_width (with spmm_width 0 this is automatic on
                                    graphs of at least 262,144 vertices whose tasks of 512 or more
                                    neighbours hold at least half the entries; such graphs also
                                    get 256-byte chunks in any case) */
#define SG2V_TUNE_ROOT_ROWS 64   /* root reduction one vertex per block step in vertex order instead
                                    of colour by colour with double-buffered rows */
#define SG2V_TUNE_BATCH_SERIAL 512 /* sg2v_count_batch: templates one after another in one workspace
                                      instead of parallel graph branches with a workspace each */
#define SG2V_TUNE_ROOT_THREAD 256 /* narrow root tables read by one thread per vertex from global
                                     memory instead of staged in LDS a tile of rows at a time */
#define SG2V_TUNE_GRAD_RECOMPUTE 2048 /* sg2v_count_grad: recompute the forward tables up to each
                                        split instead of keeping them from one forward pass per
                                        colouring (the default when they fit half the free
                                        device memory or the budget) */
#define SG2V_TUNE_BATCH_PERSISTENT 4096 /* sg2v_count_batch: every launch of every template
                                          recorded and run by one persistent kernel (a task
                                          queue over the launches' blocks with a completion
                                          counter per launch; each template's launches wait
                                          for their predecessor) instead of a HIP graph;
                                          implies SG2V_TUNE_NO_COLOR_EMA and
                                          SG2V_TUNE_ROOT_ROWS, and rejects
                                          SG2V_TUNE_SPMM_PANEL with SG2V_EINVAL; a
                                          wait longer than 30 s (or than the
                                          environment's SG2V_PERSIST_WAIT_US
                                          microseconds) stops the kernel and the
                                          call returns SG2V_EDEVICE */
#define SG2V_TUNE_SPMM_PANEL 1024 /* SpMM over row panels with column-sorted entries (the
                                     CSC-Split layout of Alg. 6): up to 32 consecutive tasks per
                                     panel, the panel's entries sorted by neighbour, one wave per
                                     panel accumulating its rows in LDS; built on first use per
                                     graph (about 5 bytes per entry, plus 4 with weights) */
typedef struct {
  int32_t spmm_width;
  int32_t ema_rows;
  int32_t batch;
  int32_t flags;
  int64_t budget_bytes;
  int32_t xsplit_group;  /* column chunks per launch of the neighbour-range split
                            (0: as many as 8 GB of range-partial rows hold) */
  int32_t launch_chunks; /* column chunks per SpMM launch without the split
                            (0: 65,535, the grid limit) */
  int32_t xsplit_min;    /* tasks of at least this many neighbours take the neighbour-range
                            split (0: 512) */
} sg2v_tuning_t;

sg2v_status sg2v_set_tuning(const sg2v_tuning_t *t);
sg2v_status sg2v_get_tuning(sg2v_tuning_t *t);

/* Autotuner: time sg2v_count of `plan` on `g` (n_colorings probe colourings,
 * `mode`) over a small set of candidate settings -- SpMM chunk width, colour
 * skipping, gathers in flight, neighbour-range split and its threshold,
 * row-panel SpMM, eMA rows per tile,
 * colourings per pass; widths that give the same row segments are tried once;
 * each candidate runs once untimed, then the median of three timed runs
 * counts -- and install the fastest
 * with sg2v_set_tuning.  Results are cached per (template, n, nnz, mode,
 * n_colorings) in the process and, if the environment variable
 * SG2V_TUNE_CACHE names a file, in that file (one line per key).
 *   out : nullable; receives the chosen settings.
 * Errors: as sg2v_count. */
sg2v_status sg2v_autotune(const sg2v_plan *plan, const sg2v_graph *g, sg2v_mode mode,
                          int32_t n_colorings, void *stream, sg2v_tuning_t *out);

#ifdef __cplusplus
}
#endif

#endif /* SG2V_H */
