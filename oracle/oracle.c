/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, obviously correct CPU implementation of colour-coding tree
 * counting (Zhang et al., "SubGraph2Vec", arXiv 2009.11665).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * library; the product path never does.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * Arithmetic: IEEE double ("FP64") or unsigned 64-bit integers taken modulo
 * 2^64 ("U64", with an overflow flag).  Loops run in the order the paper's
 * definitions give them; the only parallelism is an OpenMP split of the
 * vertex loop, which does not change the order of any sum.
 *
 * What each function follows:
 *   orc_colors        -- Sec. 2.2.2 / Sec. 2.3.1 (random colouring, colours
 *                        0..k-1).  The paper does not fix the generator; the
 *                        counter-based hash below is this project's reading.
 *   orc_count         -- Alg. 1 (estimator) around the dynamic programme of
 *                        Alg. 3 (neighbour sum B = A M_p, then the
 *                        element-wise multiply-add), or of Alg. 2 when
 *                        alg2 != 0 (neighbour loop inside the split loop).
 *   orc_node_table    -- the count table M_s of one sub-template (Table 1).
 *   orc_neighbour_sum -- B = A_G M_p (Eq. 1's right-hand factor, Alg. 4).
 *   orc_brute         -- emb(T,G) by definition (Sec. 2.2.1): enumeration
 *                        of injective edge-preserving maps, or of colourful
 *                        ones; optional per-edge derivative of the weighted sum.
 *   orc_automorphisms -- alpha of Alg. 1: maps of T onto itself, by brute force.
 *   orc_grad          -- reverse-mode derivative of the weighted colourful
 *                        count with respect to each directed CSR entry, by
 *                        differentiating the Alg. 3 recurrence loop by loop.
 *
 * Template encoding: parent[v] is v's parent, parent[root] = -1.  Children of
 * a vertex are kept in increasing vertex order.  Sub-template (v, lo, hi) is
 * v together with the full subtrees of its children lo..hi-1.  Partitioning
 * (Sec. 2.3.2) cuts the edge from v to its last kept child (cut = 0) or to
 * its first kept child (cut = 1); the active child keeps v, the passive child
 * is the full subtree of the cut-off child.
 *
 * Colour sets are k-bit masks.  The column index I_C of a set C (Table 1) is
 * its position among all sets of the same size in increasing mask order,
 * which this file builds by enumerating masks with Gosper's hack.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOTTREE -2
#define ORC_ENOMEM -3

/* ----------------------------------------------------------------------- */
/* colouring                                                               */

static uint64_t splitmix64_finalise(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* One SplitMix64 step from `state` (Steele, Lea & Flood 2014): add the golden
 * gamma, then finalise.  Exposed so the tests can check published values. */
uint64_t orc_splitmix64_next(uint64_t *state) {
  *state += 0x9E3779B97F4A7C15ULL;
  return splitmix64_finalise(*state);
}

uint64_t orc_mix64(uint64_t z) { return splitmix64_finalise(z); }

/* colour of vertex v in colouring j:
 *   h = F(seed XOR F((j << 40) | v)),  colour = floor(hi32(h) * k / 2^32)
 * with F the SplitMix64 finaliser and the last step Lemire's multiply-shift. */
int orc_colors(int64_t n, int32_t k, uint64_t seed, int32_t j, uint8_t *out) {
  if (n < 0 || k < 1 || k > 255 || j < 0 || n >= ((int64_t)1 << 40)) return ORC_EINVAL;
  for (int64_t v = 0; v < n; ++v) {
    uint64_t h = splitmix64_finalise(seed ^ splitmix64_finalise(((uint64_t)j << 40) | (uint64_t)v));
    out[v] = (uint8_t)(((h >> 32) * (uint64_t)k) >> 32);
  }
  return ORC_OK;
}

/* ----------------------------------------------------------------------- */
/* templates                                                                */

typedef struct {
  int t;
  int root;
  int *nch;      /* number of children */
  int **ch;      /* children in increasing vertex order */
  int *subsize;  /* size of the full subtree of each vertex */
} tree;

static void tree_free(tree *T) {
  if (!T->nch) return;
  for (int v = 0; v < T->t; ++v) free(T->ch[v]);
  free(T->ch);
  free(T->nch);
  free(T->subsize);
  T->nch = NULL;
}

static int subtree_size(tree *T, int v) {
  int s = 1;
  for (int c = 0; c < T->nch[v]; ++c) s += subtree_size(T, T->ch[v][c]);
  T->subsize[v] = s;
  return s;
}

/* validate: exactly one root, parents in range, every vertex reaches the root */
static int tree_build(const int32_t *parent, int t, tree *T) {
  memset(T, 0, sizeof(*T));
  if (!parent || t < 1 || t > 64) return ORC_EINVAL;
  int root = -1;
  for (int v = 0; v < t; ++v) {
    if (parent[v] == -1) {
      if (root >= 0) return ORC_ENOTTREE;
      root = v;
    } else if (parent[v] < 0 || parent[v] >= t || parent[v] == v) {
      return ORC_ENOTTREE;
    }
  }
  if (root < 0) return ORC_ENOTTREE;
  for (int v = 0; v < t; ++v) { /* walk up at most t steps */
    int u = v, steps = 0;
    while (u != root && steps <= t) { u = parent[u]; ++steps; }
    if (u != root) return ORC_ENOTTREE;
  }
  T->t = t;
  T->root = root;
  T->nch = (int *)calloc(t, sizeof(int));
  T->ch = (int **)calloc(t, sizeof(int *));
  T->subsize = (int *)calloc(t, sizeof(int));
  for (int v = 0; v < t; ++v)
    if (v != root) T->nch[parent[v]]++;
  for (int v = 0; v < t; ++v) {
    T->ch[v] = (int *)malloc((T->nch[v] + 1) * sizeof(int));
    T->nch[v] = 0;
  }
  for (int v = 0; v < t; ++v)
    if (v != root) T->ch[parent[v]][T->nch[parent[v]]++] = v;
  subtree_size(T, root);
  return ORC_OK;
}

typedef struct { int v, lo, hi; } subtpl; /* v with the subtrees of children lo..hi-1 */

static int subtpl_size(const tree *T, subtpl s) {
  int z = 1;
  for (int c = s.lo; c < s.hi; ++c) z += T->subsize[T->ch[s.v][c]];
  return z;
}

static void subtpl_split(const tree *T, subtpl s, int cut, subtpl *act, subtpl *pas) {
  int tau = (cut == 0) ? T->ch[s.v][s.hi - 1] : T->ch[s.v][s.lo];
  *act = s;
  if (cut == 0) act->hi--; else act->lo++;
  pas->v = tau;
  pas->lo = 0;
  pas->hi = T->nch[tau];
}

/* ----------------------------------------------------------------------- */
/* colour-set column indices                                                */

typedef struct {
  int k;
  int32_t *rank;     /* rank[mask] = index of mask among sets of its size */
  int64_t ncols[65]; /* ncols[m] = number of sets of size m */
  uint32_t **sets;   /* sets[m][r] = mask with index r */
} csets;

static void csets_free(csets *S) {
  if (!S->rank) return;
  for (int m = 0; m <= S->k; ++m) free(S->sets[m]);
  free(S->sets);
  free(S->rank);
  S->rank = NULL;
}

static int csets_build(int k, csets *S) {
  memset(S, 0, sizeof(*S));
  if (k < 1 || k > 24) return ORC_EINVAL;
  S->k = k;
  S->rank = (int32_t *)malloc(sizeof(int32_t) << k);
  S->sets = (uint32_t **)calloc(k + 1, sizeof(uint32_t *));
  if (!S->rank || !S->sets) return ORC_ENOMEM;
  uint32_t full = (k == 32) ? 0xFFFFFFFFu : ((1u << k) - 1u);
  for (int m = 0; m <= k; ++m) {
    /* count sets of size m */
    int64_t cnt = 0;
    for (uint64_t x = 0; x <= full; ++x)
      if (__builtin_popcountll(x) == m) cnt++;
    S->ncols[m] = cnt;
    S->sets[m] = (uint32_t *)malloc((cnt ? cnt : 1) * sizeof(uint32_t));
    if (m == 0) {
      S->sets[0][0] = 0;
      S->rank[0] = 0;
      continue;
    }
    /* Gosper's hack: next larger integer with the same number of set bits */
    uint64_t x = (1ull << m) - 1ull;
    int64_t r = 0;
    while (x <= full) {
      S->sets[m][r] = (uint32_t)x;
      S->rank[x] = (int32_t)r;
      ++r;
      uint64_t c = x & (~x + 1ull);
      uint64_t y = x + c;
      x = (((x ^ y) >> 2) / c) | y;
    }
  }
  return ORC_OK;
}

/* ----------------------------------------------------------------------- */
/* graph view                                                               */

typedef struct {
  int64_t n;
  const int64_t *row_ptr;
  const int32_t *col_idx;
  const double *w; /* nullable: 0/1 adjacency */
} graph;

/* ----------------------------------------------------------------------- */
/* dynamic programme                                                        */

typedef struct {
  const graph *G;
  const tree *T;
  const csets *S;
  const uint8_t *col;
  int k;
  int u64;   /* 0: double, 1: uint64 mod 2^64 */
  int alg2;  /* 1: Alg. 2 recurrence */
  int cut;
  int overflow;
} dp;

typedef struct {
  int64_t ncols;
  int size;
  double *f;
  uint64_t *u;
} table;

static int table_alloc(table *M, int64_t n, int64_t ncols, int size, int u64) {
  M->ncols = ncols;
  M->size = size;
  M->f = NULL;
  M->u = NULL;
  if (u64) M->u = (uint64_t *)calloc((size_t)(n * ncols), sizeof(uint64_t));
  else M->f = (double *)calloc((size_t)(n * ncols), sizeof(double));
  return (M->f || M->u) ? ORC_OK : ORC_ENOMEM;
}

static void table_free(table *M) {
  free(M->f);
  free(M->u);
  M->f = NULL;
  M->u = NULL;
}

static inline uint64_t addu(uint64_t a, uint64_t b, int *ovf) {
  uint64_t r;
  if (__builtin_add_overflow(a, b, &r)) *ovf = 1;
  return r;
}

static inline uint64_t mulu(uint64_t a, uint64_t b, int *ovf) {
  uint64_t r;
  if (__builtin_mul_overflow(a, b, &r)) *ovf = 1;
  return r;
}

/* B = A_G M (Alg. 4): B(i,c) = sum over CSR entries e of row i of
 * w_e * M(col_idx[e], c), in CSR order. */
static void neighbour_sum(const dp *D, const table *M, table *B) {
  const graph *G = D->G;
  int64_t nc = M->ncols;
  int ovf = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : ovf)
  for (int64_t i = 0; i < G->n; ++i) {
    for (int64_t e = G->row_ptr[i]; e < G->row_ptr[i + 1]; ++e) {
      int64_t j = G->col_idx[e];
      for (int64_t c = 0; c < nc; ++c) {
        if (D->u64) {
          B->u[i * nc + c] = addu(B->u[i * nc + c], M->u[j * nc + c], &ovf);
        } else {
          double wij = G->w ? G->w[e] : 1.0;
          B->f[i * nc + c] += wij * M->f[j * nc + c];
        }
      }
    }
  }
  if (ovf) ((dp *)D)->overflow = 1;
}

static int count_table(dp *D, subtpl s, table *out);

/* M_s(i,C) = sum over (C_a, C_p) splitting C with |C_a| = |T_a| of
 *            M_a(i, I_{C_a}) * B(i, I_{C_p})                    (Alg. 3, stage 2)
 * where B = A_G M_p (Alg. 3, stage 1).  With alg2 set, the neighbour sum sits
 * inside the split loop as in Alg. 2:
 * M_s(i,C) = sum_{j in N(i)} sum_splits M_a(i,C_a) M_p(j,C_p).
 * Bkeep (nullable) receives B when alg2 is off.                               */
static int combine(dp *D, int size, table *Ma, table *Mp, table *out, table *Bkeep) {
  const csets *S = D->S;
  const graph *G = D->G;
  int64_t n = G->n;
  if (table_alloc(out, n, S->ncols[size], size, D->u64)) return ORC_ENOMEM;
  int ma = Ma->size;
  int64_t nc = out->ncols;
  const uint32_t *sets = S->sets[size];
  int ovf = 0;
  if (!D->alg2) {
    table B;
    if (table_alloc(&B, n, Mp->ncols, Mp->size, D->u64)) return ORC_ENOMEM;
    neighbour_sum(D, Mp, &B);
#pragma omp parallel for schedule(dynamic, 64) reduction(| : ovf)
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t r = 0; r < nc; ++r) {
        uint32_t C = sets[r];
        /* every sub-mask of C with |T_a| bits is one split (C_a, C \ C_a) */
        for (uint32_t sub = C; sub; sub = (sub - 1) & C) {
          if (__builtin_popcount(sub) != ma) continue;
          int64_t ia = S->rank[sub], ip = S->rank[C & ~sub];
          if (D->u64) {
            out->u[i * nc + r] =
                addu(out->u[i * nc + r], mulu(Ma->u[i * Ma->ncols + ia], B.u[i * B.ncols + ip], &ovf), &ovf);
          } else {
            out->f[i * nc + r] += Ma->f[i * Ma->ncols + ia] * B.f[i * B.ncols + ip];
          }
        }
      }
    }
    if (Bkeep) *Bkeep = B; else table_free(&B);
  } else {
#pragma omp parallel for schedule(dynamic, 64) reduction(| : ovf)
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t r = 0; r < nc; ++r) {
        uint32_t C = sets[r];
        for (uint32_t sub = C; sub; sub = (sub - 1) & C) {
          if (__builtin_popcount(sub) != ma) continue;
          int64_t ia = S->rank[sub], ip = S->rank[C & ~sub];
          for (int64_t e = G->row_ptr[i]; e < G->row_ptr[i + 1]; ++e) {
            int64_t j = G->col_idx[e];
            if (D->u64) {
              out->u[i * nc + r] = addu(out->u[i * nc + r],
                                        mulu(Ma->u[i * Ma->ncols + ia], Mp->u[j * Mp->ncols + ip], &ovf), &ovf);
            } else {
              double wij = G->w ? G->w[e] : 1.0;
              out->f[i * nc + r] += Ma->f[i * Ma->ncols + ia] * (wij * Mp->f[j * Mp->ncols + ip]);
            }
          }
        }
      }
    }
  }
  if (ovf) D->overflow = 1;
  return ORC_OK;
}

/* single vertex: M(i, {colour of i}) = 1, zero elsewhere (Alg. 2) */
static int leaf_table(dp *D, table *out) {
  const csets *S = D->S;
  int64_t n = D->G->n;
  if (table_alloc(out, n, S->ncols[1], 1, D->u64)) return ORC_ENOMEM;
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = S->rank[1u << D->col[i]];
    if (D->u64) out->u[i * out->ncols + c] = 1; else out->f[i * out->ncols + c] = 1.0;
  }
  return ORC_OK;
}

/* tables are built in reverse order of partitioning: children first */
static int count_table(dp *D, subtpl s, table *out) {
  int size = subtpl_size(D->T, s);
  if (size == 1) return leaf_table(D, out);
  subtpl a, p;
  subtpl_split(D->T, s, D->cut, &a, &p);
  table Ma, Mp;
  int rc = count_table(D, a, &Ma);
  if (rc) return rc;
  rc = count_table(D, p, &Mp);
  if (!rc) rc = combine(D, size, &Ma, &Mp, out, NULL);
  table_free(&Ma);
  table_free(&Mp);
  return rc;
}

static int dp_setup(dp *D, graph *G, tree *T, csets *S, int64_t n, const int64_t *row_ptr,
                    const int32_t *col_idx, const double *w, const int32_t *parent, int32_t t,
                    int32_t k, const uint8_t *colors, int32_t u64, int32_t alg2, int32_t cut) {
  if (n < 0 || !row_ptr || (row_ptr[n] > 0 && !col_idx) || !colors || k < t || k > 24) return ORC_EINVAL;
  if (u64 && w) return ORC_EINVAL; /* exact mode counts on the 0/1 adjacency */
  if (cut != 0 && cut != 1) return ORC_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    if (colors[i] >= k) return ORC_EINVAL;
  G->n = n;
  G->row_ptr = row_ptr;
  G->col_idx = col_idx;
  G->w = w;
  int rc = tree_build(parent, t, T);
  if (rc) return rc;
  rc = csets_build(k, S);
  if (rc) { tree_free(T); return rc; }
  memset(D, 0, sizeof(*D));
  D->G = G;
  D->T = T;
  D->S = S;
  D->col = colors;
  D->k = k;
  D->u64 = u64;
  D->alg2 = alg2;
  D->cut = cut;
  return ORC_OK;
}

/* Colourful count of one colouring: sum_i sum_{|C| = t} M_0(i, I_C)
 * (Alg. 1, the double sum in finalCount before the 1/(P alpha) factor).
 * This counts colourful labelled maps of T into G. */
int orc_count(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *w,
              const int32_t *parent, int32_t t, int32_t k, const uint8_t *colors, int32_t u64,
              int32_t alg2, int32_t cut, double *out_f64, uint64_t *out_u64, int32_t *overflow) {
  dp D;
  graph G;
  tree T;
  csets S;
  int rc = dp_setup(&D, &G, &T, &S, n, row_ptr, col_idx, w, parent, t, k, colors, u64, alg2, cut);
  if (rc) return rc;
  subtpl root = {T.root, 0, T.nch[T.root]};
  table M0;
  rc = count_table(&D, root, &M0);
  if (!rc) {
    double sf = 0.0;
    uint64_t su = 0;
    int ovf = 0;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t c = 0; c < M0.ncols; ++c) {
        if (u64) su = addu(su, M0.u[i * M0.ncols + c], &ovf);
        else sf += M0.f[i * M0.ncols + c];
      }
    if (ovf) D.overflow = 1;
    if (out_f64) *out_f64 = u64 ? (double)su : sf;
    if (out_u64) *out_u64 = su;
    if (overflow) *overflow = D.overflow;
    table_free(&M0);
  }
  csets_free(&S);
  tree_free(&T);
  return rc;
}

/* Count table of sub-template (v, first `nkept` children) under the last-child
 * cut (cut = 0) or of (v, children from index n_ch - nkept on) under the
 * first-child cut (cut = 1), written row-major into out (n x C(k, size)). */
int orc_node_table(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *w,
                   const int32_t *parent, int32_t t, int32_t k, const uint8_t *colors, int32_t u64,
                   int32_t cut, int32_t v, int32_t nkept, double *out_f64, uint64_t *out_u64,
                   int64_t *out_ncols) {
  dp D;
  graph G;
  tree T;
  csets S;
  int rc = dp_setup(&D, &G, &T, &S, n, row_ptr, col_idx, w, parent, t, k, colors, u64, 0, cut);
  if (rc) return rc;
  if (v < 0 || v >= t || nkept < 0 || nkept > T.nch[v]) { csets_free(&S); tree_free(&T); return ORC_EINVAL; }
  subtpl s = {v, 0, nkept};
  if (cut == 1) { s.lo = T.nch[v] - nkept; s.hi = T.nch[v]; }
  table M;
  rc = count_table(&D, s, &M);
  if (!rc) {
    if (out_ncols) *out_ncols = M.ncols;
    if (u64 && out_u64) memcpy(out_u64, M.u, (size_t)(n * M.ncols) * sizeof(uint64_t));
    if (!u64 && out_f64) memcpy(out_f64, M.f, (size_t)(n * M.ncols) * sizeof(double));
    table_free(&M);
  }
  csets_free(&S);
  tree_free(&T);
  return rc;
}

/* B = A_G M for a row-major n x ncols table M (Alg. 4). */
int orc_neighbour_sum(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *w,
                      int64_t ncols, int32_t u64, const double *M_f64, const uint64_t *M_u64,
                      double *B_f64, uint64_t *B_u64, int32_t *overflow) {
  if (u64 && w) return ORC_EINVAL;
  graph G = {n, row_ptr, col_idx, w};
  dp D;
  memset(&D, 0, sizeof(D));
  D.G = &G;
  D.u64 = u64;
  table M = {ncols, 0, (double *)M_f64, (uint64_t *)M_u64};
  table B = {ncols, 0, B_f64, B_u64};
  if (u64) memset(B_u64, 0, (size_t)(n * ncols) * sizeof(uint64_t));
  else memset(B_f64, 0, (size_t)(n * ncols) * sizeof(double));
  neighbour_sum(&D, &M, &B);
  if (overflow) *overflow = D.overflow;
  return ORC_OK;
}

/* ----------------------------------------------------------------------- */
/* probability and estimator (Alg. 1)                                       */

/* P = probability that a fixed set of t vertices gets t distinct colours out
 * of k: k (k-1) ... (k-t+1) / k^t. */
double orc_colorful_probability(int32_t t, int32_t k) {
  double p = 1.0;
  for (int i = 0; i < t; ++i) p *= (double)(k - i) / (double)k;
  return p;
}

/* ----------------------------------------------------------------------- */
/* brute force                                                              */

typedef struct {
  const graph *G;
  const tree *T;
  const uint8_t *col; /* NULL: exact (injective) maps; else colourful maps */
  int *order;         /* template vertices, each after its parent */
  int *par;
  int64_t *img;       /* image of each template vertex */
  int64_t *ent;       /* CSR entry used by the edge (parent image -> image) */
  uint8_t *used_v;    /* exact mode: graph vertices in use */
  uint32_t used_c;    /* colourful mode: colours in use */
  double total;
  uint64_t total_u;
  double *grad;       /* nullable: per directed entry */
  int64_t limit, visited;
} brute;

static void brute_leaf(brute *B) {
  int t = B->T->t;
  double prod = 1.0;
  for (int q = 1; q < t; ++q) {
    int u = B->order[q];
    prod *= B->G->w ? B->G->w[B->ent[u]] : 1.0;
  }
  B->total += prod;
  B->total_u += 1;
  if (B->grad) {
    for (int q = 1; q < t; ++q) {
      int u = B->order[q];
      double others = 1.0;
      for (int r = 1; r < t; ++r) {
        if (r == q) continue;
        int x = B->order[r];
        others *= B->G->w ? B->G->w[B->ent[x]] : 1.0;
      }
      B->grad[B->ent[u]] += others;
    }
  }
}

static void brute_rec(brute *B, int q) {
  if (B->limit && B->visited > B->limit) return;
  B->visited++;
  int t = B->T->t;
  if (q == t) {
    brute_leaf(B);
    return;
  }
  int u = B->order[q];
  int64_t pi = B->img[B->par[u]];
  for (int64_t e = B->G->row_ptr[pi]; e < B->G->row_ptr[pi + 1]; ++e) {
    int64_t x = B->G->col_idx[e];
    if (B->col) {
      uint32_t cm = 1u << B->col[x];
      if (B->used_c & cm) continue;
      B->used_c |= cm;
      B->img[u] = x;
      B->ent[u] = e;
      brute_rec(B, q + 1);
      B->used_c &= ~cm;
    } else {
      if (B->used_v[x]) continue;
      B->used_v[x] = 1;
      B->img[u] = x;
      B->ent[u] = e;
      brute_rec(B, q + 1);
      B->used_v[x] = 0;
    }
  }
}

/* Enumerate every map phi of template vertices to graph vertices that sends
 * each template edge (p, u) onto a graph edge (phi(p), phi(u)) and is
 * injective (colors == NULL) or colourful (colours of the images distinct).
 * total = sum over maps of the product of the weights of the t-1 edges used
 * (the number of maps when w is NULL).  grad (nullable, [nnz]) receives, for
 * each directed CSR entry (phi(p) -> phi(u)) with p the parent of u in the
 * rooted template, the sum over maps of the product of the other t-2 weights.
 * limit > 0 stops after that many search nodes (returns 1). */
int orc_brute(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *w,
              const int32_t *parent, int32_t t, const uint8_t *colors, int64_t limit,
              double *total, uint64_t *total_u64, double *grad) {
  tree T;
  int rc = tree_build(parent, t, &T);
  if (rc) return rc;
  graph G = {n, row_ptr, col_idx, w};
  brute B;
  memset(&B, 0, sizeof(B));
  B.G = &G;
  B.T = &T;
  B.col = colors;
  B.order = (int *)malloc(t * sizeof(int));
  B.par = (int *)malloc(t * sizeof(int));
  B.img = (int64_t *)malloc(t * sizeof(int64_t));
  B.ent = (int64_t *)malloc(t * sizeof(int64_t));
  B.used_v = (uint8_t *)calloc(n > 0 ? n : 1, 1);
  B.grad = grad;
  B.limit = limit;
  if (grad) memset(grad, 0, (size_t)row_ptr[n] * sizeof(double));
  /* breadth-first order from the root */
  int head = 0, tail = 0;
  B.order[tail++] = T.root;
  B.par[T.root] = -1;
  while (head < tail) {
    int v = B.order[head++];
    for (int c = 0; c < T.nch[v]; ++c) {
      B.order[tail++] = T.ch[v][c];
      B.par[T.ch[v][c]] = v;
    }
  }
  for (int64_t x = 0; x < n; ++x) {
    B.img[T.root] = x;
    if (colors) {
      B.used_c = 1u << colors[x];
    } else {
      B.used_v[x] = 1;
    }
    brute_rec(&B, 1);
    if (!colors) B.used_v[x] = 0;
  }
  if (total) *total = B.total;
  if (total_u64) *total_u64 = B.total_u;
  int hit = (limit && B.visited > limit) ? 1 : 0;
  free(B.order);
  free(B.par);
  free(B.img);
  free(B.ent);
  free(B.used_v);
  tree_free(&T);
  return hit;
}

/* alpha of Alg. 1: the number of maps of T onto itself that preserve
 * adjacency, counted by brute force over T viewed as a graph. */
int64_t orc_automorphisms(const int32_t *parent, int32_t t) {
  tree T;
  if (tree_build(parent, t, &T)) return -1;
  tree_free(&T);
  int64_t *rp = (int64_t *)calloc(t + 1, sizeof(int64_t));
  int32_t *ci = (int32_t *)malloc(2 * (t > 1 ? t - 1 : 1) * sizeof(int32_t));
  for (int v = 0; v < t; ++v)
    if (parent[v] >= 0) { rp[v + 1]++; rp[parent[v] + 1]++; }
  for (int v = 0; v < t; ++v) rp[v + 1] += rp[v];
  int64_t *cur = (int64_t *)malloc(t * sizeof(int64_t));
  memcpy(cur, rp, t * sizeof(int64_t));
  for (int v = 0; v < t; ++v)
    if (parent[v] >= 0) { ci[cur[v]++] = parent[v]; ci[cur[parent[v]]++] = v; }
  uint64_t cnt = 0;
  orc_brute(t, rp, ci, NULL, parent, t, NULL, 0, NULL, &cnt, NULL);
  free(rp);
  free(ci);
  free(cur);
  return (int64_t)cnt;
}

/* ----------------------------------------------------------------------- */
/* reverse-mode derivative                                                  */

typedef struct gnode {
  subtpl s;
  int size;
  table M;          /* forward table */
  table B;          /* A_G M_p (only for split nodes) */
  struct gnode *a, *p;
} gnode;

static int gforward(dp *D, subtpl s, gnode **out) {
  gnode *g = (gnode *)calloc(1, sizeof(gnode));
  *out = g;
  g->s = s;
  g->size = subtpl_size(D->T, s);
  if (g->size == 1) return leaf_table(D, &g->M);
  subtpl a, p;
  subtpl_split(D->T, s, D->cut, &a, &p);
  int rc = gforward(D, a, &g->a);
  if (!rc) rc = gforward(D, p, &g->p);
  if (!rc) rc = combine(D, g->size, &g->a->M, &g->p->M, &g->M, &g->B);
  return rc;
}

static void gfree(gnode *g) {
  if (!g) return;
  gfree(g->a);
  gfree(g->p);
  table_free(&g->M);
  table_free(&g->B);
  free(g);
}

/* Given Mbar = d f / d M_s, accumulate d f / d w into grad and recurse:
 *   Mbar_a(i, C_a) = sum_{C = C_a + C_p} Mbar(i, C) B(i, C_p)
 *   Bbar(i, C_p)   = sum_{C = C_a + C_p} Mbar(i, C) M_a(i, C_a)
 *   grad(e = i->j) += sum_{C_p} Bbar(i, C_p) M_p(j, C_p)
 *   Mbar_p(j, C_p) = sum_{e = i->j} w_e Bbar(i, C_p)                        */
static int gbackward(dp *D, gnode *g, const double *Mbar, double *grad) {
  if (g->size == 1) return ORC_OK;
  const graph *G = D->G;
  const csets *S = D->S;
  int64_t n = G->n;
  int64_t nc = g->M.ncols, na = g->a->M.ncols, np = g->p->M.ncols;
  int ma = g->a->size;
  const uint32_t *sets = S->sets[g->size];
  double *Ma_bar = (double *)calloc((size_t)(n * na), sizeof(double));
  double *B_bar = (double *)calloc((size_t)(n * np), sizeof(double));
  double *Mp_bar = (double *)calloc((size_t)(n * np), sizeof(double));
  if (!Ma_bar || !B_bar || !Mp_bar) return ORC_ENOMEM;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t r = 0; r < nc; ++r) {
      uint32_t C = sets[r];
      double mb = Mbar[i * nc + r];
      for (uint32_t sub = C; sub; sub = (sub - 1) & C) {
        if (__builtin_popcount(sub) != ma) continue;
        int64_t ia = S->rank[sub], ip = S->rank[C & ~sub];
        Ma_bar[i * na + ia] += mb * g->B.f[i * np + ip];
        B_bar[i * np + ip] += mb * g->a->M.f[i * na + ia];
      }
    }
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = G->row_ptr[i]; e < G->row_ptr[i + 1]; ++e) {
      int64_t j = G->col_idx[e];
      double s = 0.0;
      for (int64_t c = 0; c < np; ++c) s += B_bar[i * np + c] * g->p->M.f[j * np + c];
      grad[e] += s;
    }
  }
  /* Mbar_p = A_G^T Bbar: scatter over entries, sequential for a fixed order */
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = G->row_ptr[i]; e < G->row_ptr[i + 1]; ++e) {
      int64_t j = G->col_idx[e];
      double wij = G->w ? G->w[e] : 1.0;
      for (int64_t c = 0; c < np; ++c) Mp_bar[j * np + c] += wij * B_bar[i * np + c];
    }
  }
  free(B_bar);
  int rc = gbackward(D, g->a, Ma_bar, grad);
  if (!rc) rc = gbackward(D, g->p, Mp_bar, grad);
  free(Ma_bar);
  free(Mp_bar);
  return rc;
}

/* d(colourful count)/d(w_e) for every directed CSR entry e, at weights w
 * (NULL: all ones).  The colourful count is sum_i sum_{|C|=t} M_0(i, C). */
int orc_grad(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *w,
             const int32_t *parent, int32_t t, int32_t k, const uint8_t *colors, int32_t cut,
             double *f_out, double *grad) {
  dp D;
  graph G;
  tree T;
  csets S;
  int rc = dp_setup(&D, &G, &T, &S, n, row_ptr, col_idx, w, parent, t, k, colors, 0, 0, cut);
  if (rc) return rc;
  subtpl root = {T.root, 0, T.nch[T.root]};
  gnode *g = NULL;
  rc = gforward(&D, root, &g);
  if (!rc) {
    int64_t nc = g->M.ncols;
    double f = 0.0;
    for (int64_t x = 0; x < n * nc; ++x) f += g->M.f[x];
    if (f_out) *f_out = f;
    double *Mbar = (double *)malloc((size_t)(n * nc) * sizeof(double));
    for (int64_t x = 0; x < n * nc; ++x) Mbar[x] = 1.0;
    memset(grad, 0, (size_t)row_ptr[n] * sizeof(double));
    rc = gbackward(&D, g, Mbar, grad);
    free(Mbar);
  }
  gfree(g);
  csets_free(&S);
  tree_free(&T);
  return rc;
}

int orc_num_threads(void) { return omp_get_max_threads(); }
