/*
 * Seeded synthetic graph generators shared by the oracle tests and the GPU
 * path.  This file holds input synthesis only: no part of the colour-coding
 * count is computed here.
 *
 * Every random draw is a pure function of (seed, stream, counter) through the
 * SplitMix64 output finaliser (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), so results do not depend on
 * the thread count.
 *
 * Edge sets: samples are drawn in counter order; the graph is the set of the
 * first m distinct undirected non-loop edges in that order ("draw until
 * exactly m unique edges").  Distinctness is resolved with a lock-free hash
 * set that keeps, per key, the smallest sample index that produced it, which
 * makes the selected set independent of thread timing.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC gen.c -o libgraphgen.so
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t fin64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* 64 random bits for (seed, stream, counter). */
static inline uint64_t rnd(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return fin64(fin64(seed + GOLDEN * (stream + 1)) ^ (ctr * GOLDEN + 0x632BE59BD9B4E019ULL));
}

/* uniform double in [0,1) from the top 53 bits */
static inline double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* uniform integer in [0,n) (Lemire multiply-shift on 32 bits; n < 2^32) */
static inline uint32_t below(uint32_t r32, uint32_t n) {
  return (uint32_t)(((uint64_t)r32 * (uint64_t)n) >> 32);
}

/* ------------------------------------------------------------------------ */
/* distinct-edge hash set                                                     */

#define EMPTY_KEY 0xFFFFFFFFFFFFFFFFULL

typedef struct {
  uint64_t cap;     /* power of two */
  uint64_t *key;
  uint32_t *first;  /* smallest sample index that produced key */
} eset;

static int eset_init(eset *s, uint64_t cap) {
  s->cap = cap;
  s->key = (uint64_t *)malloc(cap * sizeof(uint64_t));
  s->first = (uint32_t *)malloc(cap * sizeof(uint32_t));
  if (!s->key || !s->first) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)cap; ++i) {
    s->key[i] = EMPTY_KEY;
    s->first[i] = 0xFFFFFFFFu;
  }
  return 0;
}

static void eset_free(eset *s) {
  free(s->key);
  free(s->first);
}

/* returns 1 if the key was new */
static inline int eset_insert(eset *s, uint64_t k, uint32_t idx) {
  uint64_t h = fin64(k) & (s->cap - 1);
  for (;;) {
    uint64_t cur = __atomic_load_n(&s->key[h], __ATOMIC_RELAXED);
    if (cur == EMPTY_KEY) {
      uint64_t exp = EMPTY_KEY;
      if (__atomic_compare_exchange_n(&s->key[h], &exp, k, 0, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED)) {
        uint32_t f = __atomic_load_n(&s->first[h], __ATOMIC_RELAXED);
        while (idx < f && !__atomic_compare_exchange_n(&s->first[h], &f, idx, 0, __ATOMIC_ACQ_REL,
                                                       __ATOMIC_RELAXED)) {
        }
        return 1;
      }
      cur = exp;
    }
    if (cur == k) {
      uint32_t f = __atomic_load_n(&s->first[h], __ATOMIC_RELAXED);
      while (idx < f && !__atomic_compare_exchange_n(&s->first[h], &f, idx, 0, __ATOMIC_ACQ_REL,
                                                     __ATOMIC_RELAXED)) {
      }
      return 0;
    }
    h = (h + 1) & (s->cap - 1);
  }
}

/* A sampler writes the canonical key (u<v, key = u<<32|v) of sample s, or
 * EMPTY_KEY for a rejected sample (self-loop). */
typedef uint64_t (*sampler_fn)(const void *ctx, uint64_t s);

static inline uint64_t canon(uint32_t u, uint32_t v) {
  if (u == v) return EMPTY_KEY;
  if (u > v) {
    uint32_t t = u;
    u = v;
    v = t;
  }
  return ((uint64_t)u << 32) | v;
}

/* Draw samples in counter order until m distinct keys exist; write the m keys
 * with the smallest first-sample index (sorted ascending by key) to out. */
static int first_m_distinct(sampler_fn fn, const void *ctx, int64_t m, uint64_t *out) {
  if (m <= 0) return 0;
  uint64_t cap = 1024;
  while (cap < (uint64_t)(m * 5 / 2)) cap <<= 1;
  eset s;
  if (eset_init(&s, cap)) return -1;
  int64_t drawn = 0, distinct = 0;
  int64_t batch = m + m / 4 + 64;
  while (distinct < m) {
    if (drawn + batch > 0xFFFFFFF0LL) { eset_free(&s); return -2; }
    if ((uint64_t)(distinct + batch) * 10 > cap * 7) { eset_free(&s); return -3; }
    int64_t added = 0;
#pragma omp parallel for schedule(static) reduction(+ : added)
    for (int64_t i = drawn; i < drawn + batch; ++i) {
      uint64_t k = fn(ctx, (uint64_t)i);
      if (k != EMPTY_KEY) added += eset_insert(&s, k, (uint32_t)i);
    }
    drawn += batch;
    distinct += added;
    batch = (m - distinct) * 2 + 64;
  }
  /* threshold T: exactly m first-indices are < T */
  uint8_t *mark = (uint8_t *)calloc((size_t)drawn, 1);
  if (!mark) { eset_free(&s); return -1; }
#pragma omp parallel for schedule(static)
  for (int64_t h = 0; h < (int64_t)cap; ++h)
    if (s.key[h] != EMPTY_KEY) mark[s.first[h]] = 1;
  int64_t cnt = 0, T = drawn;
  for (int64_t i = 0; i < drawn; ++i) {
    cnt += mark[i];
    if (cnt == m) { T = i + 1; break; }
  }
  free(mark);
  int64_t pos = 0;
  for (int64_t h = 0; h < (int64_t)cap; ++h)
    if (s.key[h] != EMPTY_KEY && (int64_t)s.first[h] < T) out[pos++] = s.key[h];
  eset_free(&s);
  if (pos != m) return -4;
  /* canonical order: ascending key (LSD radix, 16-bit digits) */
  uint64_t *tmp = (uint64_t *)malloc((size_t)m * sizeof(uint64_t));
  if (!tmp) return -1;
  uint64_t *a = out, *b = tmp;
  for (int sh = 0; sh < 64; sh += 16) {
    int64_t *cntv = (int64_t *)calloc(65536, sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) cntv[(a[i] >> sh) & 0xFFFF]++;
    int64_t acc = 0;
    for (int d = 0; d < 65536; ++d) { int64_t c = cntv[d]; cntv[d] = acc; acc += c; }
    for (int64_t i = 0; i < m; ++i) b[cntv[(a[i] >> sh) & 0xFFFF]++] = a[i];
    free(cntv);
    uint64_t *t = a; a = b; b = t;
  }
  /* four passes: result is back in out */
  free(tmp);
  return 0;
}

static void split_keys(const uint64_t *keys, int64_t m, int32_t *eu, int32_t *ev) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    eu[i] = (int32_t)(keys[i] >> 32);
    ev[i] = (int32_t)(keys[i] & 0xFFFFFFFFu);
  }
}

/* ------------------------------------------------------------------------ */
/* Erdos-Renyi G(n, m): uniform distinct pairs                               */

typedef struct { uint64_t seed; uint32_t n; } er_ctx;

static uint64_t er_sample(const void *c, uint64_t s) {
  const er_ctx *x = (const er_ctx *)c;
  uint64_t r = rnd(x->seed, 1, s);
  return canon(below((uint32_t)r, x->n), below((uint32_t)(r >> 32), x->n));
}

int gg_er(int64_t n, int64_t m, uint64_t seed, int32_t *eu, int32_t *ev) {
  if (n < 2 || n >= 0x7FFFFFFF || m < 0 || m > n * (n - 1) / 2) return -10;
  er_ctx c = {seed, (uint32_t)n};
  uint64_t *keys = (uint64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
  int rc = first_m_distinct(er_sample, &c, m, keys);
  if (!rc) split_keys(keys, m, eu, ev);
  free(keys);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* RMAT (Chakrabarti, Zhan & Faloutsos 2004): recursive quadrant choice with  */
/* probabilities (a, b, c, d = 1-a-b-c), one 32-bit draw per level.          */

typedef struct {
  uint64_t seed;
  int scale;
  uint32_t ta, tb, tc; /* cumulative thresholds on 2^32 */
  const uint32_t *perm; /* optional vertex relabel */
} rmat_ctx;

static uint64_t rmat_sample(const void *c, uint64_t s) {
  const rmat_ctx *x = (const rmat_ctx *)c;
  uint32_t u = 0, v = 0;
  uint64_t r = 0;
  for (int l = 0; l < x->scale; ++l) {
    if ((l & 1) == 0) r = rnd(x->seed, 2, s * 32 + (uint64_t)(l >> 1));
    uint32_t q = (l & 1) ? (uint32_t)(r >> 32) : (uint32_t)r;
    uint32_t bu = 0, bv = 0;
    if (q < x->ta) { bu = 0; bv = 0; }
    else if (q < x->tb) { bu = 0; bv = 1; }
    else if (q < x->tc) { bu = 1; bv = 0; }
    else { bu = 1; bv = 1; }
    u = (u << 1) | bu;
    v = (v << 1) | bv;
  }
  if (x->perm) { u = x->perm[u]; v = x->perm[v]; }
  return canon(u, v);
}

/* seeded Fisher-Yates permutation of [0, n) */
int gg_permutation(int64_t n, uint64_t seed, uint32_t *perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    uint64_t r = rnd(seed, 3, (uint64_t)i);
    int64_t j = (int64_t)(((unsigned __int128)r * (uint64_t)(i + 1)) >> 64);
    uint32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
  return 0;
}

int gg_rmat(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed, int32_t relabel,
            int32_t *eu, int32_t *ev) {
  if (scale < 1 || scale > 30 || m < 0) return -10;
  double d = 1.0 - a - b - c;
  if (a < 0 || b < 0 || c < 0 || d < -1e-12) return -10;
  int64_t n = (int64_t)1 << scale;
  if (m > n * (n - 1) / 2) return -10;
  rmat_ctx x;
  x.seed = seed;
  x.scale = scale;
  x.ta = (uint32_t)fmin(4294967295.0, a * 4294967296.0);
  x.tb = (uint32_t)fmin(4294967295.0, (a + b) * 4294967296.0);
  x.tc = (uint32_t)fmin(4294967295.0, (a + b + c) * 4294967296.0);
  uint32_t *perm = NULL;
  if (relabel) {
    perm = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    gg_permutation(n, seed ^ 0xA5A5A5A5ULL, perm);
  }
  x.perm = perm;
  uint64_t *keys = (uint64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
  int rc = first_m_distinct(rmat_sample, &x, m, keys);
  if (!rc) split_keys(keys, m, eu, ev);
  free(keys);
  free(perm);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Chung-Lu with power-law expected degrees w_i = C (i + i0)^(-1/(gamma-1)),  */
/* i0 chosen so w_0 = sqrt(n * avg) (structural cut-off) and C so that the    */
/* mean of w is avg.  Endpoints are drawn independently with probability      */
/* proportional to w (inverse CDF by binary search).                         */

typedef struct {
  uint64_t seed;
  int64_t n;
  const double *cdf; /* cdf[i] = sum_{l<=i} w_l / W */
} cl_ctx;

static inline uint32_t cl_pick(const cl_ctx *x, double r) {
  int64_t lo = 0, hi = x->n - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (x->cdf[mid] > r) hi = mid; else lo = mid + 1;
  }
  return (uint32_t)lo;
}

static uint64_t cl_sample(const void *c, uint64_t s) {
  const cl_ctx *x = (const cl_ctx *)c;
  uint64_t r1 = rnd(x->seed, 4, 2 * s), r2 = rnd(x->seed, 4, 2 * s + 1);
  return canon(cl_pick(x, u01(r1)), cl_pick(x, u01(r2)));
}

static double cl_mean(int64_t n, double beta, double i0, double target_w0) {
  double cst = target_w0 * pow(i0, beta), sum = 0.0;
  for (int64_t i = 0; i < n; ++i) sum += pow((double)i + i0, -beta);
  return cst * sum / (double)n;
}

int gg_chung_lu(int64_t n, int64_t m, double gamma, uint64_t seed, int32_t *eu, int32_t *ev,
                double *expected_degree /* nullable, [n] */) {
  if (n < 2 || n >= 0x7FFFFFFF || m < 0 || gamma <= 1.0) return -10;
  double avg = 2.0 * (double)m / (double)n;
  double beta = 1.0 / (gamma - 1.0);
  double w0 = sqrt((double)n * avg);
  /* the mean of w grows monotonically with i0 (w0 fixed); bisect in log space */
  double lo = 1e-6, hi = (double)n * 1e3;
  for (int it = 0; it < 200; ++it) {
    double mid = sqrt(lo * hi);
    if (cl_mean(n, beta, mid, w0) > avg) hi = mid; else lo = mid;
  }
  double i0 = sqrt(lo * hi);
  double cst = w0 * pow(i0, beta);
  double *cdf = (double *)malloc((size_t)n * sizeof(double));
  double acc = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double w = cst * pow((double)i + i0, -beta);
    if (expected_degree) expected_degree[i] = w;
    acc += w;
    cdf[i] = acc;
  }
  for (int64_t i = 0; i < n; ++i) cdf[i] /= acc;
  cdf[n - 1] = 1.0;
  cl_ctx x = {seed, n, cdf};
  uint64_t *keys = (uint64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
  int rc = first_m_distinct(cl_sample, &x, m, keys);
  if (!rc) split_keys(keys, m, eu, ev);
  free(keys);
  free(cdf);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Symmetric CSR from an undirected edge list (no loops, no duplicates).       */
/* Each edge appears as (u,v) and (v,u); columns sorted within each row.       */
/* Optional weights: one value per undirected edge, copied to both entries.   */

static void sort_row(int32_t *c, float *w, int64_t len) {
  /* insertion sort for short rows, heap sort otherwise (in-place, O(1) mem) */
  if (len < 32) {
    for (int64_t i = 1; i < len; ++i) {
      int32_t x = c[i];
      float y = w ? w[i] : 0.f;
      int64_t j = i - 1;
      while (j >= 0 && c[j] > x) {
        c[j + 1] = c[j];
        if (w) w[j + 1] = w[j];
        --j;
      }
      c[j + 1] = x;
      if (w) w[j + 1] = y;
    }
    return;
  }
  /* heap sort */
  for (int64_t start = len / 2 - 1; start >= 0; --start) {
    int64_t root = start;
    for (;;) {
      int64_t ch = 2 * root + 1;
      if (ch >= len) break;
      if (ch + 1 < len && c[ch + 1] > c[ch]) ch++;
      if (c[root] >= c[ch]) break;
      int32_t t = c[root]; c[root] = c[ch]; c[ch] = t;
      if (w) { float tw = w[root]; w[root] = w[ch]; w[ch] = tw; }
      root = ch;
    }
  }
  for (int64_t end = len - 1; end > 0; --end) {
    int32_t t = c[0]; c[0] = c[end]; c[end] = t;
    if (w) { float tw = w[0]; w[0] = w[end]; w[end] = tw; }
    int64_t root = 0;
    for (;;) {
      int64_t ch = 2 * root + 1;
      if (ch >= end) break;
      if (ch + 1 < end && c[ch + 1] > c[ch]) ch++;
      if (c[root] >= c[ch]) break;
      int32_t t2 = c[root]; c[root] = c[ch]; c[ch] = t2;
      if (w) { float tw = w[root]; w[root] = w[ch]; w[ch] = tw; }
      root = ch;
    }
  }
}

int gg_csr(int64_t n, int64_t m, const int32_t *eu, const int32_t *ev, const float *ew,
           int64_t *row_ptr, int32_t *col_idx, float *w) {
  if (n <= 0 || m < 0) return -10;
  for (int64_t i = 0; i <= n; ++i) row_ptr[i] = 0;
  for (int64_t e = 0; e < m; ++e) {
    if (eu[e] < 0 || eu[e] >= n || ev[e] < 0 || ev[e] >= n || eu[e] == ev[e]) return -11;
    row_ptr[eu[e] + 1]++;
    row_ptr[ev[e] + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
  int64_t *cur = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  memcpy(cur, row_ptr, (size_t)n * sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) {
    int64_t p = cur[eu[e]]++;
    col_idx[p] = ev[e];
    if (w) w[p] = ew ? ew[e] : 1.0f;
    p = cur[ev[e]]++;
    col_idx[p] = eu[e];
    if (w) w[p] = ew ? ew[e] : 1.0f;
  }
  free(cur);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i)
    sort_row(col_idx + row_ptr[i], w ? w + row_ptr[i] : NULL, row_ptr[i + 1] - row_ptr[i]);
  return 0;
}

/* uniform weights in [lo, hi) per undirected edge, keyed by the edge itself */
int gg_edge_weights(int64_t m, const int32_t *eu, const int32_t *ev, uint64_t seed, double lo,
                    double hi, float *w) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint64_t k = canon((uint32_t)eu[e], (uint32_t)ev[e]);
    w[e] = (float)(lo + (hi - lo) * u01(rnd(seed, 5, k)));
  }
  return 0;
}

int gg_num_threads(void) { return omp_get_max_threads(); }
