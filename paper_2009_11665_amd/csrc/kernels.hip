// Kernels of the colour-coding dynamic programme (SubGraph2Vec, arXiv
// 2009.11665) for gfx950.  Host-side launchers are at the end of the file.
#include <algorithm>
#include <climits>
#include <cstring>
#include <type_traits>

#include "kernels.h"
#include "launch.h"

namespace sg2v {

// ===========================================================================
// Random colouring (Sec. 2.3.1): colour of v in colouring j is
//   h = F(seed ^ F((j << 40) | v)),  colour = (hi32(h) * k) >> 32,
// F = SplitMix64's output finaliser (Steele, Lea & Flood 2014).

__device__ inline uint64_t fin64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// orig (nullable): caller's vertex id of each stored vertex (graphs renumbered
// by degree), so a vertex keeps its colour under the renumbering.
template <class BK>
__device__ __forceinline__ void b_color(BK bk, uint8_t *__restrict__ out, int64_t n, int32_t k, uint64_t seed,
                        int32_t first, int32_t count, const int32_t *__restrict__ orig) {
  int64_t total = n * count;
  for (int64_t x = (int64_t)bk.x() * BLOCK + threadIdx.x; x < total;
       x += (int64_t)bk.gx() * BLOCK) {
    int64_t j = x / n, v = x - j * n;
    const uint64_t u = orig ? (uint64_t)orig[v] : (uint64_t)v;
    uint64_t h = fin64(seed ^ fin64(((uint64_t)(first + j) << 40) | u));
    out[x] = (uint8_t)(((h >> 32) * (uint64_t)k) >> 32);
  }
}
__global__ void k_color(uint8_t *__restrict__ out, int64_t n, int32_t k, uint64_t seed,
                        int32_t first, int32_t count, const int32_t *__restrict__ orig) {
  b_color(HwBlk{}, out, n, k, seed, first, count, orig);
}


// out[idx[e]] = in[e] (per-entry gradients back to the caller's entry order)
__global__ void k_scatter_f64(const double *__restrict__ in, const int64_t *__restrict__ idx,
                              double *__restrict__ out, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    out[idx[e]] = in[e];
}


// ===========================================================================
// Neighbour-colour histogram: B = A_G M_1 where M_1 is the one-hot table of a
// single-vertex passive child (Alg. 2 sets M_s(i, colour of i) = 1), so
//   H(i, jj*k + c) = sum_{e in row i} w_e [colour_jj(col_idx[e]) == c].
// One wave per SpMM task (a row, or a segment of at most 4096 neighbours of
// a long row whose partial row goes to its slot and is summed by
// k_spmm_combine); lanes over neighbours, D blocks of 64 neighbours and JG
// colourings of the pass in flight; lane c keeps colour c's sum.  Unweighted
// counts use a ballot per colour, weighted sums a fixed-order butterfly, so
// the result does not depend on scheduling.

template <class BK, typename T, bool WEIGHTED, int D, int JG>
__device__ __forceinline__ void b_hist(BK bk, const HistArgs &a) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t wave = ((int64_t)bk.x() * BLOCK + threadIdx.x) / WAVE;
  const int64_t nwaves = (int64_t)bk.gx() * WAVES_PER_BLOCK;
  T *H = (T *)a.H;
  T *Pt = (T *)a.partial;
  for (int64_t t = wave; t < a.n_tasks; t += nwaves) {
    const int64_t beg = a.task_beg[t];
    const int len = a.task_len[t];
    const int slot = a.task_slot[t];
    T *dst = slot < 0 ? H + (int64_t)a.task_row[t] * a.ldh : Pt + (int64_t)slot * a.ldh;
    // colourings JG at a time: the neighbour indices are loaded once per group
    // and the group's colour gathers are in flight together
    for (int jg = 0; jg < a.b; jg += JG) {
      T acc[JG];
#pragma unroll
      for (int u = 0; u < JG; ++u) acc[u] = T(0);
      for (int base = 0; base < len; base += D * WAVE) {
        int j[D], c[D][JG];
        float wv[D];
#pragma unroll
        for (int q = 0; q < D; ++q) {
          const int e = base + q * WAVE + lane;
          j[q] = e < len ? a.col_idx[beg + e] : -1;
          wv[q] = 1.0f;
          if constexpr (WEIGHTED) wv[q] = e < len ? a.w[beg + e] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < D; ++q)
#pragma unroll
          for (int u = 0; u < JG; ++u)
            c[q][u] = (j[q] >= 0 && jg + u < a.b) ? (int)a.colors[(int64_t)(a.j0 + jg + u) * a.n + j[q]] : 255;
#pragma unroll
        for (int q = 0; q < D; ++q) {
          if (base + q * WAVE >= len) break;  // uniform
#pragma unroll
          for (int u = 0; u < JG; ++u) {
            if (jg + u >= a.b) break;  // uniform
            for (int cc = 0; cc < a.k; ++cc) {
              if constexpr (!WEIGHTED) {
                const uint64_t m = __ballot(c[q][u] == cc);
                if (lane == cc) acc[u] += (T)__popcll(m);
              } else {
                T v = (c[q][u] == cc) ? (T)wv[q] : T(0);
                for (int off = 1; off < WAVE; off <<= 1) v += shfl_xor(v, off);
                if (lane == cc) acc[u] += v;
              }
            }
          }
        }
      }
      if (lane < a.k) {
#pragma unroll
        for (int u = 0; u < JG; ++u)
          if (jg + u < a.b) dst[(int64_t)(jg + u) * a.k + lane] = acc[u];
      }
    }
    // partial rows are summed over the whole padded width: clear the padding
    if (slot >= 0)
      for (int64_t cidx = (int64_t)a.b * a.k + lane; cidx < a.ldh; cidx += WAVE) dst[cidx] = T(0);
  }
}
template <typename T, bool WEIGHTED, int D, int JG>
__global__ void __launch_bounds__(BLOCK) k_hist(HistArgs a) {
  b_hist<HwBlk, T, WEIGHTED, D, JG>(HwBlk{}, a);
}

// ===========================================================================
// BEGIN k_spmm
// Neighbour aggregation B = A_G M_p (Sec. 5.1, Alg. 4; the SpMV step of Alg. 5) as a
// CSR SpMM over one column chunk of W = G * N columns per blockIdx.y.
//
// Rows are cut into tasks of at most a fixed number of neighbours (long rows
// become several tasks that write partial rows, combined by k_spmm_combine in
// a fixed order).  Tasks are sorted by length, longest first, and grouped in
// units of WAVES_PER_BLOCK * rpw tasks: each wave serves rpw tasks, each task
// 64/rpw lanes = (64/rpw)/G streams of G lanes, and each stream of G lanes
// reads one neighbour row segment of W elements with 16-byte loads.  The
// neighbour indices of a task are loaded once per 64/rpw neighbours and
// broadcast with ds_bpermute.  Blocks walk units with a grid stride.
//
// The column maximum of B (FP32S) is reduced in registers, then across the
// block in LDS, then one atomicMax per column per block.

// the column-maximum reduction buffer, one for every instantiation (a kernel
// that holds several of them allocates it once)
__shared__ float spmm_red[WAVES_PER_BLOCK][WAVE];

template <class BK, typename T, int G, bool WEIGHTED, int UNR>
__device__ __forceinline__ void b_spmm(BK bk, const SpmmArgs &a) {
  constexpr int N = V16<T>::N;
  constexpr int W = G * N;
  using A = Arith<T>;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int sub = lane % G;
  const int64_t chunk = a.chunk0 + bk.y();
  const int64_t col0 = chunk * W + sub * N;
  // Neighbour-range split of the first xunits units (the long tasks): block b
  // gathers only neighbours in range b % xsplit (workgroups go to the XCDs
  // round-robin, so each XCD's L2 serves one range) and writes a partial row
  // per task, summed in range order by k_xsplit_combine.  The other units are
  // processed whole by every block.
  const int xr = a.xsplit ? (int)(bk.x() % a.xsplit) : 0;
  // colour skipping for this chunk
  const int jb = a.chunk_jb ? a.chunk_jb[chunk] : -1;
  const uint8_t *colj = jb >= 0 ? a.colors + (int64_t)(a.j0 + jb) * a.n : nullptr;
  const uint32_t umask = jb >= 0 ? a.chunk_union[chunk] : 0xFFFFFFFFu;
  const uint32_t imask = jb >= 0 ? a.chunk_inter[chunk] : 0u;
  const T *__restrict__ M = (const T *)a.M;
  T *__restrict__ B = (T *)a.B;
  T *__restrict__ Pt = (T *)a.partial;
  bool ovf = false;
  T cmax[N];
#pragma unroll
  for (int u = 0; u < N; ++u) cmax[u] = T(0);

  for (int phase = a.xsplit ? 0 : 1; phase < 2; ++phase) {
  const bool split = phase == 0;
  const int64_t ustart = split ? bk.x() / a.xsplit : a.xunits + bk.x();
  const int64_t ustep = split ? bk.gx() / a.xsplit : bk.gx();
  const int64_t uend = split ? a.xunits : a.n_units;
  for (int64_t unit = ustart; unit < uend; unit += ustep) {
    const int rpw = a.unit_rpw[unit];
    const int lpt = WAVE / rpw;        // lanes per task
    const int tloc = lane / lpt;       // task within the wave
    const int tl = lane - tloc * lpt;  // lane within the task
    const int streams = lpt / G;
    const int stream = tl / G;
    const int gbase = tloc * lpt;      // first lane of the task's group
    const int tidx = wv * rpw + tloc;
    const bool valid = tidx < a.unit_ntask[unit];
    int64_t beg = 0, t = 0;
    int len = 0, row = 0, slot = -1;
    if (valid) {
      t = (int64_t)a.unit_task[unit] + tidx;
      row = a.task_row[t];
      beg = a.task_beg[t];
      len = a.task_len[t];
      slot = a.task_slot[t];
      if (split) {
        const uint16_t *sp = a.tsplit + t * (a.xsplit + 1);
        beg += sp[xr];
        len = sp[xr + 1] - sp[xr];
      }
      if (colj && (imask >> colj[row] & 1u)) len = 0;  // row never read here: zeros
    }
    const uint64_t gmask = (lpt == 64) ? ~0ull : (((1ull << lpt) - 1ull) << gbase);
    const uint64_t lt = (1ull << lane) - 1ull;
    V16<T> acc0, acc1;
#pragma unroll
    for (int u = 0; u < N; ++u) acc0.x[u] = acc1.x[u] = T(0);

    // neighbour indices (and colours) of the next block of lpt neighbours are
    // loaded while the current block's rows are gathered
    const uint8_t *ncol = colj ? a.nbr_col + (int64_t)jb * a.nnz + beg : nullptr;
    int nx_j = 0, nx_c = 0;
    float nx_w = 1.0f;
    if (tl < len) {
      nx_j = a.col_idx[beg + tl];
      if constexpr (WEIGHTED) nx_w = a.w[beg + tl];
      if (ncol) nx_c = ncol[tl];
    }
    for (int base = 0; base < len; base += lpt) {
      const int e = base + tl;
      int my_j = nx_j;
      float my_w = nx_w;
      const bool keep = e < len && (!ncol || ((umask >> nx_c) & 1u) != 0);
      const int en = e + lpt;
      if (en < len) {
        nx_j = a.col_idx[beg + en];
        if constexpr (WEIGHTED) nx_w = a.w[beg + en];
        if (ncol) nx_c = ncol[en];
      }
      // compact the kept neighbours to the first lanes of the task's group,
      // preserving their order (a permutation of the group's lanes)
      int cnt;
      {
        const uint64_t km = __ballot(keep) & gmask;
        const uint64_t dm = ~km & gmask;
        cnt = __popcll(km);
        const int dst = keep ? gbase + __popcll(km & lt) : gbase + cnt + __popcll(dm & lt);
        my_j = __builtin_amdgcn_ds_permute(dst << 2, my_j);
        if constexpr (WEIGHTED)
          my_w = __builtin_bit_cast(float, __builtin_amdgcn_ds_permute(dst << 2, __builtin_bit_cast(int, my_w)));
      }
      // Every lane of the task's group runs the same iterations (cnt is
      // uniform within the group), so each ds_bpermute reads an active lane;
      // slots past cnt load nothing and add zero.
      for (int t0 = 0; t0 < cnt; t0 += UNR * streams) {
        int jq[UNR];
        bool ok[UNR];
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
          const int sq = t0 + stream + q * streams;
          ok[q] = sq < cnt;
          jq[q] = shfl_i32(my_j, gbase + (ok[q] ? sq : 0));
        }
        V16<T> v[UNR];
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
          if (ok[q]) {
            v[q] = *(const V16<T> *)(M + (int64_t)jq[q] * a.ldm + col0);
          } else {
#pragma unroll
            for (int u = 0; u < N; ++u) v[q].x[u] = T(0);
          }
        }
        T wq[UNR];
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
          wq[q] = T(1);
          if constexpr (WEIGHTED) {
            const int sq = t0 + stream + q * streams;
            wq[q] = (T)shfl(my_w, gbase + (ok[q] ? sq : 0));
          }
        }
#pragma unroll
        for (int q = 0; q < UNR; q += 2) {
#pragma unroll
          for (int u = 0; u < N; ++u) {
            if constexpr (WEIGHTED) {
              acc0.x[u] = A::fma(wq[q + 0], v[q + 0].x[u], acc0.x[u], ovf);
              acc1.x[u] = A::fma(wq[q + 1], v[q + 1].x[u], acc1.x[u], ovf);
            } else {
              acc0.x[u] = A::add(acc0.x[u], v[q + 0].x[u], ovf);
              acc1.x[u] = A::add(acc1.x[u], v[q + 1].x[u], ovf);
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < N; ++u) {
      T x = A::add(acc0.x[u], acc1.x[u], ovf);
      // butterfly across the task's streams (lanes differing in bits >= log2 G)
      for (int off = G; off < lpt; off <<= 1) x = A::add(x, shfl_xor(x, off), ovf);
      acc0.x[u] = x;
    }
    if (valid && stream == 0 && split) {
      *(V16<T> *)((T *)a.partial8 + ((int64_t)xr * a.n_tasks + t) * a.ldp + (int64_t)bk.y() * W + sub * N) = acc0;
    } else if (valid && stream == 0) {
      if (slot < 0) {
        if (a.accumulate) {
          const V16<T> old = *(const V16<T> *)(B + (int64_t)row * a.ldb + col0);
#pragma unroll
          for (int u = 0; u < N; ++u) acc0.x[u] = A::add(acc0.x[u], old.x[u], ovf);
        }
        *(V16<T> *)(B + (int64_t)row * a.ldb + col0) = acc0;
#pragma unroll
        for (int u = 0; u < N; ++u)
          if (col0 + u < a.ncols_valid && acc0.x[u] > cmax[u]) cmax[u] = acc0.x[u];
      } else {
        *(V16<T> *)(Pt + (int64_t)slot * a.ldb + col0) = acc0;
      }
    }
  }
  }  // phase
  if constexpr (is_u64<T>) {
    // U64: flags only for valid columns are meaningful; padding columns may
    // hold arbitrary bits and are excluded by the caller zeroing padding.
    if (ovf) atomicOr(a.ovf, 1);
  }
  if (a.mx) {
    // lanes with equal `sub` hold the same columns
#pragma unroll
    for (int u = 0; u < N; ++u) {
      float x = (float)cmax[u];
      for (int off = G; off < WAVE; off <<= 1) x = fmaxf(x, shfl_xor(x, off));
      cmax[u] = (T)x;
    }
    for (int u = 0; u < N; ++u) {
      if (lane < G) spmm_red[wv][lane] = (float)cmax[u];
      __syncthreads();
      if (wv == 0 && lane < G) {
        float x = spmm_red[0][lane];
        for (int q = 1; q < WAVES_PER_BLOCK; ++q) x = fmaxf(x, spmm_red[q][lane]);
        const int64_t c = chunk * W + lane * N + u;
        if (c < a.ncols_valid && x > 0.f) atomicMax(a.mx + c, __float_as_uint(x));
      }
      __syncthreads();
    }
  }
}
template <typename T, int G, bool WEIGHTED, int UNR>
__global__ void __launch_bounds__(BLOCK) k_spmm(SpmmArgs a) {
  b_spmm<HwBlk, T, G, WEIGHTED, UNR>(HwBlk{}, a);
}

// Sum the xsplit partial rows of every task in range order: rows held in one
// task go to B (and the column maximum), segments of long rows to their slot
// of the long-row partial buffer.  Grid: (column vectors of the chunk group,
// groups of tasks).
template <class BK, typename T>
__device__ __forceinline__ void b_xsplit_combine(BK bk, const XsplitCombineArgs &a) {
  constexpr int N = V16<T>::N;
  using A = Arith<T>;
  const int64_t v = (int64_t)bk.x() * BLOCK + threadIdx.x;  // vector within the group
  const int64_t cl = v * N;                                       // column within the group
  if (cl >= a.ldp) return;
  const int64_t cg = a.col_first + cl;  // column of B
  const T *P = (const T *)a.partial8;
  T *B = (T *)a.B;
  T *H = (T *)a.hub;
  bool ovf = false;
  T cmax[N];
#pragma unroll
  for (int u = 0; u < N; ++u) cmax[u] = T(0);
  for (int64_t t = bk.y(); t < a.n_tasks; t += bk.gy()) {
    // the eight range partials are loaded together, then summed in range order
    V16<T> w[8];
#pragma unroll
    for (int x = 0; x < 8; ++x)
      if (x < a.xsplit) w[x] = *(const V16<T> *)(P + ((int64_t)x * a.n_tasks + t) * a.ldp + cl);
    V16<T> acc = w[0];
#pragma unroll
    for (int x = 1; x < 8; ++x) {
      if (x < a.xsplit) {
#pragma unroll
        for (int u = 0; u < N; ++u) acc.x[u] = A::add(acc.x[u], w[x].x[u], ovf);
      }
    }
    const int slot = a.task_slot[t];
    if (slot < 0) {
      T *dst = B + (int64_t)a.task_row[t] * a.ldb + cg;
      if (a.accumulate) {
        const V16<T> old = *(const V16<T> *)dst;
#pragma unroll
        for (int u = 0; u < N; ++u) acc.x[u] = A::add(acc.x[u], old.x[u], ovf);
      }
      *(V16<T> *)dst = acc;
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (cg + u < a.ncols_valid && acc.x[u] > cmax[u]) cmax[u] = acc.x[u];
    } else {
      *(V16<T> *)(H + (int64_t)slot * a.ldb + cg) = acc;
    }
  }
  if constexpr (is_u64<T>) {
    if (ovf && cg < a.ncols_valid) atomicOr(a.ovf, 1);
  }
  if (a.mx) {
#pragma unroll
    for (int u = 0; u < N; ++u)
      if (cg + u < a.ncols_valid && (float)cmax[u] > 0.f)
        atomicMax(a.mx + cg + u, __float_as_uint((float)cmax[u]));
  }
}
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_xsplit_combine(XsplitCombineArgs a) {
  b_xsplit_combine<HwBlk, T>(HwBlk{}, a);
}

// Split points of every task's neighbour list at the range boundaries
// r * ceil(n / xs), r = 0..xs (neighbour lists are sorted).
// bounds (nullable): xs + 1 range starts in vertex ids, else equal ranges of n / xs
template <class BK>
__device__ __forceinline__ void b_task_split(BK bk, const int32_t *col_idx, const int64_t *task_beg, const int32_t *task_len,
                             int64_t n_tasks, int64_t n, int xs, const int64_t *bounds,
                             uint16_t *out) {
  const int64_t span = (n + xs - 1) / xs;
  for (int64_t q = (int64_t)bk.x() * BLOCK + threadIdx.x; q < n_tasks * (xs + 1);
       q += (int64_t)bk.gx() * BLOCK) {
    const int64_t t = q / (xs + 1);
    const int r = (int)(q - t * (xs + 1));
    const int32_t *c = col_idx + task_beg[t];
    int lo = 0, hi = task_len[t];
    const int64_t bound = bounds ? bounds[r] : (int64_t)r * span;
    while (lo < hi) {  // first entry with column >= bound
      const int mid = (lo + hi) >> 1;
      if (c[mid] < bound) lo = mid + 1; else hi = mid;
    }
    out[q] = (uint16_t)lo;
  }
}
__global__ void k_task_split(const int32_t *col_idx, const int64_t *task_beg, const int32_t *task_len,
                             int64_t n_tasks, int64_t n, int xs, const int64_t *bounds,
                             uint16_t *out) {
  b_task_split(HwBlk{}, col_idx, task_beg, task_len, n_tasks, n, xs, bounds, out);
}

// Sum the partial rows of long rows in slot order, write them to B and fold
// them into the column maximum.  Grid: (column vectors, groups of rows).
template <class BK, typename T>
__device__ __forceinline__ void b_spmm_combine(BK bk, const CombineArgs &a) {
  constexpr int N = V16<T>::N;
  using A = Arith<T>;
  const int64_t vcol = (int64_t)bk.x() * BLOCK + threadIdx.x;  // vector column index
  const int64_t c0 = vcol * N;
  if (c0 >= a.ld) return;
  const T *P = (const T *)a.partial;
  T *B = (T *)a.B;
  bool ovf = false;
  T cmax[N];
#pragma unroll
  for (int u = 0; u < N; ++u) cmax[u] = T(0);
  for (int h = bk.y(); h < a.n_long; h += bk.gy()) {
    const int row = a.long_row[h];
    const int s0 = a.long_slot0[h], ns = a.long_nslot[h];
    V16<T> acc = *(const V16<T> *)(P + (int64_t)s0 * a.ld + c0);
    for (int s = 1; s < ns; ++s) {
      const V16<T> v = *(const V16<T> *)(P + (int64_t)(s0 + s) * a.ld + c0);
#pragma unroll
      for (int u = 0; u < N; ++u) acc.x[u] = A::add(acc.x[u], v.x[u], ovf);
    }
    if (a.accumulate) {
      const V16<T> old = *(const V16<T> *)(B + (int64_t)row * a.ld + c0);
#pragma unroll
      for (int u = 0; u < N; ++u) acc.x[u] = A::add(acc.x[u], old.x[u], ovf);
    }
    *(V16<T> *)(B + (int64_t)row * a.ld + c0) = acc;
#pragma unroll
    for (int u = 0; u < N; ++u)
      if (acc.x[u] > cmax[u]) cmax[u] = acc.x[u];
  }
  if constexpr (is_u64<T>) {
    if (ovf && c0 < a.ncols_valid) atomicOr(a.ovf, 1);
  }
  if (a.mx) {
#pragma unroll
    for (int u = 0; u < N; ++u)
      if (c0 + u < a.ncols_valid && (float)cmax[u] > 0.f)
        atomicMax(a.mx + c0 + u, __float_as_uint((float)cmax[u]));
  }
}
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_spmm_combine(CombineArgs a) {
  b_spmm_combine<HwBlk, T>(HwBlk{}, a);
}

// END k_spmm
// ===========================================================================
// Count combination, general split (Alg. 3 stage 2; the eMA step of Alg. 5):
//   M_s(i, C) = sum over pairs (I_a, I_p) of C of M_a(i, I_a) * B(i, I_p).
// A block stages R rows of M_a and B (one colouring, blockIdx.y) in LDS --
// scaled to a common exponent in FP32S mode -- then each thread owns output
// columns C and keeps R accumulators.  Pair indices are stored
// pair-major ([q][C]) so that a wave reads them coalesced.  Blocks walk row
// tiles with a grid stride; the running column maximum sits in LDS.

// ===========================================================================
// Row-panel SpMM with column-sorted entries (the CSC-Split layout of Alg. 6,
// Sec. 5.3): the tasks are grouped in panels of at most PANEL_TASKS
// consecutive tasks; a panel's entries are sorted by neighbour id, so entries
// that gather the same neighbour row are adjacent (one cache line request
// serves the lanes that share it) and the gathered rows are visited in
// increasing address order.  One wave owns a panel: its rows accumulate in
// the wave's own LDS rows (LDS atomics, so entries of one instruction that
// hit the same row are added in the hardware's fixed lane order; no other
// wave touches them, so results do not depend on scheduling), then go to B
// or to the long-row partial slots like k_spmm's.  One column chunk of
// W = G * N columns per blockIdx.y.

template <typename T>
__device__ inline void lds_add(T *p, T v, bool &ovf) {
  if constexpr (is_u64<T>) {
    const T old = atomicAdd((unsigned long long *)p, (unsigned long long)v);
    ovf |= old + v < old;
  } else {
    (void)ovf;
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  }
}

template <typename T, int G, bool WEIGHTED>
__global__ void __launch_bounds__(BLOCK) k_spmm_panel(SpmmPanelArgs a) {
  constexpr int N = V16<T>::N;
  constexpr int W = G * N;
  constexpr int E = WAVE / G;  // entries per wave step
  constexpr int UNR = 4;       // steps in flight
  using A = Arith<T>;
  extern __shared__ __align__(16) unsigned char panel_lds[];
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int sub = lane % G;
  const int q = lane / G;
  T *acc = (T *)panel_lds + (size_t)wv * PANEL_TASKS * W;  // [PANEL_TASKS][W]
  const int64_t chunk = a.chunk0 + blockIdx.y;
  const int64_t col0 = chunk * W + sub * N;
  const int jb = a.chunk_jb ? a.chunk_jb[chunk] : -1;
  const uint8_t *colj = jb >= 0 ? a.colors + (int64_t)(a.j0 + jb) * a.n : nullptr;
  const uint32_t umask = jb >= 0 ? a.chunk_union[chunk] : 0xFFFFFFFFu;
  const uint32_t imask = jb >= 0 ? a.chunk_inter[chunk] : 0u;
  const T *__restrict__ M = (const T *)a.M;
  T *__restrict__ B = (T *)a.B;
  T *__restrict__ Pt = (T *)a.partial;
  bool ovf = false;
  T cmax[N];
#pragma unroll
  for (int u = 0; u < N; ++u) cmax[u] = T(0);
  for (int64_t p = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wv; p < a.n_panels;
       p += (int64_t)gridDim.x * WAVES_PER_BLOCK) {
    const int t0 = a.p_task0[p];
    const int nt = a.p_ntask[p];
    for (int x = lane; x < PANEL_TASKS * W; x += WAVE) acc[x] = T(0);
    // rows whose colour is in the chunk's intersection are never read: zeros
    uint64_t dead = 0;
    if (colj) dead = __ballot(lane < nt && ((imask >> colj[a.task_row[t0 + lane]]) & 1u));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int64_t beg = a.p_beg[p], end = a.p_beg[p + 1];
    for (int64_t e0 = beg; e0 < end; e0 += (int64_t)E * UNR) {
      V16<T> v[UNR];
      int loc[UNR];
      T wq[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int64_t e = e0 + (int64_t)u * E + q;
        loc[u] = -1;
        wq[u] = T(1);
        if (e < end) {
          const int j = a.e_col[e];
          const int l = a.e_loc[e];
          if (!((dead >> l) & 1ull) && (!colj || ((umask >> colj[j]) & 1u))) {
            loc[u] = l;
            v[u] = *(const V16<T> *)(M + (int64_t)j * a.ldm + col0);
            if constexpr (WEIGHTED) wq[u] = (T)a.e_w[e];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        if (loc[u] >= 0) {
#pragma unroll
          for (int x = 0; x < N; ++x) {
            T val = v[u].x[x];
            if constexpr (WEIGHTED) val = wq[u] * val;
            lds_add(acc + loc[u] * W + sub * N + x, val, ovf);
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int r = q; r < nt; r += E) {
      V16<T> out = *(const V16<T> *)(acc + r * W + sub * N);
      const int64_t t = (int64_t)t0 + r;
      const int row = a.task_row[t];
      const int slot = a.task_slot[t];
      if (slot < 0) {
        if (a.accumulate) {
          const V16<T> old = *(const V16<T> *)(B + (int64_t)row * a.ldb + col0);
#pragma unroll
          for (int u = 0; u < N; ++u) out.x[u] = A::add(out.x[u], old.x[u], ovf);
        }
        *(V16<T> *)(B + (int64_t)row * a.ldb + col0) = out;
#pragma unroll
        for (int u = 0; u < N; ++u)
          if (col0 + u < a.ncols_valid && out.x[u] > cmax[u]) cmax[u] = out.x[u];
      } else {
        *(V16<T> *)(Pt + (int64_t)slot * a.ldb + col0) = out;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  if constexpr (is_u64<T>) {
    if (ovf) atomicOr(a.ovf, 1);
  }
  if (a.mx) {
    // each wave's first G floats of its own LDS rows carry its column maxima
    auto red = [&](int w2, int l) -> float & {
      return ((float *)(panel_lds + (size_t)w2 * PANEL_TASKS * W * sizeof(T)))[l];
    };
#pragma unroll
    for (int u = 0; u < N; ++u) {
      float x = (float)cmax[u];
      for (int off = G; off < WAVE; off <<= 1) x = fmaxf(x, shfl_xor(x, off));
      cmax[u] = (T)x;
    }
    for (int u = 0; u < N; ++u) {
      __syncthreads();
      if (lane < G) red(wv, lane) = (float)cmax[u];
      __syncthreads();
      if (wv == 0 && lane < G) {
        float x = red(0, lane);
        for (int w2 = 1; w2 < WAVES_PER_BLOCK; ++w2) x = fmaxf(x, red(w2, lane));
        const int64_t c = chunk * W + lane * N + u;
        if (c < a.ncols_valid && x > 0.f) atomicMax(a.mx + c, __float_as_uint(x));
      }
      __syncthreads();
    }
  }
}

template <class BK, typename T, int R, bool SCALED, bool STAGE>
__device__ __forceinline__ void b_ema_general(BK bk, const EmaArgs &a) {
  using A = Arith<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int j = bk.y();
  const int sa = a.Ca | 1, sb = a.Cb | 1;  // odd row strides in LDS
  T *la = (T *)smem;
  T *lb = la + (STAGE ? R * sa : 0);
  float *lmx = (float *)(lb + (STAGE ? R * sb : 0));
  const T *Ma = (const T *)a.Ma;
  const T *Bt = (const T *)a.B;
  T *Ms = (T *)a.Ms;
  const int2 *pairs = (const int2 *)a.pairs;
  const float *fa = SCALED ? a.fa + (int64_t)j * a.Ca : nullptr;
  const float *fb = SCALED ? a.fb + (int64_t)j * a.Cb : nullptr;
  bool ovf = false;
  const bool track = SCALED && a.mx != nullptr;  // else measured afterwards
  if (track)
    for (int c = threadIdx.x; c < a.Cs; c += BLOCK) lmx[c] = 0.f;
  const int64_t ntiles = (a.n + R - 1) / R;
  for (int64_t tile = bk.x(); tile < ntiles; tile += bk.gx()) {
    const int64_t r0 = tile * R;
    if constexpr (STAGE) {
      __syncthreads();
      for (int x = threadIdx.x; x < R * a.Ca; x += BLOCK) {
        const int r = x / a.Ca, c = x - r * a.Ca;
        const int64_t row = r0 + r;
        T v = T(0);
        if (row < a.n) {
          v = Ma[row * a.lda + (int64_t)j * a.Ca + c];
          if constexpr (SCALED) v *= fa[c];
        }
        la[r * sa + c] = v;
      }
      for (int x = threadIdx.x; x < R * a.Cb; x += BLOCK) {
        const int r = x / a.Cb, c = x - r * a.Cb;
        const int64_t row = r0 + r;
        T v = T(0);
        if (row < a.n) {
          v = Bt[row * a.ldb + (int64_t)j * a.Cb + c];
          if constexpr (SCALED) v *= fb[c];
        }
        lb[r * sb + c] = v;
      }
      __syncthreads();
    }
    for (int C = threadIdx.x; C < a.Cs; C += BLOCK) {
      T acc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = T(0);
      if constexpr (STAGE) {
        // eight pair indices in flight
        for (int q0 = 0; q0 < a.np; q0 += 8) {
          int2 pp[8];
#pragma unroll
          for (int qq = 0; qq < 8; ++qq) pp[qq] = pairs[(int64_t)min(q0 + qq, a.np - 1) * a.Cs + C];
#pragma unroll
          for (int qq = 0; qq < 8; ++qq) {
            if (q0 + qq >= a.np) break;  // uniform
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = A::fma(la[r * sa + pp[qq].x], lb[r * sb + pp[qq].y], acc[r], ovf);
          }
        }
      }
      for (int q = 0; q < (STAGE ? 0 : a.np); ++q) {
        const int2 p = pairs[(int64_t)q * a.Cs + C];
        {
          T sxa = T(1), sxb = T(1);
          if constexpr (SCALED) {
            sxa = fa[p.x];
            sxb = fb[p.y];
          }
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int64_t row = r0 + r;
            if (row < a.n) {
              T x = Ma[row * a.lda + (int64_t)j * a.Ca + p.x];
              T y = Bt[row * a.ldb + (int64_t)j * a.Cb + p.y];
              if constexpr (SCALED) {
                x *= sxa;
                y *= sxb;
              }
              acc[r] = A::fma(x, y, acc[r], ovf);
            }
          }
        }
      }
      float m = 0.f;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t row = r0 + r;
        if (row < a.n) {
          if (a.accumulate) acc[r] = A::add(acc[r], Ms[row * a.lds + (int64_t)j * a.Cs + C], ovf);
          Ms[row * a.lds + (int64_t)j * a.Cs + C] = acc[r];
          if constexpr (SCALED) m = fmaxf(m, (float)acc[r]);
        }
      }
      if (track) lmx[C] = fmaxf(lmx[C], m);
    }
  }
  if constexpr (is_u64<T>) {
    if (ovf) atomicOr(a.ovf, 1);
  }
  if constexpr (SCALED) {
    __syncthreads();
    for (int c = threadIdx.x; c < a.Cs; c += BLOCK) {
      if (track && lmx[c] > 0.f) atomicMax(a.mx + (int64_t)j * a.Cs + c, __float_as_uint(lmx[c]));
      if (bk.x() == 0) a.es[(int64_t)j * a.Cs + c] = a.Ea[j] + a.Eb[j];
    }
  }
}
template <typename T, int R, bool SCALED, bool STAGE>
__global__ void __launch_bounds__(BLOCK) k_ema_general(EmaArgs a) {
  b_ema_general<HwBlk, T, R, SCALED, STAGE>(HwBlk{}, a);
}

// Colour of every CSR entry's neighbour, per colouring of the pass, so that
// the SpMM reads it alongside col_idx instead of gathering it.
template <class BK>
__device__ __forceinline__ void b_nbr_colors(BK bk, const int32_t *col_idx, int64_t nnz, const uint8_t *colors,
                             int64_t n, int32_t j0, uint8_t *nbr) {
  const int jj = bk.y();
  const uint8_t *col = colors + (int64_t)(j0 + jj) * n;
  uint8_t *out = nbr + (int64_t)jj * nnz;
  for (int64_t e = (int64_t)bk.x() * BLOCK + threadIdx.x; e < nnz;
       e += (int64_t)bk.gx() * BLOCK)
    out[e] = col[col_idx[e]];
}
__global__ void k_nbr_colors(const int32_t *col_idx, int64_t nnz, const uint8_t *colors,
                             int64_t n, int32_t j0, uint8_t *nbr) {
  b_nbr_colors(HwBlk{}, col_idx, nnz, colors, n, j0, nbr);
}

// Rows grouped by colour for the colour-restricted multiply-add.
__global__ void k_bucket_count(const uint8_t *colors, int64_t n, int32_t j0, int32_t k,
                               int32_t *counts) {
  __shared__ int h[32];
  const int j = blockIdx.y;
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  const uint8_t *col = colors + (int64_t)(j0 + j) * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&h[col[i]], 1);
  __syncthreads();
  if (threadIdx.x < k && h[threadIdx.x]) atomicAdd(&counts[j * k + threadIdx.x], h[threadIdx.x]);
}

// Tiles of BLOCK * 8 rows: positions within the tile from LDS counters, one
// global reservation per colour and tile.
__global__ void __launch_bounds__(BLOCK) k_bucket_scatter(const uint8_t *colors, int64_t n, int32_t j0,
                                                         int32_t k, const int32_t *counts,
                                                         int32_t *cursor, int32_t *perm) {
  constexpr int ITEMS = 8;
  __shared__ int off[32], cnt[32], base[32];
  const int j = blockIdx.y;
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int c = 0; c < k; ++c) {
      off[c] = acc;
      acc += counts[j * k + c];
    }
  }
  const uint8_t *col = colors + (int64_t)(j0 + j) * n;
  int32_t *out = perm + (int64_t)j * n;
  for (int64_t t0 = (int64_t)blockIdx.x * BLOCK * ITEMS; t0 < n; t0 += (int64_t)gridDim.x * BLOCK * ITEMS) {
    if (threadIdx.x < 32) cnt[threadIdx.x] = 0;
    __syncthreads();
    int c[ITEMS], pos[ITEMS];
#pragma unroll
    for (int q = 0; q < ITEMS; ++q) {
      const int64_t i = t0 + (int64_t)q * BLOCK + threadIdx.x;
      c[q] = i < n ? (int)col[i] : -1;
      pos[q] = c[q] >= 0 ? atomicAdd(&cnt[c[q]], 1) : 0;
    }
    __syncthreads();
    if (threadIdx.x < k) base[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(&cursor[j * k + threadIdx.x], cnt[threadIdx.x]) : 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < ITEMS; ++q) {
      const int64_t i = t0 + (int64_t)q * BLOCK + threadIdx.x;
      if (c[q] >= 0) out[off[c[q]] + base[c[q]] + pos[q]] = (int32_t)i;
    }
    __syncthreads();  // cnt and base are reused by the next tile
  }
}

// Stage the columns idx[0..S) of R rows (row index -1: zeros) into LDS
// transposed, dst[q * RP + r] (times f[idx[q]] when SCALED), eight loads in
// flight per thread.
template <typename T, int R, bool SCALED, int NT>
__device__ inline void stage_cols(const T *__restrict__ M, int64_t ld, int64_t off, const int *rows,
                                  const int32_t *__restrict__ idx, const float *__restrict__ f, int S,
                                  T *__restrict__ dst, int RP) {
  constexpr int U = 8;
  const int total = R * S;
  for (int x0 = threadIdx.x; x0 < total; x0 += U * NT) {
    // every load is issued (indices clamped into range) before any is used
    int rr[U], q[U], col[U], row[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int x = min(x0 + u * NT, total - 1);
      rr[u] = x / S;
      q[u] = x - rr[u] * S;
      col[u] = idx[q[u]];
      row[u] = rows[rr[u]];
    }
    T v[U];
    float fv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = M[(int64_t)max(row[u], 0) * ld + off + col[u]];
      fv[u] = SCALED ? f[col[u]] : 1.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (x0 + u * NT < total) {
        T w = row[u] >= 0 ? v[u] : T(0);
        if constexpr (SCALED) w *= fv[u];
        dst[q[u] * RP + rr[u]] = w;
      }
    }
  }
}

// Colour-restricted multiply-add.  For a vertex of colour c, M_a(i, S) = 0
// unless c is in S (the active child's root is i), so M_s(i, C) = 0 for C
// without c and only pairs whose active set holds c contribute.  A block
// takes R rows of one colour (rows grouped by colour), stages the active
// columns holding c and the passive columns without c in LDS, and each thread
// owns output columns (in their natural order, so that whole lines are
// written): columns holding c from their pairs, the others 0.
template <typename T, int R, bool SCALED, int NT>
__global__ void __launch_bounds__(NT) k_ema_colour(EmaColourArgs a) {
  using A = Arith<T>;
  constexpr int N = V16<T>::N;
  // staged columns are R rows long, padded by one 16-byte vector so that
  // lanes reading different columns spread over the LDS banks
  constexpr int RP = R + N;
  static_assert(R % N == 0, "R");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int rows[R];
  const int j = blockIdx.y;
  // la holds one extra all-zero column (index Sa) that pads the pair lists
  T *la = (T *)smem;
  T *lb = la + (int64_t)RP * (a.Sa + 1);
  // FP32S column maxima of the block, kept as exponent codes: 0 for no
  // positive value, else the float's exponent field + 1 (what the frame
  // exponent needs is floor(log2 max), which the code determines exactly)
  uint8_t *lmx = (uint8_t *)(lb + (int64_t)RP * a.Sb);
  for (int r = threadIdx.x; r < RP; r += NT) la[(int64_t)a.Sa * RP + r] = T(0);
  const T *Ma = (const T *)a.Ma;
  const T *Bt = (const T *)a.B;
  T *Ms = (T *)a.Ms;
  const float *fa = SCALED ? a.fa + (int64_t)j * a.Ca : nullptr;
  const float *fb = SCALED ? a.fb + (int64_t)j * a.Cb : nullptr;
  const int32_t *cnt = a.counts + (int64_t)j * a.k;
  bool ovf = false;
  // column maxima (FP32S) unless the caller measures them afterwards (mx null)
  const bool track = SCALED && a.mx != nullptr;
  if (track)
    for (int c = threadIdx.x; c < a.Cs; c += NT) lmx[c] = 0;
  int64_t ntiles = 0;
  for (int c = 0; c < a.k; ++c) ntiles += (cnt[c] + R - 1) / R;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    // colour and first row of this tile
    int c = 0;
    int64_t acc_t = 0, off = 0;
    for (; c < a.k; ++c) {
      const int64_t tc = (cnt[c] + R - 1) / R;
      if (t < acc_t + tc) break;
      acc_t += tc;
      off += cnt[c];
    }
    const int64_t first = (t - acc_t) * R;
    const int nrow = (int)min<int64_t>(R, cnt[c] - first);
    __syncthreads();
    if (threadIdx.x < R)
      rows[threadIdx.x] = threadIdx.x < nrow ? a.perm[(int64_t)j * a.n + off + first + threadIdx.x] : -1;
    __syncthreads();
    const int32_t *ca = a.ca + (int64_t)c * a.Sa;
    const int32_t *cb = a.cb + (int64_t)c * a.Sb;
    stage_cols<T, R, SCALED, NT>(Ma, a.lda, (int64_t)j * a.Ca, rows, ca, fa, a.Sa, la, RP);
    stage_cols<T, R, SCALED, NT>(Bt, a.ldb, (int64_t)j * a.Cb, rows, cb, fb, a.Sb, lb, RP);
    __syncthreads();
    // output columns in their natural order, so that each wave writes whole
    // lines: columns holding c from their pairs, the others zero
    const uint32_t *cp = a.cp + (int64_t)c * a.Q * a.U;
    const int32_t *cu = a.cu + (int64_t)c * a.Cs;
    for (int C = threadIdx.x; C < a.Cs; C += NT) {
      const int u = cu[C];
      T acc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = T(0);
      if (u >= 0) {
        // eight pair indices in flight
        for (int q0 = 0; q0 < a.Q; q0 += 8) {
          // past the end of the list: the zero column, which adds nothing
          uint32_t p[8];
#pragma unroll
          for (int qq = 0; qq < 8; ++qq)
            p[qq] = q0 + qq < a.Q ? cp[(int64_t)(q0 + qq) * a.U + u] : (uint32_t)a.Sa;
#pragma unroll
          for (int qq = 0; qq < 8; ++qq) {
            const V16<T> *xa = (const V16<T> *)(la + (int)(p[qq] & 0xFFFFu) * RP);
            const V16<T> *yb = (const V16<T> *)(lb + (int)(p[qq] >> 16) * RP);
#pragma unroll
            for (int v = 0; v < R / N; ++v) {
              const V16<T> xv = xa[v], yv = yb[v];
#pragma unroll
              for (int e = 0; e < N; ++e) acc[v * N + e] = A::fma(xv.x[e], yv.x[e], acc[v * N + e], ovf);
            }
          }
        }
      }
      float m = 0.f;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (rows[r] >= 0) {
          Ms[(int64_t)rows[r] * a.lds + (int64_t)j * a.Cs + C] = acc[r];
          if constexpr (SCALED) m = fmaxf(m, (float)acc[r]);
        }
      }
      if (track) {
        // column C belongs to this thread in every tile
        const uint32_t code = m > 0.f ? (__float_as_uint(m) >> 23) + 1u : 0u;
        if (code > lmx[C]) lmx[C] = (uint8_t)code;
      }
    }
  }
  if constexpr (is_u64<T>) {
    if (ovf) atomicOr(a.ovf, 1);
  }
  if constexpr (SCALED) {
    __syncthreads();
    for (int c = threadIdx.x; c < a.Cs; c += NT) {
      // a float with the same floor(log2): 2^(field - 127), or the smallest
      // subnormal for a subnormal maximum
      const uint32_t code = track ? lmx[c] : 0u;
      if (code) atomicMax(a.mx + (int64_t)j * a.Cs + c, code == 1u ? 1u : (code - 1u) << 23);
      if (blockIdx.x == 0) a.es[(int64_t)j * a.Cs + c] = a.Ea[j] + a.Eb[j];
    }
  }
}

// Count combination when the active child is one vertex (Alg. 2's
// single-vertex table): M_s(i, C) = [col(i) in C] * B(i, C \ {col(i)}).
// A block takes tiles of rows with all nb colourings of the pass, threads
// over (row, colouring, column) in row-major order so that the writes are
// contiguous; eight elements' loads (colour, drop index, B entry) are in
// flight per thread.  Also the adjoint's B-bar(i, P) = M-bar(i, P + col(i))
// (drop = the plan's add table).
template <class BK, typename T, bool SCALED>
__device__ __forceinline__ void b_ema_single(BK bk, const EmaArgs &a) {
  constexpr int U = 8;
  extern __shared__ __align__(16) unsigned char smem[];
  const bool track = SCALED && a.mx != nullptr;
  const int W = a.Cs * a.nb;  // output entries per row
  const int R = max(1, (4 * U * BLOCK) / W);  // rows per tile: about four rounds of loads
  // LDS: [nb * Cs] column maxima (FP32S, when tracked), the drop table as
  // uint16 (0xFFFF: C lacks c) when kc > 0, the tile's colours [R][nb]
  unsigned *lmx = (unsigned *)smem;
  const int64_t off_drop = track ? ((int64_t)W * 4 + 15) / 16 * 16 : 0;
  uint16_t *ldrop = (uint16_t *)(smem + off_drop);
  uint8_t *lcol = smem + off_drop + (a.kc ? ((int64_t)a.kc * a.Cs * 2 + 15) / 16 * 16 : 0);
  const T *Bt = (const T *)a.B;
  T *Ms = (T *)a.Ms;
  if (track)
    for (int c = threadIdx.x; c < W; c += BLOCK) lmx[c] = 0u;
  for (int q = threadIdx.x; q < a.kc * a.Cs; q += BLOCK) {
    const int d = a.drop[q];
    ldrop[q] = d < 0 ? (uint16_t)0xFFFFu : (uint16_t)d;
  }
  __syncthreads();
  // entry e = r * W + jj * Cs + cl of a tile; a thread starts at e =
  // threadIdx.x and advances by BLOCK entries, tracked without divisions
  const int r_first = threadIdx.x / W, cc_first = threadIdx.x - r_first * W;
  const int jj_first = cc_first / a.Cs, cl_first = cc_first - jj_first * a.Cs;
  const int dr = BLOCK / W, dcc = BLOCK - dr * W;
  // offsets within a tile fit 32 bits: R * ld is about 4 * U * BLOCK * (ld / W),
  // and ld / W (input or output columns over output columns) is at most 20
  const int ldb32 = (int)a.ldb, lds32 = (int)a.lds;
  const int djj = dcc / a.Cs, dcl = dcc - djj * a.Cs;
  for (int64_t i0 = (int64_t)bk.x() * R; i0 < a.n; i0 += (int64_t)bk.gx() * R) {
    const int nrow = (int)min<int64_t>(R, a.n - i0);
    const int E = nrow * W;  // below 2^31: R * W <= 4 * U * BLOCK + W
    __syncthreads();  // previous tile's colours consumed
    for (int q = threadIdx.x; q < nrow * a.nb; q += BLOCK) {
      const int rr = q / a.nb, j = q - rr * a.nb;
      lcol[q] = a.colors[(int64_t)(a.j0 + j) * a.n + i0 + rr];
    }
    __syncthreads();
    int r = r_first, jc = jj_first, lc = cl_first;
    const T *Btile = Bt + i0 * a.ldb;
    T *Mtile = Ms + i0 * a.lds;
    for (int e0 = threadIdx.x; e0 < E; e0 += U * BLOCK) {
      int row[U];  // within the tile
      int jj[U], cl[U], cc[U], c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // entries past the tile load from its last row and store nothing
        const int rr = min(r, nrow - 1);
        row[u] = rr;
        jj[u] = jc;
        cl[u] = lc;
        cc[u] = jc * a.Cs + lc;
        c[u] = lcol[rr * a.nb + jc];
        lc += dcl;
        jc += djj;
        if (lc >= a.Cs) {
          lc -= a.Cs;
          ++jc;
        }
        r += dr;
        if (jc >= a.nb) {
          jc -= a.nb;
          ++r;
        }
      }
      int idx[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (a.kc) {
          const int d = ldrop[c[u] * a.Cs + cl[u]];
          idx[u] = d == 0xFFFF ? -1 : d;
        } else {
          idx[u] = a.drop[(int64_t)c[u] * a.Cs + cl[u]];
        }
      }
      T v[U];
      float f[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = jj[u] * a.Cb + max(idx[u], 0);
        v[u] = Btile[row[u] * ldb32 + src];
        f[u] = SCALED ? a.fb[src] : 1.0f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (e0 + u * BLOCK < E) {
          T w = idx[u] >= 0 ? v[u] : T(0);
          if constexpr (SCALED) w *= f[u];
          Mtile[row[u] * lds32 + cc[u]] = w;
          if (track && (float)w > 0.f) atomicMax(&lmx[cc[u]], __float_as_uint((float)w));
        }
      }
    }
  }
  if constexpr (SCALED) {
    __syncthreads();
    for (int c = threadIdx.x; c < W; c += BLOCK) {
      if (track && lmx[c]) atomicMax(a.mx + c, lmx[c]);
      if (bk.x() == 0) a.es[c] = a.Eb[c / a.Cs];
    }
  }
}
template <typename T, bool SCALED>
__global__ void __launch_bounds__(BLOCK) k_ema_single(EmaArgs a) {
  b_ema_single<HwBlk, T, SCALED>(HwBlk{}, a);
}

// FP32S column maxima of a single-vertex-active split, bounded without a pass
// over the output: M_s(i, C) = B(i, C \ c) f_B(C \ c) for the vertices of a
// colour c in C, so max_i M_s(i, C) <= max over c in C of mx_B(C \ c) f_B(C \ c)
// (an upper bound suffices for the frame exponent).  One thread per
// (colouring, output column).
template <class BK>
__device__ __forceinline__ void b_single_bound(BK bk, const int32_t *drop, int k, int Cs, int Cb, int b, const unsigned *mxB,
                               const float *fb, unsigned *mx) {
  const int64_t q = (int64_t)bk.x() * BLOCK + threadIdx.x;
  if (q >= (int64_t)b * Cs) return;
  const int jj = (int)(q / Cs), C = (int)(q - (int64_t)jj * Cs);
  float m = 0.f;
  for (int c = 0; c < k; ++c) {
    const int d = drop[(int64_t)c * Cs + C];
    if (d >= 0) m = fmaxf(m, __uint_as_float(mxB[(int64_t)jj * Cb + d]) * fb[(int64_t)jj * Cb + d]);
  }
  mx[q] = __float_as_uint(m);
}
__global__ void k_single_bound(const int32_t *drop, int k, int Cs, int Cb, int b, const unsigned *mxB,
                               const float *fb, unsigned *mx) {
  b_single_bound(HwBlk{}, drop, k, Cs, Cb, b, mxB, fb, mx);
}

// ===========================================================================
// Root reduction (Alg. 1: sum_i sum_C M_0(i, I_C)).  For a vertex of colour c
// the row sum of M_0 equals sum over list[c] of X(i, x) * Y(i, y), where the
// list comes from the root split (see the planner).  One wave per row; lanes
// stride over the list; the row value is reduced in the table type (FP32
// mantissas in FP32S) and accumulated over rows in double (uint64 in U64).
// Per-block partials are summed in block order by k_root_final.

template <class BK, typename T, bool SCALED, bool HASY>
__device__ __forceinline__ void b_root(BK bk, const RootArgs &a) {
  using A = Arith<T>;
  using Acc = typename std::conditional<is_u64<T>, uint64_t, double>::type;
  __shared__ Acc red[WAVES_PER_BLOCK];
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int j = bk.y();
  const uint8_t *col = a.colors + (int64_t)(a.j0 + j) * a.n;
  const T *X = (const T *)a.X;
  const T *Y = (const T *)a.Y;
  const float *fx = SCALED ? a.fx + (int64_t)j * a.Cx : nullptr;
  const float *fy = (SCALED && HASY) ? a.fy + (int64_t)j * a.Cy : nullptr;
  const int2 *list = (const int2 *)a.list;
  bool ovf = false;
  Acc tot = Acc(0);
  const int64_t wave = (int64_t)bk.x() * WAVES_PER_BLOCK + wv;
  const int64_t nwaves = (int64_t)bk.gx() * WAVES_PER_BLOCK;
  for (int64_t i = wave; i < a.n; i += nwaves) {
    const int c = col[i];
    const int2 *lc = list + (int64_t)c * a.L;
    const T *xr = X + i * a.ldx + (int64_t)j * a.Cx;
    const T *yr = HASY ? Y + i * a.ldy + (int64_t)j * a.Cy : nullptr;
    T s = T(0);
    for (int64_t q = lane; q < a.L; q += WAVE) {
      const int2 p = lc[q];
      T x = xr[p.x];
      if constexpr (SCALED) x *= fx[p.x];
      if constexpr (HASY) {
        T y = yr[p.y];
        if constexpr (SCALED) y *= fy[p.y];
        s = A::fma(x, y, s, ovf);
      } else {
        s = A::add(s, x, ovf);
      }
    }
    for (int off = 1; off < WAVE; off <<= 1) s = A::add(s, shfl_xor(s, off), ovf);
    if constexpr (is_u64<Acc>) {
      tot = A::add(tot, s, ovf);
    } else {
      tot += (double)s;
    }
  }
  if (lane == 0) red[wv] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    Acc b = red[0];
    for (int q = 1; q < WAVES_PER_BLOCK; ++q) {
      if constexpr (is_u64<Acc>) b = A::add(b, red[q], ovf);
      else b += red[q];
    }
    ((Acc *)a.partial)[(int64_t)j * bk.gx() + bk.x()] = b;
  }
  if constexpr (is_u64<T>) {
    if (ovf) atomicOr(a.ovf, 1);
  }
}
template <typename T, bool SCALED, bool HASY>
__global__ void __launch_bounds__(BLOCK) k_root(RootArgs a) {
  b_root<HwBlk, T, SCALED, HASY>(HwBlk{}, a);
}

// Root reduction with the vertex's rows staged in LDS (multiplied by the
// column factors in FP32S): one block per row at a time, threads stride over
// the colour's list, a fixed-order reduction gives the row value, which is
// accumulated over the block's rows in double (uint64 in U64).
template <class BK, typename T, bool SCALED, bool HASY>
__device__ __forceinline__ void b_root_lds(BK bk, const RootArgs &a) {
  using A = Arith<T>;
  using Acc = typename std::conditional<is_u64<T>, uint64_t, double>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ T red[WAVES_PER_BLOCK];
  T *lx = (T *)smem;
  T *ly = (HASY && !a.same_xy) ? lx + a.Cx : lx;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int j = bk.y();
  const uint8_t *col = a.colors + (int64_t)(a.j0 + j) * a.n;
  const T *X = (const T *)a.X;
  const T *Y = (const T *)a.Y;
  const float *fx = SCALED ? a.fx + (int64_t)j * a.Cx : nullptr;
  const float *fy = (SCALED && HASY) ? a.fy + (int64_t)j * a.Cy : nullptr;
  bool ovf = false;
  Acc tot = Acc(0);
  for (int64_t i = bk.x(); i < a.n; i += bk.gx()) {
    __syncthreads();
    const T *xr = X + i * a.ldx + (int64_t)j * a.Cx;
    for (int c = threadIdx.x; c < a.Cx; c += BLOCK) {
      T v = xr[c];
      if constexpr (SCALED) v *= fx[c];
      lx[c] = v;
    }
    if (HASY && !a.same_xy) {
      const T *yr = Y + i * a.ldy + (int64_t)j * a.Cy;
      for (int c = threadIdx.x; c < a.Cy; c += BLOCK) {
        T v = yr[c];
        if constexpr (SCALED) v *= fy[c];
        ly[c] = v;
      }
    }
    __syncthreads();
    const int c = col[i];
    const uint32_t *lc = a.list16 + (int64_t)c * a.L;
    T s = T(0);
    // eight list entries in flight per thread
    for (int64_t q0 = threadIdx.x; q0 < a.L; q0 += 8 * BLOCK) {
      uint32_t p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) p[u] = lc[min<int64_t>(q0 + u * BLOCK, a.L - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (q0 + u * BLOCK < a.L) {
          if constexpr (HASY) s = A::fma(lx[p[u] & 0xFFFFu], ly[p[u] >> 16], s, ovf);
          else s = A::add(s, lx[p[u] & 0xFFFFu], ovf);
        }
      }
    }
    for (int off = 1; off < WAVE; off <<= 1) s = A::add(s, shfl_xor(s, off), ovf);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      T r = red[0];
      for (int q = 1; q < WAVES_PER_BLOCK; ++q) r = A::add(r, red[q], ovf);
      if constexpr (is_u64<Acc>) tot = A::add(tot, r, ovf);
      else tot += (double)r;
    }
  }
  if (threadIdx.x == 0) ((Acc *)a.partial)[(int64_t)j * bk.gx() + bk.x()] = tot;
  if constexpr (is_u64<T>) {
    if (ovf) atomicOr(a.ovf, 1);
  }
}
template <typename T, bool SCALED, bool HASY>
__global__ void __launch_bounds__(BLOCK) k_root_lds(RootArgs a) {
  b_root_lds<HwBlk, T, SCALED, HASY>(HwBlk{}, a);
}

// Root reduction, colour by colour: block b takes the contiguous vertex
// range [b n / gridDim.x, (b + 1) n / gridDim.x) and, for each colour c in
// turn, lists the range's vertices of colour c (in vertex order) and walks
// them with c's (x, y) list held in registers (LPT entries per thread).
// Rows (one table: Y is X or absent) are staged in LDS double-buffered with
// 16-byte loads: the next row's loads are in flight while the current row
// is summed; the column factors stay in registers.  Each thread accumulates
// its share of every vertex's terms (summed per vertex in T) in double
// (uint64 in U64); the block then reduces its threads in a fixed order.
// Needs Cx <= PV * N * BLOCK, L <= LPT * BLOCK and 16-byte aligned rows.
template <typename T, bool SCALED, bool HASY, int LPT, int PV, bool DB>
__global__ void __launch_bounds__(BLOCK) k_root_tile(RootArgs a) {
  using A = Arith<T>;
  using Acc = typename std::conditional<is_u64<T>, uint64_t, double>::type;
  constexpr int N = V16<T>::N;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int rowlist[BLOCK];
  __shared__ int wcount[WAVES_PER_BLOCK];
  __shared__ Acc red[WAVES_PER_BLOCK];
  const int nvec = (a.Cx + N - 1) / N;
  T *lx0 = (T *)smem;
  T *lx1 = DB ? lx0 + (int64_t)nvec * N : lx0;  // single buffer: fetch after the sum
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int j = blockIdx.y;
  const uint8_t *col = a.colors + (int64_t)(a.j0 + j) * a.n;
  const T *X = (const T *)a.X;
  const int64_t r0 = (int64_t)blockIdx.x * a.n / gridDim.x;
  const int64_t r1 = (int64_t)(blockIdx.x + 1) * a.n / gridDim.x;
  bool ovf = false;
  Acc tot = Acc(0);
  // column factors of this thread's vectors
  float f[PV][N];
#pragma unroll
  for (int u = 0; u < PV; ++u) {
#pragma unroll
    for (int e = 0; e < N; ++e) {
      const int c = (threadIdx.x + u * BLOCK) * N + e;
      f[u][e] = 1.0f;
      if constexpr (SCALED) f[u][e] = c < a.Cx ? a.fx[(int64_t)j * a.Cx + c] : 0.0f;
    }
  }
  V16<T> v[PV];
  auto fetch = [&](int64_t i) {
    const V16<T> *xr = (const V16<T> *)(X + i * a.ldx + (int64_t)j * a.Cx);
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int q = threadIdx.x + u * BLOCK;
      if (q < nvec) v[u] = xr[q];
    }
  };
  auto store = [&](T *lx) {
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int q = threadIdx.x + u * BLOCK;
      if (q < nvec) {
        V16<T> w = v[u];
        if constexpr (SCALED) {
#pragma unroll
          for (int e = 0; e < N; ++e) w.x[e] *= f[u][e];
        }
        ((V16<T> *)lx)[q] = w;
      }
    }
  };
  for (int c = 0; c < a.k; ++c) {
    // this colour's (x, y) pairs, LPT per thread
    const uint32_t *lc = a.list16 + (int64_t)c * a.L;
    uint32_t p[LPT];
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int64_t q = threadIdx.x + (int64_t)u * BLOCK;
      p[u] = q < a.L ? lc[q] : 0u;
    }
    for (int64_t base = r0; base < r1; base += BLOCK) {
      // the chunk's vertices of colour c, in vertex order
      const int64_t i = base + threadIdx.x;
      const bool hit = i < r1 && col[i] == c;
      const uint64_t m = __ballot(hit);
      __syncthreads();  // rowlist and the row buffers are free again
      if (lane == 0) wcount[wv] = __popcll(m);
      __syncthreads();
      int pos = __popcll(m & ((1ull << lane) - 1ull)), cnt = 0;
      for (int w = 0; w < WAVES_PER_BLOCK; ++w) {
        if (w < wv) pos += wcount[w];
        cnt += wcount[w];
      }
      if (hit) rowlist[pos] = (int)i;
      __syncthreads();
      if (cnt == 0) continue;
      fetch(rowlist[0]);
      for (int t = 0; t < cnt; ++t) {
        T *lx = (t & 1) ? lx1 : lx0;
        store(lx);
        __syncthreads();
        if (DB && t + 1 < cnt) fetch(rowlist[t + 1]);  // in flight during the sum
        T s = T(0);
#pragma unroll
        for (int u = 0; u < LPT; ++u) {
          if (threadIdx.x + u * BLOCK < a.L) {
            if constexpr (HASY) s = A::fma(lx[p[u] & 0xFFFFu], lx[p[u] >> 16], s, ovf);
            else s = A::add(s, lx[p[u] & 0xFFFFu], ovf);
          }
        }
        if constexpr (is_u64<Acc>) tot = A::add(tot, s, ovf);
        else tot += (double)s;
        if (!DB) {
          __syncthreads();  // the buffer is free for the next row
          if (t + 1 < cnt) fetch(rowlist[t + 1]);
        }
      }
    }
  }
  // fixed-order block reduction
  for (int off = 1; off < WAVE; off <<= 1) {
    if constexpr (is_u64<Acc>) tot = A::add(tot, shfl_xor(tot, off), ovf);
    else tot += shfl_xor(tot, off);
  }
  __syncthreads();
  if (lane == 0) red[wv] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    Acc b = red[0];
    for (int q = 1; q < WAVES_PER_BLOCK; ++q) {
      if constexpr (is_u64<Acc>) b = A::add(b, red[q], ovf);
      else b += red[q];
    }
    ((Acc *)a.partial)[(int64_t)j * gridDim.x + blockIdx.x] = b;
  }
  if constexpr (is_u64<T>) {
    if (ovf) atomicOr(a.ovf, 1);
  }
}

// Root reduction for narrow tables and short lists: one thread per vertex
// (grid stride), every colour's (x, y) list staged in LDS, row entries read
// directly (they share a few cache lines).  Each thread accumulates its
// vertices in double (uint64 in U64); fixed-order block reduction.
template <typename T, bool SCALED, bool HASY>
__global__ void __launch_bounds__(BLOCK) k_root_thread(RootArgs a) {
  using A = Arith<T>;
  using Acc = typename std::conditional<is_u64<T>, uint64_t, double>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Acc red[WAVES_PER_BLOCK];
  uint32_t *lists = (uint32_t *)smem;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int j = blockIdx.y;
  for (int64_t q = threadIdx.x; q < (int64_t)a.k * a.L; q += BLOCK) lists[q] = a.list16[q];
  __syncthreads();
  const uint8_t *col = a.colors + (int64_t)(a.j0 + j) * a.n;
  const T *X = (const T *)a.X;
  const T *Y = (const T *)a.Y;
  const float *fx = SCALED ? a.fx + (int64_t)j * a.Cx : nullptr;
  const float *fy = (SCALED && HASY) ? a.fy + (int64_t)j * a.Cy : nullptr;
  bool ovf = false;
  Acc tot = Acc(0);
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * BLOCK) {
    const uint32_t *lc = lists + (int64_t)col[i] * a.L;
    const T *xr = X + i * a.ldx + (int64_t)j * a.Cx;
    const T *yr = HASY ? Y + i * a.ldy + (int64_t)j * a.Cy : nullptr;
    T s = T(0);
    for (int q = 0; q < a.L; ++q) {
      const uint32_t p = lc[q];
      T x = xr[p & 0xFFFFu];
      if constexpr (SCALED) x *= fx[p & 0xFFFFu];
      if constexpr (HASY) {
        T y = yr[p >> 16];
        if constexpr (SCALED) y *= fy[p >> 16];
        s = A::fma(x, y, s, ovf);
      } else {
        s = A::add(s, x, ovf);
      }
    }
    if constexpr (is_u64<Acc>) tot = A::add(tot, s, ovf);
    else tot += (double)s;
  }
  for (int off = 1; off < WAVE; off <<= 1) {
    if constexpr (is_u64<Acc>) tot = A::add(tot, shfl_xor(tot, off), ovf);
    else tot += shfl_xor(tot, off);
  }
  if (lane == 0) red[wv] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    Acc b = red[0];
    for (int q = 1; q < WAVES_PER_BLOCK; ++q) {
      if constexpr (is_u64<Acc>) b = A::add(b, red[q], ovf);
      else b += red[q];
    }
    ((Acc *)a.partial)[(int64_t)j * gridDim.x + blockIdx.x] = b;
  }
  if constexpr (is_u64<T>) {
    if (ovf) atomicOr(a.ovf, 1);
  }
}

// Root sum for narrow tables (same list as k_root_thread): per tile, R
// vertex rows of X and Y for colouring blockIdx.y are staged in LDS with
// consecutive lanes on consecutive columns (coalesced; rows are padded to
// cpw = 2^lg columns in the lane mapping only), then BLOCK / R lanes per
// vertex walk its colour's list from LDS.
// LDS: k * L list words, then R * Cx (and R * Cy) elements of T.
template <typename T, bool SCALED, bool HASY>
__global__ void __launch_bounds__(BLOCK) k_root_stage(RootArgs a, int R, int lgx, int lgy) {
  using A = Arith<T>;
  using Acc = typename std::conditional<is_u64<T>, uint64_t, double>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Acc red[WAVES_PER_BLOCK];
  uint32_t *lists = (uint32_t *)smem;
  const int64_t kl = (int64_t)a.k * a.L;
  T *xs = (T *)(smem + ((kl * 4 + 15) & ~(int64_t)15));
  T *ys = xs + (int64_t)R * a.Cx;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int j = blockIdx.y;
  for (int64_t q = threadIdx.x; q < kl; q += BLOCK) lists[q] = a.list16[q];
  const uint8_t *col = a.colors + (int64_t)(a.j0 + j) * a.n;
  const T *X = (const T *)a.X + (int64_t)j * a.Cx;
  const T *Y = HASY ? (const T *)a.Y + (int64_t)j * a.Cy : nullptr;
  const float *fx = SCALED ? a.fx + (int64_t)j * a.Cx : nullptr;
  const float *fy = (SCALED && HASY) ? a.fy + (int64_t)j * a.Cy : nullptr;
  const int lpv = BLOCK / R;  // lanes per vertex
  const int r = threadIdx.x / lpv, l = threadIdx.x - r * lpv;
  bool ovf = false;
  Acc tot = Acc(0);
  for (int64_t i0 = (int64_t)blockIdx.x * R; i0 < a.n; i0 += (int64_t)gridDim.x * R) {
    const int rows = (int)((a.n - i0) < R ? (a.n - i0) : R);
    __syncthreads();  // lists loaded / previous tile consumed
    // X slots [0, nx), then Y slots [nx, nx + ny): eight loads in flight per lane
    const int nx = rows << lgx, ny = HASY ? rows << lgy : 0;
    for (int q0 = threadIdx.x; q0 < nx + ny; q0 += 8 * BLOCK) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * BLOCK;
        v[u] = T(0);
        if (q < nx) {
          const int rr = q >> lgx, c = q & ((1 << lgx) - 1);
          if (c < a.Cx) v[u] = X[(i0 + rr) * a.ldx + c];
        } else if (HASY && q < nx + ny) {
          const int rr = (q - nx) >> lgy, c = (q - nx) & ((1 << lgy) - 1);
          if (c < a.Cy) v[u] = Y[(i0 + rr) * a.ldy + c];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * BLOCK;
        if (q < nx) {
          const int rr = q >> lgx, c = q & ((1 << lgx) - 1);
          if (c < a.Cx) {
            T x = v[u];
            if constexpr (SCALED) x *= fx[c];
            xs[rr * a.Cx + c] = x;
          }
        } else if (HASY && q < nx + ny) {
          const int rr = (q - nx) >> lgy, c = (q - nx) & ((1 << lgy) - 1);
          if (c < a.Cy) {
            T y = v[u];
            if constexpr (SCALED) y *= fy[c];
            ys[rr * a.Cy + c] = y;
          }
        }
      }
    }
    __syncthreads();
    if (r < rows) {
      const uint32_t *lc = lists + (int64_t)col[i0 + r] * a.L;
      const T *xr = xs + r * a.Cx;
      const T *yr = ys + r * a.Cy;
      T s = T(0);
      for (int q = l; q < a.L; q += lpv) {
        const uint32_t p = lc[q];
        if constexpr (HASY) s = A::fma(xr[p & 0xFFFFu], yr[p >> 16], s, ovf);
        else s = A::add(s, xr[p & 0xFFFFu], ovf);
      }
      if constexpr (is_u64<Acc>) tot = A::add(tot, s, ovf);
      else tot += (double)s;
    }
  }
  for (int off = 1; off < WAVE; off <<= 1) {
    if constexpr (is_u64<Acc>) tot = A::add(tot, shfl_xor(tot, off), ovf);
    else tot += shfl_xor(tot, off);
  }
  if (lane == 0) red[wv] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    Acc b = red[0];
    for (int q = 1; q < WAVES_PER_BLOCK; ++q) {
      if constexpr (is_u64<Acc>) b = A::add(b, red[q], ovf);
      else b += red[q];
    }
    ((Acc *)a.partial)[(int64_t)j * gridDim.x + blockIdx.x] = b;
  }
  if constexpr (is_u64<T>) {
    if (ovf) atomicOr(a.ovf, 1);
  }
}

template <class BK, typename Acc>
__device__ __forceinline__ void b_root_final(BK bk, const Acc *partial, int nblk, int b, Acc *out, int *ovf) {
  // one 64-lane wave per colouring: lane l sums the partials l, l + 64, ...
  // in order, then a fixed butterfly (the result does not depend on timing)
  const int j = bk.x();
  if (j >= b) return;
  const int lane = threadIdx.x;
  const Acc *pj = partial + (int64_t)j * nblk;
  Acc s = Acc(0);
  bool o = false;
  for (int q = lane; q < nblk; q += 64) {
    if constexpr (std::is_same<Acc, double>::value) s += pj[q];
    else s = Arith<uint64_t>::add(s, pj[q], o);
  }
  for (int off = 1; off < 64; off <<= 1) {
    if constexpr (std::is_same<Acc, double>::value) s += shfl_xor(s, off);
    else s = Arith<uint64_t>::add(s, shfl_xor(s, off), o);
  }
  if (lane == 0) {
    out[j] = s;
    if (o) atomicOr(ovf, 1);
  }
}
template <typename Acc>
__global__ void k_root_final(const Acc *partial, int nblk, int b, Acc *out, int *ovf) {
  b_root_final<HwBlk, Acc>(HwBlk{}, partial, nblk, b, out, ovf);
}

// Column maxima of an FP32S table (float bits, atomicMax), for producers too
// wide to keep them in LDS.  Grid: (column vectors, row groups).
template <class BK>
__device__ __forceinline__ void b_colmax(BK bk, const float *X, int64_t n, int64_t ld, int64_t cols,
                                                   unsigned *mx) {
  const int64_t c = (int64_t)bk.x() * BLOCK + threadIdx.x;
  if (c >= cols) return;
  const int64_t r0 = (int64_t)bk.y() * n / bk.gy(), r1 = (int64_t)(bk.y() + 1) * n / bk.gy();
  float m = 0.f;
  for (int64_t i = r0; i < r1; ++i) m = fmaxf(m, X[i * ld + c]);
  if (m > 0.f) atomicMax(mx + c, __float_as_uint(m));
}
__global__ void __launch_bounds__(BLOCK) k_colmax(const float *X, int64_t n, int64_t ld, int64_t cols,
                                                   unsigned *mx) {
  b_colmax(HwBlk{}, X, n, ld, cols, mx);
}

// ===========================================================================
// FP32S bookkeeping.  For every colouring j of a table X with per-column
// exponents e and column maxima mx (float bits):
//   E[j] = max_c (e[c] + floor(log2 mx[c])) + 1   over columns with mx > 0
//   f[c] = 2^(e[c] - E[j])                          (exact power of two)
// so that consumers read X(i, c) * f[c] <= 1 in the common frame 2^E[j].

template <class BK>
__device__ __forceinline__ void b_norm_prep(BK bk, const int *e, const unsigned *mx, int C, float *f, int *E) {
  const int j = bk.x();
  __shared__ int red[BLOCK];
  int best = INT_MIN;
  for (int c = threadIdx.x; c < C; c += BLOCK) {
    const unsigned m = mx[(int64_t)j * C + c];
    if (m != 0u) best = max(best, e[(int64_t)j * C + c] + ilog2_bits(m));
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const int Ej = red[0] == INT_MIN ? 0 : red[0] + 1;
  for (int c = threadIdx.x; c < C; c += BLOCK) {
    const unsigned m = mx[(int64_t)j * C + c];
    f[(int64_t)j * C + c] = m ? exp2_int(e[(int64_t)j * C + c] - Ej) : 0.f;
  }
  if (threadIdx.x == 0) E[j] = Ej;
}
__global__ void k_norm_prep(const int *e, const unsigned *mx, int C, float *f, int *E) {
  b_norm_prep(HwBlk{}, e, mx, C, f, E);
}

template <class BK>
__device__ __forceinline__ void b_root_exp(BK bk, const int *EX, const int *EY, int *out, int b) {
  const int j = bk.x() * 64 + threadIdx.x;
  if (j < b) out[j] = EX[j] + (EY ? EY[j] : 0);
}
__global__ void k_root_exp(const int *EX, const int *EY, int *out, int b) {
  b_root_exp(HwBlk{}, EX, EY, out, b);
}

template <class BK>
__device__ __forceinline__ void b_fill_u32(BK bk, unsigned *p, int64_t n, unsigned v) {
  for (int64_t x = (int64_t)bk.x() * BLOCK + threadIdx.x; x < n;
       x += (int64_t)bk.gx() * BLOCK)
    p[x] = v;
}
__global__ void k_fill_u32(unsigned *p, int64_t n, unsigned v) {
  b_fill_u32(HwBlk{}, p, n, v);
}

template <class BK>
__device__ __forceinline__ void b_copy_i32(BK bk, const int *src, int *dst, int64_t n) {
  for (int64_t x = (int64_t)bk.x() * BLOCK + threadIdx.x; x < n;
       x += (int64_t)bk.gx() * BLOCK)
    dst[x] = src[x];
}
__global__ void k_copy_i32(const int *src, int *dst, int64_t n) {
  b_copy_i32(HwBlk{}, src, dst, n);
}

// zero the padding columns [c_from, ld) of a row-major table
template <class BK, typename T>
__device__ __forceinline__ void b_zero_pad(BK bk, T *X, int64_t n, int64_t ld, int64_t c_from) {
  const int64_t w = ld - c_from;
  for (int64_t x = (int64_t)bk.x() * BLOCK + threadIdx.x; x < n * w;
       x += (int64_t)bk.gx() * BLOCK) {
    const int64_t i = x / w, c = c_from + (x - i * w);
    X[i * ld + c] = T(0);
  }
}
template <typename T>
__global__ void k_zero_pad(T *X, int64_t n, int64_t ld, int64_t c_from) {
  b_zero_pad<HwBlk, T>(HwBlk{}, X, n, ld, c_from);
}

// ===========================================================================
// Edge gradient of the neighbour aggregation (the adjoint of B = A_G M_p with
// respect to the CSR weights): grad[e] += sum_c Bbar(i, c) M_p(j, c) for
// e = (i -> j).  One wave per row, four neighbours at a time with 16 lanes
// each; every entry is owned by one lane, so no atomics.  With a one-vertex
// passive child M_p(j, .) is the colour indicator and the sum is
// sum_jj Bbar(i, jj*k + colour_jj(j)).

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_sddmm(SddmmArgs a) {
  using A = Arith<T>;
  const int lane = threadIdx.x & (WAVE - 1);
  const int grp = lane >> 4, sub = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE;
  const int64_t nwaves = (int64_t)gridDim.x * WAVES_PER_BLOCK;
  const T *Bb = (const T *)a.Bbar;
  const T *M = (const T *)a.Mp;
  bool ovf = false;
  for (int64_t i = wave; i < a.n; i += nwaves) {
    const int64_t beg = a.row_ptr[i], end = a.row_ptr[i + 1];
    const T *brow = Bb + i * a.ldb;
    for (int64_t e0 = beg; e0 < end; e0 += 4) {
      const int64_t e = e0 + grp;
      T s = T(0);
      if (e < end) {
        const int64_t j = a.col_idx[e];
        if (M) {
          const T *mrow = M + j * a.ldm;
          if (a.fm) {  // FP32S: the passive table's column factors
            for (int64_t c = sub; c < a.ncols; c += 16) s = A::fma(brow[c], mrow[c] * (T)a.fm[c], s, ovf);
          } else {
            for (int64_t c = sub; c < a.ncols; c += 16) s = A::fma(brow[c], mrow[c], s, ovf);
          }
        } else {
          for (int jj = sub; jj < a.b; jj += 16)
            s = A::add(s, brow[(int64_t)jj * a.k + a.colors[(int64_t)(a.j0 + jj) * a.n + j]], ovf);
        }
      }
      for (int off = 1; off < 16; off <<= 1) s = A::add(s, shfl_xor(s, off), ovf);
      if (e < end && sub == 0) a.grad[e] += a.scale * (double)s;
    }
  }
}

// Y = Y * so + X * sn over n rows of `cols` columns (FP32S adjoint: a
// contribution added to a table after both are brought to a common exponent)
__global__ void k_scale_add(float *Y, int64_t ldy, const float *X, int64_t ldx, int64_t n, int64_t cols,
                            float so, float sn) {
  const int64_t total = n * cols;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q / cols, c = q - i * cols;
    Y[i * ldy + c] = Y[i * ldy + c] * so + X[i * ldx + c] * sn;
  }
}

template <class BK, typename T>
__device__ __forceinline__ void b_fill_value(BK bk, T *X, int64_t count, T v) {
  for (int64_t x = (int64_t)bk.x() * BLOCK + threadIdx.x; x < count;
       x += (int64_t)bk.gx() * BLOCK)
    X[x] = v;
}
template <typename T>
__global__ void k_fill_value(T *X, int64_t count, T v) {
  b_fill_value<HwBlk, T>(HwBlk{}, X, count, v);
}

// ===========================================================================
// Persistent schedule: one kernel runs the recorded launches of several
// independent chains (the templates of a batch).  Every virtual block of a
// recorded launch is a task; each chain numbers its tasks in launch order.
// A block of k_persist looks for a chain whose next task can start (its
// launch's predecessor has completed), else any chain with tasks left, takes
// that chain's next ticket, waits if needed (thread 0, bounded by a
// wall-clock limit) until the predecessor of the ticket's launch has
// completed all of its tasks, runs the launch's kernel body with the virtual
// block coordinates, and counts the task as done.  Within a chain every
// predecessor launch has smaller tickets, a block holds one ticket at a time
// and a ticket is only taken by a running block, so every wait ends (by
// induction over each chain's tickets) whatever the number of resident
// blocks.  Ordering across the XCDs: after a task every wave waits for its
// stores, then one agent-scope release (L2 write-back) precedes the done
// counter's increment; a block that starts a launch whose predecessor it
// has not yet seen complete waits for it, then acquires at agent scope (L1
// and L2 invalidate) before any of its threads reads; a block remembers per
// chain the latest predecessor it has seen complete, so it waits and
// acquires once per launch boundary.

// argument blocks of the launchers with scalar parameters
struct ColorPA {
  uint8_t *out;
  int64_t n;
  int32_t k, first, count, pad;
  uint64_t seed;
  const int32_t *orig;
};
struct FillPA {
  unsigned *p;
  int64_t n;
  unsigned v;
};
struct CopyPA {
  const int *src;
  int *dst;
  int64_t n;
};
struct NbrColPA {
  const int32_t *col_idx;
  int64_t nnz;
  const uint8_t *colors;
  int64_t n;
  int32_t j0;
  uint8_t *nbr;
};
struct ColmaxPA {
  const float *X;
  int64_t n, ld, cols;
  unsigned *mx;
};
struct NormPrepPA {
  const int *e;
  const unsigned *mx;
  int C;
  float *f;
  int *E;
};
struct RootExpPA {
  const int *EX, *EY;
  int *out;
  int b;
};
struct SingleBoundPA {
  const int32_t *drop;
  int k, Cs, Cb, b;
  const unsigned *mxB;
  const float *fb;
  unsigned *mx;
};
struct TaskSplitPA {
  const int32_t *col_idx;
  const int64_t *task_beg;
  const int32_t *task_len;
  int64_t n_tasks, n;
  int xs;
  const int64_t *bounds;
  uint16_t *out;
};
struct RootFinalPA {
  const void *partial;
  int nblk, b;
  void *out;
  int *ovf;
};
struct ZeroPadPA {
  void *X;
  int64_t n, ld, c_from;
};

enum PBody : int32_t {
  PB_COLOR = 0,
  PB_FILL_U32,
  PB_COPY_I32,
  PB_NBR_COLORS,
  PB_COLMAX,
  PB_NORM_PREP,
  PB_ROOT_EXP,
  PB_SINGLE_BOUND,
  PB_TASK_SPLIT,
  PB_XSPLIT_COMBINE,
  PB_SPMM_COMBINE,
  PB_EMA_SINGLE,
  PB_ROOT_FINAL,
  PB_ZERO_PAD,
  PB_HIST,                           // + 2 * weighted + (b > 1)
  PB_ROOT = PB_HIST + 4,             // + (Y present)
  PB_ROOT_LDS = PB_ROOT + 2,         // + (Y present)
  PB_EMA_GENERAL = PB_ROOT_LDS + 2,  // + 2 * log2(R) + staged
  PB_SPMM = PB_EMA_GENERAL + 10,     // + 4 * log2(G / 2) + 2 * weighted + (8 gathers in flight)
  PB_COUNT = PB_SPMM + 20
};

#define P_EMA(ri, R)                                                                   \
  case PB_EMA_GENERAL + 2 * ri:                                                        \
    b_ema_general<VBlk, T, R, SC, false>(bk, *(const EmaArgs *)A);                     \
    break;                                                                             \
  case PB_EMA_GENERAL + 2 * ri + 1:                                                    \
    b_ema_general<VBlk, T, R, SC, true>(bk, *(const EmaArgs *)A);                      \
    break;
#define P_SPMM(gi, G)                                                                  \
  case PB_SPMM + 4 * gi:                                                               \
    b_spmm<VBlk, T, G, false, 4>(bk, *(const SpmmArgs *)A);                            \
    break;                                                                             \
  case PB_SPMM + 4 * gi + 1:                                                           \
    b_spmm<VBlk, T, G, false, 8>(bk, *(const SpmmArgs *)A);                            \
    break;                                                                             \
  case PB_SPMM + 4 * gi + 2:                                                           \
    b_spmm<VBlk, T, G, true, 4>(bk, *(const SpmmArgs *)A);                             \
    break;                                                                             \
  case PB_SPMM + 4 * gi + 3:                                                           \
    b_spmm<VBlk, T, G, true, 8>(bk, *(const SpmmArgs *)A);                             \
    break;

template <typename T>
__device__ __forceinline__ void p_run(int body, const unsigned char *A, const VBlk &bk) {
  constexpr bool SC = std::is_same<T, float>::value;
  using Acc = typename std::conditional<is_u64<T>, uint64_t, double>::type;
  switch (body) {
    case PB_COLOR: {
      const ColorPA &q = *(const ColorPA *)A;
      b_color(bk, q.out, q.n, q.k, q.seed, q.first, q.count, q.orig);
    } break;
    case PB_FILL_U32: {
      const FillPA &q = *(const FillPA *)A;
      b_fill_u32(bk, q.p, q.n, q.v);
    } break;
    case PB_COPY_I32: {
      const CopyPA &q = *(const CopyPA *)A;
      b_copy_i32(bk, q.src, q.dst, q.n);
    } break;
    case PB_NBR_COLORS: {
      const NbrColPA &q = *(const NbrColPA *)A;
      b_nbr_colors(bk, q.col_idx, q.nnz, q.colors, q.n, q.j0, q.nbr);
    } break;
    case PB_COLMAX: {
      const ColmaxPA &q = *(const ColmaxPA *)A;
      b_colmax(bk, q.X, q.n, q.ld, q.cols, q.mx);
    } break;
    case PB_NORM_PREP: {
      const NormPrepPA &q = *(const NormPrepPA *)A;
      b_norm_prep(bk, q.e, q.mx, q.C, q.f, q.E);
    } break;
    case PB_ROOT_EXP: {  // a 64-thread kernel
      const RootExpPA &q = *(const RootExpPA *)A;
      if (threadIdx.x < 64) b_root_exp(bk, q.EX, q.EY, q.out, q.b);
    } break;
    case PB_SINGLE_BOUND: {
      const SingleBoundPA &q = *(const SingleBoundPA *)A;
      b_single_bound(bk, q.drop, q.k, q.Cs, q.Cb, q.b, q.mxB, q.fb, q.mx);
    } break;
    case PB_TASK_SPLIT: {
      const TaskSplitPA &q = *(const TaskSplitPA *)A;
      b_task_split(bk, q.col_idx, q.task_beg, q.task_len, q.n_tasks, q.n, q.xs, q.bounds, q.out);
    } break;
    case PB_XSPLIT_COMBINE:
      b_xsplit_combine<VBlk, T>(bk, *(const XsplitCombineArgs *)A);
      break;
    case PB_SPMM_COMBINE:
      b_spmm_combine<VBlk, T>(bk, *(const CombineArgs *)A);
      break;
    case PB_EMA_SINGLE:
      b_ema_single<VBlk, T, SC>(bk, *(const EmaArgs *)A);
      break;
    case PB_ROOT_FINAL: {  // a 64-thread kernel
      const RootFinalPA &q = *(const RootFinalPA *)A;
      if (threadIdx.x < 64) b_root_final<VBlk, Acc>(bk, (const Acc *)q.partial, q.nblk, q.b, (Acc *)q.out, q.ovf);
    } break;
    case PB_ZERO_PAD: {
      const ZeroPadPA &q = *(const ZeroPadPA *)A;
      b_zero_pad<VBlk, T>(bk, (T *)q.X, q.n, q.ld, q.c_from);
    } break;
    case PB_HIST:
      b_hist<VBlk, T, false, 4, 1>(bk, *(const HistArgs *)A);
      break;
    case PB_HIST + 1:
      b_hist<VBlk, T, false, 2, 4>(bk, *(const HistArgs *)A);
      break;
    case PB_HIST + 2:
      b_hist<VBlk, T, true, 4, 1>(bk, *(const HistArgs *)A);
      break;
    case PB_HIST + 3:
      b_hist<VBlk, T, true, 2, 4>(bk, *(const HistArgs *)A);
      break;
    case PB_ROOT:
      b_root<VBlk, T, SC, false>(bk, *(const RootArgs *)A);
      break;
    case PB_ROOT + 1:
      b_root<VBlk, T, SC, true>(bk, *(const RootArgs *)A);
      break;
    case PB_ROOT_LDS:
      b_root_lds<VBlk, T, SC, false>(bk, *(const RootArgs *)A);
      break;
    case PB_ROOT_LDS + 1:
      b_root_lds<VBlk, T, SC, true>(bk, *(const RootArgs *)A);
      break;
    P_EMA(0, 1)
    P_EMA(1, 2)
    P_EMA(2, 4)
    P_EMA(3, 8)
    P_EMA(4, 16)
    P_SPMM(0, 2)
    P_SPMM(1, 4)
    P_SPMM(2, 8)
    P_SPMM(3, 16)
    P_SPMM(4, 32)
    default:
      break;
  }
}
#undef P_EMA
#undef P_SPMM

template <typename T>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4, 8))) k_persist(PersistArgs p) {
  __shared__ long long s_t;
  __shared__ int s_cur;
  // thread 0 only, per chain: the latest predecessor seen complete, and the
  // launch holding the chain's last ticket looked at (tickets only grow)
  __shared__ int s_seen[kPMaxChains];
  __shared__ int s_ccur[kPMaxChains];
  for (int c = threadIdx.x; c < p.n_chain; c += BLOCK) {
    s_seen[c] = -1;
    s_ccur[c] = p.chain_first[c];
  }
  int home = (int)(blockIdx.x % (unsigned)p.n_chain);  // thread 0: chain looked at first
  for (;;) {
    __syncthreads();  // the previous task's reads of s_t and s_cur are done
    if (threadIdx.x == 0) {
      long long t = -1;
      int ch = -1;
      // the first chain (from home) whose next task can start now, else the
      // first with tasks left (the block then waits for its predecessor)
      while (t < 0 && __hip_atomic_load(p.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        int pick = -1, any = -1;
        for (int i = 0; i < p.n_chain && pick < 0; ++i) {
          const int c = (home + i) % p.n_chain;
          const long long q = (long long)__hip_atomic_load(p.next + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (q >= p.chain_total[c]) continue;
          if (any < 0) any = c;
          int l = s_ccur[c];
          while (l + 1 < p.chain_first[c + 1] && p.L[l + 1].first <= q) ++l;
          s_ccur[c] = l;
          const int pr = p.L[l].pred;
          if (pr < 0 || s_seen[c] >= pr ||
              __hip_atomic_load(p.done + pr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (unsigned)p.L[pr].ntask)
            pick = c;
        }
        if (pick < 0) pick = any;
        if (pick < 0) break;  // every chain handed out
        const long long q = (long long)atomicAdd(p.next + pick, 1ull);
        if (q < p.chain_total[pick]) {
          t = q;
          ch = pick;
        }
      }
      int cur = -1;
      if (t >= 0) {
        home = ch;
        int l = s_ccur[ch];
        while (l + 1 < p.chain_first[ch + 1] && p.L[l + 1].first <= t) ++l;
        s_ccur[ch] = l;
        cur = l;
        const int pred = p.L[cur].pred;
        if (pred >= 0 && s_seen[ch] < pred) {
          const unsigned need = (unsigned)p.L[pred].ntask;
          const long long t0 = wall_clock64();
          while (__hip_atomic_load(p.done + pred, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            if (__hip_atomic_load(p.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                (uint64_t)(wall_clock64() - t0) > p.timeout) {
              atomicOr(p.err, 1);
              t = -1;
              break;
            }
            __builtin_amdgcn_s_sleep(8);
          }
          if (t >= 0) {
            // invalidates this CU's L1 and this XCD's L2 for the whole block
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_seen[ch] = pred;
          }
        }
      }
      s_t = t;
      s_cur = cur;
    }
    __syncthreads();
    // the same for every thread: read through the first lane so that the
    // compiler treats the task (and the body's arguments) as wave-uniform
    const long long st = s_t;
    const long long t = (long long)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(st >> 32)) << 32) |
                                    (uint32_t)__builtin_amdgcn_readfirstlane((int)st));
    if (t < 0) break;
    const int cur = __builtin_amdgcn_readfirstlane(s_cur);
    const PLaunch &L = p.L[cur];
    const long long vb = t - L.first;
    const VBlk bk{(unsigned)(vb % L.gx), (unsigned)(vb / L.gx), L.gx, L.gy};
    p_run<T>(L.body, L.args, bk);
    // every wave's stores have reached its XCD's L2 (the barrier alone does
    // not wait for them); then one agent-scope release writes that L2 back
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(p.done + cur, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ===========================================================================
// launchers

static inline unsigned grid_cap(int64_t want, int64_t cap) {
  if (want < 1) want = 1;
  return (unsigned)(want < cap ? want : cap);
}

thread_local PRecorder *t_prec = nullptr;

// append a launch to the recorder of this thread
template <typename A>
static void prec_add(int body, int dtype, const A &args, dim3 grid, size_t lds) {
  static_assert(sizeof(A) <= kPArgBytes, "argument block larger than PLaunch::args");
  static_assert(std::is_trivially_copyable<A>::value, "argument block must be plain data");
  PRecord r;
  r.body = body;
  r.dtype = dtype;
  r.chain = t_prec->chain;
  r.gx = grid.x;
  r.gy = grid.y;
  r.lds = lds;
  std::memset(r.args, 0, sizeof(r.args));
  std::memcpy(r.args, &args, sizeof(A));
  if (grid.z != 1 && t_prec->err.empty()) t_prec->err = "a launch with a 3-D grid";
  t_prec->rec.push_back(r);
}

static void prec_reject(const char *what) {
  if (t_prec->err.empty()) t_prec->err = what;
}

static int log2i(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

void launch_color(uint8_t *out, int64_t n, int32_t k, uint64_t seed, int32_t first,
                  int32_t count, const int32_t *orig, hipStream_t s) {
  int64_t total = n * count;
  int64_t blocks = (total + BLOCK - 1) / BLOCK;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  if (t_prec) {
    prec_add(PB_COLOR, -1, ColorPA{out, n, k, first, count, 0, seed, orig}, dim3((unsigned)blocks), 0);
    return;
  }
  k_color<<<dim3((unsigned)blocks), dim3(BLOCK), 0, s>>>(out, n, k, seed, first, count, orig);
}

void launch_scatter_f64(const double *in, const int64_t *idx, double *out, int64_t n,
                        hipStream_t s) {
  if (n <= 0) return;
  if (t_prec) return prec_reject("launch_scatter_f64");
  int64_t blocks = std::min<int64_t>((n + BLOCK - 1) / BLOCK, 65536);
  k_scatter_f64<<<dim3((unsigned)blocks), dim3(BLOCK), 0, s>>>(in, idx, out, n);
}

template <typename T>
static void hist_dispatch(const HistArgs &a, int blocks, hipStream_t s) {
  // one colouring: four neighbour blocks in flight; more: two blocks of four
  // colourings each
  if (a.b == 1) {
    if (a.w) k_hist<T, true, 4, 1><<<blocks, BLOCK, 0, s>>>(a);
    else k_hist<T, false, 4, 1><<<blocks, BLOCK, 0, s>>>(a);
  } else {
    if (a.w) k_hist<T, true, 2, 4><<<blocks, BLOCK, 0, s>>>(a);
    else k_hist<T, false, 2, 4><<<blocks, BLOCK, 0, s>>>(a);
  }
}

void launch_hist(int dtype, const HistArgs &a, int blocks, hipStream_t s) {
  if (t_prec) return prec_add(PB_HIST + (a.w ? 2 : 0) + (a.b == 1 ? 0 : 1), dtype, a, dim3(blocks), 0);
  if (dtype == DT_F32) hist_dispatch<float>(a, blocks, s);
  else if (dtype == DT_F64) hist_dispatch<double>(a, blocks, s);
  else hist_dispatch<uint64_t>(a, blocks, s);
}

template <typename T, int G, int UNR>
static void spmm_g(const SpmmArgs &a, dim3 grid, hipStream_t s) {
  if (a.w) k_spmm<T, G, true, UNR><<<grid, BLOCK, 0, s>>>(a);
  else k_spmm<T, G, false, UNR><<<grid, BLOCK, 0, s>>>(a);
}

template <typename T, int UNR>
static int spmm_t(const SpmmArgs &a, int G, dim3 grid, hipStream_t s) {
  switch (G) {
    case 2: spmm_g<T, 2, UNR>(a, grid, s); return 0;
    case 4: spmm_g<T, 4, UNR>(a, grid, s); return 0;
    case 8: spmm_g<T, 8, UNR>(a, grid, s); return 0;
    case 16: spmm_g<T, 16, UNR>(a, grid, s); return 0;
    case 32: spmm_g<T, 32, UNR>(a, grid, s); return 0;
    default: return -1;
  }
}

int launch_spmm(int dtype, const SpmmArgs &a, int G, int unroll, dim3 grid, hipStream_t s) {
  if (t_prec) {
    if (G != 2 && G != 4 && G != 8 && G != 16 && G != 32) return -1;
    prec_add(PB_SPMM + 4 * (log2i(G) - 1) + (a.w ? 2 : 0) + (unroll == 8 ? 1 : 0), dtype, a, grid, 0);
    return 0;
  }
  if (unroll == 8) {
    if (dtype == DT_F32) return spmm_t<float, 8>(a, G, grid, s);
    if (dtype == DT_F64) return spmm_t<double, 8>(a, G, grid, s);
    return spmm_t<uint64_t, 8>(a, G, grid, s);
  }
  if (dtype == DT_F32) return spmm_t<float, 4>(a, G, grid, s);
  if (dtype == DT_F64) return spmm_t<double, 4>(a, G, grid, s);
  return spmm_t<uint64_t, 4>(a, G, grid, s);
}

template <typename T, int G>
static void panel_g(const SpmmPanelArgs &a, dim3 grid, hipStream_t s) {
  const size_t lds = (size_t)WAVES_PER_BLOCK * PANEL_TASKS * G * 16;
  if (a.e_w) k_spmm_panel<T, G, true><<<grid, BLOCK, lds, s>>>(a);
  else k_spmm_panel<T, G, false><<<grid, BLOCK, lds, s>>>(a);
}

template <typename T>
static int panel_t(const SpmmPanelArgs &a, int G, dim3 grid, hipStream_t s) {
  switch (G) {
    case 2: panel_g<T, 2>(a, grid, s); return 0;
    case 4: panel_g<T, 4>(a, grid, s); return 0;
    case 8: panel_g<T, 8>(a, grid, s); return 0;
    case 16: panel_g<T, 16>(a, grid, s); return 0;
    case 32: panel_g<T, 32>(a, grid, s); return 0;
    default: return -1;
  }
}

int launch_spmm_panel(int dtype, const SpmmPanelArgs &a, int G, dim3 grid, hipStream_t s) {
  if (t_prec) {
    prec_reject("the row-panel SpMM");
    return 0;
  }
  if (dtype == DT_F32) return panel_t<float>(a, G, grid, s);
  if (dtype == DT_F64) return panel_t<double>(a, G, grid, s);
  return panel_t<uint64_t>(a, G, grid, s);
}

void launch_xsplit_combine(int dtype, const XsplitCombineArgs &a, hipStream_t s) {
  const int N = (dtype == DT_F32) ? 4 : 2;
  const int64_t nvec = (a.ldp + N - 1) / N;
  dim3 grid(grid_cap((nvec + BLOCK - 1) / BLOCK, 1 << 20), grid_cap((a.n_tasks + 63) / 64, 8192));
  if (t_prec) return prec_add(PB_XSPLIT_COMBINE, dtype, a, grid, 0);
  if (dtype == DT_F32) k_xsplit_combine<float><<<grid, BLOCK, 0, s>>>(a);
  else if (dtype == DT_F64) k_xsplit_combine<double><<<grid, BLOCK, 0, s>>>(a);
  else k_xsplit_combine<uint64_t><<<grid, BLOCK, 0, s>>>(a);
}

void launch_task_split(const int32_t *col_idx, const int64_t *task_beg, const int32_t *task_len,
                       int64_t n_tasks, int64_t n, int xs, const int64_t *bounds, uint16_t *out,
                       hipStream_t s) {
  const int64_t total = n_tasks * (xs + 1);
  if (total == 0) return;
  if (t_prec)
    return prec_add(PB_TASK_SPLIT, -1, TaskSplitPA{col_idx, task_beg, task_len, n_tasks, n, xs, bounds, out},
                    dim3(grid_cap((total + BLOCK - 1) / BLOCK, 65536)), 0);
  k_task_split<<<grid_cap((total + BLOCK - 1) / BLOCK, 65536), BLOCK, 0, s>>>(col_idx, task_beg, task_len,
                                                                            n_tasks, n, xs, bounds, out);
}

void launch_spmm_combine(int dtype, const CombineArgs &a, hipStream_t s) {
  const int N = (dtype == DT_F32) ? 4 : 2;
  const int64_t nvec = (a.ld + N - 1) / N;
  dim3 grid(grid_cap((nvec + BLOCK - 1) / BLOCK, 1 << 20), grid_cap((a.n_long + 31) / 32, 4096));
  if (a.n_long == 0) return;
  if (t_prec) return prec_add(PB_SPMM_COMBINE, dtype, a, grid, 0);
  if (dtype == DT_F32) k_spmm_combine<float><<<grid, BLOCK, 0, s>>>(a);
  else if (dtype == DT_F64) k_spmm_combine<double><<<grid, BLOCK, 0, s>>>(a);
  else k_spmm_combine<uint64_t><<<grid, BLOCK, 0, s>>>(a);
}

template <typename T, int R, bool SC, bool ST>
static void ema_g_launch(const EmaArgs &a, dim3 grid, size_t lds, hipStream_t s) {
  auto kern = k_ema_general<T, R, SC, ST>;
  if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  kern<<<grid, BLOCK, lds, s>>>(a);
}

template <typename T, bool SC, bool ST>
static int ema_g_r(const EmaArgs &a, int R, dim3 grid, size_t lds, hipStream_t s) {
  switch (R) {
    case 1: ema_g_launch<T, 1, SC, ST>(a, grid, lds, s); return 0;
    case 2: ema_g_launch<T, 2, SC, ST>(a, grid, lds, s); return 0;
    case 4: ema_g_launch<T, 4, SC, ST>(a, grid, lds, s); return 0;
    case 8: ema_g_launch<T, 8, SC, ST>(a, grid, lds, s); return 0;
    case 16: ema_g_launch<T, 16, SC, ST>(a, grid, lds, s); return 0;
    default: return -1;
  }
}

int launch_ema_general(int dtype, const EmaArgs &a, int R, bool stage, dim3 grid, size_t lds,
                       hipStream_t s) {
  if (t_prec) {
    if (R != 1 && R != 2 && R != 4 && R != 8 && R != 16) return -1;
    prec_add(PB_EMA_GENERAL + 2 * log2i(R) + (stage ? 1 : 0), dtype, a, grid, lds);
    return 0;
  }
  if (dtype == DT_F32)
    return stage ? ema_g_r<float, true, true>(a, R, grid, lds, s)
                 : ema_g_r<float, true, false>(a, R, grid, lds, s);
  if (dtype == DT_F64)
    return stage ? ema_g_r<double, false, true>(a, R, grid, lds, s)
                 : ema_g_r<double, false, false>(a, R, grid, lds, s);
  return stage ? ema_g_r<uint64_t, false, true>(a, R, grid, lds, s)
               : ema_g_r<uint64_t, false, false>(a, R, grid, lds, s);
}

void launch_ema_single(int dtype, const EmaArgs &a, dim3 grid, size_t lds, hipStream_t s) {
  // add the staged drop table and the tile's colours to the maxima's bytes
  const int64_t W = (int64_t)a.Cs * a.nb;
  const int64_t R = std::max<int64_t>(1, (4 * 8 * BLOCK) / W);
  const size_t total = (lds ? (lds + 15) / 16 * 16 : 0) + (a.kc ? ((size_t)a.kc * a.Cs * 2 + 15) / 16 * 16 : 0) +
                       ((size_t)R * a.nb + 15) / 16 * 16;
  if (t_prec) return prec_add(PB_EMA_SINGLE, dtype, a, grid, total);
  auto go = [&](auto kern) {
    if (total > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)total);
    kern<<<grid, BLOCK, total, s>>>(a);
  };
  if (dtype == DT_F32) go(k_ema_single<float, true>);
  else if (dtype == DT_F64) go(k_ema_single<double, false>);
  else go(k_ema_single<uint64_t, false>);
}

void launch_root(int dtype, const RootArgs &a, dim3 grid, hipStream_t s) {
  const bool hy = a.Y != nullptr;
  if (t_prec) return prec_add(PB_ROOT + (hy ? 1 : 0), dtype, a, grid, 0);
  if (dtype == DT_F32) {
    if (hy) k_root<float, true, true><<<grid, BLOCK, 0, s>>>(a);
    else k_root<float, true, false><<<grid, BLOCK, 0, s>>>(a);
  } else if (dtype == DT_F64) {
    if (hy) k_root<double, false, true><<<grid, BLOCK, 0, s>>>(a);
    else k_root<double, false, false><<<grid, BLOCK, 0, s>>>(a);
  } else {
    if (hy) k_root<uint64_t, false, true><<<grid, BLOCK, 0, s>>>(a);
    else k_root<uint64_t, false, false><<<grid, BLOCK, 0, s>>>(a);
  }
}

template <typename T, bool SC>
static void root_lds_t(const RootArgs &a, dim3 grid, size_t lds, hipStream_t s) {
  auto k1 = k_root_lds<T, SC, true>;
  auto k0 = k_root_lds<T, SC, false>;
  auto kern = a.Y ? k1 : k0;
  if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  kern<<<grid, BLOCK, lds, s>>>(a);
}

template <typename T, bool SC>
static void root_thread_t(const RootArgs &a, dim3 grid, hipStream_t s) {
  const size_t lds = (size_t)a.k * a.L * 4;
  if (a.Y) k_root_thread<T, SC, true><<<grid, BLOCK, lds, s>>>(a);
  else k_root_thread<T, SC, false><<<grid, BLOCK, lds, s>>>(a);
}

template <typename T, bool SC>
static void root_stage_t(const RootArgs &a, dim3 grid, int R, size_t lds, hipStream_t s) {
  int lgx = 0, lgy = 0;
  while ((1 << lgx) < a.Cx) ++lgx;
  while ((1 << lgy) < a.Cy) ++lgy;
  auto kern = a.Y ? k_root_stage<T, SC, true> : k_root_stage<T, SC, false>;
  if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  kern<<<grid, BLOCK, lds, s>>>(a, R, lgx, lgy);
}

void launch_root_stage(int dtype, const RootArgs &a, dim3 grid, int R, size_t lds, hipStream_t s) {
  if (t_prec) return prec_reject("the staged-row root reduction");
  if (dtype == DT_F32) root_stage_t<float, true>(a, grid, R, lds, s);
  else if (dtype == DT_F64) root_stage_t<double, false>(a, grid, R, lds, s);
  else root_stage_t<uint64_t, false>(a, grid, R, lds, s);
}

void launch_root_thread(int dtype, const RootArgs &a, dim3 grid, hipStream_t s) {
  if (t_prec) return prec_reject("the thread-per-vertex root reduction");
  if (dtype == DT_F32) root_thread_t<float, true>(a, grid, s);
  else if (dtype == DT_F64) root_thread_t<double, false>(a, grid, s);
  else root_thread_t<uint64_t, false>(a, grid, s);
}

template <typename T, bool SC>
static void root_tile_t(const RootArgs &a, dim3 grid, size_t lds, bool db, hipStream_t s) {
  // 16-byte vectors per thread: rows of up to 8192 elements
  constexpr int PV = sizeof(T) == 4 ? 8 : 16;
  auto kern = a.Y ? (db ? k_root_tile<T, SC, true, 16, PV, true> : k_root_tile<T, SC, true, 16, PV, false>)
                  : (db ? k_root_tile<T, SC, false, 16, PV, true> : k_root_tile<T, SC, false, 16, PV, false>);
  if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  kern<<<grid, BLOCK, lds, s>>>(a);
}

void launch_root_tile(int dtype, const RootArgs &a, dim3 grid, size_t lds, bool db, hipStream_t s) {
  if (t_prec) return prec_reject("the colour-by-colour root reduction");
  if (dtype == DT_F32) root_tile_t<float, true>(a, grid, lds, db, s);
  else if (dtype == DT_F64) root_tile_t<double, false>(a, grid, lds, db, s);
  else root_tile_t<uint64_t, false>(a, grid, lds, db, s);
}

void launch_root_lds(int dtype, const RootArgs &a, dim3 grid, size_t lds, hipStream_t s) {
  if (t_prec) return prec_add(PB_ROOT_LDS + (a.Y ? 1 : 0), dtype, a, grid, lds);
  if (dtype == DT_F32) root_lds_t<float, true>(a, grid, lds, s);
  else if (dtype == DT_F64) root_lds_t<double, false>(a, grid, lds, s);
  else root_lds_t<uint64_t, false>(a, grid, lds, s);
}

void launch_root_final(int dtype, const void *partial, int nblk, int b, void *out, int *ovf,
                       hipStream_t s) {
  // one 64-thread wave per colouring of the pass
  const unsigned blocks = (unsigned)b;
  if (t_prec) return prec_add(PB_ROOT_FINAL, dtype, RootFinalPA{partial, nblk, b, out, ovf}, dim3(blocks), 0);
  if (dtype == DT_U64)
    k_root_final<uint64_t><<<blocks, 64, 0, s>>>((const uint64_t *)partial, nblk, b, (uint64_t *)out, ovf);
  else
    k_root_final<double><<<blocks, 64, 0, s>>>((const double *)partial, nblk, b, (double *)out, ovf);
}

void launch_nbr_colors(const int32_t *col_idx, int64_t nnz, const uint8_t *colors, int64_t n,
                       int32_t j0, int32_t b, uint8_t *nbr, hipStream_t s) {
  if (nnz == 0) return;
  if (t_prec)
    return prec_add(PB_NBR_COLORS, -1, NbrColPA{col_idx, nnz, colors, n, j0, nbr},
                    dim3(grid_cap((nnz + BLOCK - 1) / BLOCK, 16384), b), 0);
  k_nbr_colors<<<dim3(grid_cap((nnz + BLOCK - 1) / BLOCK, 16384), b), BLOCK, 0, s>>>(col_idx, nnz, colors, n, j0, nbr);
}

void launch_bucket(const uint8_t *colors, int64_t n, int32_t j0, int32_t b, int32_t k, int32_t *counts,
                   int32_t *cursor, int32_t *perm, hipStream_t s) {
  const unsigned g = grid_cap((n + BLOCK - 1) / BLOCK, 1024);
  if (t_prec) return prec_reject("the colour bucketing of the colour-restricted multiply-add");
  k_fill_u32<<<grid_cap((2 * b * k + BLOCK - 1) / BLOCK, 64), BLOCK, 0, s>>>((unsigned *)counts, (int64_t)b * k, 0u);
  k_fill_u32<<<grid_cap((2 * b * k + BLOCK - 1) / BLOCK, 64), BLOCK, 0, s>>>((unsigned *)cursor, (int64_t)b * k, 0u);
  k_bucket_count<<<dim3(g, b), BLOCK, 0, s>>>(colors, n, j0, k, counts);
  k_bucket_scatter<<<dim3(grid_cap((n + 8 * BLOCK - 1) / (8 * BLOCK), 1024), b), BLOCK, 0, s>>>(
      colors, n, j0, k, counts, cursor, perm);
}

template <typename T, bool SC, int NT>
static int ema_colour_nt(const EmaColourArgs &a, int R, dim3 grid, size_t lds, hipStream_t s) {
  auto go = [&](auto kern) {
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    kern<<<grid, NT, lds, s>>>(a);
  };
  switch (R) {
    case 4: go(k_ema_colour<T, 4, SC, NT>); return 0;
    case 8: go(k_ema_colour<T, 8, SC, NT>); return 0;
    case 16: go(k_ema_colour<T, 16, SC, NT>); return 0;
    default: return -1;
  }
}

template <typename T, bool SC>
static int ema_colour_t(const EmaColourArgs &a, int R, int nt, dim3 grid, size_t lds, hipStream_t s) {
  if (nt == 512) return ema_colour_nt<T, SC, 512>(a, R, grid, lds, s);
  if (nt == 256) return ema_colour_nt<T, SC, 256>(a, R, grid, lds, s);
  if (nt == 128) return ema_colour_nt<T, SC, 128>(a, R, grid, lds, s);
  return -1;
}

int launch_ema_colour(int dtype, const EmaColourArgs &a, int R, int nt, dim3 grid, size_t lds, hipStream_t s) {
  if (t_prec) {
    prec_reject("the colour-restricted multiply-add");
    return 0;
  }
  if (dtype == DT_F32) return ema_colour_t<float, true>(a, R, nt, grid, lds, s);
  if (dtype == DT_F64) return ema_colour_t<double, false>(a, R, nt, grid, lds, s);
  return ema_colour_t<uint64_t, false>(a, R, nt, grid, lds, s);
}

void launch_colmax(const float *X, int64_t n, int64_t ld, int64_t cols, unsigned *mx, hipStream_t s) {
  if (n == 0 || cols == 0) return;
  const int64_t gx = (cols + BLOCK - 1) / BLOCK;
  const int64_t gy = std::max<int64_t>(1, std::min<int64_t>(n, (4096 + gx - 1) / gx));
  if (t_prec) return prec_add(PB_COLMAX, -1, ColmaxPA{X, n, ld, cols, mx}, dim3((unsigned)gx, (unsigned)gy), 0);
  k_colmax<<<dim3((unsigned)gx, (unsigned)gy), BLOCK, 0, s>>>(X, n, ld, cols, mx);
}

void launch_norm_prep(const int *e, const unsigned *mx, int C, int b, float *f, int *E,
                      hipStream_t s) {
  if (t_prec) return prec_add(PB_NORM_PREP, -1, NormPrepPA{e, mx, C, f, E}, dim3(b), 0);
  k_norm_prep<<<b, BLOCK, 0, s>>>(e, mx, C, f, E);
}

void launch_root_exp(const int *EX, const int *EY, int *out, int b, hipStream_t s) {
  if (t_prec) return prec_add(PB_ROOT_EXP, -1, RootExpPA{EX, EY, out, b}, dim3((b + 63) / 64), 0);
  k_root_exp<<<(b + 63) / 64, 64, 0, s>>>(EX, EY, out, b);
}

void launch_fill_u32(unsigned *p, int64_t n, unsigned v, hipStream_t s) {
  if (n <= 0) return;
  if (t_prec) return prec_add(PB_FILL_U32, -1, FillPA{p, n, v}, dim3(grid_cap((n + BLOCK - 1) / BLOCK, 4096)), 0);
  k_fill_u32<<<grid_cap((n + BLOCK - 1) / BLOCK, 4096), BLOCK, 0, s>>>(p, n, v);
}

void launch_copy_i32(const int *src, int *dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  if (t_prec) return prec_add(PB_COPY_I32, -1, CopyPA{src, dst, n}, dim3(grid_cap((n + BLOCK - 1) / BLOCK, 4096)), 0);
  k_copy_i32<<<grid_cap((n + BLOCK - 1) / BLOCK, 4096), BLOCK, 0, s>>>(src, dst, n);
}

void launch_scale_add(float *Y, int64_t ldy, const float *X, int64_t ldx, int64_t n, int64_t cols, float so,
                      float sn, hipStream_t s) {
  if (n == 0 || cols == 0) return;
  if (t_prec) return prec_reject("launch_scale_add");
  k_scale_add<<<grid_cap((n * cols + BLOCK - 1) / BLOCK, 65536), BLOCK, 0, s>>>(Y, ldy, X, ldx, n, cols, so, sn);
}

void launch_sddmm(int dtype, const SddmmArgs &a, hipStream_t s) {
  const unsigned g = grid_cap((a.n + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK, 4096);
  if (t_prec) return prec_reject("launch_sddmm");
  if (dtype == DT_F64) k_sddmm<double><<<g, BLOCK, 0, s>>>(a);
  else if (dtype == DT_F32) k_sddmm<float><<<g, BLOCK, 0, s>>>(a);
}

void launch_single_bound(const int32_t *drop, int k, int Cs, int Cb, int b, const unsigned *mxB,
                         const float *fb, unsigned *mx, hipStream_t s) {
  const int64_t total = (int64_t)b * Cs;
  if (total == 0) return;
  if (t_prec)
    return prec_add(PB_SINGLE_BOUND, -1, SingleBoundPA{drop, k, Cs, Cb, b, mxB, fb, mx},
                    dim3(grid_cap((total + BLOCK - 1) / BLOCK, 1 << 20)), 0);
  k_single_bound<<<grid_cap((total + BLOCK - 1) / BLOCK, 1 << 20), BLOCK, 0, s>>>(drop, k, Cs, Cb, b, mxB, fb,
                                                                                 mx);
}

void launch_fill_value(int dtype, void *X, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return;
  if (t_prec) return prec_reject("launch_fill_value");
  const unsigned g = grid_cap((count + BLOCK - 1) / BLOCK, 65536);
  if (dtype == DT_F64) k_fill_value<double><<<g, BLOCK, 0, s>>>((double *)X, count, v);
  else if (dtype == DT_F32) k_fill_value<float><<<g, BLOCK, 0, s>>>((float *)X, count, (float)v);
  else k_fill_value<uint64_t><<<g, BLOCK, 0, s>>>((uint64_t *)X, count, (uint64_t)v);
}

void launch_zero_pad(int dtype, void *X, int64_t n, int64_t ld, int64_t c_from, hipStream_t s) {
  if (c_from >= ld || n == 0) return;
  const unsigned g = grid_cap((n * (ld - c_from) + BLOCK - 1) / BLOCK, 65536);
  if (t_prec) return prec_add(PB_ZERO_PAD, dtype, ZeroPadPA{X, n, ld, c_from}, dim3(g), 0);
  if (dtype == DT_F32) k_zero_pad<float><<<g, BLOCK, 0, s>>>((float *)X, n, ld, c_from);
  else if (dtype == DT_F64) k_zero_pad<double><<<g, BLOCK, 0, s>>>((double *)X, n, ld, c_from);
  else k_zero_pad<uint64_t><<<g, BLOCK, 0, s>>>((uint64_t *)X, n, ld, c_from);
}

template <typename T>
static int persist_occ(size_t lds) {
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void *)k_persist<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<T>, BLOCK, lds) != hipSuccess) return 0;
  return nb;
}

int persist_blocks_per_cu(int dtype, size_t lds) {
  if (dtype == DT_F32) return persist_occ<float>(lds);
  if (dtype == DT_F64) return persist_occ<double>(lds);
  return persist_occ<uint64_t>(lds);
}

void launch_persist(int dtype, const PersistArgs &a, unsigned blocks, size_t lds, hipStream_t s) {
  if (dtype == DT_F32) k_persist<float><<<blocks, BLOCK, lds, s>>>(a);
  else if (dtype == DT_F64) k_persist<double><<<blocks, BLOCK, lds, s>>>(a);
  else k_persist<uint64_t><<<blocks, BLOCK, lds, s>>>(a);
}

}  // namespace sg2v
