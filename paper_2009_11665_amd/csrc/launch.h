// Kernel argument blocks and launchers (host side of kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace sg2v {

enum DType { DT_F64 = 0, DT_F32 = 1, DT_U64 = 2 };

struct HistArgs {
  const int64_t *row_ptr;
  const int32_t *col_idx;
  const float *w;        // nullable
  const uint8_t *colors; // colouring-major
  int64_t n;
  int32_t k;
  int32_t j0;            // first colouring of the pass
  int32_t b;             // colourings in the pass
  void *H;               // n x ldh
  int64_t ldh;
  // SpMM tasks (rows or segments of long rows); segments write their slot
  // of `partial` (n_slots x ldh)
  const int32_t *task_row;
  const int64_t *task_beg;
  const int32_t *task_len;
  const int32_t *task_slot;
  int64_t n_tasks;
  void *partial;
};

struct SpmmArgs {
  const int32_t *col_idx;
  const float *w;          // nullable
  const int32_t *task_row;
  const int64_t *task_beg;
  const int32_t *task_len;
  const int32_t *task_slot;  // -1: write B; else partial row index
  const int32_t *unit_task;  // first task of each unit
  const int8_t *unit_rpw;    // tasks per wave in the unit
  const int16_t *unit_ntask; // tasks in the unit
  int64_t n_units;
  const void *M;
  int64_t ldm;
  void *B;
  int64_t ldb;
  void *partial;           // n_slots x ldb
  int64_t ncols_valid;
  unsigned *mx;            // FP32S column maxima (nullable)
  int *ovf;
  int32_t accumulate;      // 1: B += A M (adjoint), 0: B = A M
  // colour skipping (nullable): per chunk, the colouring block it lies in
  // (-1: spans blocks, no skipping), the union and the intersection of its
  // colour sets.  A neighbour j whose colour is outside the union has a zero
  // row segment; a row i whose colour is in the intersection is never read
  // through this chunk (written as zeros).
  const int32_t *chunk_jb;
  const uint32_t *chunk_union;
  const uint32_t *chunk_inter;
  const uint8_t *colors;
  int32_t j0;
  int64_t n;
  const uint8_t *nbr_col;  // [b][nnz] colour of col_idx[e] in each colouring of the pass
  int64_t nnz;
  int64_t chunk0;          // first chunk of this launch (blockIdx.y is relative)
  // neighbour-range split (0: off) of units [0, xunits), whose tasks are
  // [0, n_tasks): partial rows to partial [xsplit][n_tasks][ldp]
  int32_t xsplit;
  int64_t xunits;
  const uint16_t *tsplit;  // [tasks][xsplit + 1] split offsets within each task
  int64_t n_tasks;
  int64_t ldp;
  void *partial8;
};

// Row-panel SpMM (column-sorted entries per panel of tasks)
constexpr int PANEL_TASKS = 32;  // tasks per panel (one wave's LDS rows)
struct SpmmPanelArgs {
  const int32_t *p_task0;  // first task of each panel
  const int32_t *p_ntask;  // tasks in each panel (<= PANEL_TASKS)
  const int64_t *p_beg;    // [n_panels + 1] entry offsets
  int64_t n_panels;
  const int32_t *e_col;    // neighbour of each panel entry
  const uint8_t *e_loc;    // its task within the panel
  const float *e_w;        // its weight (nullable: 0/1 adjacency)
  const int32_t *task_row;
  const int32_t *task_slot;
  const void *M;
  int64_t ldm;
  void *B;
  int64_t ldb;
  void *partial;
  int64_t ncols_valid;
  unsigned *mx;
  int *ovf;
  int32_t accumulate;
  const int32_t *chunk_jb;
  const uint32_t *chunk_union;
  const uint32_t *chunk_inter;
  const uint8_t *colors;
  int32_t j0;
  int64_t n;
  int64_t chunk0;
};

struct XsplitCombineArgs {
  const void *partial8;  // [xsplit][n_tasks][ldp]
  int32_t xsplit;        // 1..8
  int64_t n_tasks, ldp;
  int64_t col_first;     // column of B where this chunk group starts
  const int32_t *task_row, *task_slot;
  void *B;
  int64_t ldb;
  void *hub;             // long-row partial rows [n_slots][ldb]
  int64_t ncols_valid;
  unsigned *mx;
  int *ovf;
  int32_t accumulate;
};

struct CombineArgs {
  const void *partial;
  void *B;
  int64_t ld;
  int64_t ncols_valid;
  const int32_t *long_row;
  const int32_t *long_slot0;
  const int32_t *long_nslot;
  int32_t n_long;
  unsigned *mx;
  int *ovf;
  int32_t accumulate;
};

struct EmaArgs {
  const void *Ma;
  int64_t lda;
  const void *B;
  int64_t ldb;
  void *Ms;
  int64_t lds;
  const int32_t *pairs;  // int2 [np][Cs]
  const int32_t *drop;   // [k][Cs] (one-vertex active child)
  int32_t np, Cs, Ca, Cb;
  int64_t n;
  const uint8_t *colors;
  int32_t j0;
  const float *fa, *fb;  // FP32S column factors of M_a and B (per colouring block)
  const int *Ea, *Eb;    // FP32S frame exponents per colouring
  unsigned *mx;          // FP32S output column maxima
  int *es;               // FP32S output column exponents
  int *ovf;
  int32_t accumulate;    // general kernel: 1 adds into Ms (adjoint)
  int32_t nb;            // single-vertex kernel: colourings in the pass (columns j * Cs + C)
  int32_t kc;            // single-vertex kernel: colours, when the drop table is staged in
                         // LDS as uint16 (indices below 0xFFFF), else 0
};

// colour-restricted multiply-add (rows bucketed by colour)
struct EmaColourArgs {
  const void *Ma;
  int64_t lda;
  int32_t Ca;
  const void *B;
  int64_t ldb;
  int32_t Cb;
  void *Ms;
  int64_t lds;
  int32_t Cs;
  const int32_t *ca, *cb, *co, *cz;  // [k][Sa], [k][Sb], [k][U], [k][Z]
  const uint32_t *cp;                // [k][Q][U]
  const int32_t *cu;                 // [k][Cs]: u of an output column holding c, else -1
  int32_t Sa, Sb, U, Z, Q, k;
  const int32_t *perm;    // [b][n] rows grouped by colour
  const int32_t *counts;  // [b][k] rows per colour
  int64_t n;
  const float *fa, *fb;
  const int *Ea, *Eb;
  unsigned *mx;
  int *es;
  int *ovf;
};

// nbr[jj][e] = colour of col_idx[e] in colouring j0 + jj
void launch_nbr_colors(const int32_t *col_idx, int64_t nnz, const uint8_t *colors, int64_t n,
                       int32_t j0, int32_t b, uint8_t *nbr, hipStream_t s);
// rows grouped by colour: counts[j][c], then perm[j][.] (order within a colour is arbitrary)
void launch_bucket(const uint8_t *colors, int64_t n, int32_t j0, int32_t b, int32_t k, int32_t *counts,
                   int32_t *cursor, int32_t *perm, hipStream_t s);
// nt: threads per block, 128, 256 or 512 (about one output column per thread
// or more; wide outputs share each staged tile among more waves)
int launch_ema_colour(int dtype, const EmaColourArgs &a, int R, int nt, dim3 grid, size_t lds, hipStream_t s);

// edge gradient: grad[e] += sum_c Bbar(i, c) * M_p(j, c) for e = (i -> j)
struct SddmmArgs {
  const int64_t *row_ptr;
  const int32_t *col_idx;
  const void *Bbar;
  int64_t ldb;
  const void *Mp;  // null: one-vertex passive child (one-hot by colour)
  int64_t ldm;
  int64_t ncols;   // b * C(k, |T_p|)
  int64_t n;
  const uint8_t *colors;
  int32_t j0, b, k;
  double *grad;
  const float *fm;  // nullable: FP32S column factors of Mp
  double scale;     // grad[e] += scale * (per-entry sum)
};

struct RootArgs {
  const void *X;
  int64_t ldx;
  int32_t Cx;
  const void *Y;  // nullable (Y = 1)
  int64_t ldy;
  int32_t Cy;
  const int32_t *list;  // int2 [k][L]
  int64_t L;
  int64_t n;
  const uint8_t *colors;
  int32_t j0;
  const float *fx, *fy;
  void *partial;  // [b][gridDim.x] double or uint64
  int *ovf;
  const uint32_t *list16;  // nullable: (x | y << 16) [k][L], y = 0xFFFF for Y = 1
  int32_t same_xy;         // X and Y are the same table (staged once)
  int32_t k;               // colours (root lists per colour)
};

void launch_color(uint8_t *out, int64_t n, int32_t k, uint64_t seed, int32_t first,
                  int32_t count, const int32_t *orig, hipStream_t s);
void launch_scatter_f64(const double *in, const int64_t *idx, double *out, int64_t n,
                        hipStream_t s);
void launch_hist(int dtype, const HistArgs &a, int blocks, hipStream_t s);
// unroll: gathers in flight per stream (4 or 8)
int launch_spmm(int dtype, const SpmmArgs &a, int G, int unroll, dim3 grid, hipStream_t s);
void launch_spmm_combine(int dtype, const CombineArgs &a, hipStream_t s);
// mx[c] = max over rows of X(i, c) (float bits, atomicMax), c < cols; mx
// must start at zero
void launch_colmax(const float *X, int64_t n, int64_t ld, int64_t cols, unsigned *mx, hipStream_t s);
void launch_xsplit_combine(int dtype, const XsplitCombineArgs &a, hipStream_t s);
int launch_spmm_panel(int dtype, const SpmmPanelArgs &a, int G, dim3 grid, hipStream_t s);
void launch_task_split(const int32_t *col_idx, const int64_t *task_beg, const int32_t *task_len,
                       int64_t n_tasks, int64_t n, int xs, const int64_t *bounds, uint16_t *out,
                       hipStream_t s);
int launch_ema_general(int dtype, const EmaArgs &a, int R, bool stage, dim3 grid, size_t lds,
                       hipStream_t s);
// grid.y must be 1 (the kernel covers a.nb colourings); lds = nb * Cs * 4
// when FP32S column maxima are tracked (a.mx non-null), else 0 (the launcher
// adds the staged drop table and colours)
void launch_ema_single(int dtype, const EmaArgs &a, dim3 grid, size_t lds, hipStream_t s);
void launch_root(int dtype, const RootArgs &a, dim3 grid, hipStream_t s);
// block per vertex row, rows staged in LDS; lds = bytes of the staged rows
void launch_root_lds(int dtype, const RootArgs &a, dim3 grid, size_t lds, hipStream_t s);
// colour by colour over contiguous vertex ranges; needs list16, k, Y = X or
// absent, L <= 4096, Cx <= 8192, 16-byte aligned rows, and lds = (db ? 2 : 1)
// * Cx (rounded up to 16 bytes) * element size (db: double-buffered rows)
void launch_root_tile(int dtype, const RootArgs &a, dim3 grid, size_t lds, bool db, hipStream_t s);
// one thread per vertex; needs list16, k * L <= 8192 (lists staged in LDS)
void launch_root_thread(int dtype, const RootArgs &a, dim3 grid, hipStream_t s);
// R vertex rows staged per tile (R a power of two dividing BLOCK); needs
// list16, Cx, Cy <= 65536 and lds = k * L * 4 (rounded up to 16) + R * (Cx +
// Cy) * element size
void launch_root_stage(int dtype, const RootArgs &a, dim3 grid, int R, size_t lds, hipStream_t s);
void launch_root_final(int dtype, const void *partial, int nblk, int b, void *out, int *ovf,
                       hipStream_t s);
void launch_norm_prep(const int *e, const unsigned *mx, int C, int b, float *f, int *E,
                      hipStream_t s);
// FP32S: frame exponent of the root value, E_X + E_Y per colouring
void launch_root_exp(const int *EX, const int *EY, int *out, int b, hipStream_t s);
void launch_fill_u32(unsigned *p, int64_t n, unsigned v, hipStream_t s);
void launch_copy_i32(const int *src, int *dst, int64_t n, hipStream_t s);
void launch_sddmm(int dtype, const SddmmArgs &a, hipStream_t s);
// Y = Y * so + X * sn, n rows of cols columns
void launch_scale_add(float *Y, int64_t ldy, const float *X, int64_t ldx, int64_t n, int64_t cols, float so,
                      float sn, hipStream_t s);
void launch_fill_value(int dtype, void *X, int64_t count, double v, hipStream_t s);
// FP32S: mx[j * Cs + C] = an upper bound of the column maxima of a
// single-vertex-active output from the passive table's maxima and factors
void launch_single_bound(const int32_t *drop, int k, int Cs, int Cb, int b, const unsigned *mxB,
                         const float *fb, unsigned *mx, hipStream_t s);
void launch_zero_pad(int dtype, void *X, int64_t n, int64_t ld, int64_t c_from, hipStream_t s);

// ---------------------------------------------------------------------------
// Persistent schedule.  While t_prec is set on a thread, the launchers above
// append their launch (kernel body, grid, dynamic LDS and a copy of the
// arguments) to it instead of issuing it; k_persist then runs the recorded
// launches of several independent chains (one per template) in one kernel:
// each virtual block of a launch is a task, each chain hands out its tasks in
// ticket order, and a task waits until its launch's predecessor in the same
// chain has completed all of its tasks (a per-launch counter).  Launches that
// cannot run there (other block sizes, multi-kernel launchers) set `err`.

constexpr int kPArgBytes = 320;   // largest argument block (static_assert in kernels.hip)
constexpr int kPMaxChains = 256;

struct PLaunch {
  int32_t body;   // kernel body (PBody in kernels.hip)
  int32_t chain;
  int32_t pred;   // launch that must complete before this one starts (-1: none)
  uint32_t gx, gy;
  uint32_t pad;
  int64_t first;  // ticket (within its chain) of the first virtual block
  int64_t ntask;  // gx * gy
  alignas(16) unsigned char args[kPArgBytes];
};

struct PRecord {
  int32_t body = 0;
  int32_t dtype = -1;  // element type of a typed body, -1 for untyped ones
  int32_t chain = 0;
  uint32_t gx = 1, gy = 1;
  size_t lds = 0;
  unsigned char args[kPArgBytes];
};

struct PRecorder {
  int32_t chain = 0;
  std::vector<PRecord> rec;
  std::string err;  // first launch that cannot be recorded
};
extern thread_local PRecorder *t_prec;

struct PersistArgs {
  const PLaunch *L;             // grouped by chain, in order within each chain
  const int32_t *chain_first;   // [n_chain + 1]: first launch of each chain
  const int64_t *chain_total;   // [n_chain]: tickets (virtual blocks) of each chain
  int32_t n_launch;
  int32_t n_chain;
  unsigned *done;               // per launch: virtual blocks completed
  unsigned long long *next;     // per chain: ticket counter
  int *err;                     // set when a wait exceeded `timeout`
  uint64_t timeout;             // wall-clock ticks a dependency wait may take
};

// blocks of k_persist<dtype> one CU holds with `lds` bytes of dynamic LDS
int persist_blocks_per_cu(int dtype, size_t lds);
void launch_persist(int dtype, const PersistArgs &a, unsigned blocks, size_t lds, hipStream_t s);

}  // namespace sg2v
