// Host runtime of libsg2v: graph registration with degree-sorted row tasks,
// colourings, the per-pass step schedule of the dynamic programme (Alg. 5:
// neighbour aggregation then multiply-add per split, root reduction last),
// a liveness-packed device workspace, FP32 per-column exponent bookkeeping,
// and the C ABI entry points declared in include/sg2v.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <fstream>
#include <sstream>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "internal.h"
#include "launch.h"

using namespace sg2v;

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess) {                                                             \
      set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
      return SG2V_EDEVICE;                                                              \
    }                                                                                   \
  } while (0)

#define ST_TRY(expr)               \
  do {                             \
    sg2v_status _s = (expr);       \
    if (_s != SG2V_OK) return _s;  \
  } while (0)

namespace {

// ---------------------------------------------------------------------------
// tuning

sg2v_tuning_t g_tune = {0, 0, 0, 0, 0, 0, 0, 0};
std::mutex g_tune_mu;

// flags a call forces for its own duration (the persistent batch schedule
// runs only kernels with 256-thread blocks)
thread_local int32_t t_tune_or = 0;

sg2v_tuning_t tuning() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  sg2v_tuning_t t = g_tune;
  t.flags |= t_tune_or;
  return t;
}

struct TuneOr {
  int32_t old;
  explicit TuneOr(int32_t f) : old(t_tune_or) { t_tune_or |= f; }
  ~TuneOr() { t_tune_or = old; }
};

constexpr int64_t kSegment = 4096;  // neighbours per SpMM task (longer rows are split)
constexpr int kSpmmBlocks = 2048;  // blocks of an SpMM launch without the split (grid stride over units)
// blocks of an SpMM launch with the neighbour-range split (512 per XCD): more
// than one round of resident blocks, so that the blocks of a range that finish
// early pick up the remaining units (2048: 284 ms, 4096: 278 ms, 8192: 283 ms
// for the 15-vertex tree on RMAT scale 20)
constexpr int kXsplitBlocks = 4096;
constexpr int kRootBlocks = 2048;    // most root blocks (per-block partial sums)
constexpr int kXsplit = 8;          // neighbour ranges (one per XCD)
constexpr int64_t kXsplitMin = 512; // tasks at least this long are split by range
constexpr double kXpartBytes = 8.0 * (1 << 30);  // range-partial rows of one chunk group
// graphs whose 128-byte column chunk (n rows) reaches 32 MB: wider chunks and
// the neighbour-range split by default
bool large_graph(int64_t n) { return (double)n * 128.0 >= 32.0 * (1 << 20); }

// column chunks per SpMM launch without the neighbour-range split
int64_t fl_launch_chunks() {
  const sg2v_tuning_t tu = tuning();
  return tu.launch_chunks > 0 ? std::min<int64_t>(tu.launch_chunks, 65535) : 65535;
}

int dtype_of(sg2v_mode m) { return m == SG2V_FP32S ? DT_F32 : (m == SG2V_FP64 ? DT_F64 : DT_U64); }
int esize_of(int dt) { return dt == DT_F32 ? 4 : 8; }

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// A fixed device area handed out front to back (sg2v_count_noalloc): buffers
// taken from it are never allocated or freed.
struct Carver {
  char *base = nullptr;
  size_t cap = 0;
  size_t top = 0;
  bool exhausted = false;  // a request did not fit
};

// Set while sg2v_count_noalloc runs on this thread: device allocations fail
// with a message instead of calling hipMalloc.
thread_local bool t_noalloc = false;

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  uint64_t gen = 0;  // bumped on every reallocation (captured graphs hold raw pointers)
  Carver *cv = nullptr;  // set: carved from a fixed area instead of hipMalloc
  ~DevBuf() {
    if (p && !cv) (void)hipFree(p);
  }
  sg2v_status ensure(size_t want) {
    if (want <= bytes) return SG2V_OK;
    if (cv) {
      want = (want + 255) / 256 * 256;
      // the most recent buffer of the area grows in place, any other moves to the top
      size_t off = (p && (char *)p + bytes == cv->base + cv->top) ? (size_t)((char *)p - cv->base)
                                                                  : cv->top;
      if (off + want > cv->cap) {
        cv->exhausted = true;
        set_error("sg2v_count_noalloc: the count needs more than the %zu-byte scratch area "
                  "(%zu bytes requested at offset %zu)", cv->cap, want, off);
        return SG2V_ENOMEM;
      }
      p = cv->base + off;
      bytes = want;
      cv->top = off + want;
      ++gen;
      return SG2V_OK;
    }
    if (t_noalloc) {
      set_error("sg2v_count_noalloc: a device allocation of %zu bytes was requested", want);
      return SG2V_ENOMEM;
    }
    if (p) {
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      set_error("device allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
      return SG2V_ENOMEM;
    }
    bytes = want;
    ++gen;
    return SG2V_OK;
  }
};

template <typename T>
sg2v_status upload(const std::vector<T> &h, void **d, hipStream_t s) {
  *d = nullptr;
  if (h.empty()) return SG2V_OK;
  if (t_noalloc) {
    set_error("sg2v_count_noalloc: device tables of the plan or graph are not set up on this "
              "device; one sg2v_count call with the same plan and graph sets them up");
    return SG2V_ENOMEM;
  }
  HIP_TRY(hipMalloc(d, h.size() * sizeof(T)));
  HIP_TRY(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return SG2V_OK;
}

// ---------------------------------------------------------------------------
// kernel timing with HIP events (sg2v_profile_start / sg2v_profile_stop)

struct ProfRec {
  int kind;
  hipEvent_t a, b;
  double bytes, work;
};

struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};

Profiler &profiler() {
  static Profiler p;
  return p;
}

thread_local bool t_capturing = false;  // inside hipStreamBeginCapture ... EndCapture

// brackets the kernel launches of its lifetime with events when profiling
struct ProfScope {
  bool on;
  ProfRec r;
  hipStream_t s;
  ProfScope(int kind, double bytes, double work, hipStream_t st)
      : on(profiler().on && !t_capturing && !t_noalloc), s(st) {
    if (!on) return;
    r.kind = kind;
    r.bytes = bytes;
    r.work = work;
    std::lock_guard<std::mutex> lk(profiler().mu);
    r.a = profiler().get();
    r.b = profiler().get();
    (void)hipEventRecord(r.a, s);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(r.b, s);
    std::lock_guard<std::mutex> lk(profiler().mu);
    profiler().recs.push_back(r);
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// graph

struct UnitTable {
  int32_t *unit_task = nullptr;
  int8_t *unit_rpw = nullptr;
  int16_t *unit_ntask = nullptr;
  int64_t n_units = 0;
  int64_t x_units = 0;  // leading units whose tasks are split by neighbour range
  int64_t x_tasks = 0;  // tasks in those units
};

struct sg2v_graph {
  int device = 0;
  int64_t n = 0, nnz = 0;
  int64_t *row_ptr = nullptr;
  int32_t *col_idx = nullptr;
  float *w = nullptr;
  bool owns = true;
  double max_wdeg = 0.0;  // max over rows of sum_e |w_e|
  // SpMM tasks, sorted by length (longest first)
  int32_t *task_row = nullptr, *task_len = nullptr, *task_slot = nullptr;
  int64_t *task_beg = nullptr;
  int64_t n_tasks = 0, n_slots = 0;
  std::vector<int32_t> h_task_len;  // sorted lengths
  std::vector<int64_t> h_task_beg;  // their first entries
  // row panels with column-sorted entries (SG2V_TUNE_SPMM_PANEL), built on first use
  struct Panels {
    int32_t *task0 = nullptr, *ntask = nullptr;
    int64_t *beg = nullptr;
    int32_t *col = nullptr;
    uint8_t *loc = nullptr;
    float *w = nullptr;
    int64_t n = 0;
  };
  std::unique_ptr<Panels> panels;
  double long_share = 0.0;          // share of the entries in tasks of >= kXsplitMin neighbours
  int32_t *long_row = nullptr, *long_slot0 = nullptr, *long_nslot = nullptr;
  int32_t n_long = 0;
  std::map<int, UnitTable> units;  // by G (lanes per neighbour row segment)
  uint16_t *tsplit = nullptr;      // [n_tasks][kXsplit + 1] neighbour-range split offsets
  int64_t *xbounds = nullptr;      // device, kXsplit + 1 range starts (renumbered graphs), or null
  // SG2V_GRAPH_RELABEL: vertices renumbered by decreasing degree
  bool relabelled = false;
  int32_t *orig_id = nullptr;      // device, n: caller's id of each stored vertex
  int64_t *entry_orig = nullptr;   // device, nnz: caller's CSR entry of each stored entry
  std::shared_ptr<const std::vector<int32_t>> new_of;  // host, n: stored id of each caller id
  DevBuf grad_tmp;                 // per-entry gradient in stored order (renumbered graphs)
  std::vector<void *> allocs;
  ~sg2v_graph() {
    if (tsplit) (void)hipFree(tsplit);
    for (void *p : allocs) (void)hipFree(p);
    for (auto &kv : units) {
      (void)hipFree(kv.second.unit_task);
      (void)hipFree(kv.second.unit_rpw);
      (void)hipFree(kv.second.unit_ntask);
    }
  }
};

struct sg2v_colorings {
  std::shared_ptr<const std::vector<int32_t>> new_of;  // renumbered graph: stored id of a caller id
  int device = 0;
  int64_t n = 0;
  int32_t k = 0, count = 0, first = 0;
  uint64_t seed = 0;
  uint8_t *d = nullptr;
  ~sg2v_colorings() {
    if (d) (void)hipFree(d);
  }
};

namespace {

// rows per wave for a task of `len` neighbours when a neighbour row segment
// takes G lanes: enough streams for the task, at most 64/G tasks per wave.
int rpw_for(int64_t len, int G) {
  int maxr = 64 / G;
  int r = 1;
  while (r < maxr && (64 / (2 * r)) / G >= std::max<int64_t>(len, 1)) r *= 2;
  return r;
}

sg2v_status build_units(sg2v_graph *g, int G, hipStream_t s, UnitTable **out,
                        int64_t xmin_fixed = 0) {
  // units end at the split threshold (tuning's xsplit_min, 512 neighbours by default)
  const sg2v_tuning_t tu = tuning();
  const int64_t xmin = xmin_fixed > 0 ? xmin_fixed
                       : tu.xsplit_min > 0 ? std::min<int64_t>(tu.xsplit_min, kSegment)
                                           : kXsplitMin;
  const int key = G + 64 * (int)xmin;
  auto it = g->units.find(key);
  if (it != g->units.end()) {
    *out = &it->second;
    return SG2V_OK;
  }
  std::vector<int32_t> ut;
  std::vector<int8_t> ur;
  std::vector<int16_t> un;
  int64_t t = 0;
  while (t < g->n_tasks) {
    int r = rpw_for(g->h_task_len[t], G);
    int64_t cap = (int64_t)4 * r, cnt = 0;
    ut.push_back((int32_t)t);
    while (t < g->n_tasks && cnt < cap && rpw_for(g->h_task_len[t], G) == r) {
      ++t;
      ++cnt;
    }
    ur.push_back((int8_t)r);
    un.push_back((int16_t)cnt);
  }
  UnitTable U;
  U.n_units = (int64_t)ut.size();
  while (U.x_units < U.n_units && g->h_task_len[ut[U.x_units]] >= xmin) ++U.x_units;
  U.x_tasks = U.x_units < U.n_units ? ut[U.x_units] : g->n_tasks;
  ST_TRY(upload(ut, (void **)&U.unit_task, s));
  ST_TRY(upload(ur, (void **)&U.unit_rpw, s));
  ST_TRY(upload(un, (void **)&U.unit_ntask, s));
  HIP_TRY(hipStreamSynchronize(s));
  g->units[key] = U;
  *out = &g->units[key];
  return SG2V_OK;
}

// Row panels for the CSC-Split-style SpMM: consecutive tasks (in their
// longest-first order) grouped while a panel holds at most PANEL_TASKS tasks
// and kPanelEntries entries (a longer task gets a panel of its own); each
// panel's entries sorted by neighbour id, ties by task.
constexpr int64_t kPanelEntries = 8192;

sg2v_status build_panels(sg2v_graph *g, hipStream_t s, sg2v_graph::Panels **out) {
  if (g->panels) {
    *out = g->panels.get();
    return SG2V_OK;
  }
  if (t_noalloc) {
    set_error("row panels not built for this graph");
    return SG2V_ENOMEM;
  }
  const int64_t nnz = g->nnz;
  std::vector<int32_t> ci(std::max<int64_t>(nnz, 1));
  std::vector<float> wv(g->w ? nnz : 0);
  if (nnz) HIP_TRY(hipMemcpyAsync(ci.data(), g->col_idx, nnz * 4, hipMemcpyDeviceToHost, s));
  if (g->w && nnz) HIP_TRY(hipMemcpyAsync(wv.data(), g->w, nnz * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<int32_t> task0, ntask;
  std::vector<int64_t> pbeg{0};
  for (int64_t t = 0; t < g->n_tasks;) {
    int64_t cnt = 0, ent = 0;
    task0.push_back((int32_t)t);
    while (t < g->n_tasks && cnt < PANEL_TASKS && (cnt == 0 || ent + g->h_task_len[t] <= kPanelEntries)) {
      ent += g->h_task_len[t];
      ++cnt;
      ++t;
    }
    ntask.push_back((int32_t)cnt);
    pbeg.push_back(pbeg.back() + ent);
  }
  const int64_t np = (int64_t)task0.size();
  std::vector<int32_t> ecol(std::max<int64_t>(nnz, 1));
  std::vector<uint8_t> eloc(std::max<int64_t>(nnz, 1));
  std::vector<float> ew(g->w ? std::max<int64_t>(nnz, 1) : 0);
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int th = 0; th < nth; ++th)
    pool.emplace_back([&, th]() {
      std::vector<std::pair<int32_t, int64_t>> ent;  // (neighbour, local task << 40 | entry)
      for (int64_t p = th; p < np; p += nth) {
        ent.clear();
        for (int l = 0; l < ntask[p]; ++l) {
          const int64_t t = task0[p] + l;
          const int64_t b = g->h_task_beg[t];
          for (int64_t e = b; e < b + g->h_task_len[t]; ++e)
            ent.push_back({ci[e], ((int64_t)l << 40) | e});
        }
        std::sort(ent.begin(), ent.end());
        for (size_t x = 0; x < ent.size(); ++x) {
          const int64_t o = pbeg[p] + (int64_t)x;
          ecol[o] = ent[x].first;
          eloc[o] = (uint8_t)(ent[x].second >> 40);
          if (g->w) ew[o] = wv[ent[x].second & ((1ll << 40) - 1)];
        }
      }
    });
  for (auto &t : pool) t.join();
  std::unique_ptr<sg2v_graph::Panels> P(new sg2v_graph::Panels());
  void *p;
  ST_TRY(upload(task0, &p, s)); P->task0 = (int32_t *)p; g->allocs.push_back(p);
  ST_TRY(upload(ntask, &p, s)); P->ntask = (int32_t *)p; g->allocs.push_back(p);
  ST_TRY(upload(pbeg, &p, s)); P->beg = (int64_t *)p; g->allocs.push_back(p);
  ST_TRY(upload(ecol, &p, s)); P->col = (int32_t *)p; g->allocs.push_back(p);
  ST_TRY(upload(eloc, &p, s)); P->loc = (uint8_t *)p; g->allocs.push_back(p);
  if (g->w) {
    ST_TRY(upload(ew, &p, s));
    P->w = (float *)p;
    g->allocs.push_back(p);
  }
  HIP_TRY(hipStreamSynchronize(s));
  P->n = np;
  g->panels = std::move(P);
  *out = g->panels.get();
  return SG2V_OK;
}

sg2v_status graph_tasks(sg2v_graph *g, const std::vector<int64_t> &rp, hipStream_t s) {
  const int64_t n = g->n;
  std::vector<int32_t> row, len, slot;
  std::vector<int64_t> beg;
  std::vector<int32_t> lrow, lslot0, lnslot;
  row.reserve(n);
  int64_t slots = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t d = rp[i + 1] - rp[i];
    if (d <= kSegment) {
      row.push_back((int32_t)i);
      beg.push_back(rp[i]);
      len.push_back((int32_t)d);
      slot.push_back(-1);
    } else {
      const int64_t ns = (d + kSegment - 1) / kSegment;
      lrow.push_back((int32_t)i);
      lslot0.push_back((int32_t)slots);
      lnslot.push_back((int32_t)ns);
      for (int64_t q = 0; q < ns; ++q) {
        const int64_t b0 = rp[i] + d * q / ns, b1 = rp[i] + d * (q + 1) / ns;
        row.push_back((int32_t)i);
        beg.push_back(b0);
        len.push_back((int32_t)(b1 - b0));
        slot.push_back((int32_t)(slots + q));
      }
      slots += ns;
    }
  }
  const int64_t T = (int64_t)row.size();
  std::vector<int64_t> ord(T);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return len[a] > len[b]; });
  std::vector<int32_t> srow(T), slen(T), sslot(T);
  std::vector<int64_t> sbeg(T);
  for (int64_t x = 0; x < T; ++x) {
    srow[x] = row[ord[x]];
    slen[x] = len[ord[x]];
    sslot[x] = slot[ord[x]];
    sbeg[x] = beg[ord[x]];
  }
  g->n_tasks = T;
  g->n_slots = slots;
  g->h_task_len = slen;
  g->h_task_beg = sbeg;
  {
    int64_t in_long = 0, all = 0;
    for (int64_t x = 0; x < T; ++x) {
      all += slen[x];
      if (slen[x] >= kXsplitMin) in_long += slen[x];
    }
    g->long_share = all > 0 ? (double)in_long / (double)all : 0.0;
  }
  void *p;
  ST_TRY(upload(srow, &p, s)); g->task_row = (int32_t *)p; g->allocs.push_back(p);
  ST_TRY(upload(slen, &p, s)); g->task_len = (int32_t *)p; g->allocs.push_back(p);
  ST_TRY(upload(sslot, &p, s)); g->task_slot = (int32_t *)p; g->allocs.push_back(p);
  ST_TRY(upload(sbeg, &p, s)); g->task_beg = (int64_t *)p; g->allocs.push_back(p);
  g->n_long = (int32_t)lrow.size();
  ST_TRY(upload(lrow, &p, s)); g->long_row = (int32_t *)p; g->allocs.push_back(p);
  ST_TRY(upload(lslot0, &p, s)); g->long_slot0 = (int32_t *)p; g->allocs.push_back(p);
  ST_TRY(upload(lnslot, &p, s)); g->long_nslot = (int32_t *)p; g->allocs.push_back(p);
  HIP_TRY(hipStreamSynchronize(s));
  return SG2V_OK;
}

}  // namespace

extern "C" sg2v_status sg2v_graph_create(int64_t n, int64_t nnz, const int64_t *row_ptr,
                                         const int32_t *col_idx, const float *w, uint32_t flags,
                                         void *stream, sg2v_graph **out) {
  if (!out || !row_ptr || (nnz > 0 && !col_idx) || (flags & ~7u)) {
    set_error("sg2v_graph_create: null argument or unknown flag");
    return SG2V_EINVAL;
  }
  *out = nullptr;
  if (n < 1 || n >= ((int64_t)1 << 31) || nnz < 0) {
    set_error("sg2v_graph_create: n=%lld nnz=%lld out of range", (long long)n, (long long)nnz);
    return SG2V_ERANGE;
  }
  hipStream_t s = (hipStream_t)stream;
  const bool dev = flags & SG2V_GRAPH_DEVICE_PTRS;
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> ci;
  std::vector<float> wv;
  const bool relabel = flags & SG2V_GRAPH_RELABEL;
  if (dev) {
    HIP_TRY(hipMemcpyAsync(rp.data(), row_ptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if ((flags & SG2V_GRAPH_VALIDATE) || relabel) {
      ci.resize(nnz);
      if (nnz) HIP_TRY(hipMemcpyAsync(ci.data(), col_idx, nnz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    if (w) {
      wv.resize(nnz);
      if (nnz) HIP_TRY(hipMemcpyAsync(wv.data(), w, nnz * sizeof(float), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
  } else {
    std::memcpy(rp.data(), row_ptr, (n + 1) * sizeof(int64_t));
  }
  if (rp[0] != 0 || rp[n] != nnz) {
    set_error("sg2v_graph_create: row_ptr[0] must be 0 and row_ptr[n] = nnz");
    return SG2V_EGRAPH;
  }
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) {
      set_error("sg2v_graph_create: row_ptr decreases at row %lld", (long long)i);
      return SG2V_EGRAPH;
    }
  const int32_t *hc = dev ? ci.data() : col_idx;
  const float *hw = dev ? (w ? wv.data() : nullptr) : w;
  if (flags & SG2V_GRAPH_VALIDATE) {
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        if (hc[e] < 0 || hc[e] >= n || hc[e] == i || (e > rp[i] && hc[e] <= hc[e - 1])) {
          set_error("sg2v_graph_create: row %lld not sorted/unique/loop-free", (long long)i);
          return SG2V_EGRAPH;
        }
        // symmetric: (j, i) present with the same weight
        const int64_t j = hc[e];
        const int32_t *lo = hc + rp[j], *hi = hc + rp[j + 1];
        const int32_t *f = std::lower_bound(lo, hi, (int32_t)i);
        if (f == hi || *f != i || (hw && hw[f - hc] != hw[e])) {
          set_error("sg2v_graph_create: entry (%lld,%lld) has no symmetric partner", (long long)i,
                    (long long)j);
          return SG2V_EGRAPH;
        }
      }
    }
  }
  std::unique_ptr<sg2v_graph> g(new (std::nothrow) sg2v_graph());
  if (!g) return SG2V_ENOMEM;
  HIP_TRY(hipGetDevice(&g->device));
  g->n = n;
  g->nnz = nnz;
  double mw = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double sw = 0.0;
    if (hw)
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) sw += std::fabs((double)hw[e]);
    else
      sw = (double)(rp[i + 1] - rp[i]);
    mw = std::max(mw, sw);
  }
  g->max_wdeg = mw;
  if (relabel) {
    // Vertices by decreasing degree (ties in caller order), dealt round-robin
    // to the eight neighbour ranges of the XCD split: the vertex of degree
    // rank q goes to range q mod 8, at position q / 8 within it.  Each range
    // then holds an equal mix of hubs and low-degree vertices (equal work per
    // XCD), with its hubs first and together.  Rows are re-sorted.
    std::vector<int32_t> byd(n);
    std::iota(byd.begin(), byd.end(), 0);
    std::stable_sort(byd.begin(), byd.end(), [&](int32_t a, int32_t b) {
      return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
    });
    std::vector<int64_t> xb(kXsplit + 1, 0);
    for (int r = 0; r < kXsplit; ++r) xb[r + 1] = xb[r] + n / kXsplit + (r < n % kXsplit ? 1 : 0);
    std::vector<int32_t> orig(n);
    for (int64_t q = 0; q < n; ++q) orig[xb[q % kXsplit] + q / kXsplit] = byd[q];
    auto nw = std::make_shared<std::vector<int32_t>>(n);
    for (int64_t v = 0; v < n; ++v) (*nw)[orig[v]] = (int32_t)v;
    std::vector<int64_t> rp2(n + 1, 0);
    for (int64_t v = 0; v < n; ++v) rp2[v + 1] = rp2[v] + (rp[orig[v] + 1] - rp[orig[v]]);
    std::vector<int32_t> ci2(nnz);
    std::vector<float> w2(hw ? nnz : 0);
    std::vector<int64_t> eo(nnz);
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int th = 0; th < nth; ++th)
      pool.emplace_back([&, th]() {
        std::vector<std::pair<int32_t, int64_t>> row;
        for (int64_t v = th; v < n; v += nth) {
          const int64_t u = orig[v];
          row.clear();
          for (int64_t e = rp[u]; e < rp[u + 1]; ++e) row.push_back({(*nw)[hc[e]], e});
          std::sort(row.begin(), row.end());
          for (size_t q = 0; q < row.size(); ++q) {
            const int64_t e2 = rp2[v] + (int64_t)q;
            ci2[e2] = row[q].first;
            eo[e2] = row[q].second;
            if (hw) w2[e2] = hw[row[q].second];
          }
        }
      });
    for (auto &t : pool) t.join();
    g->relabelled = true;
    g->new_of = nw;
    g->owns = true;
    void *p;
    ST_TRY(upload(orig, &p, s)); g->orig_id = (int32_t *)p; g->allocs.push_back(p);
    if (nnz) { ST_TRY(upload(eo, &p, s)); g->entry_orig = (int64_t *)p; g->allocs.push_back(p); }
    ST_TRY(upload(xb, &p, s)); g->xbounds = (int64_t *)p; g->allocs.push_back(p);
    HIP_TRY(hipMalloc(&p, (n + 1) * sizeof(int64_t)));
    g->allocs.push_back(p);
    g->row_ptr = (int64_t *)p;
    HIP_TRY(hipMemcpyAsync(p, rp2.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMalloc(&p, std::max<int64_t>(nnz, 1) * sizeof(int32_t)));
    g->allocs.push_back(p);
    g->col_idx = (int32_t *)p;
    if (nnz) HIP_TRY(hipMemcpyAsync(p, ci2.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (hw) {
      HIP_TRY(hipMalloc(&p, std::max<int64_t>(nnz, 1) * sizeof(float)));
      g->allocs.push_back(p);
      g->w = (float *)p;
      if (nnz) HIP_TRY(hipMemcpyAsync(p, w2.data(), nnz * sizeof(float), hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));  // host arrays of this scope are read by the copies
    rp.swap(rp2);
  } else if (dev) {
    g->owns = false;
    g->row_ptr = (int64_t *)row_ptr;
    g->col_idx = (int32_t *)col_idx;
    g->w = (float *)w;
  } else {
    void *p;
    HIP_TRY(hipMalloc(&p, (n + 1) * sizeof(int64_t)));
    g->allocs.push_back(p);
    g->row_ptr = (int64_t *)p;
    HIP_TRY(hipMemcpyAsync(p, row_ptr, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMalloc(&p, std::max<int64_t>(nnz, 1) * sizeof(int32_t)));
    g->allocs.push_back(p);
    g->col_idx = (int32_t *)p;
    if (nnz) HIP_TRY(hipMemcpyAsync(p, col_idx, nnz * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (w) {
      HIP_TRY(hipMalloc(&p, std::max<int64_t>(nnz, 1) * sizeof(float)));
      g->allocs.push_back(p);
      g->w = (float *)p;
      if (nnz) HIP_TRY(hipMemcpyAsync(p, w, nnz * sizeof(float), hipMemcpyHostToDevice, s));
    }
  }
  ST_TRY(graph_tasks(g.get(), rp, s));
  // task units for every row-segment width at the default split threshold,
  // so that counts with the default threshold never upload them
  for (int G = 2; G <= 32; G *= 2) {
    UnitTable *U = nullptr;
    ST_TRY(build_units(g.get(), G, s, &U, kXsplitMin));
  }
  *out = g.release();
  return SG2V_OK;
}

void drop_batch_graphs(const sg2v_graph *g);

extern "C" void sg2v_graph_destroy(sg2v_graph *g) {
  drop_batch_graphs(g);
  delete g;
}

extern "C" sg2v_status sg2v_color(const sg2v_graph *g, int32_t k, uint64_t seed, int32_t first,
                                  int32_t n_colorings, void *stream, sg2v_colorings **out) {
  if (!g || !out || k < 1 || k > SG2V_KMAX || first < 0 || n_colorings < 1 ||
      (int64_t)first + n_colorings >= (1 << 24)) {
    set_error("sg2v_color: bad argument (k=%d first=%d count=%d)", k, first, n_colorings);
    return SG2V_EINVAL;
  }
  *out = nullptr;
  std::unique_ptr<sg2v_colorings> c(new (std::nothrow) sg2v_colorings());
  if (!c) return SG2V_ENOMEM;
  c->device = g->device;
  c->n = g->n;
  c->k = k;
  c->count = n_colorings;
  c->first = first;
  c->seed = seed;
  c->new_of = g->new_of;
  HIP_TRY(hipMalloc((void **)&c->d, g->n * n_colorings));
  {
    ProfScope ps(SG2V_K_COLOR, (double)g->n * n_colorings, (double)g->n * n_colorings,
                 (hipStream_t)stream);
    launch_color(c->d, g->n, k, seed, first, n_colorings, g->orig_id, (hipStream_t)stream);
  }
  HIP_TRY(hipGetLastError());
  *out = c.release();
  return SG2V_OK;
}

extern "C" void sg2v_colorings_destroy(sg2v_colorings *c) { delete c; }

extern "C" sg2v_status sg2v_colorings_download(const sg2v_colorings *c, uint8_t *out,
                                               void *stream) {
  if (!c || !out) {
    set_error("sg2v_colorings_download: null argument");
    return SG2V_EINVAL;
  }
  HIP_TRY(hipMemcpyAsync(out, c->d, c->n * c->count, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  if (c->new_of) {
    // stored order -> the caller's vertex order
    const std::vector<int32_t> &nw = *c->new_of;
    std::vector<uint8_t> row(c->n);
    for (int32_t j = 0; j < c->count; ++j) {
      uint8_t *o = out + (size_t)j * c->n;
      std::memcpy(row.data(), o, c->n);
      for (int64_t v = 0; v < c->n; ++v) o[v] = row[nw[v]];
    }
  }
  return SG2V_OK;
}

// ---------------------------------------------------------------------------
// count

namespace {

struct DevPlan {
  std::vector<int32_t *> pairs, drop;  // per node, device
  std::vector<int32_t *> tr_a, tr_p, add;
  std::vector<int32_t *> root_list;     // per template
  std::vector<uint32_t *> root_list16;
  std::vector<char *> cpr;  // colour-restricted tables per node
};

// pair-major copy ([q][col]) of a [col][np] x 2 table
std::vector<int32_t> pair_major(const std::vector<int32_t> &t, int64_t cols, int np) {
  std::vector<int32_t> o(t.size());
  for (int64_t C = 0; C < cols; ++C)
    for (int q = 0; q < np; ++q) {
      o[((size_t)q * cols + C) * 2 + 0] = t[((size_t)C * np + q) * 2 + 0];
      o[((size_t)q * cols + C) * 2 + 1] = t[((size_t)C * np + q) * 2 + 1];
    }
  return o;
}

// device copies of a plan's tables, one per device, kept with the plan
void fill_devplan(const Plan::DeviceTables &d, DevPlan *out) {
  const size_t nn = d.pairs.size();
  out->pairs.assign(nn, nullptr);
  out->drop.assign(nn, nullptr);
  out->tr_a.assign(nn, nullptr);
  out->tr_p.assign(nn, nullptr);
  out->add.assign(nn, nullptr);
  for (size_t i = 0; i < nn; ++i) {
    out->pairs[i] = (int32_t *)d.pairs[i];
    out->drop[i] = (int32_t *)d.drop[i];
    out->tr_a[i] = (int32_t *)d.tr_a[i];
    out->tr_p[i] = (int32_t *)d.tr_p[i];
    out->add[i] = (int32_t *)d.add[i];
  }
  out->root_list.clear();
  out->root_list16.clear();
  for (void *p : d.root_list) out->root_list.push_back((int32_t *)p);
  for (void *p : d.root_list16) out->root_list16.push_back((uint32_t *)p);
  out->cpr.assign(nn, nullptr);
  for (size_t i = 0; i < nn && i < d.cpr.size(); ++i) out->cpr[i] = (char *)d.cpr[i];
}

sg2v_status plan_device(const Plan &P, int device, hipStream_t s, DevPlan *out) {
  std::lock_guard<std::mutex> lk(P.mu);
  for (auto &d : P.dev)
    if (d.device == device) {
      fill_devplan(d, out);
      return SG2V_OK;
    }
  Plan::DeviceTables D;
  D.device = device;
  const size_t nn = P.nodes.size();
  D.pairs.assign(nn, nullptr);
  D.drop.assign(nn, nullptr);
  D.tr_a.assign(nn, nullptr);
  D.tr_p.assign(nn, nullptr);
  D.add.assign(nn, nullptr);
  for (size_t i = 0; i < nn; ++i) {
    const Node &nd = P.nodes[i];
    if (nd.size > 1) {
      // pair-major ([q][C]) so that consecutive columns are contiguous
      ST_TRY(upload(pair_major(nd.pairs, nd.cols, nd.np), &D.pairs[i], s));
      const int64_t ca = P.nodes[nd.active].cols, cp = P.nodes[nd.passive].cols;
      ST_TRY(upload(pair_major(nd.tr_a, ca, nd.np_ta), &D.tr_a[i], s));
      ST_TRY(upload(pair_major(nd.tr_p, cp, nd.np_tp), &D.tr_p[i], s));
    }
    if (!nd.drop.empty()) ST_TRY(upload(nd.drop, &D.drop[i], s));
    if (!nd.add.empty()) ST_TRY(upload(nd.add, &D.add[i], s));
  }
  D.cpr.assign(nn, nullptr);
  for (size_t i = 0; i < nn; ++i) {
    const Node &nd = P.nodes[i];
    if (nd.c_q == 0) continue;
    std::vector<uint32_t> blk;
    blk.insert(blk.end(), nd.ca.begin(), nd.ca.end());
    blk.insert(blk.end(), nd.cb.begin(), nd.cb.end());
    blk.insert(blk.end(), nd.co.begin(), nd.co.end());
    blk.insert(blk.end(), nd.cz.begin(), nd.cz.end());
    blk.insert(blk.end(), nd.cp.begin(), nd.cp.end());
    // inverse of co: output column -> its position among the columns holding c
    const size_t cu0 = blk.size();
    blk.resize(cu0 + (size_t)P.k * nd.cols, 0xFFFFFFFFu);
    for (int c = 0; c < P.k; ++c)
      for (int64_t u = 0; u < nd.c_u; ++u)
        blk[cu0 + (size_t)c * nd.cols + nd.co[(size_t)c * nd.c_u + u]] = (uint32_t)u;
    ST_TRY(upload(blk, &D.cpr[i], s));
  }
  D.root_list.assign(P.roots.size(), nullptr);
  D.root_list16.assign(P.roots.size(), nullptr);
  for (size_t r = 0; r < P.roots.size(); ++r) {
    const std::vector<int32_t> &rl = P.roots[r].list;
    if (rl.empty()) continue;
    ST_TRY(upload(rl, &D.root_list[r], s));
    bool fits = true;
    std::vector<uint32_t> l16(rl.size() / 2);
    for (size_t q = 0; q < l16.size(); ++q) {
      const int32_t x = rl[2 * q], y = rl[2 * q + 1];
      fits &= x >= 0 && x < 0xFFFF && y >= -1 && y < 0xFFFF;
      l16[q] = (uint32_t)x | ((uint32_t)(y < 0 ? 0xFFFF : y) << 16);
    }
    if (fits) ST_TRY(upload(l16, &D.root_list16[r], s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  P.dev.push_back(D);
  fill_devplan(P.dev.back(), out);
  return SG2V_OK;
}

enum StepKind { S_HIST, S_SPMM, S_EMA_SINGLE, S_EMA_GENERAL, S_ROOT };

struct Step {
  StepKind kind;
  int node;
};

// one table (M of a node or B of a passive node) within a pass
struct Tab {
  int64_t cols = 0;  // columns per colouring
  int64_t ld = 0;    // row stride in elements
  int64_t bytes = 0;
  int first = INT_MAX, last = -1;
  int64_t off = -1;
  void *p = nullptr;
  // FP32S bookkeeping (device)
  int *e = nullptr;
  unsigned *mx = nullptr;
  float *f = nullptr;
  int *E = nullptr;
};

struct PassPlan {
  std::vector<Step> steps;
  std::vector<Tab> M, B;  // indexed by node
  int64_t arena = 0;
  int64_t partial_bytes = 0;
  int64_t partial_off = 0;
  int64_t small_bytes = 0;
  int G = 8;
};

struct Workspace {
  DevBuf arena, small, partial, result, ovf, grad, bucket, nbrcol, xpart;
};

Workspace &workspace() {
  static thread_local std::map<int, std::unique_ptr<Workspace>> ws;
  int dev = 0;
  (void)hipGetDevice(&dev);
  auto &p = ws[dev];
  if (!p) p.reset(new Workspace());
  return *p;
}

// Lanes per row segment of the SpMM (chunk width G * N columns).  Automatic:
// 128-byte segments, or 256-byte segments (with the neighbour-range split of
// long tasks, below) on graphs whose 128-byte column chunk reaches 32 MB.
int pick_G(int dt, int64_t widest_cols_b, int64_t n) {
  sg2v_tuning_t tu = tuning();
  const int N = dt == DT_F32 ? 4 : 2;
  int G = 8;  // 128-byte row segments
  if (tu.spmm_width > 0) G = std::max(2, std::min(32, tu.spmm_width / N));
  else if (large_graph(n) && !(tu.flags & SG2V_TUNE_NO_XSPLIT)) G = 16;
  // narrow tables: do not read far past the last column
  while (G > 2 && (int64_t)G * N / 2 >= widest_cols_b) G /= 2;
  int p2 = 2;
  while (p2 * 2 <= G) p2 *= 2;
  return p2;
}

struct PassOpts {
  std::vector<std::pair<int, int>> keep;  // (node, 0: M / 1: B) kept to the end of the pass
  bool no_fuse = false;                   // materialise every non-root table
};

// Build the step list and table lifetimes for a pass over b colourings.
void build_pass(const Plan &P, int64_t n, int b, int dt, int G, int64_t n_slots, PassPlan &pp,
                const PassOpts &opt) {
  const int es = esize_of(dt);
  const int N = dt == DT_F32 ? 4 : 2;
  const int64_t align = std::max<int64_t>(128 / es, (int64_t)G * N);
  const size_t nn = P.nodes.size();
  pp.steps.clear();
  pp.M.assign(nn, Tab());
  pp.B.assign(nn, Tab());
  pp.G = G;
  std::vector<char> haveB(nn, 0);
  auto needB = [&](int p) {
    if (haveB[p]) return;
    haveB[p] = 1;
    pp.steps.push_back({P.nodes[p].size == 1 ? S_HIST : S_SPMM, p});
  };
  for (size_t s = 0; s < nn; ++s) {
    const Node &nd = P.nodes[s];
    if (nd.size == 1) continue;
    const int ri = P.root_index[s];
    if (ri >= 0) {
      if (P.roots[ri].kind == ROOT_FUSED) needB(P.nodes[nd.active].passive);
      needB(nd.passive);
      pp.steps.push_back({S_ROOT, (int)s});
      continue;
    }
    bool kept = false;
    for (auto &kp : opt.keep) kept |= kp.first == (int)s && kp.second == 0;
    if (P.fused[s] && !opt.no_fuse && !kept) continue;
    needB(nd.passive);
    pp.steps.push_back({P.nodes[nd.active].size == 1 ? S_EMA_SINGLE : S_EMA_GENERAL, (int)s});
  }
  // lifetimes
  auto touch = [](Tab &t, int step) {
    t.first = std::min(t.first, step);
    t.last = std::max(t.last, step);
  };
  for (int x = 0; x < (int)pp.steps.size(); ++x) {
    const Step &st = pp.steps[x];
    const Node &nd = P.nodes[st.node];
    switch (st.kind) {
      case S_HIST: touch(pp.B[st.node], x); break;
      case S_SPMM: touch(pp.M[st.node], x); touch(pp.B[st.node], x); break;
      case S_EMA_SINGLE: touch(pp.B[nd.passive], x); touch(pp.M[st.node], x); break;
      case S_EMA_GENERAL:
        touch(pp.M[nd.active], x); touch(pp.B[nd.passive], x); touch(pp.M[st.node], x);
        break;
      case S_ROOT:
        if (P.roots[P.root_index[st.node]].kind == ROOT_FUSED) touch(pp.B[P.nodes[nd.active].passive], x);
        if (P.roots[P.root_index[st.node]].kind == ROOT_GENERAL) touch(pp.M[nd.active], x);
        touch(pp.B[nd.passive], x);
        break;
    }
  }
  for (auto &kp : opt.keep) {
    Tab &t = kp.second == 0 ? pp.M[kp.first] : pp.B[kp.first];
    if (t.last >= 0) t.last = (int)pp.steps.size();
  }
  // sizes
  std::vector<Tab *> all;
  for (size_t s = 0; s < nn; ++s) {
    for (int kind = 0; kind < 2; ++kind) {
      Tab &t = kind == 0 ? pp.M[s] : pp.B[s];
      if (t.last < 0) continue;
      t.cols = P.nodes[s].size == 1 ? P.k : P.nodes[s].cols;
      t.ld = round_up(t.cols * b, align);
      t.bytes = round_up(n * t.ld * es, 256);
      all.push_back(&t);
    }
  }
  // greedy placement: largest first, lowest offset free over the lifetime
  std::sort(all.begin(), all.end(), [](Tab *a, Tab *c) { return a->bytes > c->bytes; });
  std::vector<Tab *> placed;
  int64_t top = 0;
  for (Tab *t : all) {
    std::vector<std::pair<int64_t, int64_t>> busy;
    for (Tab *q : placed)
      if (!(q->last < t->first || t->last < q->first)) busy.push_back({q->off, q->off + q->bytes});
    std::sort(busy.begin(), busy.end());
    int64_t off = 0;
    for (auto &bz : busy) {
      if (off + t->bytes <= bz.first) break;
      off = std::max(off, bz.second);
    }
    t->off = off;
    top = std::max(top, off + t->bytes);
    placed.push_back(t);
  }
  int64_t widest = 0;
  for (size_t s = 0; s < nn; ++s)
    if (pp.B[s].last >= 0) widest = std::max(widest, pp.B[s].ld);  // the histogram too
  pp.partial_off = top;
  pp.partial_bytes = round_up(std::max<int64_t>(n_slots, 1) * std::max<int64_t>(widest, 1) * es, 256);
  pp.arena = top + pp.partial_bytes;
  // small FP32S arrays: e, mx, f per column, E per colouring
  int64_t small = 0;
  for (Tab *t : all) small += round_up(t->cols * b * 12 + b * 4, 256);
  pp.small_bytes = small + 256;
}

}  // namespace

namespace sg2v {
int64_t graph_vertices(const sg2v_graph *g) { return g ? g->n : 0; }

int64_t pass_bytes_per_vertex(const Plan &P, int fp32) {
  const int dt = fp32 ? DT_F32 : DT_F64;
  const int64_t n = (int64_t)1 << 20;
  int64_t widest = 1;
  for (auto &nd : P.nodes)
    if (nd.n_passive_uses > 0) widest = std::max(widest, nd.size == 1 ? (int64_t)P.k : nd.cols);
  PassPlan pp;
  build_pass(P, n, 1, dt, pick_G(dt, widest, n), 0, pp, PassOpts());
  return (pp.arena + n - 1) / n;
}
}  // namespace sg2v

namespace {

struct Ctx {
  const Plan *P;
  sg2v_graph *g;
  const sg2v_colorings *c;
  int dt, es, b, j0;
  hipStream_t s;
  DevPlan dp;
  PassPlan pp;
  Workspace *ws;
  int *ovf;
  int cu_count = 256;
  size_t lds_max = 65536;
  int bucket_j0 = -1;  // pass whose colour buckets are in ws->bucket
  int bucket_b = 0;
  int nbr_j0 = -1;     // pass whose neighbour colours are in ws->nbrcol
  int nbr_b = 0;
  int64_t res_stride = 0;  // results per template (plans of several templates)
  // sg2v_count_noalloc: colour-skip masks copied into the scratch area
  std::map<std::tuple<int, int, int>, void *> tmp_masks;
  std::vector<std::vector<uint32_t>> tmp_host;
};

sg2v_status bind_tables(Ctx &x) {
  char *base = (char *)x.ws->arena.p;
  char *small = (char *)x.ws->small.p;
  int64_t so = 0;
  for (size_t s = 0; s < x.pp.M.size(); ++s) {
    for (int kind = 0; kind < 2; ++kind) {
      Tab &t = kind == 0 ? x.pp.M[s] : x.pp.B[s];
      if (t.last < 0) continue;
      t.p = base + t.off;
      if (x.dt == DT_F32) {
        const int64_t nc = t.cols * x.b;
        t.e = (int *)(small + so);
        t.mx = (unsigned *)(small + so + nc * 4);
        t.f = (float *)(small + so + nc * 8);
        t.E = (int *)(small + so + nc * 12);
        so += round_up(nc * 12 + x.b * 4, 256);
      }
    }
  }
  return SG2V_OK;
}

// FP32S: column maxima of a freshly produced table -> common frame per colouring
void norm(Ctx &x, Tab &t) {
  if (x.dt != DT_F32) return;
  launch_norm_prep(t.e, t.mx, (int)t.cols, x.b, t.f, t.E, x.s);
}

sg2v_status step_hist(Ctx &x, int node) {
  Tab &H = x.pp.B[node];
  HistArgs a{};
  a.row_ptr = x.g->row_ptr;
  a.col_idx = x.g->col_idx;
  a.w = x.g->w;
  a.colors = x.c->d;
  a.n = x.g->n;
  a.k = x.P->k;
  a.j0 = x.j0;
  a.b = x.b;
  a.H = H.p;
  a.ldh = H.ld;
  a.task_row = x.g->task_row;
  a.task_beg = x.g->task_beg;
  a.task_len = x.g->task_len;
  a.task_slot = x.g->task_slot;
  a.n_tasks = x.g->n_tasks;
  a.partial = (char *)x.ws->arena.p + x.pp.partial_off;
  const int64_t blocks = std::min<int64_t>((x.g->n_tasks + 3) / 4, 8192);  // 4 waves per block
  {
    const double nnz = (double)x.g->nnz;
    ProfScope ps(SG2V_K_HIST,
                 nnz * (4.0 + (x.g->w ? 4.0 : 0.0) + x.b) + (double)x.g->n * (8.0 + x.b * x.P->k * x.es),
                 nnz * x.b, x.s);
    launch_hist(x.dt, a, (int)std::max<int64_t>(blocks, 1), x.s);
  }
  if (x.g->n_long > 0) {
    // segments of long rows, summed in slot order
    CombineArgs cb{};
    cb.partial = a.partial;
    cb.B = H.p;
    cb.ld = H.ld;
    cb.ncols_valid = H.cols * x.b;
    cb.long_row = x.g->long_row;
    cb.long_slot0 = x.g->long_slot0;
    cb.long_nslot = x.g->long_nslot;
    cb.n_long = x.g->n_long;
    cb.mx = nullptr;
    cb.ovf = x.ovf;
    cb.accumulate = 0;
    ProfScope ps(SG2V_K_SPMM_COMBINE, (double)(x.g->n_slots + x.g->n_long) * H.ld * x.es,
                 (double)x.g->n_slots * H.ld, x.s);
    launch_spmm_combine(x.dt, cb, x.s);
  }
  if (x.dt == DT_U64) launch_zero_pad(x.dt, H.p, x.g->n, H.ld, H.cols * x.b, x.s);
  if (x.dt == DT_F32) {
    const int64_t nc = H.cols * x.b;
    launch_fill_u32((unsigned *)H.e, nc, 0u, x.s);
    float mw = (float)std::max(1.0, x.g->max_wdeg);
    unsigned bits;
    std::memcpy(&bits, &mw, 4);
    launch_fill_u32(H.mx, nc, bits, x.s);
    norm(x, H);
  }
  return SG2V_OK;
}

// Per chunk of W columns of a passive node's table (b colourings side by
// side): the colouring block holding the whole chunk (-1 if it spans two
// blocks or padding), and the union and intersection of its colour sets.
sg2v_status chunk_masks(Ctx &x, int node, int W, const int32_t **jb, const uint32_t **un,
                        const uint32_t **in) {
  const Plan &P = *x.P;
  std::lock_guard<std::mutex> lk(P.mu);
  Plan::DeviceTables *D = nullptr;
  for (auto &d : P.dev)
    if (d.device == x.g->device) D = &d;
  if (!D) {
    set_error("sg2v_count: plan tables missing on device %d", x.g->device);
    return SG2V_EINVAL;
  }
  const Node &nd = P.nodes[node];
  const int64_t C = nd.cols, nc = C * x.b, nch = (nc + W - 1) / W;
  auto key = std::make_tuple(node, x.b, W);
  auto it = D->chunks.find(key);
  const void *found = it != D->chunks.end() ? it->second : nullptr;
  if (!found) {
    auto tk = x.tmp_masks.find(key);
    if (tk != x.tmp_masks.end()) found = tk->second;
  }
  if (!found) {
    std::vector<uint32_t> h((size_t)nch * 3);
    for (int64_t ch = 0; ch < nch; ++ch) {
      const int64_t c0 = ch * W, c1 = std::min<int64_t>(c0 + W, nc);
      const int64_t b0 = c0 / C, b1 = (c1 - 1) / C;
      uint32_t u = 0, i = ~0u;
      for (int64_t c = c0; c < c1; ++c) {
        const uint32_t m = colex_unrank(c % C, nd.size, P.k);
        u |= m;
        i &= m;
      }
      const bool one = b0 == b1 && c1 - c0 == W;
      h[ch] = one ? (uint32_t)b0 : 0xFFFFFFFFu;
      h[nch + ch] = u;
      h[2 * nch + ch] = i;
    }
    void *d = nullptr;
    if (t_noalloc && x.ws->arena.cv) {
      // into the scratch area for this call; the host copy lives until the call ends
      Carver *cv = x.ws->arena.cv;
      const size_t bytes = (h.size() * 4 + 255) / 256 * 256;
      if (cv->top + bytes > cv->cap) {
        cv->exhausted = true;
        set_error("sg2v_count_noalloc: the count needs more than the %zu-byte scratch area", cv->cap);
        return SG2V_ENOMEM;
      }
      d = cv->base + cv->top;
      cv->top += bytes;
      HIP_TRY(hipMemcpyAsync(d, h.data(), h.size() * 4, hipMemcpyHostToDevice, x.s));
      x.tmp_host.push_back(std::move(h));
      x.tmp_masks[key] = d;
    } else {
      ST_TRY(upload(h, &d, x.s));
      HIP_TRY(hipStreamSynchronize(x.s));
      D->chunks.emplace(key, d);
    }
    found = d;
  }
  const uint32_t *base = (const uint32_t *)found;
  *jb = (const int32_t *)base;
  *un = base + nch;
  *in = base + 2 * nch;
  return SG2V_OK;
}

// Neighbour-range split of the SpMM's long tasks: used when one column chunk
// of the gathered table is much larger than an XCD's L2.  Returns the chunk
// group size (0: no split) after making sure the split offsets and the
// partial-row buffer exist.
sg2v_status xsplit_setup(Ctx &x, const UnitTable *U, int64_t nc, int W, int64_t *group) {
  *group = 0;
  const sg2v_tuning_t tu = tuning();
  const int fl = tu.flags;
  if ((fl & SG2V_TUNE_NO_XSPLIT) || U->x_units == 0) return SG2V_OK;
  // automatic: large graphs whose long tasks hold at least half the entries
  const bool wanted = (fl & SG2V_TUNE_XSPLIT) ||
                      (tu.spmm_width == 0 && large_graph(x.g->n) && x.g->long_share >= 0.5);
  if (!(fl & SG2V_TUNE_FORCE_XSPLIT) && (!wanted || (double)x.g->n * W * x.es < 32.0 * (1 << 20)))
    return SG2V_OK;
  sg2v_graph *g = x.g;
  if (!g->tsplit && t_noalloc) return SG2V_OK;  // offsets never built: no split (same counts)
  if (!g->tsplit) {
    HIP_TRY(hipMalloc((void **)&g->tsplit, (size_t)g->n_tasks * (kXsplit + 1) * sizeof(uint16_t)));
    launch_task_split(g->col_idx, g->task_beg, g->task_len, g->n_tasks, g->n, kXsplit, g->xbounds,
                      g->tsplit, x.s);
    HIP_TRY(hipGetLastError());
  }
  const int64_t chunks = (nc + W - 1) / W;
  const double per_chunk = (double)kXsplit * U->x_tasks * W * x.es;
  int64_t cap = (int64_t)65535;
  if (tu.xsplit_group > 0) cap = std::min<int64_t>(cap, tu.xsplit_group);
  const int64_t gch = std::max<int64_t>(
      1, std::min<int64_t>({chunks, cap, (int64_t)(kXpartBytes / per_chunk)}));
  ST_TRY(x.ws->xpart.ensure((size_t)(per_chunk * gch) + 256));
  *group = gch;
  return SG2V_OK;
}

sg2v_status step_spmm(Ctx &x, int node) {
  Tab &Mp = x.pp.M[node];
  Tab &B = x.pp.B[node];
  UnitTable *U = nullptr;
  ST_TRY(build_units(x.g, x.pp.G, x.s, &U));
  const int N = x.dt == DT_F32 ? 4 : 2;
  const int W = x.pp.G * N;
  const int64_t nc = Mp.cols * x.b;
  SpmmArgs a{};
  a.col_idx = x.g->col_idx;
  a.w = x.g->w;
  a.task_row = x.g->task_row;
  a.task_beg = x.g->task_beg;
  a.task_len = x.g->task_len;
  a.task_slot = x.g->task_slot;
  a.unit_task = U->unit_task;
  a.unit_rpw = U->unit_rpw;
  a.unit_ntask = U->unit_ntask;
  a.n_units = U->n_units;
  a.M = Mp.p;
  a.ldm = Mp.ld;
  a.B = B.p;
  a.ldb = B.ld;
  a.partial = (char *)x.ws->arena.p + x.pp.partial_off;
  a.ncols_valid = nc;
  a.mx = x.dt == DT_F32 ? B.mx : nullptr;
  a.ovf = x.ovf;
  a.accumulate = 0;
  a.chunk_jb = nullptr;
  a.chunk_union = a.chunk_inter = nullptr;
  a.colors = x.c->d;
  a.j0 = x.j0;
  a.n = x.g->n;
  a.nbr_col = nullptr;
  a.nnz = x.g->nnz;
  if (!(tuning().flags & SG2V_TUNE_NO_COLOR_SKIP)) {
    ST_TRY(chunk_masks(x, node, W, &a.chunk_jb, &a.chunk_union, &a.chunk_inter));
    if (x.nbr_j0 != x.j0 || x.nbr_b != x.b) {
      launch_nbr_colors(x.g->col_idx, x.g->nnz, x.c->d, x.g->n, x.j0, x.b, (uint8_t *)x.ws->nbrcol.p, x.s);
      x.nbr_j0 = x.j0;
      x.nbr_b = x.b;
    }
    a.nbr_col = (const uint8_t *)x.ws->nbrcol.p;
  }
  if (x.dt == DT_F32) launch_fill_u32(B.mx, nc, 0u, x.s);
  const int64_t chunks = (nc + W - 1) / W;
  // gathers in flight per stream: 8 for long neighbour lists (mean degree
  // >= 64), else 4 (fewer registers, more waves)
  const int fl = tuning().flags;
  const int unroll = (fl & SG2V_TUNE_SPMM_UNROLL4)   ? 4
                     : (fl & SG2V_TUNE_SPMM_UNROLL8) ? 8
                     : (x.g->nnz >= 64 * x.g->n)     ? 8
                                                     : 4;
  a.chunk0 = 0;
  a.xsplit = 0;
  a.xunits = 0;
  a.tsplit = nullptr;
  a.n_tasks = 0;
  a.ldp = 0;
  a.partial8 = nullptr;
  int64_t gch = 0;
  const double n = (double)x.g->n, nnz = (double)x.g->nnz;
  const double bytes = 2.0 * n * (double)nc * x.es +
                       (double)chunks * (nnz * (4.0 + (x.g->w ? 4.0 : 0.0)) + 20.0 * x.g->n_tasks);
  sg2v_graph::Panels *PN = nullptr;
  if (fl & SG2V_TUNE_SPMM_PANEL) {
    // a noalloc call on a graph whose panels were never built runs k_spmm instead
    const sg2v_status ps = build_panels(x.g, x.s, &PN);
    if (ps != SG2V_OK && !t_noalloc) return ps;
  }
  if (PN) {
    SpmmPanelArgs pa{};
    pa.p_task0 = PN->task0;
    pa.p_ntask = PN->ntask;
    pa.p_beg = PN->beg;
    pa.n_panels = PN->n;
    pa.e_col = PN->col;
    pa.e_loc = PN->loc;
    pa.e_w = PN->w;
    pa.task_row = x.g->task_row;
    pa.task_slot = x.g->task_slot;
    pa.M = a.M;
    pa.ldm = a.ldm;
    pa.B = a.B;
    pa.ldb = a.ldb;
    pa.partial = a.partial;
    pa.ncols_valid = nc;
    pa.mx = a.mx;
    pa.ovf = a.ovf;
    pa.accumulate = 0;
    pa.chunk_jb = a.chunk_jb;
    pa.chunk_union = a.chunk_union;
    pa.chunk_inter = a.chunk_inter;
    pa.colors = a.colors;
    pa.j0 = a.j0;
    pa.n = a.n;
    const int64_t per_launch = fl_launch_chunks();
    const int64_t gx = std::max<int64_t>(1, std::min<int64_t>((PN->n + 3) / 4,  // four waves per block
                                                              kSpmmBlocks));
    for (int64_t c0 = 0; c0 < chunks; c0 += per_launch) {
      const int64_t gc = std::min<int64_t>(per_launch, chunks - c0);
      const double frac = (double)gc / (double)chunks;
      pa.chunk0 = c0;
      ProfScope ps(SG2V_K_SPMM, bytes * frac, nnz * (double)nc * frac, x.s);
      if (launch_spmm_panel(x.dt, pa, x.pp.G, dim3((unsigned)gx, (unsigned)gc), x.s)) {
        set_error("sg2v_count: no panel SpMM variant for G=%d", x.pp.G);
        return SG2V_EINVAL;
      }
    }
  } else {
  ST_TRY(xsplit_setup(x, U, nc, W, &gch));
  if (gch == 0) {
    // all chunks in one launch (grid.y is at most 65535: groups beyond that)
    const int64_t per_launch = fl_launch_chunks();
    for (int64_t c0 = 0; c0 < chunks; c0 += per_launch) {
      const int64_t gc = std::min<int64_t>(per_launch, chunks - c0);
      const double frac = (double)gc / (double)chunks;
      a.chunk0 = c0;
      dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(U->n_units, kSpmmBlocks)), (unsigned)gc);
      ProfScope ps(SG2V_K_SPMM, bytes * frac, nnz * (double)nc * frac, x.s);
      if (launch_spmm(x.dt, a, x.pp.G, unroll, grid, x.s)) {
        set_error("sg2v_count: no SpMM variant for G=%d", x.pp.G);
        return SG2V_EINVAL;
      }
    }
    a.chunk0 = 0;
  } else {
    // long tasks split over the XCDs' neighbour ranges, chunk group by group
    unsigned *mx = a.mx;
    a.mx = nullptr;  // column maxima of split tasks come from the combine
    a.xsplit = kXsplit;
    a.xunits = U->x_units;
    a.tsplit = x.g->tsplit;
    a.n_tasks = U->x_tasks;
    a.partial8 = x.ws->xpart.p;
    const int64_t gx =
        std::max<int64_t>(kXsplit, std::min<int64_t>(U->n_units * kXsplit, kXsplitBlocks) / kXsplit * kXsplit);
    for (int64_t c0 = 0; c0 < chunks; c0 += gch) {
      const int64_t gc = std::min(gch, chunks - c0);
      const double frac = (double)gc / (double)chunks;
      a.chunk0 = c0;
      a.ldp = gc * W;
      a.mx = mx;  // whole (unsplit) tasks still fold their maxima in the kernel
      {
        ProfScope ps(SG2V_K_SPMM, bytes * frac, nnz * (double)nc * frac, x.s);
        if (launch_spmm(x.dt, a, x.pp.G, unroll, dim3((unsigned)gx, (unsigned)gc), x.s)) {
          set_error("sg2v_count: no SpMM variant for G=%d", x.pp.G);
          return SG2V_EINVAL;
        }
      }
      XsplitCombineArgs xc{};
      xc.partial8 = a.partial8;
      xc.xsplit = kXsplit;
      xc.n_tasks = a.n_tasks;
      xc.ldp = a.ldp;
      xc.col_first = c0 * W;
      xc.task_row = x.g->task_row;
      xc.task_slot = x.g->task_slot;
      xc.B = B.p;
      xc.ldb = B.ld;
      xc.hub = a.partial;
      xc.ncols_valid = nc;
      xc.mx = mx;
      xc.ovf = x.ovf;
      xc.accumulate = 0;
      ProfScope pc(SG2V_K_SPMM_COMBINE, 2.0 * kXsplit * (double)a.n_tasks * a.ldp * x.es,
                   (double)a.n_tasks * a.ldp, x.s);
      launch_xsplit_combine(x.dt, xc, x.s);
    }
    a.mx = mx;
  }
  }  // row panels or k_spmm
  CombineArgs cb{};
  cb.partial = a.partial;
  cb.B = B.p;
  cb.ld = B.ld;
  cb.ncols_valid = nc;
  cb.long_row = x.g->long_row;
  cb.long_slot0 = x.g->long_slot0;
  cb.long_nslot = x.g->long_nslot;
  cb.n_long = x.g->n_long;
  cb.mx = a.mx;
  cb.ovf = x.ovf;
  cb.accumulate = 0;
  if (x.g->n_long > 0) {
    ProfScope ps(SG2V_K_SPMM_COMBINE, (double)(x.g->n_slots + x.g->n_long) * nc * x.es,
                 (double)x.g->n_slots * nc, x.s);
    launch_spmm_combine(x.dt, cb, x.s);
  }
  if (x.dt == DT_F32) {
    launch_copy_i32(Mp.e, B.e, nc, x.s);
    norm(x, B);
  }
  return SG2V_OK;
}

// Multiply-add over pairs (Alg. 3 stage 2) with rows staged in LDS when they
// fit: picks the rows per tile and the grid, then launches k_ema_general.
sg2v_status launch_general(Ctx &x, EmaArgs &a) {
  const bool sc = x.dt == DT_F32;
  const size_t lmx = (sc && a.mx) ? (size_t)a.Cs * 4 : 0;
  sg2v_tuning_t tu = tuning();
  const size_t budget = std::min<size_t>(x.lds_max, 64 * 1024);
  const size_t rowb = (size_t)((a.Ca | 1) + (a.Cb | 1)) * x.es;
  int R = 16;
  if (tu.ema_rows > 0) R = tu.ema_rows;
  while (R > 1 && R * rowb + lmx > budget) R /= 2;
  const bool stage = R * rowb + lmx <= budget;
  if (!stage) R = 4;
  const size_t lds = (stage ? R * rowb : 0) + lmx;
  const int64_t ntiles = (x.g->n + R - 1) / R;
  const int64_t per_cu = std::max<int64_t>(1, (int64_t)(x.lds_max / std::max<size_t>(lds, 1)));
  const int64_t blocks =
      std::min<int64_t>(ntiles, (int64_t)x.cu_count * std::min<int64_t>(per_cu, 8));
  dim3 grid((unsigned)std::max<int64_t>(blocks, 1), (unsigned)x.b);
  if (launch_ema_general(x.dt, a, R, stage, grid, lds, x.s)) {
    set_error("sg2v_count: no eMA variant for R=%d", R);
    return SG2V_EINVAL;
  }
  return SG2V_OK;
}

// Colour-restricted multiply-add of a general split: vertices are grouped by
// colour once per pass, then k_ema_colour works on tiles of one colour.
sg2v_status ema_colour(Ctx &x, int node, const EmaArgs &g, bool *done) {
  const Node &nd = x.P->nodes[node];
  *done = false;
  const int k = x.P->k;
  int32_t *counts = (int32_t *)x.ws->bucket.p;
  int32_t *cursor = counts + (size_t)x.b * 32;
  int32_t *perm = cursor + (size_t)x.b * 32;
  if (x.bucket_j0 != x.j0 || x.bucket_b != x.b) {
    launch_bucket(x.c->d, x.g->n, x.j0, x.b, k, counts, cursor, perm, x.s);
    x.bucket_j0 = x.j0;
    x.bucket_b = x.b;
  }
  EmaColourArgs a{};
  a.Ma = g.Ma;
  a.lda = g.lda;
  a.Ca = g.Ca;
  a.B = g.B;
  a.ldb = g.ldb;
  a.Cb = g.Cb;
  a.Ms = g.Ms;
  a.lds = g.lds;
  a.Cs = g.Cs;
  const int32_t *base = (const int32_t *)x.dp.cpr[node];
  a.ca = base;
  a.cb = a.ca + (size_t)k * nd.c_sa;
  a.co = a.cb + (size_t)k * nd.c_sb;
  a.cz = a.co + (size_t)k * nd.c_u;
  a.cp = (const uint32_t *)(a.cz + (size_t)k * nd.c_z);
  a.cu = (const int32_t *)(a.cp + (size_t)k * nd.c_q * nd.c_u);
  a.Sa = (int32_t)nd.c_sa;
  a.Sb = (int32_t)nd.c_sb;
  a.U = (int32_t)nd.c_u;
  a.Z = (int32_t)nd.c_z;
  a.Q = nd.c_q;
  a.k = k;
  a.perm = perm;
  a.counts = counts;
  a.n = x.g->n;
  a.fa = g.fa;
  a.fb = g.fb;
  a.Ea = g.Ea;
  a.Eb = g.Eb;
  a.mx = g.mx;
  a.es = g.es;
  a.ovf = g.ovf;
  const bool sc = x.dt == DT_F32;
  const size_t lmx = (sc && g.mx) ? (size_t)round_up(nd.cols, 16) : 0;  // one byte per output column
  const size_t budget = std::min<size_t>(x.lds_max, 80 * 1024);
  // staged columns hold R rows plus one 16-byte vector of padding
  const int Nv = 16 / (int)x.es;
  auto lds_for = [&](int R) { return (size_t)(a.Sa + 1 + a.Sb) * (R + Nv) * x.es + lmx; };
  sg2v_tuning_t tu = tuning();
  int R = 16;
  if (tu.ema_rows > 0)
    while (R > 4 && R > tu.ema_rows) R /= 2;  // a power of two, 4..16
  while (R > 4 && lds_for(R) > budget) R /= 2;
  if (R < 4) R = 4;
  const size_t lds = lds_for(R);
  if (lds > x.lds_max) return SG2V_OK;  // staging does not fit: the general kernel runs
  // wide outputs: 512 threads share each staged tile (each still has several
  // output columns); narrow ones (256 columns or fewer) take 128 threads and
  // twice the blocks per CU, so that few threads idle
  const int nt = nd.cols >= 4 * 512 ? 512 : nd.cols <= 256 ? 128 : 256;
  const int64_t ntiles = x.g->n / R + k;
  const int64_t per_cu = std::max<int64_t>(1, (int64_t)(x.lds_max / lds));
  const int64_t blocks =
      std::min<int64_t>(ntiles, (int64_t)x.cu_count * std::min<int64_t>(per_cu, 8 * 256 / nt));
  ProfScope ps(SG2V_K_EMA_GENERAL,
               (double)x.g->n * x.b * (double)(nd.cols + nd.c_sa + nd.c_sb) * x.es,
               (double)x.g->n * x.b * (double)nd.c_u * nd.c_q, x.s);
  if (launch_ema_colour(x.dt, a, R, nt, dim3((unsigned)std::max<int64_t>(1, blocks), (unsigned)x.b), lds, x.s)) {
    set_error("sg2v_count: no colour-restricted eMA variant for R=%d", R);
    return SG2V_EINVAL;
  }
  *done = true;
  return SG2V_OK;
}

sg2v_status step_ema(Ctx &x, int node, bool single) {
  const Plan &P = *x.P;
  const Node &nd = P.nodes[node];
  Tab &Ms = x.pp.M[node];
  Tab &Bt = x.pp.B[nd.passive];
  EmaArgs a{};
  std::memset(&a, 0, sizeof(a));
  a.B = Bt.p;
  a.ldb = Bt.ld;
  a.Ms = Ms.p;
  a.lds = Ms.ld;
  a.pairs = x.dp.pairs[node];
  a.drop = x.dp.drop[node];
  a.np = nd.np;
  a.Cs = (int32_t)nd.cols;
  a.Cb = (int32_t)Bt.cols;
  a.n = x.g->n;
  a.colors = x.c->d;
  a.j0 = x.j0;
  a.ovf = x.ovf;
  const bool sc = x.dt == DT_F32;
  if (sc) {
    a.fb = Bt.f;
    a.Eb = Bt.E;
    a.mx = Ms.mx;
    a.es = Ms.e;
    launch_fill_u32(Ms.mx, Ms.cols * x.b, 0u, x.s);
  }
  // FP32S tables too wide for per-block column maxima in LDS get them from a
  // pass over the finished table instead
  // (the single-vertex kernel keeps all b colourings of the pass in a block)
  const size_t lmx_cols = (size_t)nd.cols * (single ? x.b : 1);
  const bool wide = sc && !single && lmx_cols * 4 > 32 * 1024;
  if (wide || single) a.mx = nullptr;  // single-vertex active: bounded from B's maxima below
  const size_t lmx = (sc && !wide && !single) ? lmx_cols * 4 : 0;
  if (single) {
    a.nb = x.b;
    // the drop table in LDS while it leaves room for several blocks per CU
    if ((int64_t)P.k * nd.cols * 2 <= 16 * 1024 && Bt.cols < 0xFFFF) a.kc = P.k;
    const int64_t rows = std::max<int64_t>(1, 8192 / ((int64_t)nd.cols * x.b));
    const int64_t tiles = (x.g->n + rows - 1) / rows;
    dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)x.cu_count * 8)), 1);
    ProfScope ps(SG2V_K_EMA_SINGLE, (double)x.g->n * x.b * (double)(nd.cols + Bt.cols) * x.es,
                 (double)x.g->n * x.b * (double)nd.cols, x.s);
    launch_ema_single(x.dt, a, grid, lmx, x.s);
    if (sc)
      launch_single_bound(a.drop, P.k, a.Cs, a.Cb, x.b, Bt.mx, Bt.f, Ms.mx, x.s);
  } else {
    Tab &Ma = x.pp.M[nd.active];
    a.Ma = Ma.p;
    a.lda = Ma.ld;
    a.Ca = (int32_t)Ma.cols;
    if (sc) {
      a.fa = Ma.f;
      a.Ea = Ma.E;
    }
    bool done = false;
    if (nd.c_q > 0 && x.dp.cpr[node] && !(tuning().flags & SG2V_TUNE_NO_COLOR_EMA))
      ST_TRY(ema_colour(x, node, a, &done));
    if (!done) {
      ProfScope ps(SG2V_K_EMA_GENERAL,
                   (double)x.g->n * x.b * (double)(nd.cols + Ma.cols + Bt.cols) * x.es,
                   (double)x.g->n * x.b * (double)nd.cols * nd.np, x.s);
      ST_TRY(launch_general(x, a));
    }
  }
  if (wide) launch_colmax((const float *)Ms.p, x.g->n, Ms.ld, Ms.cols * x.b, Ms.mx, x.s);
  if (x.dt == DT_U64) launch_zero_pad(x.dt, Ms.p, x.g->n, Ms.ld, Ms.cols * x.b, x.s);
  norm(x, Ms);
  return SG2V_OK;
}

// result: per-colouring raw colourful sums (double or uint64) for this pass
// go to result + j0; FP32S frame exponents to Eout + j0.
sg2v_status step_root(Ctx &x, int node, void *result, int *Eout);

}  // namespace


namespace {

sg2v_status step_root(Ctx &x, int node, void *result, int *Eout) {
  const Plan &P = *x.P;
  const Node &nd = P.nodes[node];
  const int ri = P.root_index[node];
  const RootInfo &RI = P.roots[ri];
  // template ri's results follow those of the templates before it
  result = (char *)result + (size_t)ri * x.res_stride * 8;
  Eout += (size_t)ri * x.res_stride;
  RootArgs a{};
  std::memset(&a, 0, sizeof(a));
  Tab *X = nullptr, *Y = nullptr;
  if (RI.kind == ROOT_SINGLE) {
    X = &x.pp.B[nd.passive];
  } else if (RI.kind == ROOT_FUSED) {
    X = &x.pp.B[P.nodes[nd.active].passive];
    Y = &x.pp.B[nd.passive];
  } else {
    X = &x.pp.M[nd.active];
    Y = &x.pp.B[nd.passive];
  }
  a.X = X->p;
  a.ldx = X->ld;
  a.Cx = (int32_t)X->cols;
  if (Y) {
    a.Y = Y->p;
    a.ldy = Y->ld;
    a.Cy = (int32_t)Y->cols;
  }
  a.list = x.dp.root_list[ri];
  a.L = RI.L;
  a.n = x.g->n;
  a.colors = x.c->d;
  a.j0 = x.j0;
  if (x.dt == DT_F32) {
    a.fx = X->f;
    a.fy = Y ? Y->f : nullptr;
  }
  a.partial = x.ws->partial.p;
  a.ovf = x.ovf;
  a.list16 = x.dp.root_list16[ri];
  a.same_xy = Y && Y->p == X->p;
  a.k = P.k;
  const size_t stage = (size_t)(X->cols + (Y && !a.same_xy ? Y->cols : 0)) * x.es;
  const bool use_lds = a.list16 && stage <= std::min<size_t>(x.lds_max, 64 * 1024);
  // colour by colour, double-buffered rows, lists in registers
  const int64_t Nv = 16 / x.es;
  const size_t row_lds = (size_t)round_up(X->cols, Nv) * x.es;
  const bool tile_db = 2 * row_lds <= 64 * 1024;  // else one row buffer
  const size_t tile_lds = (tile_db ? 2 : 1) * row_lds;
  const bool aligned = x.b == 1 || (X->cols * x.es) % 16 == 0;
  const bool use_tile = a.list16 && !(tuning().flags & SG2V_TUNE_ROOT_ROWS) && (!Y || a.same_xy) &&
                        aligned && RI.L <= 16 * 256 && X->cols <= 8192 && tile_lds <= 64 * 1024;
  // narrow rows and short lists: one thread per vertex
  const bool use_thread = a.list16 && !(tuning().flags & SG2V_TUNE_ROOT_ROWS) && RI.L <= 256 &&
                          (int64_t)P.k * RI.L <= 8192 && X->cols <= 512 && (!Y || Y->cols <= 512);
  // narrow rows: a tile of rows staged in LDS, a few lanes per vertex
  int stage_R = 0;
  size_t stage_lds = 0;
  if (use_thread && !(tuning().flags & SG2V_TUNE_ROOT_THREAD)) {
    const size_t lists = (size_t)round_up((int64_t)P.k * RI.L * 4, 16);
    const size_t per_row = (size_t)(X->cols + (Y ? Y->cols : 0)) * x.es;
    for (int R = 64; R >= 4 && !stage_R; R /= 2)
      if (lists + R * per_row <= 48 * 1024) stage_R = R;
    stage_lds = lists + (size_t)stage_R * per_row;
  }
  int nblk = 1024;
  if (stage_R)
    nblk = (int)std::min<int64_t>(kRootBlocks, std::max<int64_t>(1, (x.g->n + stage_R - 1) / stage_R));
  else if (use_thread)
    nblk = (int)std::min<int64_t>(kRootBlocks, std::max<int64_t>(1, (x.g->n + 255) / 256));
  else if (use_tile)
    nblk = (int)std::min<int64_t>(kRootBlocks, (int64_t)x.cu_count *
                                                   std::max<int64_t>(1, (int64_t)(x.lds_max / tile_lds)));
  {
    ProfScope ps(SG2V_K_ROOT,
                 (double)x.g->n * x.b * (double)(X->cols + (Y && !a.same_xy ? Y->cols : 0)) * x.es,
                 (double)x.g->n * x.b * (double)RI.L, x.s);
    if (stage_R) launch_root_stage(x.dt, a, dim3(nblk, x.b), stage_R, stage_lds, x.s);
    else if (use_thread) launch_root_thread(x.dt, a, dim3(nblk, x.b), x.s);
    else if (use_tile) launch_root_tile(x.dt, a, dim3(nblk, x.b), tile_lds, tile_db, x.s);
    else if (use_lds) launch_root_lds(x.dt, a, dim3(nblk, x.b), stage, x.s);
    else launch_root(x.dt, a, dim3(nblk, x.b), x.s);
  }
  const int es = 8;
  launch_root_final(x.dt, a.partial, nblk, x.b, (char *)result + (size_t)x.j0 * es, x.ovf, x.s);
  if (x.dt == DT_F32) launch_root_exp(X->E, Y ? Y->E : nullptr, Eout + x.j0, x.b, x.s);
  return SG2V_OK;
}

struct Capture {
  int node = -1, kind = 0;
  void *host = nullptr;
};

sg2v_status copy_capture(Ctx &x, const Capture &cap) {
  Tab &t = cap.kind == 0 ? x.pp.M[cap.node] : x.pp.B[cap.node];
  const int64_t n = x.g->n, nc = t.cols;
  std::vector<char> raw((size_t)n * t.ld * x.es);
  HIP_TRY(hipMemcpyAsync(raw.data(), t.p, raw.size(), hipMemcpyDeviceToHost, x.s));
  std::vector<int> e;
  if (x.dt == DT_F32) {
    e.resize(nc);
    HIP_TRY(hipMemcpyAsync(e.data(), t.e, nc * 4, hipMemcpyDeviceToHost, x.s));
  }
  HIP_TRY(hipStreamSynchronize(x.s));
  const std::vector<int32_t> *nw = x.g->new_of.get();
  for (int64_t i = 0; i < n; ++i)  // row i of the caller's vertex order
    for (int64_t c = 0; c < nc; ++c) {
      const size_t src = (size_t)((nw ? (int64_t)(*nw)[i] : i) * t.ld + c);
      if (x.dt == DT_U64) {
        ((uint64_t *)cap.host)[i * nc + c] = ((uint64_t *)raw.data())[src];
      } else if (x.dt == DT_F64) {
        ((double *)cap.host)[i * nc + c] = ((double *)raw.data())[src];
      } else {
        ((double *)cap.host)[i * nc + c] = std::ldexp((double)((float *)raw.data())[src], e[c]);
      }
    }
  return SG2V_OK;
}

sg2v_status run_pass(Ctx &x, void *result, int *Eout, const Capture *cap, int stop_node = -1) {
  for (size_t q = 0; q < x.pp.steps.size(); ++q) {
    const Step &st = x.pp.steps[q];
    if (st.node == stop_node && (st.kind == S_EMA_SINGLE || st.kind == S_EMA_GENERAL ||
                                 st.kind == S_ROOT))
      break;
    switch (st.kind) {
      case S_HIST: ST_TRY(step_hist(x, st.node)); break;
      case S_SPMM: ST_TRY(step_spmm(x, st.node)); break;
      case S_EMA_SINGLE: ST_TRY(step_ema(x, st.node, true)); break;
      case S_EMA_GENERAL: ST_TRY(step_ema(x, st.node, false)); break;
      case S_ROOT: ST_TRY(step_root(x, st.node, result, Eout)); break;
    }
    HIP_TRY(hipGetLastError());
    if (cap && cap->node == st.node) {
      const bool produced = (cap->kind == 0 && (st.kind == S_EMA_SINGLE || st.kind == S_EMA_GENERAL)) ||
                            (cap->kind == 1 && (st.kind == S_HIST || st.kind == S_SPMM));
      if (produced) ST_TRY(copy_capture(x, *cap));
    }
  }
  return SG2V_OK;
}

sg2v_status check_inputs(const sg2v_plan *plan, const sg2v_graph *g, const sg2v_colorings *c,
                         sg2v_mode mode) {
  if (!plan || !g || !c) {
    set_error("sg2v_count: null handle");
    return SG2V_EINVAL;
  }
  if (mode != SG2V_FP64 && mode != SG2V_FP32S && mode != SG2V_U64) {
    set_error("sg2v_count: unknown mode %d", mode);
    return SG2V_EINVAL;
  }
  if (c->k != plan->p.k || c->n != g->n) {
    set_error("sg2v_count: colourings have k=%d n=%lld, plan k=%d graph n=%lld", c->k,
              (long long)c->n, plan->p.k, (long long)g->n);
    return SG2V_EINVAL;
  }
  if (mode == SG2V_U64 && g->w) {
    set_error("sg2v_count: U64 mode counts the 0/1 adjacency; the graph has weights");
    return SG2V_EINVAL;
  }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != g->device || dev != c->device) {
    set_error("sg2v_count: current device %d differs from the graph's (%d)", dev, g->device);
    return SG2V_EINVAL;
  }
  return SG2V_OK;
}

int choose_batch(const Plan &P, int ncol, int dt, int64_t n, int64_t n_slots) {
  sg2v_tuning_t tu = tuning();
  int64_t widest_passive = 1;
  for (auto &nd : P.nodes)
    if (nd.n_passive_uses > 0) widest_passive = std::max(widest_passive, nd.size == 1 ? P.k : nd.cols);
  int b = tu.batch > 0 ? tu.batch : (int)std::max<int64_t>(1, 1024 / widest_passive);
  b = std::max(1, std::min({b, ncol, 65535}));  // colourings of a pass index grid.y
  // memory budget
  size_t fr = 0, tot = 0;
  (void)hipMemGetInfo(&fr, &tot);
  int64_t budget = tu.budget_bytes > 0 ? tu.budget_bytes : (int64_t)(fr * 0.85);
  while (b > 1) {
    PassPlan pp;
    build_pass(P, n, b, dt, pick_G(dt, widest_passive * b, n), n_slots, pp, PassOpts());
    if (pp.arena <= budget) break;
    b = (b + 1) / 2;
  }
  return b;
}

sg2v_status prepare(Ctx &x, const sg2v_plan *plan, sg2v_graph *g, const sg2v_colorings *c,
                    sg2v_mode mode, int b, hipStream_t s, const PassOpts &opt, Workspace *wsp = nullptr) {
  x.P = &plan->p;
  x.g = g;
  x.c = c;
  x.dt = dtype_of(mode);
  x.es = esize_of(x.dt);
  x.b = b;
  x.s = s;
  x.ws = wsp ? wsp : &workspace();
  {
    static std::mutex mu;
    static std::map<int, std::pair<int, size_t>> props;
    std::lock_guard<std::mutex> lk(mu);
    auto it = props.find(g->device);
    if (it == props.end()) {
      hipDeviceProp_t prop;
      HIP_TRY(hipGetDeviceProperties(&prop, g->device));
      it = props.emplace(g->device, std::make_pair(prop.multiProcessorCount,
                                                   (size_t)prop.sharedMemPerBlock)).first;
    }
    x.cu_count = it->second.first;
    x.lds_max = it->second.second;
  }
  ST_TRY(plan_device(plan->p, g->device, s, &x.dp));
  int64_t widest = 1;
  for (auto &nd : plan->p.nodes)
    if (nd.n_passive_uses > 0) widest = std::max(widest, nd.size == 1 ? plan->p.k : nd.cols);
  build_pass(plan->p, g->n, b, x.dt, pick_G(x.dt, widest * b, g->n), g->n_slots, x.pp, opt);
  sg2v_tuning_t tu = tuning();
  if (tu.budget_bytes > 0 && x.pp.arena > tu.budget_bytes) {
    set_error("sg2v_count: one colouring needs %lld bytes, budget is %lld",
              (long long)x.pp.arena, (long long)tu.budget_bytes);
    return SG2V_ENOMEM;
  }
  ST_TRY(x.ws->arena.ensure(x.pp.arena));
  ST_TRY(x.ws->small.ensure(x.pp.small_bytes));
  ST_TRY(x.ws->partial.ensure((size_t)kRootBlocks * b * 8));
  ST_TRY(x.ws->ovf.ensure(256));
  ST_TRY(x.ws->bucket.ensure((size_t)b * (64 + g->n) * 4 + 256));
  if (!(tuning().flags & SG2V_TUNE_NO_COLOR_SKIP))
    ST_TRY(x.ws->nbrcol.ensure((size_t)b * std::max<int64_t>(g->nnz, 1) + 256));
  x.ovf = (int *)x.ws->ovf.p;
  x.bucket_j0 = -1;
  x.nbr_j0 = -1;
  return bind_tables(x);
}

// Upload everything a pass over b colourings needs (SpMM units, colour-skip
// masks) so that the pass itself only enqueues kernels.
sg2v_status prewarm(Ctx &x, int b) {
  if (b < 1) return SG2V_OK;
  PassPlan pp;
  build_pass(*x.P, x.g->n, b, x.dt, x.pp.G, x.g->n_slots, pp, PassOpts());
  UnitTable *U = nullptr;
  ST_TRY(build_units(x.g, x.pp.G, x.s, &U));
  const int W = x.pp.G * (x.dt == DT_F32 ? 4 : 2);
  // split offsets and partial rows of the neighbour-range split
  for (auto &st : pp.steps)
    if (st.kind == S_SPMM) {
      int64_t gch = 0;
      ST_TRY(xsplit_setup(x, U, pp.M[st.node].cols * b, W, &gch));
    }
  if (tuning().flags & SG2V_TUNE_NO_COLOR_SKIP) return SG2V_OK;
  const int keep_b = x.b;
  x.b = b;
  for (auto &st : pp.steps)
    if (st.kind == S_SPMM) {
      const int32_t *a;
      const uint32_t *u, *i;
      sg2v_status r = chunk_masks(x, st.node, W, &a, &u, &i);
      if (r != SG2V_OK) {
        x.b = keep_b;
        return r;
      }
    }
  x.b = keep_b;
  return SG2V_OK;
}

// Enqueue every pass for the ncol colourings of x.c (no host synchronisation):
// raw colourful sums to res[j] (double or uint64), FP32S frame exponents to
// Ed[j].  x must come from prepare() with batch b, prewarmed for b and for the
// last, smaller pass.
sg2v_status enqueue_count(Ctx &x, int ncol, int b, void *res, int *Ed) {
  for (int j0 = 0; j0 < ncol; j0 += b) {
    const int bb = std::min(b, ncol - j0);
    if (bb != x.b) {
      // last, smaller pass: tables of the full batch still fit
      x.b = bb;
      build_pass(*x.P, x.g->n, bb, x.dt, x.pp.G, x.g->n_slots, x.pp, PassOpts());
      ST_TRY(bind_tables(x));
    }
    x.j0 = j0;
    ST_TRY(run_pass(x, res, Ed, nullptr));
  }
  return SG2V_OK;
}

void finish_counts(const RootInfo &P, int ncol, int dt, const double *rf, const uint64_t *ru,
                   const int *E, double *colorful, uint64_t *colorful_u64, double *estimate,
                   double *mean_estimate) {
  double mean = 0.0;
  for (int j = 0; j < ncol; ++j) {
    double v = dt == DT_U64 ? (double)ru[j] : rf[j];
    if (dt == DT_F32) v = std::ldexp(v, E[j]);
    if (colorful) colorful[j] = v;
    if (colorful_u64) colorful_u64[j] = dt == DT_U64 ? ru[j] : 0;
    const double est = v / (P.P * (double)P.alpha);
    if (estimate) estimate[j] = est;
    mean += est;
  }
  if (mean_estimate) *mean_estimate = mean / ncol;
}

}  // namespace

namespace {

// Raw colourful sums of every template of the plan for every colouring of c:
// rf / ru / E hold n_templates x ncol entries, template-major (FP32S sums
// still to be scaled by 2^E).  Templates of one vertex are filled on the host.
sg2v_status count_raw(const sg2v_plan *plan, const sg2v_graph *g, const sg2v_colorings *c,
                      sg2v_mode mode, hipStream_t s, std::vector<double> &rf,
                      std::vector<uint64_t> &ru, std::vector<int> &E, int *ovf_h) {
  const Plan &P = plan->p;
  const int ncol = c->count;
  const int nr = (int)P.roots.size();
  const int dt = dtype_of(mode);
  rf.assign((size_t)nr * ncol, 0.0);
  ru.assign((size_t)nr * ncol, 0);
  E.assign((size_t)nr * ncol, 0);
  *ovf_h = 0;
  bool device = false;
  for (auto &R : P.roots) device |= R.kind != ROOT_VERTEX;
  if (device) {
    const int b = choose_batch(P, ncol, dt, g->n, g->n_slots);
    Ctx x;
    ST_TRY(prepare(x, plan, (sg2v_graph *)g, c, mode, b, s, PassOpts()));
    x.res_stride = ncol;
    ST_TRY(prewarm(x, b));
    ST_TRY(prewarm(x, ncol % b));
    const size_t nres = (size_t)nr * ncol;
    ST_TRY(x.ws->result.ensure(nres * 12 + 64));
    void *res = x.ws->result.p;
    int *Ed = (int *)((char *)res + nres * 8);
    launch_fill_u32((unsigned *)x.ovf, 1, 0u, s);
    ST_TRY(enqueue_count(x, ncol, b, res, Ed));
    HIP_TRY(hipMemcpyAsync(dt == DT_U64 ? (void *)ru.data() : (void *)rf.data(), res, nres * 8,
                           hipMemcpyDeviceToHost, s));
    if (dt == DT_F32) HIP_TRY(hipMemcpyAsync(E.data(), Ed, nres * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ovf_h, x.ovf, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  // every vertex is one colourful map of a one-vertex template
  for (int r = 0; r < nr; ++r)
    if (P.roots[r].kind == ROOT_VERTEX)
      for (int j = 0; j < ncol; ++j) {
        rf[(size_t)r * ncol + j] = (double)g->n;
        ru[(size_t)r * ncol + j] = (uint64_t)g->n;
        E[(size_t)r * ncol + j] = 0;
      }
  return SG2V_OK;
}

// Scaled counts and estimates of template r (raw sums of a one-vertex
// template are doubles whatever the mode).
void finish_template(const Plan &P, int r, int ncol, int dt, const std::vector<double> &rf,
                     const std::vector<uint64_t> &ru, const std::vector<int> &E, double *colorful,
                     uint64_t *colorful_u64, double *estimate, double *mean_estimate) {
  const RootInfo &R = P.roots[r];
  const size_t o = (size_t)r * ncol;
  const bool vertex = R.kind == ROOT_VERTEX;
  finish_counts(R, ncol, vertex ? DT_F64 : dt, rf.data() + o, ru.data() + o, E.data() + o,
                colorful, colorful_u64, estimate, mean_estimate);
  if (colorful_u64 && vertex)
    for (int j = 0; j < ncol; ++j) colorful_u64[j] = ru[o + j];
}

}  // namespace

extern "C" sg2v_status sg2v_count(const sg2v_plan *plan, const sg2v_graph *g,
                                  const sg2v_colorings *c, sg2v_mode mode, void *stream,
                                  double *colorful, uint64_t *colorful_u64, double *estimate,
                                  double *mean_estimate, int32_t *overflow) {
  ST_TRY(check_inputs(plan, g, c, mode));
  if (plan->p.roots.size() != 1) {
    set_error("sg2v_count: the plan holds %d templates; use sg2v_count_multi",
              (int)plan->p.roots.size());
    return SG2V_EINVAL;
  }
  std::vector<double> rf;
  std::vector<uint64_t> ru;
  std::vector<int> E;
  int ovf_h = 0;
  ST_TRY(count_raw(plan, g, c, mode, (hipStream_t)stream, rf, ru, E, &ovf_h));
  finish_template(plan->p, 0, c->count, dtype_of(mode), rf, ru, E, colorful, colorful_u64,
                  estimate, mean_estimate);
  if (overflow) *overflow = ovf_h;
  return SG2V_OK;
}

extern "C" sg2v_status sg2v_count_multi(const sg2v_plan *plan, const sg2v_graph *g,
                                        const sg2v_colorings *c, sg2v_mode mode, void *stream,
                                        double *colorful, uint64_t *colorful_u64,
                                        double *estimate, double *mean_estimate,
                                        double *frequency, int32_t *overflow) {
  ST_TRY(check_inputs(plan, g, c, mode));
  const Plan &P = plan->p;
  const int ncol = c->count;
  const int nr = (int)P.roots.size();
  std::vector<double> rf;
  std::vector<uint64_t> ru;
  std::vector<int> E;
  int ovf_h = 0;
  ST_TRY(count_raw(plan, g, c, mode, (hipStream_t)stream, rf, ru, E, &ovf_h));
  std::vector<double> means(nr, 0.0);
  for (int r = 0; r < nr; ++r)
    finish_template(P, r, ncol, dtype_of(mode), rf, ru, E,
                    colorful ? colorful + (size_t)r * ncol : nullptr,
                    colorful_u64 ? colorful_u64 + (size_t)r * ncol : nullptr,
                    estimate ? estimate + (size_t)r * ncol : nullptr, &means[r]);
  double total = 0.0;
  for (double m : means) total += m;
  for (int r = 0; r < nr; ++r) {
    if (mean_estimate) mean_estimate[r] = means[r];
    if (frequency) frequency[r] = total > 0.0 ? means[r] / total : 0.0;
  }
  if (overflow) *overflow = ovf_h;
  return SG2V_OK;
}

// ---------------------------------------------------------------------------
// sg2v_count without device allocations: every per-call buffer is carved
// from a fixed area in the library's own device memory.

namespace {

// The area itself.  In host code its name is only a handle for
// hipGetSymbolAddress; kernels receive the device address from scratch_area().
static __device__ __align__(256) unsigned char scratch[SG2V_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on device `dev` (which must be current), looked
// up once per device and kept.
sg2v_status scratch_area(int dev, char **out) {
  static std::mutex mu;
  static std::map<int, char *> ptrs;
  std::lock_guard<std::mutex> lk(mu);
  auto it = ptrs.find(dev);
  if (it == ptrs.end()) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      set_error("sg2v_count_noalloc: hipGetSymbolAddress of the scratch area failed on device %d: %s",
                dev, hipGetErrorString(e));
      return SG2V_EDEVICE;
    }
    it = ptrs.emplace(dev, (char *)p).first;
  }
  *out = it->second;
  return SG2V_OK;
}

struct NoallocGuard {
  NoallocGuard() { t_noalloc = true; }
  ~NoallocGuard() { t_noalloc = false; }
};

}  // namespace

extern "C" sg2v_status sg2v_count_noalloc(const sg2v_plan *plan, const sg2v_graph *g,
                                          const sg2v_colorings *c, sg2v_mode mode, void *stream,
                                          double *colorful, uint64_t *colorful_u64,
                                          double *estimate, double *mean_estimate,
                                          int32_t *overflow) {
  ST_TRY(check_inputs(plan, g, c, mode));
  if (plan->p.roots.size() != 1) {
    set_error("sg2v_count_noalloc: the plan holds %d templates", (int)plan->p.roots.size());
    return SG2V_EINVAL;
  }
  const Plan &P = plan->p;
  hipStream_t s = (hipStream_t)stream;
  const int ncol = c->count;
  const int dt = dtype_of(mode);
  std::vector<double> raw_f(ncol, 0.0);
  std::vector<uint64_t> raw_u(ncol, 0);
  std::vector<int> Eh(ncol, 0);
  int ovf_h = 0;
  if (P.root_kind == ROOT_VERTEX) {
    for (int j = 0; j < ncol; ++j) {
      raw_f[j] = (double)g->n;
      raw_u[j] = (uint64_t)g->n;
    }
  } else {
    {
      std::lock_guard<std::mutex> lk(P.mu);
      bool have = false;
      for (auto &d : P.dev) have |= d.device == g->device;
      if (!have) {
        set_error("sg2v_count_noalloc: the plan's split tables are not on device %d yet; one "
                  "sg2v_count call with this plan on this device uploads them", g->device);
        return SG2V_ENOMEM;
      }
    }
    char *area = nullptr;
    ST_TRY(scratch_area(g->device, &area));
    NoallocGuard guard;
    Carver cv;
    cv.base = area;
    cv.cap = SG2V_NOALLOC_SCRATCH_BYTES;
    Workspace ws;
    DevBuf *bufs[] = {&ws.arena, &ws.small, &ws.partial, &ws.result, &ws.ovf,
                      &ws.grad,  &ws.bucket, &ws.nbrcol, &ws.xpart};
    // colourings per pass: as sg2v_count would take them, halved until the pass fits
    int b = choose_batch(P, ncol, dt, g->n, g->n_slots);
    std::unique_ptr<Ctx> x;
    for (;;) {
      cv.top = 0;
      cv.exhausted = false;
      for (DevBuf *d : bufs) {
        d->p = nullptr;
        d->bytes = 0;
        d->cv = &cv;
      }
      x.reset(new Ctx());
      sg2v_status st = prepare(*x, plan, (sg2v_graph *)g, c, mode, b, s, PassOpts(), &ws);
      x->res_stride = ncol;
      if (st == SG2V_OK) st = prewarm(*x, b);
      if (st == SG2V_OK) st = prewarm(*x, ncol % b);
      if (st == SG2V_OK) st = ws.result.ensure((size_t)ncol * 12 + 64);
      if (st == SG2V_OK) break;
      if (!cv.exhausted || b == 1) {
        HIP_TRY(hipStreamSynchronize(s));  // mask copies read host memory of this call
        return st;
      }
      HIP_TRY(hipStreamSynchronize(s));
      b = (b + 1) / 2;
    }
    void *res = ws.result.p;
    int *Ed = (int *)((char *)res + (size_t)ncol * 8);
    launch_fill_u32((unsigned *)x->ovf, 1, 0u, s);
    sg2v_status st = enqueue_count(*x, ncol, b, res, Ed);
    if (st != SG2V_OK) {
      (void)hipStreamSynchronize(s);
      return st;
    }
    HIP_TRY(hipMemcpyAsync(dt == DT_U64 ? (void *)raw_u.data() : (void *)raw_f.data(), res,
                           ncol * 8, hipMemcpyDeviceToHost, s));
    if (dt == DT_F32) HIP_TRY(hipMemcpyAsync(Eh.data(), Ed, ncol * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&ovf_h, x->ovf, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  finish_template(P, 0, ncol, dt, raw_f, raw_u, Eh, colorful, colorful_u64, estimate,
                  mean_estimate);
  if (overflow) *overflow = ovf_h;
  return SG2V_OK;
}

extern "C" sg2v_status sg2v_debug_table(const sg2v_plan *plan, const sg2v_graph *g,
                                        const sg2v_colorings *c, sg2v_mode mode, int32_t which,
                                        int32_t node, int32_t kind, void *host_out, void *stream) {
  ST_TRY(check_inputs(plan, g, c, mode));
  const Plan &P = plan->p;
  if (!host_out || which < 0 || which >= c->count || node < 0 || node >= (int)P.nodes.size() ||
      (kind != 0 && kind != 1)) {
    set_error("sg2v_debug_table: bad argument");
    return SG2V_EINVAL;
  }
  const Node &nd = P.nodes[node];
  if ((kind == 0 && (nd.size == 1 || P.root_index[node] >= 0)) || (kind == 1 && nd.n_passive_uses == 0)) {
    set_error("sg2v_debug_table: node %d has no materialised %s table", node, kind ? "B" : "M");
    return SG2V_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  Ctx x;
  PassOpts opt;
  opt.keep.push_back({node, kind});
  ST_TRY(prepare(x, plan, (sg2v_graph *)g, c, mode, 1, s, opt));
  ST_TRY(x.ws->result.ensure((size_t)c->count * 12 + 64));
  void *res = x.ws->result.p;
  int *Ed = (int *)((char *)res + (size_t)c->count * 8);
  launch_fill_u32((unsigned *)x.ovf, 1, 0u, s);
  x.j0 = which;
  Capture cap;
  cap.node = node;
  cap.kind = kind;
  cap.host = host_out;
  ST_TRY(run_pass(x, res, Ed, &cap));
  HIP_TRY(hipStreamSynchronize(s));
  return SG2V_OK;
}

namespace {

// Recorded launches of a batch run by one k_persist launch: the host copy of
// the launch table (grouped by chain) and its device copy followed by each
// chain's ticket count and first launch; the control words: per-launch done
// counters, per-chain ticket counters and the error flag.
struct PSched {
  int dtype = 0;
  int n_chain = 1;
  size_t lds = 0;
  unsigned blocks = 0;
  uint64_t timeout = 0;
  int clock_khz = 100000;  // device wall clock
  std::vector<PLaunch> h;
  std::vector<int64_t> chain_total;
  std::vector<int32_t> chain_first;
  char *d = nullptr;        // PLaunch[n] | int64 chain_total[n_chain] | int32 chain_first[n_chain + 1]
  unsigned *ctl = nullptr;  // done[n] (padded to even) | uint64 next[n_chain] | error flag
  size_t ctl_words = 0;
  ~PSched() {
    if (d) (void)hipFree(d);
    if (ctl) (void)hipFree(ctl);
  }
  size_t done_words() const { return (h.size() + 1) & ~(size_t)1; }
  unsigned *done() const { return ctl; }
  unsigned long long *next() const { return (unsigned long long *)(ctl + done_words()); }
  int *err() const { return (int *)(ctl + done_words() + 2 * (size_t)n_chain); }
};

// One captured multi-template count: colourings of every plan plus all of
// their passes, instantiated once and replayed while the workspace buffers
// it captured are unchanged.
struct BatchGraph {
  std::vector<const sg2v_plan *> plans;
  const sg2v_graph *g = nullptr;
  uint64_t seed = 0;
  int ncol = 0, mode = 0;
  sg2v_tuning_t tune{};
  uint64_t gens[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<std::unique_ptr<sg2v_colorings>> cols;
  // per-template workspaces when the templates run as parallel graph branches
  std::vector<std::unique_ptr<Workspace>> wss;
  bool conc = false;
  hipGraphExec_t exec = nullptr;
  std::unique_ptr<PSched> ps;  // persistent schedule instead of the graph
  int device = -1;
  ~BatchGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

std::mutex g_batch_mu;
std::vector<std::unique_ptr<BatchGraph>> g_batch_cache;

bool same_tuning(const sg2v_tuning_t &a, const sg2v_tuning_t &b) {
  return a.spmm_width == b.spmm_width && a.ema_rows == b.ema_rows && a.batch == b.batch &&
         a.flags == b.flags && a.budget_bytes == b.budget_bytes &&
         a.xsplit_group == b.xsplit_group && a.launch_chunks == b.launch_chunks &&
         a.xsplit_min == b.xsplit_min;
}

// The recorded launches grouped by chain (each chain's launches in recording
// order, its tasks numbered from 0), each launch's predecessor the previous
// launch of its chain.
sg2v_status build_psched(const PRecorder &rec, int dtype, int n_chain, int device, PSched *ps) {
  const size_t n = rec.rec.size();
  if (n == 0) {
    set_error("sg2v_count_batch: nothing was recorded for the persistent schedule");
    return SG2V_EINVAL;
  }
  if (n_chain < 1 || n_chain > kPMaxChains) {
    set_error("sg2v_count_batch: the persistent schedule runs 1 to %d templates", kPMaxChains);
    return SG2V_EINVAL;
  }
  size_t lds = 0;
  std::vector<std::vector<int>> of(n_chain);
  for (size_t i = 0; i < n; ++i) {
    const PRecord &r = rec.rec[i];
    if (r.dtype >= 0 && r.dtype != dtype) {
      set_error("sg2v_count_batch: a recorded launch has another element type");
      return SG2V_EINVAL;
    }
    if (r.chain < 0 || r.chain >= n_chain) {
      set_error("sg2v_count_batch: a recorded launch names chain %d of %d", r.chain, n_chain);
      return SG2V_EINVAL;
    }
    lds = std::max(lds, r.lds);
    of[r.chain].push_back((int)i);
  }
  const int per_cu = persist_blocks_per_cu(dtype, lds);
  if (per_cu < 1) {
    set_error("sg2v_count_batch: the persistent kernel does not fit a CU with %zu bytes of LDS", lds);
    return SG2V_ENOMEM;
  }
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  ps->h.assign(n, PLaunch{});
  ps->chain_total.assign(n_chain, 0);
  ps->chain_first.assign(n_chain + 1, 0);
  int64_t all = 0;
  size_t q = 0;
  for (int c = 0; c < n_chain; ++c) {
    ps->chain_first[c] = (int32_t)q;
    int64_t first = 0;
    for (size_t k = 0; k < of[c].size(); ++k, ++q) {
      const PRecord &r = rec.rec[of[c][k]];
      PLaunch &L = ps->h[q];
      std::memset(&L, 0, sizeof(L));
      L.body = r.body;
      L.chain = c;
      L.pred = k > 0 ? (int32_t)q - 1 : -1;
      L.gx = r.gx;
      L.gy = r.gy;
      L.first = first;
      L.ntask = (int64_t)r.gx * r.gy;
      std::memcpy(L.args, r.args, kPArgBytes);
      if (L.ntask < 1 || L.ntask > (int64_t)UINT32_MAX) {
        set_error("sg2v_count_batch: a recorded launch has %lld blocks", (long long)L.ntask);
        return SG2V_EINVAL;
      }
      first += L.ntask;
    }
    ps->chain_total[c] = first;
    all += first;
  }
  ps->chain_first[n_chain] = (int32_t)q;
  int clock_khz = 0;
  if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || clock_khz <= 0)
    clock_khz = 100000;
  ps->dtype = dtype;
  ps->n_chain = n_chain;
  ps->lds = lds;
  ps->blocks = (unsigned)std::min<int64_t>((int64_t)prop.multiProcessorCount * per_cu, all);
  ps->clock_khz = clock_khz;
  ps->timeout = (uint64_t)clock_khz * 1000ull * 30ull;  // 30 s per dependency wait
  const size_t lb = n * sizeof(PLaunch), tb = (size_t)n_chain * 8, fb = (size_t)(n_chain + 1) * 4;
  HIP_TRY(hipMalloc((void **)&ps->d, lb + tb + fb));
  HIP_TRY(hipMemcpy(ps->d, ps->h.data(), lb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ps->d + lb, ps->chain_total.data(), tb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ps->d + lb + tb, ps->chain_first.data(), fb, hipMemcpyHostToDevice));
  ps->ctl_words = ps->done_words() + 2 * (size_t)n_chain + 2;
  HIP_TRY(hipMalloc((void **)&ps->ctl, ps->ctl_words * 4));
  return SG2V_OK;
}

void run_psched(const PSched &ps, hipStream_t s) {
  launch_fill_u32(ps.ctl, (int64_t)ps.ctl_words, 0u, s);
  PersistArgs a{};
  const size_t lb = ps.h.size() * sizeof(PLaunch);
  a.L = (const PLaunch *)ps.d;
  a.chain_total = (const int64_t *)(ps.d + lb);
  a.chain_first = (const int32_t *)(ps.d + lb + (size_t)ps.n_chain * 8);
  a.n_launch = (int32_t)ps.h.size();
  a.n_chain = ps.n_chain;
  a.done = ps.done();
  a.next = ps.next();
  a.err = ps.err();
  a.timeout = ps.timeout;
  // SG2V_PERSIST_WAIT_US: another bound on each dependency wait, in
  // microseconds (tests of the time-out path)
  if (const char *e = std::getenv("SG2V_PERSIST_WAIT_US"))
    a.timeout = (uint64_t)std::strtoull(e, nullptr, 10) * (uint64_t)ps.clock_khz / 1000ull;
  launch_persist(ps.dtype, a, ps.blocks, ps.lds, s);
}

void ws_gens(Workspace &ws, uint64_t *out) {
  out[0] = ws.arena.gen;
  out[1] = ws.small.gen;
  out[2] = ws.partial.gen;
  out[3] = ws.result.gen;
  out[4] = ws.ovf.gen;
  out[5] = ws.grad.gen;
  out[6] = ws.bucket.gen;
  out[7] = ws.nbrcol.gen;
  out[8] = ws.xpart.gen;
}

}  // namespace

// Several templates, n_colorings colourings each, recorded as one HIP graph
// (colouring kernels and every pass of every template) and launched with a
// single hipGraphLaunch.  The executable graph is cached and replayed by later
// calls with the same arguments while the workspace is unchanged.
extern "C" sg2v_status sg2v_count_batch(const sg2v_plan *const *plans, int32_t n_plans,
                                        const sg2v_graph *g, uint64_t seed, int32_t n_colorings,
                                        sg2v_mode mode, void *stream, double *colorful,
                                        double *estimate) {
  if (!plans || n_plans < 1 || !g || n_colorings < 1) {
    set_error("sg2v_count_batch: bad argument");
    return SG2V_EINVAL;
  }
  for (int p = 0; p < n_plans; ++p) {
    if (plans[p] && plans[p]->p.roots.size() != 1) {
      set_error("sg2v_count_batch: plan %d holds several templates; use sg2v_count_multi", p);
      return SG2V_EINVAL;
    }
    if (!plans[p] || plans[p]->p.root_kind == ROOT_VERTEX) {
      set_error("sg2v_count_batch: plan %d is null or a one-vertex template", p);
      return SG2V_EINVAL;
    }
  }
  if (mode != SG2V_FP64 && mode != SG2V_FP32S && mode != SG2V_U64) {
    set_error("sg2v_count_batch: unknown mode %d", mode);
    return SG2V_EINVAL;
  }
  if (mode == SG2V_U64 && g->w) {
    set_error("sg2v_count_batch: U64 mode counts the 0/1 adjacency; the graph has weights");
    return SG2V_EINVAL;
  }
  hipStream_t us = (hipStream_t)stream;
  const int dt = dtype_of(mode);
  const int ncol = n_colorings;
  std::lock_guard<std::mutex> lk(g_batch_mu);
  Workspace &ws = workspace();
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));

  std::vector<int> bs(n_plans);
  for (int p = 0; p < n_plans; ++p) bs[p] = choose_batch(plans[p]->p, ncol, dt, g->n, g->n_slots);
  // Templates run as parallel branches of the graph, each with a workspace of
  // its own, when those fit in half of the free device memory (estimated from
  // the pass plan of each); otherwise one after another in the shared one.
  const sg2v_tuning_t tune = tuning();
  const bool persist = (tune.flags & SG2V_TUNE_BATCH_PERSISTENT) != 0;
  // the persistent schedule runs kernels of 256-thread blocks only: the
  // general multiply-add and the vertex-order root reduction
  TuneOr forced(persist ? (SG2V_TUNE_NO_COLOR_EMA | SG2V_TUNE_ROOT_ROWS) : 0);
  bool conc = n_plans > 1 && !(tune.flags & SG2V_TUNE_BATCH_SERIAL);
  if (conc) {
    size_t fr = 0, tot = 0;
    HIP_TRY(hipMemGetInfo(&fr, &tot));
    double need = 0;
    for (int p = 0; p < n_plans; ++p) {
      PassPlan pp;
      int64_t widest = 1;
      for (auto &nd : plans[p]->p.nodes)
        if (nd.n_passive_uses > 0) widest = std::max(widest, nd.size == 1 ? plans[p]->p.k : nd.cols);
      build_pass(plans[p]->p, g->n, bs[p], dt, pick_G(dt, widest * bs[p], g->n), g->n_slots, pp, PassOpts());
      need += (double)pp.arena + pp.small_bytes + (double)bs[p] * (g->nnz + 4.0 * g->n + 64.0);
    }
    conc = need <= 0.5 * (double)fr;
  }
  ST_TRY(ws.ovf.ensure(256));
  ST_TRY(ws.result.ensure((size_t)n_plans * ncol * 12 + 64));
  const std::vector<const sg2v_plan *> pv(plans, plans + n_plans);
  auto same_key = [&](const BatchGraph &e) {
    return e.g == g && e.seed == seed && e.ncol == ncol && e.mode == mode && e.device == dev && e.plans == pv &&
           same_tuning(e.tune, tune) && e.conc == conc;
  };
  uint64_t gens[9];
  ws_gens(ws, gens);
  BatchGraph *hit = nullptr;
  if (conc) {
    // a cached graph with workspaces of its own only needs the shared result
    // and flag buffers unchanged
    for (auto &e : g_batch_cache)
      if (same_key(*e) && e->gens[3] == gens[3] && e->gens[4] == gens[4]) hit = e.get();
  }
  std::unique_ptr<BatchGraph> bg;
  std::vector<Ctx> xs(n_plans);
  if (!hit) {
    // colourings and contexts (all uploads and allocations happen here)
    bg.reset(new BatchGraph());
    bg->plans = pv;
    bg->g = g;
    bg->seed = seed;
    bg->ncol = ncol;
    bg->mode = mode;
    bg->tune = tune;
    bg->device = dev;
    bg->conc = conc;
    for (int p = 0; p < n_plans; ++p) {
      std::unique_ptr<sg2v_colorings> c(new sg2v_colorings());
      c->device = dev;
      c->n = g->n;
      c->k = plans[p]->p.k;
      c->count = ncol;
      c->seed = seed;
      HIP_TRY(hipMalloc((void **)&c->d, g->n * ncol));
      bg->cols.push_back(std::move(c));
    }
    for (int p = 0; p < n_plans; ++p) {
      Workspace *wp = nullptr;
      if (conc) {
        bg->wss.emplace_back(new Workspace());
        wp = bg->wss.back().get();
      }
      ST_TRY(prepare(xs[p], plans[p], (sg2v_graph *)g, bg->cols[p].get(), mode, bs[p], us, PassOpts(), wp));
      ST_TRY(prewarm(xs[p], bs[p]));
      ST_TRY(prewarm(xs[p], ncol % bs[p]));
    }
    HIP_TRY(hipStreamSynchronize(us));
    if (!conc) {
      // reuse a cached executable graph if every input and buffer is unchanged
      ws_gens(ws, gens);
      for (auto &e : g_batch_cache)
        if (same_key(*e) && std::equal(gens, gens + 9, e->gens)) hit = e.get();
    }
  }
  char *res = (char *)ws.result.p;
  int *Ed = (int *)(res + (size_t)n_plans * ncol * 8);
  if (!hit) {
    // the prepares above may have grown the workspace: rebind every context
    for (int p = 0; p < n_plans; ++p) {
      xs[p].ovf = (int *)ws.ovf.p;
      ST_TRY(bind_tables(xs[p]));
    }
    if (persist) {
      // record every launch of every template (one chain each when they have
      // workspaces of their own) for one k_persist launch
      PRecorder rec;
      sg2v_status st = SG2V_OK;
      t_prec = &rec;
      t_capturing = true;
      for (int p = 0; p < n_plans && st == SG2V_OK; ++p) {
        rec.chain = conc ? p : 0;
        launch_color(bg->cols[p]->d, g->n, plans[p]->p.k, seed, 0, ncol, g->orig_id, us);
        xs[p].s = us;
        xs[p].c = bg->cols[p].get();
        st = enqueue_count(xs[p], ncol, bs[p], res + (size_t)p * ncol * 8, Ed + (size_t)p * ncol);
      }
      t_capturing = false;
      t_prec = nullptr;
      if (st != SG2V_OK) return st;
      if (!rec.err.empty()) {
        set_error("sg2v_count_batch: %s cannot run in the persistent schedule", rec.err.c_str());
        return SG2V_EINVAL;
      }
      bg->ps.reset(new PSched());
      ST_TRY(build_psched(rec, dt, conc ? n_plans : 1, dev, bg->ps.get()));
    } else {
      hipStream_t cs = nullptr;
      HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      // one stream (and one join event) per template for the parallel branches
      std::vector<hipStream_t> sp(n_plans, cs);
      std::vector<hipEvent_t> done(n_plans, nullptr);
      hipEvent_t fork = nullptr;
      hipError_t he = hipSuccess;
      if (conc) {
        he = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        for (int p = 0; p < n_plans && he == hipSuccess; ++p) {
          he = hipStreamCreateWithFlags(&sp[p], hipStreamNonBlocking);
          if (he == hipSuccess) he = hipEventCreateWithFlags(&done[p], hipEventDisableTiming);
        }
      }
      hipGraph_t graph = nullptr;
      sg2v_status st = SG2V_OK;
      if (he == hipSuccess) he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (he == hipSuccess) {
        t_capturing = true;
        launch_fill_u32((unsigned *)ws.ovf.p, 1, 0u, cs);
        if (conc) he = hipEventRecord(fork, cs);
        for (int p = 0; p < n_plans && st == SG2V_OK && he == hipSuccess; ++p) {
          if (conc) he = hipStreamWaitEvent(sp[p], fork, 0);
          if (he != hipSuccess) break;
          launch_color(bg->cols[p]->d, g->n, plans[p]->p.k, seed, 0, ncol, g->orig_id, sp[p]);
          xs[p].s = sp[p];
          xs[p].c = bg->cols[p].get();
          st = enqueue_count(xs[p], ncol, bs[p], res + (size_t)p * ncol * 8, Ed + (size_t)p * ncol);
          if (conc && st == SG2V_OK) {
            he = hipEventRecord(done[p], sp[p]);
            if (he == hipSuccess) he = hipStreamWaitEvent(cs, done[p], 0);
          }
        }
        t_capturing = false;
        hipError_t he2 = hipStreamEndCapture(cs, &graph);
        if (he == hipSuccess) he = he2;
      }
      if (he == hipSuccess && st == SG2V_OK) he = hipGraphInstantiate(&bg->exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (conc) {
        for (int p = 0; p < n_plans; ++p) {
          if (sp[p] && sp[p] != cs) (void)hipStreamDestroy(sp[p]);
          if (done[p]) (void)hipEventDestroy(done[p]);
        }
        if (fork) (void)hipEventDestroy(fork);
      }
      (void)hipStreamDestroy(cs);
      if (st != SG2V_OK) return st;
      if (he != hipSuccess) {
        set_error("sg2v_count_batch: graph capture failed: %s", hipGetErrorString(he));
        return SG2V_EDEVICE;
      }
    }
    ws_gens(ws, bg->gens);
    g_batch_cache.push_back(std::move(bg));
    if (g_batch_cache.size() > 8) g_batch_cache.erase(g_batch_cache.begin());
    hit = g_batch_cache.back().get();
  }
  if (hit->ps) {
    launch_fill_u32((unsigned *)ws.ovf.p, 1, 0u, us);
    run_psched(*hit->ps, us);
    HIP_TRY(hipGetLastError());
  } else {
    HIP_TRY(hipGraphLaunch(hit->exec, us));
  }
  std::vector<double> rf((size_t)n_plans * ncol);
  std::vector<uint64_t> ru((size_t)n_plans * ncol);
  std::vector<int> E((size_t)n_plans * ncol, 0);
  HIP_TRY(hipMemcpyAsync(dt == DT_U64 ? (void *)ru.data() : (void *)rf.data(), res,
                         (size_t)n_plans * ncol * 8, hipMemcpyDeviceToHost, us));
  if (dt == DT_F32)
    HIP_TRY(hipMemcpyAsync(E.data(), Ed, (size_t)n_plans * ncol * 4, hipMemcpyDeviceToHost, us));
  int perr = 0;
  if (hit->ps) HIP_TRY(hipMemcpyAsync(&perr, hit->ps->err(), 4, hipMemcpyDeviceToHost, us));
  HIP_TRY(hipStreamSynchronize(us));
  if (perr) {
    set_error("sg2v_count_batch: a dependency wait of the persistent schedule timed out");
    return SG2V_EDEVICE;
  }
  for (int p = 0; p < n_plans; ++p)
    finish_counts(plans[p]->p.roots[0], ncol, dt, rf.data() + (size_t)p * ncol, ru.data() + (size_t)p * ncol,
                  E.data() + (size_t)p * ncol, colorful ? colorful + (size_t)p * ncol : nullptr,
                  nullptr, estimate ? estimate + (size_t)p * ncol : nullptr, nullptr);
  return SG2V_OK;
}

// Reverse-mode derivative of f = sum_j g_j * colourful_j with respect to the
// CSR weights.  Splits are visited in reverse topological order with the
// adjoint Mbar_s of each node complete (all its consumers come later in the
// forward order).  For a split s = (a, p), B = A_G M_p, M_s = eMA(M_a, B):
//   Mbar_a += sum over C containing I_a of Mbar_s(i, C) B(i, C \ I_a)
//   Bbar    = sum over C containing I_p of Mbar_s(i, C) M_a(i, C \ I_p)
//   grad[e = i->j] += sum_c Bbar(i, c) M_p(j, c)
//   Mbar_p += A_G Bbar                       (A_G symmetric)
// The forward tables M_a, M_p and B of each split are recomputed by a forward
// pass that stops before the split, not stored.
// FP32S adjoint: the sweep of the FP64 adjoint below with FP32 tables.  Each
// adjoint table holds FP32 mantissas and one power-of-two exponent per
// colouring, kept on the host (INT_MIN: the table is zero).  Before an
// adjoint table is multiplied, its maximum is brought below 1 by an exact
// power of two; a contribution to a table that already holds values is added
// after both are brought to the larger exponent (k_scale_add).  The forward
// tables are recomputed in FP32S and their frame exponents read back; the
// per-entry gradient accumulates in FP64.
// Forward tables for the adjoint sweep (checkpointing).  When every table the
// sweep reads -- each split's active and passive tables and each passive
// child's aggregation -- fits the memory budget (the tuning's budget, else half
// of the free device memory), one forward pass per colouring keeps them all;
// otherwise each split recomputes a forward pass up to itself, as before.
PassOpts keep_every(const Plan &P) {
  PassOpts o;
  o.no_fuse = true;
  for (size_t q = 0; q < P.nodes.size(); ++q) {
    const Node &nd = P.nodes[q];
    if (nd.size > 1 && P.root_index[q] < 0) o.keep.push_back({(int)q, 0});
    if (nd.n_passive_uses > 0) o.keep.push_back({(int)q, 1});
  }
  return o;
}

bool keep_all_fits(const Plan &P, const sg2v_graph *g, int dt, int G, const PassOpts &every) {
  const sg2v_tuning_t tu = tuning();
  if (tu.flags & SG2V_TUNE_GRAD_RECOMPUTE) return false;
  PassPlan pp;
  build_pass(P, g->n, 1, dt, G, g->n_slots, pp, every);
  size_t fr = 0, tot = 0;
  (void)hipMemGetInfo(&fr, &tot);
  const double budget = tu.budget_bytes > 0 ? (double)tu.budget_bytes : 0.5 * (double)fr;
  return (double)pp.arena <= budget;
}

sg2v_status count_grad_fp32s(const sg2v_plan *plan, sg2v_graph *gg, const sg2v_colorings *c,
                             const double *grad_colorful, double *grad_w, hipStream_t s) {
  const Plan &P = plan->p;
  const sg2v_graph *g = gg;
  const size_t nn = P.nodes.size();
  int64_t widest = 1;
  for (auto &nd : P.nodes)
    if (nd.n_passive_uses > 0) widest = std::max(widest, nd.size == 1 ? P.k : nd.cols);
  const int G = pick_G(DT_F32, widest, g->n);
  const int W = G * 4;
  const int64_t align = std::max<int64_t>(32, W);
  std::vector<int64_t> off(nn, -1), ld(nn, 0);
  int64_t top = 0, bbar_ld = 0, maxld = 1, maxcols = 1;
  for (size_t q = 0; q < nn; ++q) {
    const Node &nd = P.nodes[q];
    if (nd.n_passive_uses > 0) bbar_ld = std::max(bbar_ld, round_up(nd.size == 1 ? P.k : nd.cols, align));
    maxcols = std::max(maxcols, nd.size == 1 ? (int64_t)P.k : nd.cols);
    if (nd.size == 1) continue;
    ld[q] = round_up(nd.cols, align);
    maxld = std::max(maxld, ld[q]);
    off[q] = top;
    top += round_up(g->n * ld[q] * 4, 256);
  }
  maxld = std::max(maxld, bbar_ld);
  const int64_t bbar_off = top;
  top += round_up(g->n * bbar_ld * 4, 256);
  const int64_t tmp_off = top;  // contributions before they are added
  top += round_up(g->n * maxld * 4, 256);
  const int64_t part_off = top;  // long-row partial rows of the adjoint SpMM
  top += round_up(std::max<int64_t>(g->n_slots, 1) * maxld * 4, 256);
  const int64_t small_off = top;  // column maxima, factors, exponents
  top += round_up(maxcols * 12 + 64, 256);
  Workspace &ws = workspace();
  ST_TRY(ws.grad.ensure(top));
  char *gbase = (char *)ws.grad.p;
  float *bbar = (float *)(gbase + bbar_off);
  float *tmp = (float *)(gbase + tmp_off);
  unsigned *mxb = (unsigned *)(gbase + small_off);
  float *fq = (float *)(gbase + small_off + maxcols * 4);
  int *esd = (int *)(gbase + small_off + maxcols * 8);
  int *zero = esd + maxcols;  // one int, 0: the exponents the FP32S kernels add
  auto mbar = [&](int q) { return (float *)(gbase + off[q]); };
  launch_fill_u32((unsigned *)zero, 1, 0u, s);

  // exponent shift d with max(X) * 2^-d < 1, INT_MIN for an all-zero table
  std::vector<unsigned> hmx((size_t)maxcols);
  auto shift_of = [&](const float *X, int64_t ldx, int64_t cols, int *d) -> sg2v_status {
    launch_fill_u32(mxb, cols, 0u, s);
    launch_colmax(X, g->n, ldx, cols, mxb, s);
    HIP_TRY(hipMemcpyAsync(hmx.data(), mxb, (size_t)cols * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    unsigned m = 0;
    for (int64_t q = 0; q < cols; ++q) m = std::max(m, hmx[q]);
    *d = m == 0 ? INT_MIN : (int)((m >> 23) & 0xFF) - 127 + 1;
    return SG2V_OK;
  };
  auto frame_of = [&](const Tab &t, int *E) -> sg2v_status {
    HIP_TRY(hipMemcpyAsync(E, t.E, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SG2V_OK;
  };
  // table Y (exponent *ey) += X (exponent ex)
  auto add_to = [&](float *Y, int64_t ldy, int *ey, const float *X, int64_t ldx, int64_t cols, int ex) {
    if (ex == INT_MIN) return;
    const int e = *ey == INT_MIN ? ex : std::max(*ey, ex);
    const float so = *ey == INT_MIN ? 0.f : std::ldexp(1.0f, *ey - e);
    launch_scale_add(Y, ldy, X, ldx, g->n, cols, so, std::ldexp(1.0f, ex - e), s);
    *ey = e;
  };

  std::vector<int> ebar(nn, INT_MIN);
  const PassOpts every = keep_every(P);
  const bool keep_all = keep_all_fits(P, g, DT_F32, G, every);
  Ctx xa;
  if (keep_all) ST_TRY(prepare(xa, plan, gg, c, SG2V_FP32S, 1, s, every));
  for (int j = 0; j < c->count; ++j) {
    if (grad_colorful[j] == 0.0) continue;
    if (keep_all) {
      ST_TRY(ws.result.ensure((size_t)c->count * 12 + 64));
      xa.j0 = j;
      ST_TRY(run_pass(xa, ws.result.p, (int *)((char *)ws.result.p + (size_t)c->count * 8), nullptr,
                      P.root));
    }
    launch_fill_value(DT_F32, gbase, bbar_off / 4, 0.0, s);
    std::fill(ebar.begin(), ebar.end(), INT_MIN);
    int eg = 0;
    // seed |g| as mantissa times 2^eg; every adjoint value carries the sign of g
    const double sg = grad_colorful[j] < 0.0 ? -1.0 : 1.0;
    const double mg = std::frexp(std::fabs(grad_colorful[j]), &eg);
    launch_fill_value(DT_F32, mbar(P.root), g->n * ld[P.root], mg, s);
    ebar[P.root] = eg;
    for (int q = (int)nn - 1; q >= 0; --q) {
      const Node &nd = P.nodes[q];
      if (nd.size == 1 || ebar[q] == INT_MIN) continue;
      const Node &A = P.nodes[nd.active];
      const Node &Pn = P.nodes[nd.passive];
      const int64_t cs = nd.cols, ca = A.size == 1 ? P.k : A.cols;
      int d = 0;
      ST_TRY(shift_of(mbar(q), ld[q], cs, &d));
      if (d == INT_MIN) continue;  // zero adjoint: no contributions
      const int eq = ebar[q] + d;
      launch_fill_value(DT_F32, fq, cs, std::ldexp(1.0, -d), s);
      Ctx xr;
      if (!keep_all) {
        PassOpts opt;
        opt.no_fuse = true;
        if (A.size > 1) opt.keep.push_back({nd.active, 0});
        if (Pn.size > 1) opt.keep.push_back({nd.passive, 0});
        opt.keep.push_back({nd.passive, 1});
        ST_TRY(prepare(xr, plan, gg, c, SG2V_FP32S, 1, s, opt));
        ST_TRY(ws.result.ensure((size_t)c->count * 12 + 64));
        xr.j0 = j;
        ST_TRY(run_pass(xr, ws.result.p, (int *)((char *)ws.result.p + (size_t)c->count * 8), nullptr, q));
      }
      Ctx &x = keep_all ? xa : xr;
      Tab &Bp = x.pp.B[nd.passive];
      const int64_t cp = Bp.cols;
      int EB = 0, EA = 0, EP = 0;
      ST_TRY(frame_of(Bp, &EB));
      if (A.size > 1) ST_TRY(frame_of(x.pp.M[nd.active], &EA));
      if (Pn.size > 1) ST_TRY(frame_of(x.pp.M[nd.passive], &EP));
      // Mbar_a += eMA^T over the active index
      if (A.size > 1) {
        EmaArgs a{};
        std::memset(&a, 0, sizeof(a));
        a.Ma = mbar(q);
        a.lda = ld[q];
        a.Ca = (int32_t)cs;
        a.fa = fq;
        a.B = Bp.p;
        a.ldb = Bp.ld;
        a.Cb = (int32_t)cp;
        a.fb = Bp.f;
        a.Ms = tmp;
        a.lds = ld[nd.active];
        a.Cs = (int32_t)ca;
        a.pairs = x.dp.tr_a[q];
        a.np = nd.np_ta;
        a.n = g->n;
        a.ovf = x.ovf;
        a.Ea = a.Eb = zero;
        a.es = esd;
        {
          ProfScope ps(SG2V_K_EMA_GENERAL, (double)g->n * (cs + cp + ca) * 4, (double)g->n * ca * nd.np_ta, s);
          ST_TRY(launch_general(x, a));
        }
        add_to(mbar(nd.active), ld[nd.active], &ebar[nd.active], tmp, ld[nd.active], ca, eq + EB);
      }
      // Bbar over the passive index
      int ebb = eq;
      {
        EmaArgs a{};
        std::memset(&a, 0, sizeof(a));
        a.Ms = bbar;
        a.lds = bbar_ld;
        a.Cs = (int32_t)cp;
        a.n = g->n;
        a.colors = c->d;
        a.j0 = j;
        a.ovf = x.ovf;
        a.es = esd;
        a.Ea = a.Eb = zero;
        if (A.size > 1) {
          Tab &Ma = x.pp.M[nd.active];
          a.Ma = mbar(q);
          a.lda = ld[q];
          a.Ca = (int32_t)cs;
          a.fa = fq;
          a.B = Ma.p;
          a.ldb = Ma.ld;
          a.Cb = (int32_t)ca;
          a.fb = Ma.f;
          a.pairs = x.dp.tr_p[q];
          a.np = nd.np_tp;
          ebb = eq + EA;
          ProfScope ps(SG2V_K_EMA_GENERAL, (double)g->n * (cs + ca + cp) * 4, (double)g->n * cp * nd.np_tp, s);
          ST_TRY(launch_general(x, a));
        } else {
          a.B = mbar(q);
          a.ldb = ld[q];
          a.Cb = (int32_t)cs;
          a.fb = fq;
          a.drop = x.dp.add[q];
          a.nb = 1;
          const int64_t rows = std::max<int64_t>(1, 8192 / cp);
          dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((g->n + rows - 1) / rows, 2048)), 1);
          ProfScope ps(SG2V_K_EMA_SINGLE, (double)g->n * (cs + cp) * 4, (double)g->n * cp, s);
          launch_ema_single(DT_F32, a, grid, 0, s);
        }
      }
      // edge gradient
      {
        SddmmArgs dd{};
        dd.row_ptr = g->row_ptr;
        dd.col_idx = g->col_idx;
        dd.Bbar = bbar;
        dd.ldb = bbar_ld;
        dd.Mp = Pn.size > 1 ? x.pp.M[nd.passive].p : nullptr;
        dd.ldm = Pn.size > 1 ? x.pp.M[nd.passive].ld : 0;
        dd.fm = Pn.size > 1 ? x.pp.M[nd.passive].f : nullptr;
        dd.scale = sg * std::ldexp(1.0, ebb + (Pn.size > 1 ? EP : 0));
        dd.ncols = cp;
        dd.n = g->n;
        dd.colors = c->d;
        dd.j0 = j;
        dd.b = 1;
        dd.k = P.k;
        dd.grad = grad_w;
        ProfScope ps(SG2V_K_SPMM, (double)g->nnz * 12 + (double)g->n * cp * 8, (double)g->nnz * cp, s);
        launch_sddmm(DT_F32, dd, s);
      }
      // Mbar_p += A_G Bbar
      if (Pn.size > 1) {
        UnitTable *U = nullptr;
        ST_TRY(build_units(gg, G, s, &U));
        SpmmArgs a{};
        a.col_idx = g->col_idx;
        a.w = g->w;
        a.task_row = g->task_row;
        a.task_beg = g->task_beg;
        a.task_len = g->task_len;
        a.task_slot = g->task_slot;
        a.unit_task = U->unit_task;
        a.unit_rpw = U->unit_rpw;
        a.unit_ntask = U->unit_ntask;
        a.n_units = U->n_units;
        a.M = bbar;
        a.ldm = bbar_ld;
        a.B = tmp;
        a.ldb = ld[nd.passive];
        a.partial = gbase + part_off;
        a.ncols_valid = cp;
        a.ovf = x.ovf;
        a.colors = c->d;
        a.j0 = j;
        a.n = g->n;
        a.nnz = g->nnz;
        const int64_t chunks = (cp + W - 1) / W;
        dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(U->n_units, kSpmmBlocks)), (unsigned)chunks);
        {
          ProfScope ps(SG2V_K_SPMM, 2.0 * g->n * cp * 4 + (double)chunks * g->nnz * 8, (double)g->nnz * cp, s);
          if (launch_spmm(DT_F32, a, G, 4, grid, s)) {
            set_error("sg2v_count_grad: no SpMM variant for G=%d", G);
            return SG2V_EINVAL;
          }
        }
        CombineArgs cb{};
        cb.partial = a.partial;
        cb.B = tmp;
        cb.ld = a.ldb;
        cb.ncols_valid = cp;
        cb.long_row = g->long_row;
        cb.long_slot0 = g->long_slot0;
        cb.long_nslot = g->long_nslot;
        cb.n_long = g->n_long;
        cb.ovf = x.ovf;
        launch_spmm_combine(DT_F32, cb, s);
        add_to(mbar(nd.passive), ld[nd.passive], &ebar[nd.passive], tmp, ld[nd.passive], cp, ebb);
      }
      HIP_TRY(hipGetLastError());
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  return SG2V_OK;
}

namespace {
sg2v_status count_grad_stored(const sg2v_plan *plan, const sg2v_graph *g, const sg2v_colorings *c,
                              sg2v_mode mode, const double *grad_colorful, void *grad_w,
                              void *stream);
}  // namespace

extern "C" sg2v_status sg2v_count_grad(const sg2v_plan *plan, const sg2v_graph *g,
                                       const sg2v_colorings *c, sg2v_mode mode,
                                       const double *grad_colorful, void *grad_w,
                                       void *stream) {
  if (!g || !g->relabelled || !grad_w)
    return count_grad_stored(plan, g, c, mode, grad_colorful, grad_w, stream);
  // renumbered graph: gradients in stored entry order, then back to the caller's
  sg2v_graph *gg = (sg2v_graph *)g;
  ST_TRY(gg->grad_tmp.ensure((size_t)std::max<int64_t>(g->nnz, 1) * 8));
  ST_TRY(count_grad_stored(plan, g, c, mode, grad_colorful, gg->grad_tmp.p, stream));
  launch_scatter_f64((const double *)gg->grad_tmp.p, g->entry_orig, (double *)grad_w, g->nnz,
                     (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return SG2V_OK;
}

namespace {
sg2v_status count_grad_stored(const sg2v_plan *plan, const sg2v_graph *g, const sg2v_colorings *c,
                              sg2v_mode mode, const double *grad_colorful, void *grad_w,
                              void *stream) {
  ST_TRY(check_inputs(plan, g, c, mode));
  if (plan->p.roots.size() != 1) {
    set_error("sg2v_count_grad: the plan holds several templates (one template only)");
    return SG2V_EINVAL;
  }
  if (mode != SG2V_FP64 && mode != SG2V_FP32S) {
    set_error("sg2v_count_grad: mode must be SG2V_FP64 or SG2V_FP32S");
    return SG2V_EINVAL;
  }
  if (!grad_colorful || !grad_w) {
    set_error("sg2v_count_grad: null gradient buffer");
    return SG2V_EINVAL;
  }
  const Plan &P = plan->p;
  hipStream_t s = (hipStream_t)stream;
  sg2v_graph *gg = (sg2v_graph *)g;
  launch_fill_value(DT_F64, grad_w, g->nnz, 0.0, s);
  HIP_TRY(hipGetLastError());
  if (P.root_kind == ROOT_VERTEX) {
    HIP_TRY(hipStreamSynchronize(s));
    return SG2V_OK;
  }
  if (mode == SG2V_FP32S) return count_grad_fp32s(plan, gg, c, grad_colorful, (double *)grad_w, s);
  const size_t nn = P.nodes.size();
  int64_t widest = 1;
  for (auto &nd : P.nodes)
    if (nd.n_passive_uses > 0) widest = std::max(widest, nd.size == 1 ? P.k : nd.cols);
  const int G = pick_G(DT_F64, widest, g->n);
  const int64_t align = std::max<int64_t>(16, (int64_t)G * 2);
  // adjoint tables of every node with more than one vertex, plus Bbar
  std::vector<int64_t> off(nn, -1), ld(nn, 0);
  int64_t top = 0, bbar_ld = 0;
  for (size_t q = 0; q < nn; ++q) {
    const Node &nd = P.nodes[q];
    if (nd.n_passive_uses > 0) bbar_ld = std::max(bbar_ld, round_up(nd.size == 1 ? P.k : nd.cols, align));
    if (nd.size == 1) continue;
    ld[q] = round_up(nd.cols, align);
    off[q] = top;
    top += round_up(g->n * ld[q] * 8, 256);
  }
  const int64_t bbar_off = top;
  top += round_up(g->n * bbar_ld * 8, 256);
  Workspace &ws = workspace();
  ST_TRY(ws.grad.ensure(top));
  char *gbase = (char *)ws.grad.p;
  double *bbar = (double *)(gbase + bbar_off);
  auto mbar = [&](int q) { return (double *)(gbase + off[q]); };

  const PassOpts every = keep_every(P);
  const bool keep_all = keep_all_fits(P, g, DT_F64, G, every);
  Ctx xa;
  if (keep_all) ST_TRY(prepare(xa, plan, gg, c, mode, 1, s, every));
  for (int j = 0; j < c->count; ++j) {
    if (keep_all) {
      ST_TRY(ws.result.ensure((size_t)c->count * 12 + 64));
      xa.j0 = j;
      ST_TRY(run_pass(xa, ws.result.p, (int *)((char *)ws.result.p + (size_t)c->count * 8), nullptr,
                      P.root));
    }
    launch_fill_value(DT_F64, gbase, bbar_off / 8, 0.0, s);
    launch_fill_value(DT_F64, mbar(P.root), g->n * ld[P.root], grad_colorful[j], s);
    for (int q = (int)nn - 1; q >= 0; --q) {
      const Node &nd = P.nodes[q];
      if (nd.size == 1) continue;
      const Node &A = P.nodes[nd.active];
      const Node &Pn = P.nodes[nd.passive];
      Ctx xr;
      if (!keep_all) {
        PassOpts opt;
        opt.no_fuse = true;
        if (A.size > 1) opt.keep.push_back({nd.active, 0});
        if (Pn.size > 1) opt.keep.push_back({nd.passive, 0});
        opt.keep.push_back({nd.passive, 1});
        ST_TRY(prepare(xr, plan, gg, c, mode, 1, s, opt));
        ST_TRY(ws.result.ensure((size_t)c->count * 12 + 64));
        xr.j0 = j;
        ST_TRY(run_pass(xr, ws.result.p, (int *)((char *)ws.result.p + (size_t)c->count * 8), nullptr,
                        q));
      }
      Ctx &x = keep_all ? xa : xr;
      Tab &Bp = x.pp.B[nd.passive];
      const int64_t cs = nd.cols, ca = A.size == 1 ? P.k : A.cols, cp = Bp.cols;
      // Mbar_a += eMA^T over the active index
      if (A.size > 1) {
        EmaArgs a{};
        std::memset(&a, 0, sizeof(a));
        a.Ma = mbar(q);
        a.lda = ld[q];
        a.Ca = (int32_t)cs;
        a.B = Bp.p;
        a.ldb = Bp.ld;
        a.Cb = (int32_t)cp;
        a.Ms = mbar(nd.active);
        a.lds = ld[nd.active];
        a.Cs = (int32_t)ca;
        a.pairs = x.dp.tr_a[q];
        a.np = nd.np_ta;
        a.n = g->n;
        a.ovf = x.ovf;
        a.accumulate = 1;
        ProfScope ps(SG2V_K_EMA_GENERAL, (double)g->n * (cs + cp + 2 * ca) * 8,
                     (double)g->n * ca * nd.np_ta, s);
        ST_TRY(launch_general(x, a));
      }
      // Bbar over the passive index
      {
        EmaArgs a{};
        std::memset(&a, 0, sizeof(a));
        a.Ms = bbar;
        a.lds = bbar_ld;
        a.Cs = (int32_t)cp;
        a.n = g->n;
        a.colors = c->d;
        a.j0 = j;
        a.ovf = x.ovf;
        if (A.size > 1) {
          Tab &Ma = x.pp.M[nd.active];
          a.Ma = mbar(q);
          a.lda = ld[q];
          a.Ca = (int32_t)cs;
          a.B = Ma.p;
          a.ldb = Ma.ld;
          a.Cb = (int32_t)ca;
          a.pairs = x.dp.tr_p[q];
          a.np = nd.np_tp;
          ProfScope ps(SG2V_K_EMA_GENERAL, (double)g->n * (cs + ca + cp) * 8,
                       (double)g->n * cp * nd.np_tp, s);
          ST_TRY(launch_general(x, a));
        } else {
          a.B = mbar(q);
          a.ldb = ld[q];
          a.Cb = (int32_t)cs;
          a.drop = x.dp.add[q];
          a.nb = 1;
          const int64_t rows = std::max<int64_t>(1, 8192 / cp);
          dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((g->n + rows - 1) / rows, 2048)), 1);
          ProfScope ps(SG2V_K_EMA_SINGLE, (double)g->n * (cs + cp) * 8, (double)g->n * cp, s);
          launch_ema_single(DT_F64, a, grid, 0, s);
        }
      }
      // edge gradient
      {
        SddmmArgs d{};
        d.row_ptr = g->row_ptr;
        d.col_idx = g->col_idx;
        d.Bbar = bbar;
        d.ldb = bbar_ld;
        d.Mp = Pn.size > 1 ? x.pp.M[nd.passive].p : nullptr;
        d.ldm = Pn.size > 1 ? x.pp.M[nd.passive].ld : 0;
        d.ncols = cp;
        d.n = g->n;
        d.colors = c->d;
        d.j0 = j;
        d.b = 1;
        d.k = P.k;
        d.grad = (double *)grad_w;
        d.scale = 1.0;
        ProfScope ps(SG2V_K_SPMM, (double)g->nnz * 12 + (double)g->n * cp * 16,
                     (double)g->nnz * cp, s);
        launch_sddmm(DT_F64, d, s);
      }
      // Mbar_p += A_G Bbar
      if (Pn.size > 1) {
        UnitTable *U = nullptr;
        ST_TRY(build_units(gg, x.pp.G, s, &U));
        const int W = x.pp.G * 2;
        SpmmArgs a{};
        a.col_idx = g->col_idx;
        a.w = g->w;
        a.task_row = g->task_row;
        a.task_beg = g->task_beg;
        a.task_len = g->task_len;
        a.task_slot = g->task_slot;
        a.unit_task = U->unit_task;
        a.unit_rpw = U->unit_rpw;
        a.unit_ntask = U->unit_ntask;
        a.n_units = U->n_units;
        a.M = bbar;
        a.ldm = bbar_ld;
        a.B = mbar(nd.passive);
        a.ldb = ld[nd.passive];
        a.partial = (char *)x.ws->arena.p + x.pp.partial_off;
        a.ncols_valid = cp;
        a.mx = nullptr;
        a.ovf = x.ovf;
        a.accumulate = 1;
        a.chunk_jb = nullptr;
        a.chunk_union = a.chunk_inter = nullptr;
        a.colors = c->d;
        a.j0 = j;
        a.n = g->n;
        a.nbr_col = nullptr;
        a.nnz = g->nnz;
        a.chunk0 = 0;  // one launch over every chunk, no neighbour-range split
        a.xsplit = 0;
        a.xunits = 0;
        a.tsplit = nullptr;
        a.partial8 = nullptr;
        const int64_t chunks = (cp + W - 1) / W;
        dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(U->n_units, kSpmmBlocks)),
                  (unsigned)chunks);
        {
          ProfScope ps(SG2V_K_SPMM, 2.0 * g->n * cp * 8 + (double)chunks * g->nnz * 8,
                       (double)g->nnz * cp, s);
          if (launch_spmm(DT_F64, a, x.pp.G, 4, grid, s)) {
            set_error("sg2v_count_grad: no SpMM variant for G=%d", x.pp.G);
            return SG2V_EINVAL;
          }
        }
        CombineArgs cb{};
        cb.partial = a.partial;
        cb.B = a.B;
        cb.ld = a.ldb;
        cb.ncols_valid = cp;
        cb.long_row = g->long_row;
        cb.long_slot0 = g->long_slot0;
        cb.long_nslot = g->long_nslot;
        cb.n_long = g->n_long;
        cb.mx = nullptr;
        cb.ovf = x.ovf;
        cb.accumulate = 1;
        launch_spmm_combine(DT_F64, cb, s);
      }
      HIP_TRY(hipGetLastError());
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  return SG2V_OK;
}
}  // namespace

extern "C" sg2v_status sg2v_set_tuning(const sg2v_tuning_t *t) {
  if (!t) {
    set_error("sg2v_set_tuning: null");
    return SG2V_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune = *t;
  return SG2V_OK;
}

extern "C" sg2v_status sg2v_get_tuning(sg2v_tuning_t *t) {
  if (!t) {
    set_error("sg2v_get_tuning: null");
    return SG2V_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  *t = g_tune;
  return SG2V_OK;
}

void drop_batch_graphs(const sg2v_graph *g) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (size_t i = 0; i < g_batch_cache.size();) {
    if (g_batch_cache[i]->g == g)
      g_batch_cache.erase(g_batch_cache.begin() + i);
    else
      ++i;
  }
}

extern "C" void sg2v_plan_destroy(sg2v_plan *plan) {
  if (!plan) return;
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (size_t i = 0; i < g_batch_cache.size();) {
      auto &e = g_batch_cache[i];
      if (std::find(e->plans.begin(), e->plans.end(), plan) != e->plans.end())
        g_batch_cache.erase(g_batch_cache.begin() + i);
      else
        ++i;
    }
  }
  for (auto &d : plan->p.dev) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(d.device);
    for (void *q : d.pairs) (void)hipFree(q);
    for (void *q : d.drop) (void)hipFree(q);
    for (void *p : d.root_list) (void)hipFree(p);
    for (void *p : d.root_list16) (void)hipFree(p);
    for (void *q : d.tr_a) (void)hipFree(q);
    for (void *q : d.tr_p) (void)hipFree(q);
    for (void *q : d.add) (void)hipFree(q);
    for (auto &kv : d.chunks) (void)hipFree(kv.second);
    for (void *q : d.cpr) (void)hipFree(q);
    (void)hipSetDevice(cur);
  }
  delete plan;
}

extern "C" sg2v_status sg2v_profile_start(void) {
  Profiler &p = profiler();
  std::lock_guard<std::mutex> lk(p.mu);
  for (auto &r : p.recs) {
    p.pool.push_back(r.a);
    p.pool.push_back(r.b);
  }
  p.recs.clear();
  p.on = true;
  return SG2V_OK;
}

extern "C" sg2v_status sg2v_profile_stop(sg2v_prof_entry_t *out) {
  if (!out) {
    set_error("sg2v_profile_stop: null");
    return SG2V_EINVAL;
  }
  Profiler &p = profiler();
  std::lock_guard<std::mutex> lk(p.mu);
  p.on = false;
  for (int k = 0; k < SG2V_K_COUNT; ++k) {
    out[k].kind = k;
    out[k].launches = 0;
    out[k].ms = out[k].bytes = out[k].work = 0.0;
  }
  for (auto &r : p.recs) {
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    sg2v_prof_entry_t &e = out[r.kind];
    e.launches++;
    e.ms += ms;
    e.bytes += r.bytes;
    e.work += r.work;
    p.pool.push_back(r.a);
    p.pool.push_back(r.b);
  }
  p.recs.clear();
  return SG2V_OK;
}

namespace {

std::mutex g_autotune_mu;
std::map<std::string, sg2v_tuning_t> g_autotune;

std::string tune_key(const Plan &P, const sg2v_graph *g, sg2v_mode mode, int ncol) {
  std::ostringstream k;
  k << P.nodes[P.root].canon << "/k" << P.k << "/n" << g->n << "/nnz" << g->nnz << "/m" << mode
    << "/c" << ncol;
  return k.str();
}

void tune_file_load() {
  const char *f = std::getenv("SG2V_TUNE_CACHE");
  if (!f) return;
  std::ifstream in(f);
  std::string key;
  sg2v_tuning_t t{};
  while (in >> key >> t.spmm_width >> t.ema_rows >> t.batch >> t.flags >> t.budget_bytes >>
         t.xsplit_group >> t.launch_chunks >> t.xsplit_min)
    g_autotune[key] = t;
}

void tune_file_store(const std::string &key, const sg2v_tuning_t &t) {
  const char *f = std::getenv("SG2V_TUNE_CACHE");
  if (!f) return;
  std::ofstream out(f, std::ios::app);
  out << key << " " << t.spmm_width << " " << t.ema_rows << " " << t.batch << " " << t.flags
      << " " << t.budget_bytes << " " << t.xsplit_group << " " << t.launch_chunks << " "
      << t.xsplit_min << "\n";
}

}  // namespace

extern "C" sg2v_status sg2v_autotune(const sg2v_plan *plan, const sg2v_graph *g, sg2v_mode mode,
                                     int32_t n_colorings, void *stream, sg2v_tuning_t *out) {
  if (!plan || !g || n_colorings < 1 || plan->p.roots.size() != 1) {
    set_error("sg2v_autotune: bad argument (null handle, no colourings or several templates)");
    return SG2V_EINVAL;
  }
  const std::string key = tune_key(plan->p, g, mode, n_colorings);
  {
    std::lock_guard<std::mutex> lk(g_autotune_mu);
    static bool loaded = false;
    if (!loaded) {
      tune_file_load();
      loaded = true;
    }
    auto it = g_autotune.find(key);
    if (it != g_autotune.end()) {
      ST_TRY(sg2v_set_tuning(&it->second));
      if (out) *out = it->second;
      return SG2V_OK;
    }
  }
  const sg2v_tuning_t base = tuning();
  sg2v_colorings *c = nullptr;
  ST_TRY(sg2v_color(g, plan->p.k, 0x5EEDULL, 0, n_colorings, stream, &c));
  std::unique_ptr<sg2v_colorings> hold(c);
  std::vector<sg2v_tuning_t> cand;
  const int widths[] = {16, 32, 64, 128};
  const int rows[] = {4, 8, 16};
  const int skipfl = SG2V_TUNE_NO_COLOR_SKIP | SG2V_TUNE_SPMM_UNROLL4 | SG2V_TUNE_SPMM_UNROLL8 |
                     SG2V_TUNE_XSPLIT | SG2V_TUNE_SPMM_PANEL;
  for (int w : widths)
    for (int fl : {0, (int)SG2V_TUNE_NO_COLOR_SKIP, (int)SG2V_TUNE_SPMM_UNROLL4, (int)SG2V_TUNE_SPMM_UNROLL8,
                   (int)SG2V_TUNE_XSPLIT, (int)SG2V_TUNE_SPMM_PANEL}) {
      sg2v_tuning_t t = base;
      t.spmm_width = w;
      t.flags = (base.flags & ~skipfl) | fl;
      cand.push_back(t);
      if (fl == SG2V_TUNE_XSPLIT)  // the split threshold as well
        for (int xm : {256, 1024}) {
          t.xsplit_min = xm;
          cand.push_back(t);
        }
    }
  // candidates whose chunk width maps to the same row-segment lanes run the
  // same kernels: keep the first of each
  {
    int64_t widest = 1;
    for (auto &nd : plan->p.nodes)
      if (nd.n_passive_uses > 0) widest = std::max(widest, nd.size == 1 ? (int64_t)plan->p.k : nd.cols);
    const int dt = dtype_of(mode);
    std::vector<std::pair<int, int>> seen;
    std::vector<sg2v_tuning_t> uniq;
    for (auto &t : cand) {
      ST_TRY(sg2v_set_tuning(&t));
      const std::pair<int, int> key(pick_G(dt, widest, g->n), t.flags + (t.xsplit_min << 16));
      if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
      seen.push_back(key);
      uniq.push_back(t);
    }
    ST_TRY(sg2v_set_tuning(&base));
    cand.swap(uniq);
  }
  sg2v_tuning_t best = base;
  double best_ms = 1e300;
  // one untimed count, then the median of three timed ones; a candidate whose
  // untimed count takes over three times the best median so far is dropped
  auto time_one = [&](const sg2v_tuning_t &t, double *ms) -> sg2v_status {
    ST_TRY(sg2v_set_tuning(&t));
    double cf;
    auto w0 = std::chrono::steady_clock::now();
    ST_TRY(sg2v_count(plan, g, c, mode, stream, nullptr, nullptr, nullptr, &cf, nullptr));
    const double first = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
    if (first > 3.0 * best_ms) {
      *ms = first;
      return SG2V_OK;
    }
    double v[3];
    for (double &x : v) {
      auto t0 = std::chrono::steady_clock::now();
      ST_TRY(sg2v_count(plan, g, c, mode, stream, nullptr, nullptr, nullptr, &cf, nullptr));
      x = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    std::sort(v, v + 3);
    *ms = v[1];
    return SG2V_OK;
  };
  sg2v_status st = SG2V_OK;
  for (auto &t : cand) {
    double ms;
    if ((st = time_one(t, &ms)) != SG2V_OK) break;
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  if (st == SG2V_OK) {
    // then rows per eMA tile and colourings per pass around the best width
    std::vector<sg2v_tuning_t> more;
    for (int r : rows) {
      sg2v_tuning_t t = best;
      t.ema_rows = r;
      more.push_back(t);
    }
    for (int b : {1, 2, 4}) {
      if (b > n_colorings) break;
      sg2v_tuning_t t = best;
      t.batch = b;
      more.push_back(t);
    }
    for (auto &t : more) {
      double ms;
      if ((st = time_one(t, &ms)) != SG2V_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
  }
  if (st != SG2V_OK) {
    (void)sg2v_set_tuning(&base);
    return st;
  }
  ST_TRY(sg2v_set_tuning(&best));
  {
    std::lock_guard<std::mutex> lk(g_autotune_mu);
    g_autotune[key] = best;
    tune_file_store(key, best);
  }
  if (out) *out = best;
  return SG2V_OK;
}
