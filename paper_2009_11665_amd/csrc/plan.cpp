// Template planner: partition of a tree template into active/passive
// sub-templates (Sec. 2.3.2), deduplication of isomorphic rooted
// sub-templates, colour-set column indices (Table 1) and the split index
// tables consumed by the multiply-add (Alg. 3 stage 2, Alg. 5), the
// automorphism count alpha and the colourful probability P (Alg. 1).
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <new>

#include "internal.h"

namespace sg2v {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char *last_error() { return g_err; }

namespace {
// Pascal's triangle up to 64, filled when the library is loaded
struct BinomTable {
  int64_t t[65][65];
  BinomTable() {
    for (int x = 0; x <= 64; ++x) {
      t[x][0] = 1;
      for (int y = 1; y <= 64; ++y) t[x][y] = (x == 0) ? 0 : t[x - 1][y - 1] + t[x - 1][y];
    }
  }
};
const BinomTable g_binom;
}  // namespace

int64_t binom(int a, int b) {
  if (a < 0 || b < 0 || a > 64 || b > 64) return 0;
  return g_binom.t[a][b];
}

int64_t colex_rank(uint32_t mask) {
  int64_t r = 0;
  int i = 0;
  while (mask) {
    const int c = __builtin_ctz(mask);
    mask &= mask - 1;
    r += g_binom.t[c][++i];
  }
  return r;
}

uint32_t colex_unrank(int64_t rank, int m, int k) {
  // greedy from the largest element: c_m is the largest c with C(c, m) <= rank
  uint32_t mask = 0;
  int hi = k - 1;
  for (int i = m; i >= 1; --i) {
    int c = hi;
    while (binom(c, i) > rank) --c;
    mask |= 1u << c;
    rank -= binom(c, i);
    hi = c - 1;
  }
  return mask;
}

namespace {

struct Tree {
  int t = 0, root = -1;
  std::vector<std::vector<int>> ch;  // children in increasing vertex order
  std::vector<std::string> full_canon;
};

sg2v_status tree_from_parent(const int32_t *parent, int t, Tree &T) {
  T.t = t;
  T.ch.assign(t, {});
  int roots = 0;
  for (int v = 0; v < t; ++v) {
    if (parent[v] == -1) {
      T.root = v;
      ++roots;
    } else if (parent[v] < 0 || parent[v] >= t || parent[v] == v) {
      set_error("sg2v_plan_create: parent[%d] = %d out of range", v, parent[v]);
      return SG2V_ENOTTREE;
    }
  }
  if (roots != 1) {
    set_error("sg2v_plan_create: %d roots (exactly one parent entry must be -1)", roots);
    return SG2V_ENOTTREE;
  }
  // every vertex must reach the root (no cycles)
  for (int v = 0; v < t; ++v) {
    int u = v, steps = 0;
    while (u != T.root && steps++ <= t) u = parent[u];
    if (u != T.root) {
      set_error("sg2v_plan_create: vertex %d does not reach the root (cycle)", v);
      return SG2V_ENOTTREE;
    }
  }
  for (int v = 0; v < t; ++v)
    if (v != T.root) T.ch[parent[v]].push_back(v);
  // AHU canonical strings of full subtrees, leaves first
  T.full_canon.assign(t, "");
  std::function<const std::string &(int)> canon = [&](int v) -> const std::string & {
    std::vector<std::string> kids;
    for (int c : T.ch[v]) kids.push_back(canon(c));
    std::sort(kids.begin(), kids.end());
    std::string s = "(";
    for (auto &x : kids) s += x;
    s += ")";
    T.full_canon[v] = s;
    return T.full_canon[v];
  };
  canon(T.root);
  return SG2V_OK;
}

std::string kept_canon(const Tree &T, int v, int n_kept) {
  std::vector<std::string> kids;
  for (int i = 0; i < n_kept; ++i) kids.push_back(T.full_canon[T.ch[v][i]]);
  std::sort(kids.begin(), kids.end());
  std::string s = "(";
  for (auto &x : kids) s += x;
  return s + ")";
}

// |Aut| of a rooted tree: product over vertices of the automorphisms of the
// children and the factorials of the multiplicities of identical children.
int64_t rooted_aut(const std::vector<std::vector<int>> &adj, int v, int from,
                   std::vector<std::string> &canon) {
  int64_t a = 1;
  std::vector<std::string> kids;
  for (int u : adj[v]) {
    if (u == from) continue;
    a *= rooted_aut(adj, u, v, canon);
    kids.push_back(canon[u]);
  }
  std::sort(kids.begin(), kids.end());
  for (size_t i = 0; i < kids.size();) {
    size_t j = i;
    while (j < kids.size() && kids[j] == kids[i]) ++j;
    for (size_t f = 2; f <= j - i; ++f) a *= (int64_t)f;
    i = j;
  }
  std::string s = "(";
  for (auto &x : kids) s += x;
  canon[v] = s + ")";
  return a;
}

// |Aut(T)| of the unrooted tree: root at its centre; with two centres, also
// count the swap of the two halves when they are isomorphic.
int64_t tree_automorphisms(const int32_t *parent, int t) {
  if (t <= 1) return 1;
  std::vector<std::vector<int>> adj(t);
  for (int v = 0; v < t; ++v)
    if (parent[v] >= 0) {
      adj[v].push_back(parent[v]);
      adj[parent[v]].push_back(v);
    }
  std::vector<int> deg(t);
  std::vector<int> layer;
  for (int v = 0; v < t; ++v) {
    deg[v] = (int)adj[v].size();
    if (deg[v] <= 1) layer.push_back(v);
  }
  int remaining = t;
  while (remaining > 2) {
    std::vector<int> next;
    for (int v : layer) {
      --remaining;
      for (int u : adj[v])
        if (--deg[u] == 1) next.push_back(u);
    }
    layer = next;
  }
  std::vector<std::string> canon(t);
  if (remaining == 1 || layer.size() == 1) return rooted_aut(adj, layer[0], -1, canon);
  int c1 = layer[0], c2 = layer[1];
  int64_t a = rooted_aut(adj, c1, c2, canon) * rooted_aut(adj, c2, c1, canon);
  if (canon[c1] == canon[c2]) a *= 2;
  return a;
}

}  // namespace

sg2v_status plan_build(const int32_t *parent, int t, int k, Plan &out) {
  if (!parent) {
    set_error("sg2v_plan_create: parent is NULL");
    return SG2V_EINVAL;
  }
  const int32_t *ps[1] = {parent};
  const int32_t ts[1] = {t};
  return plan_build_multi(ps, ts, 1, k, out);
}

sg2v_status plan_build_multi(const int32_t *const *parents, const int32_t *ts, int n_templates,
                             int k, Plan &out) {
  if (!parents || !ts || n_templates < 1) {
    set_error("sg2v_plan_create: null template list or no template");
    return SG2V_EINVAL;
  }
  std::vector<Tree> trees(n_templates);
  for (int r = 0; r < n_templates; ++r) {
    const int t = ts[r];
    if (!parents[r]) {
      set_error("sg2v_plan_create: parent of template %d is NULL", r);
      return SG2V_EINVAL;
    }
    if (t < 1 || k < t || k > SG2V_KMAX) {
      set_error("sg2v_plan_create: need 1 <= t <= k <= %d (template %d: t=%d, k=%d)", SG2V_KMAX, r,
                t, k);
      return SG2V_ERANGE;
    }
    sg2v_status st = tree_from_parent(parents[r], t, trees[r]);
    if (st != SG2V_OK) return st;
  }
  Plan *P = &out;
  P->t = ts[0];
  P->k = k;
  P->parent.assign(parents[0], parents[0] + ts[0]);

  // Partition: node (v, n_kept) = v with its first n_kept children's subtrees.
  // Cut the edge to the last kept child: active = (v, n_kept - 1), passive =
  // (child, all its children).  Nodes are emitted after their children; a
  // rooted sub-template met again (in this template or an earlier one) reuses
  // the first node with its canonical form.
  std::map<std::string, int> by_canon;
  P->roots.assign(n_templates, RootInfo());
  for (int r = 0; r < n_templates; ++r) {
    const Tree &T = trees[r];
    std::function<int(int, int)> build = [&](int v, int n_kept) -> int {
      std::string key = kept_canon(T, v, n_kept);
      auto it = by_canon.find(key);
      if (it != by_canon.end()) return it->second;
      Node nd;
      nd.vertex = v;
      nd.n_kept = n_kept;
      nd.canon = key;
      if (n_kept > 0) {
        int tau = T.ch[v][n_kept - 1];
        nd.active = build(v, n_kept - 1);
        nd.passive = build(tau, (int)T.ch[tau].size());
        nd.size = P->nodes[nd.active].size + P->nodes[nd.passive].size;
      }
      nd.cols = binom(k, nd.size);
      P->nodes.push_back(nd);
      int id = (int)P->nodes.size() - 1;
      by_canon[key] = id;
      return id;
    };
    P->roots[r].node = build(T.root, (int)T.ch[T.root].size());
    P->roots[r].t = ts[r];
    P->roots[r].parent.assign(parents[r], parents[r] + ts[r]);
  }
  P->root = P->roots[0].node;
  for (auto &nd : P->nodes) {
    if (nd.active >= 0) P->nodes[nd.active].n_active_uses++;
    if (nd.passive >= 0) P->nodes[nd.passive].n_passive_uses++;
  }
  P->root_index.assign(P->nodes.size(), -1);
  for (int r = 0; r < n_templates; ++r) {
    const int nr = P->roots[r].node;
    if (P->root_index[nr] >= 0) {
      set_error("sg2v_plan_create: templates %d and %d are the same rooted tree",
                P->root_index[nr], r);
      return SG2V_EINVAL;
    }
    if (P->nodes[nr].n_active_uses || P->nodes[nr].n_passive_uses) {
      set_error("sg2v_plan_create: template %d is a rooted sub-template of another template", r);
      return SG2V_EINVAL;
    }
    P->root_index[nr] = r;
  }

  // Split tables: for each output set C (colex order), every subset S of C
  // with |S| = |T_a| taken in lexicographic order of positions within C.
  for (auto &nd : P->nodes) {
    if (nd.size == 1) continue;
    const Node &A = P->nodes[nd.active];
    const int m = nd.size, ma = A.size;
    nd.np = (int)binom(m, ma);
    nd.pairs.resize((size_t)nd.cols * nd.np * 2);
    std::vector<int> elem(m), pos(ma);
    for (int64_t r = 0; r < nd.cols; ++r) {
      uint32_t C = colex_unrank(r, m, k);
      for (int c = 0, i = 0; c < k; ++c)
        if (C >> c & 1u) elem[i++] = c;
      for (int i = 0; i < ma; ++i) pos[i] = i;
      for (int q = 0; q < nd.np; ++q) {
        uint32_t S = 0;
        for (int i = 0; i < ma; ++i) S |= 1u << elem[pos[i]];
        nd.pairs[((size_t)r * nd.np + q) * 2 + 0] = (int32_t)colex_rank(S);
        nd.pairs[((size_t)r * nd.np + q) * 2 + 1] = (int32_t)colex_rank(C & ~S);
        // next combination of positions
        int i = ma - 1;
        while (i >= 0 && pos[i] == m - ma + i) --i;
        if (i < 0) break;
        ++pos[i];
        for (int j = i + 1; j < ma; ++j) pos[j] = pos[j - 1] + 1;
      }
    }
    if (ma == 1) {
      nd.drop.assign((size_t)k * nd.cols, -1);
      for (int64_t r = 0; r < nd.cols; ++r) {
        uint32_t C = colex_unrank(r, m, k);
        for (int c = 0; c < k; ++c)
          if (C >> c & 1u) nd.drop[(size_t)c * nd.cols + r] = (int32_t)colex_rank(C & ~(1u << c));
      }
    }
  }

  // Adjoint tables: the same splits grouped by the active set and by the
  // passive set, and the one-vertex-active inverse (P -> P + {c}).
  for (auto &nd : P->nodes) {
    if (nd.size == 1) continue;
    const Node &A = P->nodes[nd.active];
    const Node &Pn = P->nodes[nd.passive];
    const int64_t ca = binom(k, A.size), cp = binom(k, Pn.size);
    nd.np_ta = (int)binom(k - A.size, Pn.size);
    nd.np_tp = (int)binom(k - Pn.size, A.size);
    nd.tr_a.assign((size_t)ca * nd.np_ta * 2, -1);
    nd.tr_p.assign((size_t)cp * nd.np_tp * 2, -1);
    std::vector<int> fa(ca, 0), fp(cp, 0);
    for (int64_t r = 0; r < nd.cols; ++r)
      for (int q = 0; q < nd.np; ++q) {
        const int32_t ia = nd.pairs[((size_t)r * nd.np + q) * 2 + 0];
        const int32_t ip = nd.pairs[((size_t)r * nd.np + q) * 2 + 1];
        const size_t xa = ((size_t)ia * nd.np_ta + fa[ia]++) * 2;
        nd.tr_a[xa] = (int32_t)r;
        nd.tr_a[xa + 1] = ip;
        const size_t xp = ((size_t)ip * nd.np_tp + fp[ip]++) * 2;
        nd.tr_p[xp] = (int32_t)r;
        nd.tr_p[xp + 1] = ia;
      }
    if (A.size == 1) {
      nd.add.assign((size_t)k * cp, -1);
      for (int64_t r = 0; r < cp; ++r) {
        const uint32_t Pm = colex_unrank(r, Pn.size, k);
        for (int c = 0; c < k; ++c)
          if (!(Pm >> c & 1u)) nd.add[(size_t)c * cp + r] = (int32_t)colex_rank(Pm | (1u << c));
      }
    }
  }

  // Colour-restricted tables of general splits (active child with more than
  // one vertex), built when every compact position fits 16 bits and the
  // per-colour pair lists stay below 2^26 entries.  The root split is reduced
  // from its children's tables (root lists below) and gets none.
  for (size_t ni = 0; ni < P->nodes.size(); ++ni) {
    Node &nd = P->nodes[ni];
    if (nd.size == 1 || P->root_index[ni] >= 0) continue;
    const Node &A = P->nodes[nd.active];
    const Node &Pn = P->nodes[nd.passive];
    if (A.size == 1) continue;
    const int m = nd.size, ma = A.size, mp = Pn.size;
    nd.c_sa = binom(k - 1, ma - 1);
    nd.c_sb = binom(k - 1, mp);
    nd.c_u = binom(k - 1, m - 1);
    nd.c_z = binom(k - 1, m);
    nd.c_q = (int)binom(m - 1, ma - 1);
    if (nd.c_sa >= 0xFFFF || nd.c_sb >= 0xFFFF || (double)k * nd.c_q * nd.c_u > (double)(1 << 26)) {
      nd.c_q = 0;
      continue;
    }
    const int64_t ca_cols = binom(k, ma), cb_cols = binom(k, mp);
    nd.ca.resize((size_t)k * nd.c_sa);
    nd.cb.resize((size_t)k * nd.c_sb);
    nd.co.resize((size_t)k * nd.c_u);
    nd.cz.resize((size_t)k * nd.c_z);
    nd.cp.resize((size_t)k * nd.c_q * nd.c_u);
    // compact positions: posa[c][I_a] among active sets holding c, posb[c][I_p]
    // among passive sets without c, and u[c][I_s] among output sets holding c
    std::vector<int32_t> posa((size_t)k * ca_cols, -1), posb((size_t)k * cb_cols, -1);
    std::vector<int32_t> ucol((size_t)k * nd.cols, -1);
    for (int c = 0; c < k; ++c) {
      int64_t na = 0, nb = 0, nu = 0, nz = 0;
      for (int64_t r = 0; r < ca_cols; ++r)
        if (colex_unrank(r, ma, k) >> c & 1u) {
          posa[(size_t)c * ca_cols + r] = (int32_t)na;
          nd.ca[(size_t)c * nd.c_sa + na++] = (int32_t)r;
        }
      for (int64_t r = 0; r < cb_cols; ++r)
        if (!(colex_unrank(r, mp, k) >> c & 1u)) {
          posb[(size_t)c * cb_cols + r] = (int32_t)nb;
          nd.cb[(size_t)c * nd.c_sb + nb++] = (int32_t)r;
        }
      for (int64_t r = 0; r < nd.cols; ++r) {
        if (colex_unrank(r, m, k) >> c & 1u) {
          ucol[(size_t)c * nd.cols + r] = (int32_t)nu;
          nd.co[(size_t)c * nd.c_u + nu++] = (int32_t)r;
        } else {
          nd.cz[(size_t)c * nd.c_z + nz++] = (int32_t)r;
        }
      }
    }
    // one walk over the pairs: a pair contributes to the colours of its
    // active set (M_a(i, I_a) = 0 for a vertex whose colour is not in I_a)
    std::vector<int32_t> qn(k);
    for (int64_t r = 0; r < nd.cols; ++r) {
      std::fill(qn.begin(), qn.end(), 0);
      for (int t = 0; t < nd.np; ++t) {
        const int32_t ia = nd.pairs[((size_t)r * nd.np + t) * 2 + 0];
        const int32_t ip = nd.pairs[((size_t)r * nd.np + t) * 2 + 1];
        uint32_t Am = colex_unrank(ia, ma, k);
        while (Am) {
          const int c = __builtin_ctz(Am);
          Am &= Am - 1;
          const int64_t u = ucol[(size_t)c * nd.cols + r];
          nd.cp[((size_t)c * nd.c_q + qn[c]) * nd.c_u + u] =
              (uint32_t)posa[(size_t)c * ca_cols + ia] | ((uint32_t)posb[(size_t)c * cb_cols + ip] << 16);
          ++qn[c];
        }
      }
    }
  }

  // Root reduction lists, one per template.
  P->fused.assign(P->nodes.size(), 0);
  for (int ri = 0; ri < n_templates; ++ri) {
    RootInfo &RI = P->roots[ri];
    const int t = RI.t;
    const Node &R = P->nodes[RI.node];
    if (R.size == 1) {
      RI.kind = ROOT_VERTEX;
    } else {
      const Node &A = P->nodes[R.active];
      RI.y_node = R.passive;
      std::vector<std::vector<int32_t>> lists(k);
      int64_t nout = binom(k, t);
      if (A.size == 1) {
        RI.kind = ROOT_SINGLE;
        RI.x_node = R.passive;
        RI.y_node = -1;
        for (int64_t r = 0; r < nout; ++r) {
          uint32_t C = colex_unrank(r, t, k);
          for (int c = 0; c < k; ++c)
            if (C >> c & 1u) {
              lists[c].push_back((int32_t)colex_rank(C & ~(1u << c)));
              lists[c].push_back(-1);
            }
        }
      } else {
        // fused: the active child is a one-vertex-active split used only here
        bool fuse = P->nodes[A.active].size == 1 && A.n_active_uses == 1 && A.n_passive_uses == 0;
        RI.kind = fuse ? ROOT_FUSED : ROOT_GENERAL;
        RI.x_node = fuse ? A.passive : R.active;
        if (fuse) P->fused[R.active] = 1;
        std::vector<uint32_t> amask(binom(k, A.size));
        for (size_t x = 0; x < amask.size(); ++x) amask[x] = colex_unrank((int64_t)x, A.size, k);
        for (int64_t r = 0; r < nout; ++r) {
          for (int q = 0; q < R.np; ++q) {
            int32_t ia = R.pairs[((size_t)r * R.np + q) * 2 + 0];
            int32_t ip = R.pairs[((size_t)r * R.np + q) * 2 + 1];
            uint32_t S = amask[ia];
            for (int c = 0; c < k; ++c)
              if (S >> c & 1u) {
                lists[c].push_back(fuse ? (int32_t)colex_rank(S & ~(1u << c)) : ia);
                lists[c].push_back(ip);
              }
          }
        }
      }
      RI.L = (int64_t)lists[0].size() / 2;
      RI.list.resize((size_t)k * RI.L * 2);
      for (int c = 0; c < k; ++c) {
        if ((int64_t)lists[c].size() != 2 * RI.L) {
          set_error("sg2v_plan_create: internal error (root list sizes differ)");
          return SG2V_EINVAL;
        }
        std::copy(lists[c].begin(), lists[c].end(), RI.list.begin() + (size_t)c * RI.L * 2);
      }
    }
    RI.alpha = tree_automorphisms(RI.parent.data(), t);
    double p = 1.0;
    for (int i = 0; i < t; ++i) p *= (double)(k - i) / (double)k;
    RI.P = p;
  }
  const RootInfo &R0 = P->roots[0];
  P->root_kind = R0.kind;
  P->root_x_node = R0.x_node;
  P->root_y_node = R0.y_node;
  P->root_L = R0.L;
  P->root_list = R0.list;
  P->alpha = R0.alpha;
  P->P = R0.P;
  return SG2V_OK;
}


// ---------------------------------------------------------------------------
// Choice of root and cut order (Sec. 2.3.2).  The colourful count sums the
// rooted counts over every image of the root, so it is the number of
// colourful injective maps of T and does not depend on which vertex is the
// root or in which order a vertex's children are cut; alpha is |Aut| of the
// unrooted tree.  Only the work of the decomposition changes.

namespace {

struct Rooted {
  int r = 0;
  std::vector<std::vector<int>> ch;  // children, in the order they are kept
  std::vector<int> size;
  std::vector<std::string> canon;    // AHU string of the full subtree
  std::vector<int> bfs;
};

Rooted root_at(const std::vector<std::vector<int>> &adj, int r) {
  const int t = (int)adj.size();
  Rooted R;
  R.r = r;
  R.ch.assign(t, {});
  R.size.assign(t, 1);
  R.canon.assign(t, "");
  std::vector<int> par(t, -2);
  par[r] = -1;
  R.bfs.push_back(r);
  for (size_t q = 0; q < R.bfs.size(); ++q) {
    const int v = R.bfs[q];
    for (int u : adj[v])
      if (par[u] == -2) {
        par[u] = v;
        R.ch[v].push_back(u);
        R.bfs.push_back(u);
      }
  }
  for (int q = t - 1; q >= 0; --q) {
    const int v = R.bfs[q];
    std::vector<std::string> kids;
    for (int u : R.ch[v]) {
      R.size[v] += R.size[u];
      kids.push_back(R.canon[u]);
    }
    std::sort(kids.begin(), kids.end());
    std::string s = "(";
    for (auto &x : kids) s += x;
    R.canon[v] = s + ")";
  }
  return R;
}

// Work of vertex v's splits for one child order: node (v, n) multiplies
// C(k, s_n) * C(s_n, s_{n-1}) pairs per vertex, s_n = 1 + sizes of the first
// n children; the last split of the root is its root reduction, C(k, s_{d-1}).
double local_pairs(const Rooted &R, int v, const std::vector<int> &order, int k) {
  double c = 0;
  int s = 1;
  for (size_t n = 0; n < order.size(); ++n) {
    const int s1 = s + R.size[order[n]];
    if (v == R.r && n + 1 == order.size()) c += (double)binom(k, s);
    else c += (double)binom(k, s1) * (double)binom(s1, s);
    s = s1;
  }
  return c;
}

// Per vertex, the child order with the least local work (every distinct order
// of the isomorphism classes while there are at most 8! of them, else by
// increasing subtree size); ties keep the current order.
void choose_orders(Rooted &R, int k) {
  for (size_t v = 0; v < R.ch.size(); ++v) {
    std::vector<int> &ch = R.ch[v];
    if (ch.size() < 2) continue;
    std::vector<int> best = ch;
    double best_c = local_pairs(R, (int)v, ch, k);
    std::vector<int> idx(ch.size());
    for (size_t i = 0; i < ch.size(); ++i) idx[i] = (int)i;
    auto cls = [&](int i) -> const std::string & { return R.canon[ch[i]]; };
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return cls(a) < cls(b) || (cls(a) == cls(b) && a < b); });
    double perms = 1;
    for (size_t i = 2; i <= ch.size(); ++i) perms *= (double)i;
    std::vector<int> order(ch.size());
    if (perms <= 40320.0) {
      // distinct arrangements of the class sequence: permute class labels
      std::vector<int> lab(ch.size());
      for (size_t i = 0; i < idx.size(); ++i)
        lab[i] = (i > 0 && cls(idx[i]) == cls(idx[i - 1])) ? lab[i - 1] : (int)i;
      std::vector<int> seq = lab;
      do {
        // the p-th member of a class goes to its p-th occurrence in seq
        std::map<int, int> used;
        for (size_t i = 0; i < seq.size(); ++i) {
          int p = used[seq[i]]++;
          order[i] = ch[idx[seq[i] + p]];
        }
        const double c = local_pairs(R, (int)v, order, k);
        if (c < best_c) {
          best_c = c;
          best = order;
        }
      } while (std::next_permutation(seq.begin(), seq.end()));
    } else {
      order = ch;
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return R.size[a] < R.size[b]; });
      const double c = local_pairs(R, (int)v, order, k);
      if (c < best_c) best = order;
    }
    ch = best;
  }
}

// Total work of the rooted, ordered tree with isomorphic sub-templates
// counted once (as the planner shares their tables).
double decomposition_cost(const Rooted &R, int k, double spmm_weight) {
  std::map<std::string, int> seen;  // kept-children key -> size
  std::map<std::string, int> passive;
  double pairs = 0;
  std::function<int(int, int, std::string *)> build = [&](int v, int n, std::string *key_out) -> int {
    std::vector<std::string> kids;
    for (int i = 0; i < n; ++i) kids.push_back(R.canon[R.ch[v][i]]);
    std::sort(kids.begin(), kids.end());
    std::string key = "(";
    for (auto &x : kids) key += x;
    key += ")";
    if (key_out) *key_out = key;
    auto it = seen.find(key);
    if (it != seen.end()) return it->second;
    int s = 1;
    if (n > 0) {
      const int tau = R.ch[v][n - 1];
      const int sa = build(v, n - 1, nullptr);
      std::string pk;
      const int sp = build(tau, (int)R.ch[tau].size(), &pk);
      s = sa + sp;
      if (sp >= 2) passive[pk] = sp;
      if (v == R.r && n == (int)R.ch[v].size()) pairs += (double)binom(k, sa);
      else pairs += (double)binom(k, s) * (double)binom(s, sa);
    }
    seen[key] = s;
    return s;
  };
  build(R.r, (int)R.ch[R.r].size(), nullptr);
  double cols = 0;
  for (auto &p : passive) cols += (double)binom(k, p.second);
  return spmm_weight * cols + pairs;
}

}  // namespace

sg2v_status template_reroot(const int32_t *parent, int t, int k, double spmm_weight,
                            int32_t *parent_out, int32_t *perm_out) {
  if (!parent || !parent_out) {
    set_error("sg2v_template_reroot: null argument");
    return SG2V_EINVAL;
  }
  if (t < 1 || k < t || k > SG2V_KMAX) {
    set_error("sg2v_template_reroot: need 1 <= t <= k <= %d (t=%d, k=%d)", SG2V_KMAX, t, k);
    return SG2V_ERANGE;
  }
  if (!(spmm_weight >= 0.0)) {
    set_error("sg2v_template_reroot: spmm_weight must be >= 0");
    return SG2V_EINVAL;
  }
  Tree T;
  sg2v_status st = tree_from_parent(parent, t, T);
  if (st != SG2V_OK) return st;
  std::vector<std::vector<int>> adj(t);
  for (int v = 0; v < t; ++v)
    if (v != T.root) {
      adj[v].push_back(parent[v]);
      adj[parent[v]].push_back(v);
    }
  for (auto &a : adj) std::sort(a.begin(), a.end());
  // the given root first, so that ties keep it
  Rooted best = root_at(adj, T.root);
  choose_orders(best, k);
  double best_c = decomposition_cost(best, k, spmm_weight);
  for (int r = 0; r < t; ++r) {
    if (r == T.root) continue;
    Rooted R = root_at(adj, r);
    choose_orders(R, k);
    const double c = decomposition_cost(R, k, spmm_weight);
    if (c < best_c) {
      best_c = c;
      best = std::move(R);
    }
  }
  // relabel breadth first, children in their chosen order, root 0
  std::vector<int> lab(t, -1), order{best.r};
  lab[best.r] = 0;
  for (size_t q = 0; q < order.size(); ++q)
    for (int u : best.ch[order[q]]) {
      lab[u] = (int)order.size();
      order.push_back(u);
    }
  parent_out[0] = -1;
  for (int v : order)
    for (int u : best.ch[v]) parent_out[lab[u]] = lab[v];
  if (perm_out)
    for (int v = 0; v < t; ++v) perm_out[v] = lab[v];
  return SG2V_OK;
}

}  // namespace sg2v

using namespace sg2v;

extern "C" {

const char *sg2v_last_error(void) { return sg2v::last_error(); }

const char *sg2v_version(void) { return "sg2v 0.1 (gfx950)"; }

sg2v_status sg2v_plan_create(const int32_t *parent, int32_t t, int32_t k, sg2v_plan **out) {
  if (!out) {
    set_error("sg2v_plan_create: out is NULL");
    return SG2V_EINVAL;
  }
  *out = nullptr;
  try {
    sg2v_plan *h = new sg2v_plan;
    sg2v_status st = plan_build(parent, t, k, h->p);
    if (st != SG2V_OK) {
      delete h;
      return st;
    }
    *out = h;
    return SG2V_OK;
  } catch (const std::bad_alloc &) {
    set_error("sg2v_plan_create: out of host memory");
    return SG2V_ENOMEM;
  }
}

sg2v_status sg2v_plan_create_multi(const int32_t *parents, const int32_t *sizes,
                                   int32_t n_templates, int32_t k, sg2v_plan **out) {
  if (!out || !parents || !sizes || n_templates < 1) {
    set_error("sg2v_plan_create_multi: null argument or no template");
    return SG2V_EINVAL;
  }
  *out = nullptr;
  try {
    std::vector<const int32_t *> ps(n_templates);
    int64_t off = 0;
    for (int r = 0; r < n_templates; ++r) {
      if (sizes[r] < 1 || sizes[r] > SG2V_KMAX) {
        set_error("sg2v_plan_create_multi: template %d has %d vertices", r, sizes[r]);
        return SG2V_ERANGE;
      }
      ps[r] = parents + off;
      off += sizes[r];
    }
    sg2v_plan *h = new sg2v_plan;
    sg2v_status st = plan_build_multi(ps.data(), sizes, n_templates, k, h->p);
    if (st != SG2V_OK) {
      delete h;
      return st;
    }
    *out = h;
    return SG2V_OK;
  } catch (const std::bad_alloc &) {
    set_error("sg2v_plan_create_multi: out of host memory");
    return SG2V_ENOMEM;
  }
}

sg2v_status sg2v_template_reroot(const int32_t *parent, int32_t t, int32_t k, double spmm_weight,
                                 int32_t *parent_out, int32_t *perm_out) {
  try {
    return template_reroot(parent, t, k, spmm_weight, parent_out, perm_out);
  } catch (const std::bad_alloc &) {
    set_error("sg2v_template_reroot: out of host memory");
    return SG2V_ENOMEM;
  }
}

sg2v_status sg2v_plan_info(const sg2v_plan *plan, sg2v_plan_info_t *out) {
  if (!plan || !out) {
    set_error("sg2v_plan_info: null argument");
    return SG2V_EINVAL;
  }
  const Plan &P = plan->p;
  memset(out, 0, sizeof(*out));
  out->t = P.t;
  out->k = P.k;
  out->n_nodes = (int32_t)P.nodes.size();
  out->root_node = P.root;
  out->alpha = P.alpha;
  out->colorful_prob = P.P;
  out->n_templates = (int32_t)P.roots.size();
  out->bytes_per_vertex_fp32 = pass_bytes_per_vertex(P, 1);
  out->bytes_per_vertex_fp64 = pass_bytes_per_vertex(P, 0);
  for (auto &nd : P.nodes) {
    if (nd.size > 1) {
      out->n_splits++;
      out->pairs_per_vertex += nd.cols * nd.np;
    }
    if (nd.n_passive_uses > 0) {
      out->n_passive++;
      out->spmm_columns += nd.cols;
    }
    out->widest_table = std::max(out->widest_table, nd.cols);
  }
  return SG2V_OK;
}

sg2v_status sg2v_plan_node(const sg2v_plan *plan, int32_t node, sg2v_node_info_t *out) {
  if (!plan || !out || node < 0 || node >= (int32_t)plan->p.nodes.size()) {
    set_error("sg2v_plan_node: bad argument");
    return SG2V_EINVAL;
  }
  const Node &nd = plan->p.nodes[node];
  out->size = nd.size;
  out->active = nd.active;
  out->passive = nd.passive;
  out->vertex = nd.vertex;
  out->n_kept = nd.n_kept;
  out->is_passive = nd.n_passive_uses > 0;
  out->columns = nd.cols;
  return SG2V_OK;
}

sg2v_status sg2v_plan_pairs(const sg2v_plan *plan, int32_t node, int32_t *out) {
  if (!plan || !out || node < 0 || node >= (int32_t)plan->p.nodes.size() ||
      plan->p.nodes[node].size < 2) {
    set_error("sg2v_plan_pairs: bad argument");
    return SG2V_EINVAL;
  }
  const Node &nd = plan->p.nodes[node];
  std::copy(nd.pairs.begin(), nd.pairs.end(), out);
  return SG2V_OK;
}

}  // extern "C"
