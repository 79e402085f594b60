// Internal structures shared by the planner (plan.cpp) and the device
// runtime (runtime.hip).  Not part of the public interface.
#pragma once

#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/sg2v.h"

namespace sg2v {

void set_error(const char *fmt, ...);

// binomial coefficients C(a, b) for 0 <= a, b <= 64 (exact in int64 for the
// sizes used here: a <= SG2V_KMAX).
int64_t binom(int a, int b);

// colexicographic rank of a colour set given as a bit mask (bit c = colour c):
// rank = sum_i C(c_i, i) over the sorted elements c_1 < ... < c_m.
int64_t colex_rank(uint32_t mask);
// inverse: the mask of size m with the given rank among k colours.
uint32_t colex_unrank(int64_t rank, int m, int k);

// One distinct rooted sub-template.  Nodes are stored children first.
struct Node {
  int size = 1;
  int active = -1;   // node id of the active child (keeps the root)
  int passive = -1;  // node id of the passive child (cut-off subtree)
  int vertex = 0;    // template vertex rooting the first occurrence
  int n_kept = 0;    // number of that vertex's first children it keeps
  int64_t cols = 0;  // C(k, size)
  int n_active_uses = 0;   // splits using this node as active child
  int n_passive_uses = 0;  // splits using this node as passive child
  std::string canon;       // rooted canonical form
  // split tables (size > 1):
  int np = 0;                  // pairs per output column = C(size, size_a)
  std::vector<int32_t> pairs;  // [cols][np] x (ia, ip)
  std::vector<int32_t> drop;   // active child is one vertex: [k][cols] -> rank(C\{c}) or -1
  // adjoint tables (reverse-mode derivative of the multiply-add):
  int np_ta = 0;               // pairs per active column = C(k - size_a, size_p)
  std::vector<int32_t> tr_a;   // [cols_a][np_ta] x (I_s, I_p): output sets containing I_a
  int np_tp = 0;               // pairs per passive column = C(k - size_p, size_a)
  std::vector<int32_t> tr_p;   // [cols_p][np_tp] x (I_s, I_a): output sets containing I_p
  std::vector<int32_t> add;    // active child is one vertex: [k][cols_p] -> rank(P + {c}) or -1
  // colour-restricted multiply-add (general splits): a vertex of colour c has
  // M_s(i, C) = 0 unless c is in C, and only pairs whose active set holds c
  // contribute.  Per colour c (all sizes are equal across colours):
  //   ca[c][*]  active columns holding c      (Sa = C(k-1, |T_a|-1))
  //   cb[c][*]  passive columns not holding c (Sb = C(k-1, |T_p|))
  //   co[c][*]  output columns holding c      (U  = C(k-1, |T_s|-1))
  //   cz[c][*]  output columns not holding c  (Z  = C(k-1, |T_s|))
  //   cp[c][q][u] = position in ca | position in cb << 16, q < Q = C(|T_s|-1, |T_a|-1)
  int64_t c_sa = 0, c_sb = 0, c_u = 0, c_z = 0;
  int c_q = 0;
  std::vector<int32_t> ca, cb, co, cz;
  std::vector<uint32_t> cp;
};

enum RootKind {
  ROOT_SINGLE = 0,   // root split's active child is one vertex:  X = B_Q, no Y
  ROOT_FUSED = 1,    // active child is itself a one-vertex-active split used only
                     // here: X = B of its passive, Y = B_Q
  ROOT_GENERAL = 2,  // X = M of the active child, Y = B_Q
  ROOT_VERTEX = 3,   // the template is one vertex
};

// Root reduction of one template of a plan.
struct RootInfo {
  int node = -1;               // node id of the template itself
  int t = 0;                   // template vertices
  int kind = ROOT_VERTEX;
  int x_node = -1, y_node = -1;
  int64_t L = 0;
  std::vector<int32_t> list;   // [k][L] x (x, y)
  int64_t alpha = 1;           // |Aut(T)|
  double P = 1.0;              // colourful probability
  std::vector<int32_t> parent; // the template as given
};

struct Plan {
  // The first (or only) template: t, parent, root, alpha, P and the root_*
  // fields below describe it.  A plan of several templates (treelet
  // distributions) shares its sub-template nodes across them and keeps one
  // RootInfo per template in `roots`.
  int t = 0, k = 0;
  std::vector<int32_t> parent;
  std::vector<Node> nodes;
  int root = -1;
  int64_t alpha = 1;
  double P = 1.0;
  // root reduction: for every colour c, L entries (x, y): the sum over the
  // list of X(i, x) * Y(i, y) equals sum_C M_0(i, C) for a vertex of colour c.
  int root_kind = ROOT_VERTEX;
  int root_x_node = -1;  // node whose B (or M for ROOT_GENERAL) is X
  int root_y_node = -1;  // node whose B is Y (-1: Y = 1)
  int64_t root_L = 0;
  std::vector<int32_t> root_list;  // [k][L] x (x, y)
  // nodes whose tables are never materialised (fused into the root)
  std::vector<char> fused;
  std::vector<RootInfo> roots;   // one per template, roots[0] = the fields above
  std::vector<int> root_index;   // per node: index into roots, or -1

  // device copies of the tables, uploaded on first use per device
  struct DeviceTables {
    int device = -1;
    std::vector<void *> pairs, drop;  // per node
    std::vector<void *> tr_a, tr_p, add;
    std::vector<void *> cpr;  // colour-restricted tables, one block per node
    std::vector<void *> root_list;    // per template
    std::vector<void *> root_list16;  // (x | y << 16), when every index fits 16 bits
    // SpMM colour-skip masks per (node, colourings per pass, chunk width)
    std::map<std::tuple<int, int, int>, void *> chunks;
  };
  mutable std::mutex mu;
  mutable std::vector<DeviceTables> dev;
};

sg2v_status plan_build(const int32_t *parent, int t, int k, Plan &out);
// Several templates over the same k, sharing isomorphic rooted sub-templates.
sg2v_status plan_build_multi(const int32_t *const *parents, const int32_t *ts, int n, int k,
                             Plan &out);
// Device workspace of one pass over one colouring, per vertex (runtime).
int64_t pass_bytes_per_vertex(const Plan &P, int fp32);
// Vertices of a registered graph (runtime).
int64_t graph_vertices(const sg2v_graph *g);

}  // namespace sg2v

struct sg2v_plan {
  sg2v::Plan p;
};
