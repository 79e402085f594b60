// Enumeration of the non-isomorphic (free, unlabelled) trees with t vertices:
// the template set of a treelet distribution (Sec. 2.1: the 47 treelets of
// nine vertices).  Host only.
//
// Trees of t vertices are all obtained by hanging one leaf on some vertex of a
// tree of t - 1 vertices, so the set is grown one vertex at a time and kept
// free of duplicates by a canonical form: the tree rooted at its centre (the
// one or two vertices left after stripping leaves repeatedly), written as the
// nested-parenthesis code whose children codes are sorted (Aho, Hopcroft and
// Ullman's rooted-tree isomorphism code); with two centres the smaller of the
// two codes.  Isomorphic trees have the same centres up to isomorphism, hence
// the same code, and the code determines the tree.
#include <algorithm>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

using namespace sg2v;

namespace {

using Adj = std::vector<std::vector<int>>;

std::string rooted_code(const Adj &adj, int v, int from) {
  std::vector<std::string> sub;
  for (int u : adj[v])
    if (u != from) sub.push_back(rooted_code(adj, u, v));
  std::sort(sub.begin(), sub.end());
  std::string s = "(";
  for (auto &x : sub) s += x;
  s += ")";
  return s;
}

std::vector<int> centres(const Adj &adj) {
  const int t = (int)adj.size();
  if (t <= 2) {
    std::vector<int> c;
    for (int v = 0; v < t; ++v) c.push_back(v);
    return c;
  }
  std::vector<int> deg(t), layer;
  for (int v = 0; v < t; ++v) {
    deg[v] = (int)adj[v].size();
    if (deg[v] == 1) layer.push_back(v);
  }
  int left = t;
  while (left > 2) {
    left -= (int)layer.size();
    std::vector<int> next;
    for (int v : layer)
      for (int u : adj[v])
        if (--deg[u] == 1) next.push_back(u);
    layer.swap(next);
  }
  return layer;
}

// Canonical code and a centre achieving it.
std::string free_code(const Adj &adj, int *root) {
  std::string best;
  int br = 0;
  for (int c : centres(adj)) {
    std::string s = rooted_code(adj, c, -1);
    if (best.empty() || s < best) {
      best = s;
      br = c;
    }
  }
  if (root) *root = br;
  return best;
}

// Parent array of the tree with the given code: root 0, vertices numbered
// breadth first, children in increasing code order.
std::vector<int32_t> parents_of_code(const std::string &code) {
  // parse the nested code into a rooted tree
  std::vector<int32_t> par;
  std::vector<std::vector<int>> ch;
  std::vector<int> stack;
  for (char x : code) {
    if (x == '(') {
      const int v = (int)par.size();
      par.push_back(stack.empty() ? -1 : stack.back());
      ch.emplace_back();
      if (!stack.empty()) ch[stack.back()].push_back(v);
      stack.push_back(v);
    } else {
      stack.pop_back();
    }
  }
  // breadth-first relabel
  std::vector<int> order{0}, label(par.size(), -1);
  label[0] = 0;
  for (size_t q = 0; q < order.size(); ++q)
    for (int u : ch[order[q]]) {
      label[u] = (int)order.size();
      order.push_back(u);
    }
  std::vector<int32_t> out(par.size());
  for (size_t v = 0; v < par.size(); ++v) out[label[v]] = par[v] < 0 ? -1 : label[par[v]];
  return out;
}

}  // namespace

extern "C" sg2v_status sg2v_trees(int32_t t, int64_t max_trees, int32_t *parents_out,
                                  int64_t *n_trees) {
  if (!n_trees || max_trees < 0 || (max_trees > 0 && !parents_out)) {
    set_error("sg2v_trees: null argument or negative max_trees");
    return SG2V_EINVAL;
  }
  if (t < 1 || t > SG2V_KMAX) {
    set_error("sg2v_trees: need 1 <= t <= %d (t=%d)", SG2V_KMAX, t);
    return SG2V_ERANGE;
  }
  std::vector<std::string> cur{"()"};
  for (int s = 1; s < t; ++s) {
    std::map<std::string, char> next;
    for (const std::string &code : cur) {
      const std::vector<int32_t> par = parents_of_code(code);
      Adj adj(s + 1);
      for (int v = 1; v < s; ++v) {
        adj[v].push_back(par[v]);
        adj[par[v]].push_back(v);
      }
      for (int v = 0; v < s; ++v) {
        adj[v].push_back(s);
        adj[s].push_back(v);
        next.emplace(free_code(adj, nullptr), 0);
        adj[v].pop_back();
        adj[s].clear();
      }
    }
    cur.clear();
    for (auto &kv : next) cur.push_back(kv.first);
  }
  *n_trees = (int64_t)cur.size();
  const int64_t w = std::min<int64_t>(max_trees, (int64_t)cur.size());
  for (int64_t i = 0; i < w; ++i) {
    const std::vector<int32_t> p = parents_of_code(cur[i]);
    std::copy(p.begin(), p.end(), parents_out + i * t);
  }
  return SG2V_OK;
}
