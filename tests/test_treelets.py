"""Treelet distribution (Sec. 2.1: the normalised counts of every
non-isomorphic tree of a given size, 47 trees of nine vertices).

CPU: the enumeration (sg2v_trees) against the number of unlabelled trees
(tests/golden/unlabelled_trees.txt: Cayley/Otter's counts for 1..16
vertices; the paper's 47 for nine vertices) and against a brute-force
isomorphism check written here (minimum over every root of the rooted code);
the plan of several templates (sg2v_plan_create_multi) shares sub-templates.
GPU: every template's count from one sg2v_count_multi call against the oracle
(U64 exact, FP32 with per-column exponents within 1e-5) and the frequencies
summing to 1."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle as O
import paper_2009_11665_amd as sg

def _golden_tree_counts():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "unlabelled_trees.txt")
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                t, c = line.split()
                out[int(t)] = int(c)
    return out


UNLABELLED_TREES = _golden_tree_counts()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def adjacency(par):
    adj = [[] for _ in par]
    for v, p in enumerate(par):
        if p >= 0:
            adj[v].append(p)
            adj[p].append(v)
    return adj


def code_at(adj, v, frm):
    return "[" + "".join(sorted(code_at(adj, u, v) for u in adj[v] if u != frm)) + "]"


def brute_canonical(par):
    """Isomorphism class of a free tree: the least rooted code over all roots."""
    adj = adjacency(par)
    return min(code_at(adj, r, -1) for r in range(len(par)))


def is_tree(par):
    t = len(par)
    if par.count(-1) != 1 or par[0] != -1:
        return False
    seen = {0}
    for v in range(1, t):  # breadth-first numbering: parents come first
        if not (0 <= par[v] < v) or par[v] not in seen:
            return False
        seen.add(v)
    return True


@pytest.mark.parametrize("t", sorted(UNLABELLED_TREES))
def test_tree_enumeration_counts(t):
    trees = sg.trees(t)
    assert len(trees) == UNLABELLED_TREES[t]
    assert all(len(p) == t and is_tree(p) for p in trees)
    if t <= 12:
        codes = [brute_canonical(p) for p in trees]
        assert len(set(codes)) == len(codes)  # pairwise non-isomorphic


def test_paper_nine_vertex_treelets():
    """Sec. 2.1: 47 unlabelled treelets of nine vertices; path and star among them."""
    trees = sg.trees(9)
    assert len(trees) == 47
    codes = {brute_canonical(p) for p in trees}
    assert brute_canonical([-1, 0, 1, 2, 3, 4, 5, 6, 7]) in codes
    assert brute_canonical([-1] + [0] * 8) in codes


def test_enumeration_rejects_bad_sizes():
    with pytest.raises(sg.Sg2vError):
        sg.trees(0)
    with pytest.raises(sg.Sg2vError):
        sg.trees(21)


def test_multi_plan_shares_subtemplates():
    trees = sg.trees(9)
    multi = sg.Plan.multi(trees)
    info = multi.info()
    assert info.n_templates == 47 and info.k == 9 and info.t == 9
    single = [sg.Plan(p).info() for p in trees]
    assert info.n_nodes < sum(i.n_nodes for i in single)
    assert info.alpha == O.automorphisms(trees[0])
    assert info.bytes_per_vertex_fp64 >= info.bytes_per_vertex_fp32 > 0
    # every node appears once: distinct rooted sub-templates of all 47 trees
    say("nodes shared:", info.n_nodes, "unshared:", sum(i.n_nodes for i in single))


def test_multi_plan_rejects_repeats_and_subtemplates():
    with pytest.raises(sg.Sg2vError) as e:
        sg.Plan.multi([gg.PATH5, gg.PATH5])
    assert e.value.status == -1
    # a rooted path of 3 vertices is the passive child of a rooted path of 4
    with pytest.raises(sg.Sg2vError) as e:
        sg.Plan.multi([[-1, 0, 1, 2], [-1, 0, 1]], k=4)
    assert e.value.status == -1


@pytest.mark.gpu
def test_treelet_distribution_against_oracle():
    G = gg.rmat(9, 2400, seed=31)
    trees = sg.trees(9)
    k, seed, ncol = 9, 17, 2
    g = sg.Graph.from_csr(G)
    c = sg.Colorings(g, k, seed, ncol)
    plan = sg.Plan.multi(trees, k)
    say("treelets: 47 nine-vertex trees on RMAT scale 9, u64")
    ru = sg.count_multi(plan, g, c, "u64")
    assert not ru["overflow"]
    r32 = sg.count_multi(plan, g, c, "fp32s")
    for j in range(ncol):
        col = O.colors(G.n, k, seed, j)
        for r, par in enumerate(trees):
            f, u, _ = O.count(G, par, k, col, mode=O.U64)
            assert int(ru["colorful_u64"][r, j]) == u, (r, j)
            assert r32["colorful"][r, j] == pytest.approx(float(u), rel=1e-5, abs=1e-300)
    for res in (ru, r32):
        assert res["frequency"].sum() == pytest.approx(1.0, rel=1e-12)
        m = res["mean_estimate"]
        np.testing.assert_allclose(res["frequency"], m / m.sum(), rtol=1e-12)
    # the same counts template by template through sg2v_count
    for r in (0, 13, 46):
        one = sg.count(sg.Plan(trees[r], k), g, c, "u64")
        np.testing.assert_array_equal(one["colorful_u64"], ru["colorful_u64"][r])


@pytest.mark.gpu
def test_multi_plan_of_uneven_sizes_and_k_above_t():
    """Templates of 5, 6 and 7 vertices with k = 8 in one count."""
    G = gg.tiny_er()
    pars = [gg.PATH5, [-1, 0, 0, 0, 1, 1], gg.BINTREE7]
    k, seed = 8, 5
    g = sg.Graph.from_csr(G)
    c = sg.Colorings(g, k, seed, 3)
    res = sg.count_multi(sg.Plan.multi(pars, k), g, c, "u64")
    for j in range(3):
        col = O.colors(G.n, k, seed, j)
        for r, par in enumerate(pars):
            _, u, _ = O.count(G, par, k, col, mode=O.U64)
            assert int(res["colorful_u64"][r, j]) == u
