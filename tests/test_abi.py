"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function its header declares, the planner's partition, split
tables, alpha and P agree with independent enumerations and the oracle, and
malformed inputs are rejected with the documented status codes."""
import math
import os
import re
from itertools import combinations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
import paper_2009_11665_amd as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sg2v.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sg2v_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = sg.lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(sg.EXPORTS)
    assert "gfx950" in sg.version()


def colex_rank(s):
    return sum(math.comb(c, i + 1) for i, c in enumerate(sorted(s)))


def test_colex_order_matches_oracle_mask_order():
    # the oracle indexes colour sets by increasing mask; colex rank must agree
    k = 9
    for m in range(1, k + 1):
        sets = sorted(combinations(range(k), m), key=lambda s: sum(1 << c for c in s))
        assert [colex_rank(s) for s in sets] == list(range(math.comb(k, m)))


TEMPLATES = [gg.PATH5, gg.BINTREE7, gg.CATERPILLAR10, gg.PATH8, gg.BINTREE15, [-1, 0, 0, 0],
             [-1, 0], [-1], [2, 2, -1, 0, 0, 1, 3]]


@pytest.mark.parametrize("par", TEMPLATES)
def test_plan_alpha_and_probability(par):
    t = len(par)
    for k in sorted({t, t + 1, min(t + 3, 20)}):
        p = sg.Plan(par, k)
        info = p.info()
        assert info.alpha == O.automorphisms(par)
        assert info.colorful_prob == pytest.approx(O.colorful_probability(t, k), rel=1e-14)
        assert info.t == t and info.k == k


@pytest.mark.parametrize("par", TEMPLATES)
def test_split_tables_enumerate_every_split_once(par):
    t = len(par)
    k = min(t + 1, 20) if t < 12 else t
    p = sg.Plan(par, k)
    nodes = p.nodes()
    for idx, nd in enumerate(nodes):
        assert nd.columns == math.comb(k, nd.size)
        if nd.size == 1:
            continue
        A, Pn = nodes[nd.active], nodes[nd.passive]
        assert A.size + Pn.size == nd.size
        pairs = p.pairs(idx)
        out_sets = sorted(combinations(range(k), nd.size), key=colex_rank)
        for r, C in enumerate(out_sets):
            expect = set()
            for S in combinations(C, A.size):
                expect.add((colex_rank(S), colex_rank(set(C) - set(S))))
            got = {(int(a), int(b)) for a, b in pairs[r]}
            assert got == expect and len(pairs[r]) == len(expect)


def test_bintree15_partition_shape():
    """The 15-vertex complete binary tree splits into 6 distinct sub-templates
    (sizes 2, 3, 4, 7, 8, 15) with 3 distinct passive children."""
    p = sg.Plan(gg.BINTREE15, 15)
    info = p.info()
    assert info.n_splits == 6 and info.n_passive == 3
    assert info.spmm_columns == 15 + 455 + 6435
    assert info.pairs_per_vertex == 210 + 1365 + 5460 + 225225 + 51480 + 6435
    assert info.widest_table == 6435
    sizes = sorted(nd.size for nd in p.nodes())
    assert sizes == [1, 2, 3, 4, 7, 8, 15]


def test_dedup_preserves_first_occurrence():
    p = sg.Plan(gg.BINTREE7, 7)
    for nd in p.nodes():
        # (vertex, n_kept) is a valid sub-template of the input
        assert 0 <= nd.vertex < 7


@pytest.mark.parametrize("bad,t,k,status", [
    ([-1, -1, 0], 3, 3, -2), ([0, 1, 2], 3, 3, -2), ([-1, 0, 5], 3, 3, -2),
    ([-1, 2, 1], 3, 3, -2), ([-1, 0, 1], 3, 2, -3), ([-1] + [0] * 20, 21, 21, -3)])
def test_plan_rejects_bad_input(bad, t, k, status):
    with pytest.raises(sg.Sg2vError) as e:
        sg.Plan(bad, k)
    assert e.value.status == status
    assert len(sg.lib().sg2v_last_error()) > 0


def test_graph_validation_errors_on_host():
    # these are detected before any device call
    rp = np.array([0, 2, 3, 4], np.int64)
    ci = np.array([1, 1, 0, 0], np.int32)  # duplicate in row 0
    with pytest.raises(sg.Sg2vError) as e:
        sg.Graph(3, rp, ci, validate=True)
    assert e.value.status == -5
    rp = np.array([0, 1, 1], np.int64)
    ci = np.array([1], np.int32)  # (0,1) without (1,0)
    with pytest.raises(sg.Sg2vError) as e:
        sg.Graph(2, rp, ci, validate=True)
    assert e.value.status == -5
    rp = np.array([0, 1, 2], np.int64)
    ci = np.array([0, 1], np.int32)  # self-loops
    with pytest.raises(sg.Sg2vError) as e:
        sg.Graph(2, rp, ci, validate=True)
    assert e.value.status == -5
    with pytest.raises(sg.Sg2vError) as e:
        sg.Graph(2, np.array([1, 1, 1], np.int64), np.zeros(0, np.int32))
    assert e.value.status == -5


def test_tuning_roundtrip():
    old = sg.get_tuning()
    try:
        sg.set_tuning(spmm_width=64, ema_rows=8, batch=3, budget_bytes=123456)
        t = sg.get_tuning()
        assert (t.spmm_width, t.ema_rows, t.batch, t.budget_bytes) == (64, 8, 3, 123456)
    finally:
        sg.restore_tuning(old)


def _edges(par):
    return {frozenset((v, p)) for v, p in enumerate(par) if p >= 0}


def _random_tree(t, rng):
    par = [-1] + [int(rng.integers(0, v)) for v in range(1, t)]
    perm = rng.permutation(t)
    out = [0] * t
    for v in range(t):
        out[perm[v]] = -1 if par[v] < 0 else int(perm[par[v]])
    return out


REROOT_CASES = TEMPLATES + [_random_tree(t, np.random.default_rng(t)) for t in (6, 9, 12, 14)]


@pytest.mark.parametrize("par", REROOT_CASES)
def test_reroot_is_a_relabelling_with_no_more_work(par):
    """sg2v_template_reroot returns the same tree under a vertex bijection
    (edges map to edges), rooted at 0 with children numbered after their
    parent, and a decomposition whose work (aggregated columns, multiply-add
    pairs) does not exceed the input's for any column weight."""
    t = len(par)
    k = min(t + 1, 20)
    for w in (0.0, 0.5, 4.0):
        out, perm = sg.reroot(par, k, w)
        assert sorted(perm) == list(range(t))
        assert out[0] == -1 and all(0 <= out[v] < v for v in range(1, t))
        assert {frozenset((perm[a], perm[b])) for a, b in map(tuple, _edges(par))} == _edges(out)
        a, b = sg.Plan(par, k).info(), sg.Plan(out, k).info()
        assert b.alpha == a.alpha == O.automorphisms(out)
        assert w * b.spmm_columns + b.pairs_per_vertex <= w * a.spmm_columns + a.pairs_per_vertex + 1e-9


def test_reroot_twenty_vertices_is_a_relabelling():
    for seed in range(4):
        par = _random_tree(20, np.random.default_rng(100 + seed))
        out, perm = sg.reroot(par, 20, 0.5)
        assert sorted(perm) == list(range(20)) and out[0] == -1
        assert {frozenset((perm[a], perm[b])) for a, b in map(tuple, _edges(par))} == _edges(out)
        assert O.automorphisms(out) == O.automorphisms(par)


def test_reroot_moves_path_root_to_the_middle():
    out, _ = sg.reroot(gg.PATH8, 8, 0.5)
    root_kids = [v for v in range(8) if out[v] == 0]
    assert len(root_kids) == 2  # an inner vertex, not an end
    p0, p1 = sg.Plan(gg.PATH8, 8).info(), sg.Plan(out, 8).info()
    assert p1.spmm_columns < p0.spmm_columns and p1.pairs_per_vertex < p0.pairs_per_vertex
    # the complete binary tree is already best rooted at its centre
    out, _ = sg.reroot(gg.BINTREE15, 15, 0.5)
    assert sg.Plan(out, 15).info().spmm_columns == sg.Plan(gg.BINTREE15, 15).info().spmm_columns


@pytest.mark.parametrize("par", [gg.PATH8, gg.CATERPILLAR10, _random_tree(9, np.random.default_rng(3))])
def test_reroot_keeps_the_colourful_count(par):
    """The colourful count of the relabelled template equals the input's
    (exact, by the oracle, which decomposes each rooting on its own)."""
    G = gg.tiny_er(4)
    t = len(par)
    out, _ = sg.reroot(par, t, 0.5)
    for j in range(2):
        col = O.colors(G.n, t, 11, j)
        assert O.count(G, par, t, col, mode=O.U64)[1] == O.count(G, out, t, col, mode=O.U64)[1]


def test_reroot_rejects_bad_input():
    with pytest.raises(sg.Sg2vError) as e:
        sg.reroot([-1, 2, 1], 3)
    assert e.value.status == -2
    with pytest.raises(sg.Sg2vError) as e:
        sg.reroot([-1, 0], 2, -1.0)
    assert e.value.status == -1


def test_python_tuning_flags_match_header():
    """The binding's SG2V_TUNE_* constants carry the header's values."""
    txt = open(HEADER).read()
    defs = dict(re.findall(r"#define SG2V_(TUNE_[A-Z0-9_]+)\s+(\d+)", txt))
    assert "TUNE_BATCH_PERSISTENT" in defs
    for name, val in defs.items():
        assert getattr(sg, name) == int(val), name
