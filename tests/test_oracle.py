"""Pins for the oracle: each test checks the CPU reference against something
other than itself -- published values, closed forms, brute-force enumeration
by definition, invariants of the mathematics -- so that a dropped term, a
wrong index or a transposed operand anywhere in it fails at least one test.

Sections cited are those of the SubGraph2Vec paper (arXiv 2009.11665).
"""
import math
import os
from itertools import permutations

import numpy as np
import pytest

import graphgen as gg
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def random_tree(t, rng):
    """Random labelled tree as a parent array, vertices shuffled so the parent
    array is not in breadth-first order."""
    par = [-1] + [int(rng.integers(0, v)) for v in range(1, t)]
    perm = rng.permutation(t)
    out = [0] * t
    for v in range(t):
        out[perm[v]] = -1 if par[v] < 0 else int(perm[par[v]])
    return out


def random_graph(n, p, rng, weighted=False):
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    w = rng.uniform(0.5, 1.5, len(edges)) if weighted else None
    return gg.from_edge_list(n, edges, w)


def complete_graph(n):
    return gg.from_edge_list(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def tree_graph(parent):
    return gg.from_edge_list(len(parent), [(v, p) for v, p in enumerate(parent) if p >= 0])


# --------------------------------------------------------------------------
# colouring (Sec. 2.2.2 / 2.3.1)

def test_splitmix64_published_values():
    for row in _golden_rows("splitmix64.txt"):
        seed, outs = int(row[0]), [int(x) for x in row[1:]]
        assert O.splitmix64_sequence(seed, len(outs)) == outs


def test_colors_range_and_uniformity():
    for k in (5, 7, 15):
        c = O.colors(200_000, k, 11, 3)
        assert c.min() >= 0 and c.max() < k
        cnt = np.bincount(c, minlength=k)
        exp = len(c) / k
        chi2 = ((cnt - exp) ** 2 / exp).sum()
        # chi-square with k-1 dof: mean k-1, sd sqrt(2(k-1)); 6 sd margin
        assert chi2 < (k - 1) + 6 * math.sqrt(2 * (k - 1))


def test_colors_follow_the_stated_hash():
    # colour = floor(hi32(F(seed ^ F((j<<40)|v))) * k / 2^32), F = finaliser
    seed, j, k = 123456789, 5, 13
    c = O.colors(64, k, seed, j)
    for v in range(64):
        h = O._load().orc_mix64(seed ^ O._load().orc_mix64((j << 40) | v))
        assert c[v] == ((h >> 32) * k) >> 32
    # the finaliser itself: first output of SplitMix64 from state 0 is F(gamma)
    assert O._load().orc_mix64(0x9E3779B97F4A7C15) == O.splitmix64_sequence(0, 1)[0]


def test_colorings_differ_across_index_and_seed():
    a, b, c = O.colors(1000, 7, 1, 0), O.colors(1000, 7, 1, 1), O.colors(1000, 7, 2, 0)
    assert (a != b).mean() > 0.7 and (a != c).mean() > 0.7


# --------------------------------------------------------------------------
# alpha = |Aut(T)| (Alg. 1)

def test_automorphisms_golden():
    for name, alpha, par in _golden_rows("automorphisms.txt"):
        parent = [int(x) for x in par.split(",")]
        assert O.automorphisms(parent) == int(alpha), name


def test_automorphisms_vs_permutations():
    """Brute force over all t! vertex permutations for random trees, t <= 7."""
    rng = np.random.default_rng(1)
    for _ in range(25):
        t = int(rng.integers(1, 8))
        par = random_tree(t, rng)
        edges = {frozenset((v, p)) for v, p in enumerate(par) if p >= 0}
        n_aut = sum(1 for pi in permutations(range(t))
                    if all(frozenset((pi[a], pi[b])) in edges for a, b in map(tuple, edges)))
        assert O.automorphisms(par) == n_aut


def test_identity_colouring_on_template_counts_alpha():
    """G = T with vertex v coloured v: every colourful map of T is an
    automorphism, so the colourful count equals alpha."""
    rng = np.random.default_rng(2)
    for par in ([-1, 0, 1, 2, 3], gg.BINTREE7, gg.CATERPILLAR10, [-1, 0, 0, 0, 0]) + tuple(
            random_tree(int(rng.integers(2, 10)), rng) for _ in range(8)):
        G = tree_graph(par)
        t = len(par)
        col = np.arange(t, dtype=np.uint8)
        f, u, _ = O.count(G, par, t, col, mode=O.U64)
        assert u == O.automorphisms(par)
        f64, _, _ = O.count(G, par, t, col)
        assert f64 == float(u)


# --------------------------------------------------------------------------
# DP (Alg. 3) against brute-force enumeration by definition (Sec. 2.2.1)

@pytest.mark.parametrize("seed", range(6))
def test_dp_equals_brute_force_colourful(seed):
    rng = np.random.default_rng(100 + seed)
    G = random_graph(int(rng.integers(8, 16)), float(rng.uniform(0.2, 0.5)), rng)
    for _ in range(6):
        t = int(rng.integers(1, 8))
        par = random_tree(t, rng)
        k = t + int(rng.integers(0, 2))
        col = O.colors(G.n, k, int(rng.integers(1 << 30)), 0)
        _, bc, _ = O.brute(G, par, col)
        f, _, _ = O.count(G, par, k, col)
        _, u, ov = O.count(G, par, k, col, mode=O.U64)
        _, u2, _ = O.count(G, par, k, col, mode=O.U64, alg2=True)
        _, u3, _ = O.count(G, par, k, col, mode=O.U64, cut=O.CUT_FIRST)
        assert not ov
        assert u == bc and u2 == bc and u3 == bc and f == float(bc)


def test_dp_weighted_equals_brute_force():
    rng = np.random.default_rng(7)
    for _ in range(5):
        G = random_graph(12, 0.4, rng, weighted=True)
        t = int(rng.integers(2, 7))
        par = random_tree(t, rng)
        col = O.colors(G.n, t, int(rng.integers(1 << 30)), 0)
        bt, _, _ = O.brute(G, par, col)
        f, _, _ = O.count(G, par, t, col)
        f2, _, _ = O.count(G, par, t, col, alg2=True)
        f3, _, _ = O.count(G, par, t, col, cut=O.CUT_FIRST)
        for x in (f, f2, f3):
            assert x == pytest.approx(bt, rel=1e-12, abs=1e-12)


def test_partition_invariance_on_er_graph():
    """The count cannot depend on which edge is cut (Sec. 2.3.2)."""
    G = gg.tiny_er()
    for par in (gg.PATH5, gg.BINTREE7, [-1, 0, 0, 0, 1, 1]):
        k = len(par)
        col = O.colors(G.n, k, 1, 0)
        a = O.count(G, par, k, col, mode=O.U64)
        b = O.count(G, par, k, col, mode=O.U64, cut=O.CUT_FIRST)
        c = O.count(G, par, k, col, mode=O.U64, alg2=True)
        assert a[1] == b[1] == c[1] and not a[2]


def test_tiny_config_brute_force():
    """Path5 on ER(1000, 4000): DP = colourful brute-force enumeration."""
    G = gg.tiny_er()
    col = O.colors(G.n, 5, 1, 0)
    _, bc, _ = O.brute(G, gg.PATH5, col)
    _, u, ov = O.count(G, gg.PATH5, 5, col, mode=O.U64)
    f, _, _ = O.count(G, gg.PATH5, 5, col)
    assert u == bc and f == float(bc) and not ov and bc > 0


# --------------------------------------------------------------------------
# closed forms

@pytest.mark.parametrize("n,par", [(9, [-1, 0, 1, 2]), (8, [-1, 0, 0, 1, 1]), (10, [-1, 0, 0, 0]),
                                   (7, [-1, 0, 1, 1, 0, 4])])
def test_complete_graph_colourful_closed_form(n, par):
    """In K_n with k = t colours, every injective map is a homomorphism, so
    the colourful labelled maps number t! * prod_c n_c."""
    G = complete_graph(n)
    t = len(par)
    for seed in range(4):
        col = O.colors(n, t, seed, 0)
        nc = np.bincount(col, minlength=t)
        expect = math.factorial(t) * int(np.prod(nc.astype(object)))
        _, u, _ = O.count(G, par, t, col, mode=O.U64)
        assert u == expect


@pytest.mark.parametrize("n,t", [(7, 3), (8, 4), (9, 5)])
def test_paths_in_complete_graph(n, t):
    """Copies of the t-vertex path in K_n: n! / (2 (n-t)!)."""
    G = complete_graph(n)
    par = [-1] + list(range(t - 1))
    _, maps, _ = O.brute(G, par, None)
    alpha = O.automorphisms(par)
    assert alpha == 2
    assert maps == math.factorial(n) // math.factorial(n - t)
    assert maps // alpha == math.factorial(n) // (2 * math.factorial(n - t))


def test_star_closed_forms():
    """Star S_t (centre + t-1 leaves): copies = sum_v C(deg v, t-1); colourful
    maps with k = t = sum_v (t-1)! prod_{c != col(v)} d_c(v)."""
    rng = np.random.default_rng(3)
    G = random_graph(14, 0.45, rng)
    deg = G.degrees()
    for t in (3, 4, 5):
        par = [-1] + [0] * (t - 1)
        _, maps, _ = O.brute(G, par, None)
        assert maps // O.automorphisms(par) == sum(math.comb(int(d), t - 1) for d in deg)
        for seed in range(3):
            col = O.colors(G.n, t, seed, 0)
            expect = 0
            for v in range(G.n):
                nb = G.col_idx[G.row_ptr[v]:G.row_ptr[v + 1]]
                dc = np.bincount(col[nb], minlength=t)
                expect += math.factorial(t - 1) * int(
                    np.prod([int(dc[c]) for c in range(t) if c != col[v]], dtype=object))
            _, u, _ = O.count(G, par, t, col, mode=O.U64)
            assert u == expect


# --------------------------------------------------------------------------
# invariants

def test_colourful_count_divisible_by_alpha():
    G = gg.tiny_er()
    for par in (gg.PATH5, gg.BINTREE7, gg.CATERPILLAR10):
        k = len(par)
        for j in range(2):
            _, u, ov = O.count(G, par, k, O.colors(G.n, k, 9, j), mode=O.U64)
            assert not ov and u % O.automorphisms(par) == 0


def test_estimator_is_unbiased():
    """The mean of colourful/(P alpha) over colourings converges to emb(T,G)
    (Sec. 2.2.2): within 4 standard errors after N colourings."""
    rng = np.random.default_rng(4)
    G = random_graph(14, 0.35, rng)
    for par in ([-1, 0, 1, 2], [-1, 0, 0, 1]):
        t = len(par)
        alpha = O.automorphisms(par)
        _, maps, _ = O.brute(G, par, None)
        emb = maps / alpha
        N = 400
        est = np.array([O.estimate(O.count(G, par, t, O.colors(G.n, t, 77, j))[0], par, t)
                        for j in range(N)])
        se = est.std(ddof=1) / math.sqrt(N)
        assert abs(est.mean() - emb) < 4 * se + 1e-9


def test_u64_overflow_flag():
    """A star template on a star graph: colourful maps = (t-1)! prod_c d_c,
    far beyond 2^64; the exact mode must raise its overflow flag and the FP64
    mode must match the closed form."""
    D, t = 1200, 12
    G = gg.from_edge_list(D + 1, [(0, v) for v in range(1, D + 1)])
    par = [-1] + [0] * (t - 1)
    col = O.colors(G.n, t, 5, 0)
    dc = np.bincount(col[1:], minlength=t)
    expect = math.factorial(t - 1) * math.prod(int(dc[c]) for c in range(t) if c != col[0])
    f, u, ov = O.count(G, par, t, col, mode=O.U64)
    assert ov and expect > 2 ** 64 and u == expect % 2 ** 64
    f64, _, ov64 = O.count(G, par, t, col)
    assert f64 == pytest.approx(expect, rel=1e-12)


# --------------------------------------------------------------------------
# weighted count and its derivative

def _weighted_instance(seed, n=11, p=0.45):
    rng = np.random.default_rng(seed)
    G = random_graph(n, p, rng, weighted=True)
    t = int(rng.integers(3, 7))
    par = random_tree(t, rng)
    col = O.colors(G.n, t, seed, 0)
    return G, par, t, col


@pytest.mark.parametrize("seed", range(4))
def test_grad_equals_brute_force_per_entry(seed):
    G, par, t, col = _weighted_instance(seed)
    f, g = O.grad(G, par, t, col)
    bt, _, bg = O.brute(G, par, col, grad=True)
    assert f == pytest.approx(bt, rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(g, bg, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_grad_euler_homogeneity(seed):
    """f is a sum of products of t-1 edge weights: sum_e w_e df/dw_e = (t-1) f."""
    G, par, t, col = _weighted_instance(seed + 10)
    f, g = O.grad(G, par, t, col)
    assert float(np.dot(G.w.astype(np.float64), g)) == pytest.approx((t - 1) * f, rel=1e-12,
                                                                      abs=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_grad_affine_in_each_edge(seed):
    """An injective map uses an undirected edge at most once, so f is affine in
    each edge weight: f(w_e=1) - f(w_e=0) = df/dw_e (both directed entries
    tied), and a central difference is exact up to rounding."""
    G, par, t, col = _weighted_instance(seed + 20)
    f, g = O.grad(G, par, t, col)
    gu = O.fold_undirected(G, g)
    rows = np.repeat(np.arange(G.n), np.diff(G.row_ptr))
    rng = np.random.default_rng(seed)
    for e in rng.choice(G.nnz, size=min(8, G.nnz), replace=False):
        i, j = int(rows[e]), int(G.col_idx[e])
        rev = int(G.row_ptr[j] + np.searchsorted(G.col_idx[G.row_ptr[j]:G.row_ptr[j + 1]], i))

        def f_at(x):
            w = G.w.astype(np.float64).copy()
            w[e] = x
            w[rev] = x
            return O.count(G, par, t, col, weights=w)[0]

        assert f_at(1.0) - f_at(0.0) == pytest.approx(gu[e], rel=1e-10, abs=1e-9)
        h = 1e-3
        w0 = float(G.w[e])
        assert (f_at(w0 + h) - f_at(w0 - h)) / (2 * h) == pytest.approx(gu[e], rel=1e-7, abs=1e-6)


def test_grad_at_unit_weights_counts_edge_participation():
    """At w = 1 the folded derivative of an edge is the number of colourful
    maps using it, so the sum over undirected edges is (t-1) * colourful."""
    rng = np.random.default_rng(5)
    G = random_graph(13, 0.4, rng)
    par = gg.PATH5
    col = O.colors(G.n, 5, 3, 0)
    f, g = O.grad(G, par, 5, col)
    assert g.sum() == pytest.approx(4 * f, rel=1e-12)
    _, _, bg = O.brute(G, par, col, grad=True)
    np.testing.assert_allclose(g, bg, rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# intermediate tables

def test_node_tables_and_neighbour_sum():
    """The single-vertex table is the colour indicator; B = A M equals a
    dense product; the root table summed equals the count."""
    rng = np.random.default_rng(6)
    G = random_graph(15, 0.3, rng, weighted=True)
    par = gg.BINTREE7
    k = 7
    col = O.colors(G.n, k, 2, 0)
    leaf = O.node_table(G, par, k, col, 3, 0)
    assert leaf.shape == (G.n, k)
    np.testing.assert_array_equal(leaf, np.eye(k)[col])
    A = np.zeros((G.n, G.n))
    rows = np.repeat(np.arange(G.n), np.diff(G.row_ptr))
    A[rows, G.col_idx] = G.w
    M = O.node_table(G, par, k, col, 1, 2)
    np.testing.assert_allclose(O.neighbour_sum(G, M), A @ M, rtol=1e-13)
    M0 = O.node_table(G, par, k, col, 0, 2)
    assert M0.shape == (G.n, 1)
    assert M0.sum() == pytest.approx(O.count(G, par, k, col)[0], rel=1e-13)
    # the edge table: M(i,{a,b}) = sum_j w_ij [colours of i, j are a, b]
    E = O.node_table(G, par, k, col, 1, 1)
    from itertools import combinations
    sets = sorted(combinations(range(k), 2), key=lambda s: sum(1 << c for c in s))
    E2 = np.zeros_like(E)
    for i in range(G.n):
        for e in range(G.row_ptr[i], G.row_ptr[i + 1]):
            j = G.col_idx[e]
            if col[i] != col[j]:
                E2[i, sets.index(tuple(sorted((col[i], col[j]))))] += G.w[e]
    np.testing.assert_allclose(E, E2, rtol=1e-13)


def test_probability():
    assert O.colorful_probability(5, 5) == pytest.approx(math.factorial(5) / 5 ** 5)
    assert O.colorful_probability(3, 5) == pytest.approx(5 * 4 * 3 / 125)


def test_rejects_bad_templates():
    G = gg.tiny_er()
    col = O.colors(G.n, 3, 1, 0)
    for bad in ([-1, -1, 0], [0, 1, 2], [-1, 0, 5], [-1, 2, 1]):
        with pytest.raises(O.OracleError):
            O.count(G, bad, 3, col)
