"""GPU parity: the HIP path through the C ABI against the oracle on the same
seeded inputs.  Exact for U64 and colours, relative 1e-12 for FP64 and 1e-5
for FP32 with per-column scaling (against the FP64 oracle)."""
import math
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle as O
import paper_2009_11665_amd as sg

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def random_tree(t, rng):
    par = [-1] + [int(rng.integers(0, v)) for v in range(1, t)]
    perm = rng.permutation(t)
    out = [0] * t
    for v in range(t):
        out[perm[v]] = -1 if par[v] < 0 else int(perm[par[v]])
    return out


def gpu_counts(G, par, k, seed, ncol, mode, weighted=None):
    g = sg.Graph.from_csr(G, weighted=weighted)
    c = sg.Colorings(g, k, seed, ncol)
    return sg.count(sg.Plan(par, k), g, c, mode)


def oracle_counts(G, par, k, seed, ncol, mode=O.FP64, weights=None):
    out = []
    for j in range(ncol):
        col = O.colors(G.n, k, seed, j)
        out.append(O.count(G, par, k, col, mode=mode, weights=weights))
    return out


@pytest.fixture(scope="module")
def small_rmat():
    return gg.rmat(11, 12_000, seed=21)


def test_colors_match_oracle():
    G = gg.tiny_er()
    g = sg.Graph.from_csr(G)
    for k, seed in ((5, 1), (15, 7), (20, 123456789)):
        c = sg.Colorings(g, k, seed, 3, first=2).download()
        for j in range(3):
            np.testing.assert_array_equal(c[j], O.colors(G.n, k, seed, 2 + j))
    G2 = gg.rmat16()
    c = sg.Colorings(sg.Graph.from_csr(G2), 7, 99, 1).download()
    np.testing.assert_array_equal(c[0], O.colors(G2.n, 7, 99, 0))


def test_tiny_config_all_modes():
    """path5 on ER(1000, 4000), k = 5: exact vs oracle and brute force."""
    G = gg.tiny_er()
    col = O.colors(G.n, 5, 1, 0)
    _, bc, _ = O.brute(G, gg.PATH5, col)
    ou = O.count(G, gg.PATH5, 5, col, mode=O.U64)
    r = gpu_counts(G, gg.PATH5, 5, 1, 1, "u64")
    say("tiny u64", r["colorful_u64"][0], ou[1], bc)
    assert int(r["colorful_u64"][0]) == ou[1] == bc and not r["overflow"]
    r64 = gpu_counts(G, gg.PATH5, 5, 1, 1, "fp64")
    assert r64["colorful"][0] == pytest.approx(float(bc), rel=FP64_TOL)
    r32 = gpu_counts(G, gg.PATH5, 5, 1, 1, "fp32s")
    assert r32["colorful"][0] == pytest.approx(float(bc), rel=FP32_TOL)
    est = bc / (O.colorful_probability(5, 5) * 2)
    assert r64["estimate"][0] == pytest.approx(est, rel=FP64_TOL)


TEMPLATES = [gg.PATH5, gg.BINTREE7, gg.CATERPILLAR10, [-1, 0, 0, 0], [-1, 0], [-1, 0, 0, 1, 1],
             [-1, 0, 0, 0, 0, 0]]


@pytest.mark.parametrize("ti", range(len(TEMPLATES)))
def test_templates_u64_exact(small_rmat, ti):
    par = TEMPLATES[ti]
    t = len(par)
    for k in (t, t + 1):
        say("u64 template", par, "k", k)
        r = gpu_counts(small_rmat, par, k, 5, 3, "u64")
        for j, (f, u, ov) in enumerate(oracle_counts(small_rmat, par, k, 5, 3, O.U64)):
            assert int(r["colorful_u64"][j]) == u, (par, k, j)
        assert r["overflow"] == any(x[2] for x in oracle_counts(small_rmat, par, k, 5, 3, O.U64))


@pytest.mark.parametrize("flags", [0, 256])
@pytest.mark.parametrize("par", [gg.PATH8, gg.CATERPILLAR10, random_tree(12, np.random.default_rng(8))])
def test_rerooted_template_same_counts(small_rmat, par, flags):
    """A template re-rooted by sg2v_template_reroot counts exactly what the
    oracle counts for the template as given (U64), FP64 and FP32S agree; the
    narrow root tables go through the staged root (flags 0) or the
    thread-per-vertex root (ROOT_THREAD)."""
    t = len(par)
    out, _ = sg.reroot(par, t, 0.5)
    say("rerooted", par, "->", out, "flags", flags)
    ref = oracle_counts(small_rmat, par, t, 9, 2, O.U64)
    old = sg.get_tuning()
    try:
        sg.set_tuning(flags=flags)
        r = gpu_counts(small_rmat, out, t, 9, 2, "u64")
        for j in range(2):
            assert int(r["colorful_u64"][j]) == ref[j][1]
        for mode, tol in (("fp64", FP64_TOL), ("fp32s", FP32_TOL)):
            rf = gpu_counts(small_rmat, out, t, 9, 2, mode)
            for j in range(2):
                assert rf["colorful"][j] == pytest.approx(float(ref[j][1]), rel=tol)
    finally:
        sg.restore_tuning(old)


def test_staged_root_several_tiles_per_block():
    """262,144 vertices: more row tiles than root blocks, so every block
    walks several tiles (path8 re-rooted: distinct narrow X and Y)."""
    G = gg.rmat(18, 600_000, seed=13)
    out, _ = sg.reroot(gg.PATH8, 8, 0.5)
    ref = oracle_counts(G, gg.PATH8, 8, 4, 1, O.U64)
    say("staged root rmat18 path8")
    r = gpu_counts(G, out, 8, 4, 1, "u64")
    assert int(r["colorful_u64"][0]) == ref[0][1]
    r = gpu_counts(G, out, 8, 4, 1, "fp32s")
    assert r["colorful"][0] == pytest.approx(float(ref[0][1]), rel=FP32_TOL)


def test_random_trees_all_modes(small_rmat):
    rng = np.random.default_rng(5)
    for _ in range(6):
        t = int(rng.integers(2, 9))
        par = random_tree(t, rng)
        k = t + int(rng.integers(0, 3))
        say("random tree", par, "k", k)
        ref = oracle_counts(small_rmat, par, k, 11, 2, O.U64)
        ref64 = oracle_counts(small_rmat, par, k, 11, 2, O.FP64)
        ru = gpu_counts(small_rmat, par, k, 11, 2, "u64")
        r64 = gpu_counts(small_rmat, par, k, 11, 2, "fp64")
        r32 = gpu_counts(small_rmat, par, k, 11, 2, "fp32s")
        for j in range(2):
            assert int(ru["colorful_u64"][j]) == ref[j][1]
            assert r64["colorful"][j] == pytest.approx(ref64[j][0], rel=FP64_TOL)
            assert r32["colorful"][j] == pytest.approx(ref64[j][0], rel=FP32_TOL)


def _colex_sets(k, m):
    from itertools import combinations
    return sorted(combinations(range(k), m), key=lambda s: sum(math.comb(c, i + 1) for i, c in enumerate(s)))


@pytest.mark.parametrize("mode", ["u64", "fp64", "fp32s"])
@pytest.mark.parametrize("skip", [False, True])
def test_intermediate_tables(small_rmat, mode, skip):
    """Every materialised table M_s and B = A M_p against the oracle's.  With
    colour skipping, B(i, C) is only defined for sets C not holding i's colour
    (the only entries any multiply-add reads) and is zero elsewhere."""
    G = small_rmat
    old = sg.get_tuning()
    sg.set_tuning(flags=0 if skip else (sg.TUNE_NO_COLOR_SKIP | sg.TUNE_NO_COLOR_EMA))
    try:
        for par, k in ((gg.BINTREE7, 7), (gg.CATERPILLAR10, 10)):
            p = sg.Plan(par, k)
            g = sg.Graph.from_csr(G)
            c = sg.Colorings(g, k, 3, 2)
            col1 = O.colors(G.n, k, 3, 1)
            om = O.U64 if mode == "u64" else O.FP64
            info = p.info()
            for idx, nd in enumerate(p.nodes()):
                ref_M = O.node_table(G, par, k, col1, nd.vertex, nd.n_kept, mode=om)
                if nd.size > 1 and idx != info.root_node:
                    say("table M", par, idx, mode, skip)
                    got = sg.debug_table(p, g, c, idx, 0, which=1, mode=mode)
                    _cmp(got, ref_M, mode)
                if nd.is_passive:
                    say("table B", par, idx, mode, skip)
                    got = sg.debug_table(p, g, c, idx, 1, which=1, mode=mode)
                    ref_B = O.neighbour_sum(G, ref_M, mode=om)
                    if skip and nd.size > 1:
                        sets = _colex_sets(k, nd.size)
                        holds = np.array([[c in s for s in sets] for c in range(k)])[col1]
                        ref_B = np.where(holds, ref_B.dtype.type(0), ref_B)
                        got = np.where(holds, got.dtype.type(0), got)
                    _cmp(got, ref_B, mode)
    finally:
        sg.restore_tuning(old)


def _cmp(got, ref, mode):
    assert got.shape == ref.shape
    if mode == "u64":
        np.testing.assert_array_equal(got, ref)
    else:
        tol = FP64_TOL if mode == "fp64" else FP32_TOL
        np.testing.assert_allclose(got, ref, rtol=tol, atol=tol * max(1.0, float(np.abs(ref).max())) * 1e-3)


def test_weighted_counts():
    G = gg.chung_lu(6000, 10.0, 2.1, seed=8, weighted=True)
    for par in (gg.CATERPILLAR10, gg.PATH5):
        k = len(par)
        say("weighted", par)
        ref = oracle_counts(G, par, k, 4, 2)
        r64 = gpu_counts(G, par, k, 4, 2, "fp64")
        r32 = gpu_counts(G, par, k, 4, 2, "fp32s")
        for j in range(2):
            assert r64["colorful"][j] == pytest.approx(ref[j][0], rel=FP64_TOL)
            assert r32["colorful"][j] == pytest.approx(ref[j][0], rel=FP32_TOL)


def test_batching_invariance(small_rmat):
    """Colourings as extra columns (batch > 1) give the same counts as one
    colouring per pass."""
    par, k = gg.BINTREE7, 7
    g = sg.Graph.from_csr(small_rmat)
    c = sg.Colorings(g, k, 17, 5)
    p = sg.Plan(par, k)
    old = sg.get_tuning()
    try:
        res = {}
        for b in (1, 2, 5):
            sg.set_tuning(batch=b)
            res[b] = sg.count(p, g, c, "u64")["colorful_u64"].copy()
            res[("f", b)] = sg.count(p, g, c, "fp32s")["colorful"].copy()
        np.testing.assert_array_equal(res[1], res[2])
        np.testing.assert_array_equal(res[1], res[5])
        np.testing.assert_allclose(res[("f", 1)], res[("f", 5)], rtol=1e-6)
    finally:
        sg.restore_tuning(old)


def test_spmm_widths_agree(small_rmat):
    par, k = gg.CATERPILLAR10, 10
    g = sg.Graph.from_csr(small_rmat)
    assert small_rmat.degrees().max() >= 128  # some tasks take the neighbour-range split
    c = sg.Colorings(g, k, 2, 2)
    p = sg.Plan(par, k)
    ref = [x[1] for x in oracle_counts(small_rmat, par, k, 2, 2, O.U64)]
    old = sg.get_tuning()
    try:
        for w in (8, 16, 32, 64, 128):
            for fl in (0, sg.TUNE_NO_COLOR_SKIP, sg.TUNE_NO_COLOR_EMA, sg.TUNE_SPMM_UNROLL4,
                       sg.TUNE_FORCE_XSPLIT, sg.TUNE_FORCE_XSPLIT | sg.TUNE_NO_COLOR_SKIP,
                       sg.TUNE_NO_COLOR_SKIP | sg.TUNE_NO_COLOR_EMA | sg.TUNE_SPMM_UNROLL4,
                       sg.TUNE_XSPLIT, sg.TUNE_ROOT_ROWS, sg.TUNE_SPMM_UNROLL8,
                       sg.TUNE_SPMM_UNROLL8 | sg.TUNE_FORCE_XSPLIT, sg.TUNE_ROOT_THREAD):
                sg.set_tuning(spmm_width=w, flags=fl)
                say("spmm width", w, "flags", fl)
                got = sg.count(p, g, c, "u64")["colorful_u64"]
                assert [int(x) for x in got] == ref
    finally:
        sg.restore_tuning(old)


def test_edge_cases():
    # isolated vertices only
    G0 = gg.from_edge_list(50, [])
    g0 = sg.Graph.from_csr(G0)
    for par in (gg.PATH5, [-1, 0]):
        r = sg.count(sg.Plan(par), g0, sg.Colorings(g0, len(par), 1, 2), "u64")
        assert list(r["colorful_u64"]) == [0, 0]
    # one-vertex template: every vertex is one map
    G = gg.tiny_er()
    g = sg.Graph.from_csr(G)
    r = sg.count(sg.Plan([-1], 1), g, sg.Colorings(g, 1, 1, 1), "fp64")
    assert r["colorful"][0] == G.n
    # fewer vertices than a tile, ragged sizes
    Gs = gg.from_edge_list(7, [(0, 1), (1, 2), (2, 3), (3, 4), (1, 5), (5, 6), (0, 6)])
    for par in (gg.PATH5, [-1, 0, 0]):
        t = len(par)
        ref = oracle_counts(Gs, par, t, 3, 4, O.U64)
        r = gpu_counts(Gs, par, t, 3, 4, "u64")
        assert [int(x) for x in r["colorful_u64"]] == [x[1] for x in ref]


def test_budget_too_small_is_enomem():
    """A device-memory budget below one colouring's tables fails with ENOMEM
    before any kernel runs; the next count with the budget lifted works."""
    G = gg.tiny_er()
    g = sg.Graph.from_csr(G)
    p = sg.Plan(gg.CATERPILLAR10, 10)
    c = sg.Colorings(g, 10, 1, 1)
    old = sg.get_tuning()
    try:
        sg.set_tuning(budget_bytes=4096)
        with pytest.raises(sg.Sg2vError) as e:
            sg.count(p, g, c, "fp32s")
        assert e.value.status == -4
    finally:
        sg.restore_tuning(old)
    r = sg.count(p, g, c, "u64")
    assert int(r["colorful_u64"][0]) == O.count(G, gg.CATERPILLAR10, 10, O.colors(G.n, 10, 1, 0), mode=O.U64)[1]


@pytest.mark.parametrize("flags", [0, 16])
def test_long_rows_split_across_tasks(flags):
    """Rows longer than one SpMM task are split and their partial rows summed
    (flags 16: also split every long task over the neighbour ranges)."""
    rng = np.random.default_rng(9)
    n = 12_000
    edges = {(0, v) for v in range(1, 9001)} | {(1, v) for v in range(2, 5002)}
    while len(edges) < 30_000:
        a, b = (int(x) for x in rng.integers(0, n, 2))
        if a != b:
            edges.add((min(a, b), max(a, b)))
    G = gg.from_edge_list(n, sorted(edges))
    old = sg.get_tuning()
    sg.set_tuning(flags=flags)
    try:
        for par in (gg.PATH5, gg.BINTREE7):
            k = len(par)
            say("long rows", par, flags)
            ref = oracle_counts(G, par, k, 6, 2, O.U64)
            ref64 = oracle_counts(G, par, k, 6, 2, O.FP64)
            r = gpu_counts(G, par, k, 6, 2, "u64")
            r32 = gpu_counts(G, par, k, 6, 2, "fp32s")
            for j in range(2):
                assert int(r["colorful_u64"][j]) == ref[j][1]
                assert r32["colorful"][j] == pytest.approx(ref64[j][0], rel=FP32_TOL)
    finally:
        sg.restore_tuning(old)


def test_u64_overflow_flag():
    D, t = 1200, 12
    G = gg.from_edge_list(D + 1, [(0, v) for v in range(1, D + 1)])
    par = [-1] + [0] * (t - 1)
    col = O.colors(G.n, t, 5, 0)
    f, u, ov = O.count(G, par, t, col, mode=O.U64)
    r = gpu_counts(G, par, t, 5, 1, "u64")
    assert ov and r["overflow"] and int(r["colorful_u64"][0]) == u
    r64 = gpu_counts(G, par, t, 5, 1, "fp64")
    f64, _, _ = O.count(G, par, t, col)
    assert r64["colorful"][0] == pytest.approx(f64, rel=FP64_TOL)


def test_mid_config_rmat16_bintree7():
    """RMAT scale 16 (nnz 2,097,152), bintree7, k = 7, 8 colourings:
    FP32S within 1e-5 of the FP64 oracle; U64 exact (mod 2^64)."""
    G = gg.rmat16()
    par, k, seed, ncol = gg.BINTREE7, 7, 2, 8
    ref = oracle_counts(G, par, k, seed, ncol)
    refu = oracle_counts(G, par, k, seed, ncol, O.U64)
    r32 = gpu_counts(G, par, k, seed, ncol, "fp32s")
    ru = gpu_counts(G, par, k, seed, ncol, "u64")
    r64 = gpu_counts(G, par, k, seed, ncol, "fp64")
    for j in range(ncol):
        say("mid", j, r32["colorful"][j], ref[j][0])
        assert r32["colorful"][j] == pytest.approx(ref[j][0], rel=FP32_TOL)
        assert r64["colorful"][j] == pytest.approx(ref[j][0], rel=FP64_TOL)
        assert int(ru["colorful_u64"][j]) == refu[j][1]
    assert ru["overflow"] == any(x[2] for x in refu)


def test_bintree15_on_rmat12_against_oracle():
    """The large configuration's template (15-vertex binary tree, k = 15) on a
    smaller RMAT graph that the oracle finishes: FP32S and FP64 vs oracle."""
    G = gg.rmat(12, 60_000, seed=5)
    par, k = gg.BINTREE15, 15
    ref = oracle_counts(G, par, k, 5, 1)
    r64 = gpu_counts(G, par, k, 5, 1, "fp64")
    r32 = gpu_counts(G, par, k, 5, 1, "fp32s")
    say("bt15", ref[0][0], r64["colorful"][0], r32["colorful"][0])
    assert ref[0][0] > 0
    assert r64["colorful"][0] == pytest.approx(ref[0][0], rel=FP64_TOL)
    assert r32["colorful"][0] == pytest.approx(ref[0][0], rel=FP32_TOL)


@pytest.mark.parametrize("flags", [0, 64])
def test_bintree15_u64_exact_both_root_paths(flags):
    """Exact (mod 2^64) count of the 15-vertex binary tree, root reduced colour
    by colour over vertex ranges (flags 0) and one vertex per block step
    (flags 64), against the oracle's exact mode."""
    G = gg.rmat(11, 25_000, seed=8)
    par, k = gg.BINTREE15, 15
    ref = [x[1] for x in oracle_counts(G, par, k, 9, 2, O.U64)]  # mod 2^64
    ref64 = [x[0] for x in oracle_counts(G, par, k, 9, 2, O.FP64)]
    old = sg.get_tuning()
    sg.set_tuning(flags=flags)
    try:
        r = gpu_counts(G, par, k, 9, 2, "u64")
        r32 = gpu_counts(G, par, k, 9, 2, "fp32s")
    finally:
        sg.restore_tuning(old)
    say("bt15 u64", flags, ref, list(r["colorful_u64"]))
    assert [int(x) for x in r["colorful_u64"]] == ref
    np.testing.assert_allclose(r32["colorful"], ref64, rtol=FP32_TOL)


def _complete_graph(n):
    return gg.from_edge_list(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def _colourful_in_complete(t, colours, k):
    """Colourful maps of any t-vertex tree into K_n: every injective map is a
    homomorphism, so the count is t! times the number of t-sets of vertices
    with distinct colours, e_t(n_0, ..., n_{k-1}) (elementary symmetric
    polynomial of the colour class sizes)."""
    sizes = np.bincount(colours, minlength=k)
    e = [1] + [0] * t
    for s in sizes:
        for q in range(t, 0, -1):
            e[q] += e[q - 1] * int(s)
    return math.factorial(t) * e[t]


@pytest.mark.parametrize("par,k", [
    (list(range(-1, 19)), 20),                 # 20-vertex path, the largest template
    (gg.BINTREE15, 17),
    ([-1, 0, 0, 0, 1, 1, 2, 2, 3, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13], 20),
    (gg.CATERPILLAR10, 17),
    (gg.PATH8, 8),
])
def test_large_k_on_complete_graph(par, k):
    """k up to 20 (tables of C(20, 10) columns, splits beyond the 16-bit
    colour-restricted tables) on K_40 against the closed form t! e_t(n_c):
    exact mod 2^64, FP64 and FP32 within their tolerances."""
    G = _complete_graph(40)
    g = sg.Graph.from_csr(G)
    t = len(par)
    c = sg.Colorings(g, k, 31, 2)
    cols = c.download()
    p = sg.Plan(par, k)
    ru = sg.count(p, g, c, "u64")
    r64 = sg.count(p, g, c, "fp64")
    r32 = sg.count(p, g, c, "fp32s")
    for j in range(2):
        exact = _colourful_in_complete(t, cols[j], k)
        say("complete", t, k, j, exact)
        np.testing.assert_array_equal(cols[j], O.colors(G.n, k, 31, j))
        assert int(ru["colorful_u64"][j]) == exact % (1 << 64)
        assert r64["colorful"][j] == pytest.approx(float(exact), rel=FP64_TOL)
        assert r32["colorful"][j] == pytest.approx(float(exact), rel=FP32_TOL)


def test_gpu_estimator_is_unbiased():
    """End to end on the GPU: the mean of colourful/(P alpha) over 2000
    colourings (FP32, batched) is within 4 standard errors of the number of
    copies of the template counted by brute force (Sec. 2.2.2), for k = t and
    k > t; every colouring's count equals the oracle's on the same colouring."""
    rng = np.random.default_rng(4)
    n = 40
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.12]
    G = gg.from_edge_list(n, edges)
    g = sg.Graph.from_csr(G)
    for par, k in ((gg.PATH5, 5), ([-1, 0, 0, 1, 1], 5), (gg.PATH5, 7)):
        alpha = O.automorphisms(par)
        _, maps, _ = O.brute(G, par, None)
        copies = maps / alpha
        N = 2000
        r = sg.count(sg.Plan(par, k), g, sg.Colorings(g, k, 123, N), "fp32s")
        est = np.asarray(r["estimate"])
        se = est.std(ddof=1) / math.sqrt(N)
        say("estimator", par, k, copies, est.mean(), se)
        assert abs(est.mean() - copies) < 4 * se + 1e-9
        assert r["mean_estimate"] == pytest.approx(est.mean(), rel=1e-12)
        for j in (0, 1, N - 1):
            f = O.count(G, par, k, O.colors(G.n, k, 123, j))[0]
            assert r["colorful"][j] == pytest.approx(f, rel=FP32_TOL)


@pytest.mark.parametrize("mode", ["u64", "fp64", "fp32s"])
def test_many_colourings_per_pass(mode):
    """Small templates batch hundreds of colourings per pass (colourings as
    extra table columns); every one of 300 colourings matches the oracle."""
    rng = np.random.default_rng(8)
    n = 60
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.1]
    G = gg.from_edge_list(n, edges)
    g = sg.Graph.from_csr(G)
    par, k, N = gg.PATH5, 5, 300
    r = sg.count(sg.Plan(par, k), g, sg.Colorings(g, k, 42, N), mode)
    for j in range(N):
        f, u, _ = O.count(G, par, k, O.colors(G.n, k, 42, j), mode=O.U64)
        if mode == "u64":
            assert int(r["colorful_u64"][j]) == u, j
        else:
            assert r["colorful"][j] == pytest.approx(float(u), rel=FP64_TOL if mode == "fp64" else FP32_TOL), j


@pytest.mark.parametrize("split", [True, False])
def test_spmm_chunk_groups_against_oracle(split):
    """A wide table aggregated in several SpMM launches, each starting at a
    later column chunk, as on the large workload: with the neighbour-range
    split over 256-byte row segments in chunk groups of 3 chunks (the
    6435-column table of the 15-vertex tree takes 34 launches plus their
    range combines, every launch after the first with a column offset), and
    without the split in launches of 2 chunks.  U64 exact (mod 2^64) and FP32S
    within 1e-5 of the FP64 oracle."""
    G = gg.rmat(12, 60_000, seed=5)
    assert (G.degrees() >= 512).sum() > 0  # tasks the range split applies to
    par, k, seed = gg.BINTREE15, 15, 3
    col = O.colors(G.n, k, seed, 0)
    _, ref_u, _ = O.count(G, par, k, col, mode=O.U64)
    ref_f, _, _ = O.count(G, par, k, col, mode=O.FP64)
    kw = (dict(spmm_width=64, flags=sg.TUNE_XSPLIT | sg.TUNE_FORCE_XSPLIT, xsplit_group=3) if split
          else dict(spmm_width=64, flags=sg.TUNE_NO_XSPLIT, launch_chunks=2))
    g = sg.Graph.from_csr(G)
    c = sg.Colorings(g, k, seed, 1)
    p = sg.Plan(par, k)
    with sg.tuned(**kw):
        for mode in ("u64", "fp32s"):
            say("chunk groups", "split" if split else "plain", mode)
            sg.profile_start()
            r = sg.count(p, g, c, mode)
            prof = sg.profile_stop()
            # 101 chunks of the 6435-column table + 8 of the 455-column one
            assert prof["spmm"]["launches"] >= (34 + 3 if split else 51 + 4), prof["spmm"]
            if split:
                assert prof["spmm_combine"]["launches"] >= 34 + 3
            if mode == "u64":
                assert int(r["colorful_u64"][0]) == ref_u
            else:
                assert r["colorful"][0] == pytest.approx(ref_f, rel=FP32_TOL)
