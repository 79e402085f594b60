"""Row-panel SpMM with column-sorted entries (SG2V_TUNE_SPMM_PANEL, the
CSC-Split layout of Alg. 6) against the oracle: U64 exact, FP64 1e-12 and
FP32S 1e-5 relative; every chunk width; long rows split over several tasks
(partial rows in slots); weighted graphs; several launches per table; the
intermediate B tables element by element."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle as O
import paper_2009_11665_amd as sg

pytestmark = pytest.mark.gpu
PANEL = sg.TUNE_SPMM_PANEL


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_u64(G, par, k, seed, j):
    return O.count(G, par, k, O.colors(G.n, k, seed, j), mode=O.U64)[1]


def test_panel_widths_and_skipping():
    G = gg.rmat(11, 12_000, seed=21)
    par, k = gg.CATERPILLAR10, 10
    g = sg.Graph.from_csr(G)
    c = sg.Colorings(g, k, 2, 2)
    p = sg.Plan(par, k)
    ref = [oracle_u64(G, par, k, 2, j) for j in range(2)]
    for w in (8, 16, 32, 64, 128):
        for fl in (PANEL, PANEL | sg.TUNE_NO_COLOR_SKIP, PANEL | sg.TUNE_NO_COLOR_EMA):
            with sg.tuned(spmm_width=w, flags=fl):
                say("panel width", w, "flags", fl)
                got = sg.count(p, g, c, "u64")["colorful_u64"]
                assert [int(x) for x in got] == ref


def test_panel_long_rows_and_modes():
    rng = np.random.default_rng(9)
    n = 12_000
    edges = {(0, v) for v in range(1, 9001)} | {(1, v) for v in range(2, 5002)}
    while len(edges) < 30_000:
        a, b = (int(x) for x in rng.integers(0, n, 2))
        if a != b:
            edges.add((min(a, b), max(a, b)))
    G = gg.from_edge_list(n, sorted(edges))
    g = sg.Graph.from_csr(G)
    for par in (gg.PATH5, gg.BINTREE7):
        k = len(par)
        c = sg.Colorings(g, k, 6, 2)
        p = sg.Plan(par, k)
        with sg.tuned(flags=PANEL):
            say("panel long rows", par)
            ru = sg.count(p, g, c, "u64")
            r64 = sg.count(p, g, c, "fp64")
            r32 = sg.count(p, g, c, "fp32s")
        for j in range(2):
            col = O.colors(G.n, k, 6, j)
            f, u, _ = O.count(G, par, k, col, mode=O.U64)
            f64, _, _ = O.count(G, par, k, col, mode=O.FP64)
            assert int(ru["colorful_u64"][j]) == u
            assert r64["colorful"][j] == pytest.approx(f64, rel=1e-12)
            assert r32["colorful"][j] == pytest.approx(f64, rel=1e-5)


def test_panel_weighted_and_tables():
    G = gg.chung_lu(4000, 10.0, 2.1, seed=13, weighted=True)
    par, k, seed = gg.BINTREE7, 7, 3
    g = sg.Graph.from_csr(G)
    c = sg.Colorings(g, k, seed, 1)
    p = sg.Plan(par, k)
    col = O.colors(G.n, k, seed, 0)
    f64, _, _ = O.count(G, par, k, col, mode=O.FP64, weights=G.w)
    with sg.tuned(flags=PANEL):
        r64 = sg.count(p, g, c, "fp64")
        r32 = sg.count(p, g, c, "fp32s")
        assert r64["colorful"][0] == pytest.approx(f64, rel=1e-12)
        assert r32["colorful"][0] == pytest.approx(f64, rel=1e-5)
    # every aggregated table against the oracle's neighbour sums (without colour
    # skipping, which leaves entries no multiply-add reads at zero)
    with sg.tuned(flags=PANEL | sg.TUNE_NO_COLOR_SKIP):
        for node, ni in enumerate(p.nodes()):
            if ni.size > 1 and ni.is_passive:
                got = sg.debug_table(p, g, c, node, 1, mode="fp64")
                M = O.node_table(G, par, k, col, ni.vertex, ni.n_kept, weights=G.w)
                ref = O.neighbour_sum(G, M, weights=G.w)
                np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_panel_many_launches_wide_table():
    G = gg.rmat(12, 60_000, seed=5)
    par, k, seed = gg.BINTREE15, 15, 3
    col = O.colors(G.n, k, seed, 0)
    _, ref_u, _ = O.count(G, par, k, col, mode=O.U64)
    ref_f, _, _ = O.count(G, par, k, col, mode=O.FP64)
    g = sg.Graph.from_csr(G)
    c = sg.Colorings(g, k, seed, 1)
    p = sg.Plan(par, k)
    with sg.tuned(spmm_width=64, flags=PANEL, launch_chunks=7):
        say("panel bintree15 u64")
        assert int(sg.count(p, g, c, "u64")["colorful_u64"][0]) == ref_u
        assert sg.count(p, g, c, "fp32s")["colorful"][0] == pytest.approx(ref_f, rel=1e-5)


@pytest.mark.parametrize("xmin", [128, 1024])
def test_split_threshold_tuning(xmin):
    """The neighbour-range split's task threshold (a tuning knob the
    autotuner searches) changes which tasks are split, not the counts."""
    G = gg.rmat(12, 60_000, seed=5)
    par, k, seed = gg.BINTREE7, 7, 4
    g = sg.Graph.from_csr(G)
    c = sg.Colorings(g, k, seed, 2)
    p = sg.Plan(par, k)
    ref = [oracle_u64(G, par, k, seed, j) for j in range(2)]
    with sg.tuned(spmm_width=32, flags=sg.TUNE_XSPLIT | sg.TUNE_FORCE_XSPLIT, xsplit_min=xmin):
        got = sg.count(p, g, c, "u64")["colorful_u64"]
    assert [int(x) for x in got] == ref
