"""SG2V_GRAPH_RELABEL (vertices stored by decreasing degree): invisible to the
caller.  Colourings, counts (U64 exact, FP64 and FP32S within their
tolerances of the oracle), intermediate tables and per-entry gradients in the
caller's order are the same with and without it, also through the
neighbour-range split over the renumbered ranges."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle as O
import paper_2009_11665_amd as sg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_relabel_colourings_and_counts():
    G = gg.rmat(12, 30_000, seed=8)
    par, k, seed = gg.BINTREE7, 7, 4
    g0 = sg.Graph.from_csr(G)
    g1 = sg.Graph.from_csr(G, relabel=True)
    c0 = sg.Colorings(g0, k, seed, 3)
    c1 = sg.Colorings(g1, k, seed, 3)
    np.testing.assert_array_equal(c0.download(), c1.download())
    np.testing.assert_array_equal(c1.download()[1], O.colors(G.n, k, seed, 1))
    p = sg.Plan(par, k)
    say("relabel: counts rmat12 bintree7")
    u0 = sg.count(p, g0, c0, "u64")
    u1 = sg.count(p, g1, c1, "u64")
    np.testing.assert_array_equal(u0["colorful_u64"], u1["colorful_u64"])
    for j in range(3):
        _, u, _ = O.count(G, par, k, O.colors(G.n, k, seed, j), mode=O.U64)
        assert int(u1["colorful_u64"][j]) == u
    f1 = sg.count(p, g1, c1, "fp64")
    s1 = sg.count(p, g1, c1, "fp32s")
    for j in range(3):
        ref = float(u1["colorful_u64"][j])
        assert f1["colorful"][j] == pytest.approx(ref, rel=1e-12)
        assert s1["colorful"][j] == pytest.approx(ref, rel=1e-5)


def test_relabel_tables_in_caller_order():
    G = gg.rmat(10, 6_000, seed=9)
    par, k, seed = gg.BINTREE7, 7, 2
    p = sg.Plan(par, k)
    g0, g1 = sg.Graph.from_csr(G), sg.Graph.from_csr(G, relabel=True)
    c0, c1 = sg.Colorings(g0, k, seed, 1), sg.Colorings(g1, k, seed, 1)
    for node, ni in enumerate(p.nodes()):
        if ni.size == 1 or node == p.info().root_node:
            continue
        kinds = [0] + ([1] if ni.is_passive else [])
        for kind in kinds:
            a = sg.debug_table(p, g0, c0, node, kind, mode="u64")
            b = sg.debug_table(p, g1, c1, node, kind, mode="u64")
            np.testing.assert_array_equal(a, b)


def test_relabel_gradients_in_caller_entry_order():
    G = gg.chung_lu(3000, 8.0, 2.1, seed=12, weighted=True)
    par, k, seed = [-1, 0, 1, 2, 3], 5, 6
    p = sg.Plan(par, k)
    g0, g1 = sg.Graph.from_csr(G), sg.Graph.from_csr(G, relabel=True)
    c0, c1 = sg.Colorings(g0, k, seed, 1), sg.Colorings(g1, k, seed, 1)
    say("relabel: gradients chung-lu 3000 path5 weighted")
    d0 = sg.count_grad(p, g0, c0, [1.0], "fp64").cpu().numpy()
    d1 = sg.count_grad(p, g1, c1, [1.0], "fp64").cpu().numpy()
    scale = np.abs(d0).max()
    np.testing.assert_allclose(d1, d0, rtol=1e-12, atol=1e-12 * scale)
    f, ref = O.grad(G, par, k, O.colors(G.n, k, seed, 0))
    np.testing.assert_allclose(d1, ref, rtol=1e-10, atol=1e-10 * scale)


def test_relabel_with_neighbour_range_split():
    """Round-robin degree-ordered ranges on the stored ids."""
    G = gg.rmat(12, 60_000, seed=5)
    par, k, seed = gg.BINTREE15, 15, 3
    col = O.colors(G.n, k, seed, 0)
    _, ref_u, _ = O.count(G, par, k, col, mode=O.U64)
    ref_f, _, _ = O.count(G, par, k, col, mode=O.FP64)
    g = sg.Graph.from_csr(G, relabel=True)
    c = sg.Colorings(g, k, seed, 1)
    p = sg.Plan(par, k)
    with sg.tuned(spmm_width=64, flags=sg.TUNE_XSPLIT | sg.TUNE_FORCE_XSPLIT, xsplit_group=3):
        say("relabel: split u64")
        r = sg.count(p, g, c, "u64")
        assert int(r["colorful_u64"][0]) == ref_u
        r = sg.count(p, g, c, "fp32s")
        assert r["colorful"][0] == pytest.approx(ref_f, rel=1e-5)
