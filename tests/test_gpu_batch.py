"""Multi-template batches recorded as one HIP graph (sg2v_count_batch):
equal to one-template counts and to the oracle, stable across replays of
the cached graph with eager work in between."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle as O
import paper_2009_11665_amd as sg

pytestmark = pytest.mark.gpu

TEMPLATES = (gg.BINTREE7, gg.PATH8, gg.CATERPILLAR10)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("flags", [0, 512])
def test_batch_equals_single_and_oracle(flags):
    """flags 0: templates as parallel graph branches with a workspace each;
    512 (BATCH_SERIAL): one after another in the shared workspace."""
    G = gg.chung_lu(20_000, 12.0, 2.1, seed=4)
    g = sg.Graph.from_csr(G)
    plans = [sg.Plan(p) for p in TEMPLATES]
    seed, ncol = 7, 4
    old = sg.get_tuning()
    sg.set_tuning(flags=flags)
    try:
        _batch_vs_single(G, g, plans, seed, ncol)
    finally:
        sg.restore_tuning(old)


def _batch_vs_single(G, g, plans, seed, ncol):
    for mode in ("u64", "fp32s", "fp64"):
        say("batch", mode)
        cf, est = sg.count_batch(plans, g, seed, ncol, mode)
        for p, par in enumerate(TEMPLATES):
            c = sg.Colorings(g, len(par), seed, ncol)
            r = sg.count(plans[p], g, c, mode)
            if mode == "u64":
                np.testing.assert_array_equal(cf[p], r["colorful"])
                for j in range(2):
                    u = O.count(G, par, len(par), O.colors(G.n, len(par), seed, j), mode=O.U64)[1]
                    assert int(r["colorful_u64"][j]) == u
            else:
                np.testing.assert_allclose(cf[p], r["colorful"], rtol=1e-12)
            np.testing.assert_allclose(est[p], r["estimate"], rtol=1e-12)


def test_batch_of_rerooted_templates():
    """The batch workload's re-rooted templates: the graph-recorded batch
    equals the oracle's counts of the templates as given (U64), and FP32S
    agrees with FP64."""
    G = gg.chung_lu(20_000, 12.0, 2.1, seed=5)
    g = sg.Graph.from_csr(G)
    pars = [sg.reroot(p, len(p), 0.05)[0] for p in TEMPLATES]
    plans = [sg.Plan(p) for p in pars]
    seed, ncol = 3, 3
    say("batch rerooted", pars)
    cu, _ = sg.count_batch(plans, g, seed, ncol, "u64")
    c64, _ = sg.count_batch(plans, g, seed, ncol, "fp64")
    c32, _ = sg.count_batch(plans, g, seed, ncol, "fp32s")
    for p, par in enumerate(TEMPLATES):
        for j in range(ncol):
            u = O.count(G, par, len(par), O.colors(G.n, len(par), seed, j), mode=O.U64)[1]
            assert cu[p][j] == pytest.approx(float(u), rel=1e-15)  # U64 counts returned as float64
            assert c64[p][j] == pytest.approx(float(u), rel=1e-12)
            assert c32[p][j] == pytest.approx(float(u), rel=1e-5)


def test_batch_graph_replays_with_eager_work_between():
    G = gg.rmat(12, 40_000, seed=9)
    g = sg.Graph.from_csr(G)
    plans = [sg.Plan(p) for p in TEMPLATES]
    first, _ = sg.count_batch(plans, g, 3, 3, "fp32s")
    for rep in range(3):
        # eager work on the same workspace between replays
        c = sg.Colorings(g, 7, 11 + rep, 2)
        sg.count(plans[0], g, c, "fp32s")
        again, _ = sg.count_batch(plans, g, 3, 3, "fp32s")
        say("replay", rep)
        np.testing.assert_array_equal(first, again)


def test_batch_config_chung_lu_500k():
    """The batching workload: Chung-Lu n=500,000, mean degree 20, gamma 2.1;
    bintree7, path8, caterpillar10 x 16 colourings in one graph launch, FP32
    with per-column scaling, against the FP64 path (all colourings) and the
    oracle (first colouring of every template)."""
    G = gg.chung_lu_500k()
    g = sg.Graph.from_csr(G)
    plans = [sg.Plan(p) for p in TEMPLATES]
    seed, ncol = 4, 16
    cf32, est32 = sg.count_batch(plans, g, seed, ncol, "fp32s")
    cf64, _ = sg.count_batch(plans, g, seed, ncol, "fp64")
    np.testing.assert_allclose(cf32, cf64, rtol=1e-5)
    for p, par in enumerate(TEMPLATES):
        k = len(par)
        f = O.count(G, par, k, O.colors(G.n, k, seed, 0))[0]
        say("oracle", par, f, cf64[p][0])
        assert cf64[p][0] == pytest.approx(f, rel=1e-12)
        assert cf32[p][0] == pytest.approx(f, rel=1e-5)


def test_autotune_installs_a_candidate_and_keeps_results():
    G = gg.rmat(12, 40_000, seed=9)
    g = sg.Graph.from_csr(G)
    p = sg.Plan(gg.CATERPILLAR10)
    old = sg.get_tuning()
    try:
        c = sg.Colorings(g, 10, 5, 2)
        ref = sg.count(p, g, c, "u64")["colorful_u64"].copy()
        t = sg.autotune(p, g, "u64", 2)
        cur = sg.get_tuning()
        assert (cur.spmm_width, cur.ema_rows, cur.batch, cur.flags) == (
            t.spmm_width, t.ema_rows, t.batch, t.flags)
        assert t.spmm_width in (16, 32, 64, 128)  # the autotuner's candidate widths
        np.testing.assert_array_equal(sg.count(p, g, c, "u64")["colorful_u64"], ref)
    finally:
        sg.restore_tuning(old)
