"""Multi-template batches run by the persistent schedule (sg2v_count_batch
with TUNE_BATCH_PERSISTENT): every launch of every template is recorded and
one kernel runs them as a task queue with a completion counter per launch.
Checked against the oracle (U64, exact) and against the graph-recorded batch
in every mode, with templates of uneven k, as independent chains and as one
chain, and across replays of the cached schedule."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle as O
import paper_2009_11665_amd as sg

pytestmark = pytest.mark.gpu

# uneven k: 5, 7, 8 and 10 colours
TEMPLATES = (gg.PATH5, gg.BINTREE7, gg.PATH8, gg.CATERPILLAR10)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _batch(plans, g, seed, ncol, mode, flags):
    with sg.tuned(flags=flags):
        return sg.count_batch(plans, g, seed, ncol, mode)


@pytest.mark.parametrize("serial", [False, True])
def test_persistent_equals_oracle_and_graph(serial):
    """serial False: one chain per template (a workspace each); True
    (BATCH_SERIAL): all templates in one chain in the shared workspace."""
    G = gg.chung_lu(20_000, 12.0, 2.1, seed=4)
    g = sg.Graph.from_csr(G)
    plans = [sg.Plan(p) for p in TEMPLATES]
    seed, ncol = 11, 3
    extra = sg.TUNE_BATCH_SERIAL if serial else 0
    for mode in ("u64", "fp64", "fp32s"):
        say("persistent", "serial" if serial else "chains", mode)
        cp, ep = _batch(plans, g, seed, ncol, mode, sg.TUNE_BATCH_PERSISTENT | extra)
        cg, eg = _batch(plans, g, seed, ncol, mode, extra)
        if mode == "u64":
            np.testing.assert_array_equal(cp, cg)
            for p, par in enumerate(TEMPLATES):
                for j in range(ncol):
                    u = O.count(G, par, len(par), O.colors(G.n, len(par), seed, j), mode=O.U64)[1]
                    assert cp[p][j] == float(u)
        elif mode == "fp64":
            np.testing.assert_allclose(cp, cg, rtol=1e-12)
        else:
            # the persistent schedule uses the general multiply-add and the
            # vertex-order root (other summation orders): FP32 tolerance
            np.testing.assert_allclose(cp, cg, rtol=1e-5)
        np.testing.assert_allclose(ep, eg, rtol=1e-5 if mode == "fp32s" else 1e-12)


def test_persistent_replays_and_rmat():
    """The cached schedule replayed with eager work between the replays, on an
    RMAT graph whose long rows take the long-row combine, with 16 colourings
    as table columns (several passes for the wider templates)."""
    G = gg.rmat(12, 40_000, seed=9)
    g = sg.Graph.from_csr(G)
    plans = [sg.Plan(p) for p in TEMPLATES]
    seed, ncol = 5, 16
    say("persistent rmat u64")
    ref = [[O.count(G, par, len(par), O.colors(G.n, len(par), seed, j), mode=O.U64)[1] for j in range(ncol)]
           for par in TEMPLATES]
    first = None
    for rep in range(3):
        cp, _ = _batch(plans, g, seed, ncol, "u64", sg.TUNE_BATCH_PERSISTENT)
        for p in range(len(TEMPLATES)):
            for j in range(ncol):
                assert cp[p][j] == float(ref[p][j]), (rep, p, j)
        if first is None:
            first = cp.copy()
        np.testing.assert_array_equal(cp, first)
        # eager work between replays
        c = sg.Colorings(g, 7, seed + rep, 2)
        sg.count(plans[1], g, c, "fp64")
    say("persistent rmat fp32s")
    # counts of the longer templates exceed 2^64 here (U64 is exact modulo
    # 2^64): FP32S against the FP64 oracle on four colourings
    c32, _ = _batch(plans, g, seed, ncol, "fp32s", sg.TUNE_BATCH_PERSISTENT)
    for p, par in enumerate(TEMPLATES):
        for j in range(4):
            f = O.count(G, par, len(par), O.colors(G.n, len(par), seed, j), mode=O.FP64)[0]
            assert c32[p][j] == pytest.approx(f, rel=1e-5), (p, j)


def test_persistent_split_rows():
    """The neighbour-range split (forced on a small graph): its task-split
    and range-combine launches run as tasks of the persistent kernel."""
    G = gg.rmat(12, 40_000, seed=3)
    g = sg.Graph.from_csr(G)
    plans = [sg.Plan(p) for p in (gg.BINTREE7, gg.PATH8)]
    seed, ncol = 2, 2
    say("persistent forced split")
    flags = sg.TUNE_BATCH_PERSISTENT | sg.TUNE_FORCE_XSPLIT | sg.TUNE_XSPLIT
    with sg.tuned(flags=flags, spmm_width=32, xsplit_min=16):
        cp, _ = sg.count_batch(plans, g, seed, ncol, "u64")
    for p, par in enumerate((gg.BINTREE7, gg.PATH8)):
        for j in range(ncol):
            u = O.count(G, par, len(par), O.colors(G.n, len(par), seed, j), mode=O.U64)[1]
            assert cp[p][j] == float(u)


def test_persistent_rejects_panel_spmm():
    """The row-panel SpMM has no body in the persistent kernel: rejected on
    the host before anything runs."""
    G = gg.chung_lu(5_000, 8.0, 2.1, seed=2)
    g = sg.Graph.from_csr(G)
    plans = [sg.Plan(gg.BINTREE7)]
    with pytest.raises(RuntimeError, match="persistent"):
        _batch(plans, g, 1, 2, "u64", sg.TUNE_BATCH_PERSISTENT | sg.TUNE_SPMM_PANEL)


def test_persistent_wait_timeout_reports_error(monkeypatch):
    """A zero bound on the dependency waits, set from the host: a block that
    finds its launch's predecessor unfinished raises the error flag, every
    block stops taking tasks and the kernel ends normally; the call reports
    the time-out, and the next call without the bound is exact."""
    G = gg.chung_lu(20_000, 12.0, 2.1, seed=4)
    g = sg.Graph.from_csr(G)
    pars = (gg.BINTREE7, gg.PATH8)
    plans = [sg.Plan(p) for p in pars]
    seed, ncol = 3, 2
    say("persistent time-out path")
    monkeypatch.setenv("SG2V_PERSIST_WAIT_US", "0")
    with pytest.raises(RuntimeError, match="timed out"):
        _batch(plans, g, seed, ncol, "u64", sg.TUNE_BATCH_PERSISTENT)
    monkeypatch.delenv("SG2V_PERSIST_WAIT_US")
    cp, _ = _batch(plans, g, seed, ncol, "u64", sg.TUNE_BATCH_PERSISTENT)
    for p, par in enumerate(pars):
        for j in range(ncol):
            u = O.count(G, par, len(par), O.colors(G.n, len(par), seed, j), mode=O.U64)[1]
            assert cp[p][j] == float(u)


def test_persistent_many_chains():
    """All 23 trees of eight vertices as one batch (23 chains, one per
    template): U64 counts equal the graph-recorded batch's and, for three
    of them, the oracle's."""
    G = gg.rmat(10, 6_000, seed=12)
    g = sg.Graph.from_csr(G)
    pars = sg.trees(8)
    assert len(pars) == 23
    plans = [sg.Plan(p) for p in pars]
    seed, ncol = 6, 2
    say("persistent 23 chains")
    cp, _ = _batch(plans, g, seed, ncol, "u64", sg.TUNE_BATCH_PERSISTENT)
    cg, _ = _batch(plans, g, seed, ncol, "u64", 0)
    np.testing.assert_array_equal(cp, cg)
    for p in (0, 11, 22):
        par = pars[p]
        u = O.count(G, par, len(par), O.colors(G.n, len(par), seed, 1), mode=O.U64)[1]
        assert cp[p][1] == float(u)
