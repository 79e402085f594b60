"""GPU adjoint (d colourful count / d edge weight) against the oracle's
reverse-mode derivative, brute-force per-edge counts and finite differences
of the GPU's own FP64 forward."""
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


def random_tree(t, rng):
    par = [-1] + [int(rng.integers(0, v)) for v in range(1, t)]
    perm = rng.permutation(t)
    out = [0] * t
    for v in range(t):
        out[perm[v]] = -1 if par[v] < 0 else int(perm[par[v]])
    return out


def gpu_grad(G, par, k, seed, ncol, gcol, w=None):
    g = sg.Graph(G.n, G.row_ptr, G.col_idx, G.w if w is None else w)
    c = sg.Colorings(g, k, seed, ncol)
    p = sg.Plan(par, k)
    r = sg.count(p, g, c, "fp64")
    gw = sg.count_grad(p, g, c, gcol, "fp64")
    return r["colorful"], gw.cpu().numpy()


def test_grad_small_graphs_vs_oracle():
    rng = np.random.default_rng(1)
    for trial in range(6):
        n = int(rng.integers(20, 60))
        edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.15]
        G = gg.from_edge_list(n, edges, rng.uniform(0.5, 1.5, len(edges)))
        t = int(rng.integers(2, 8))
        par = random_tree(t, rng)
        say("grad small", trial, par)
        f, gw = gpu_grad(G, par, t, 3, 1, [1.0])
        fo, go = O.grad(G, par, t, O.colors(G.n, t, 3, 0))
        assert f[0] == pytest.approx(fo, rel=1e-12, abs=1e-12)
        np.testing.assert_allclose(gw, go, rtol=1e-11, atol=1e-11 * max(1.0, np.abs(go).max()))


def test_grad_weights_colourings_combination():
    """Several colourings, each weighted by grad_colorful[j]."""
    rng = np.random.default_rng(2)
    G = gg.chung_lu(3000, 8.0, 2.1, seed=11, weighted=True)
    par, k = gg.CATERPILLAR10, 10
    gc = [0.5, -2.0, 1.25]
    _, gw = gpu_grad(G, par, k, 9, 3, gc)
    ref = np.zeros(G.nnz)
    for j, a in enumerate(gc):
        _, go = O.grad(G, par, k, O.colors(G.n, k, 9, j))
        ref += a * go
    np.testing.assert_allclose(gw, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_grad_brute_force_edge_counts():
    """The folded derivative of the weighted count of an edge equals the sum,
    over the colourful maps using that edge, of the product of the other edge
    weights (brute-force enumeration on a 200-vertex subgraph)."""
    G = gg.chung_lu_262k_weighted()
    deg = G.degrees()
    # breadth-first ball of 200 vertices through vertices of degree <= 32
    # (hubs would make the enumeration explode), induced subgraph
    cap = 32
    start = int(np.nonzero((deg >= 8) & (deg <= cap))[0][0])
    seen, order, head = {start}, [start], 0
    while head < len(order) and len(order) < 200:
        v = order[head]
        head += 1
        for u in G.col_idx[G.row_ptr[v]:G.row_ptr[v + 1]]:
            u = int(u)
            if u not in seen and deg[u] <= cap and len(order) < 200:
                seen.add(u)
                order.append(u)
    idx = {v: i for i, v in enumerate(order)}
    edges, ws = [], []
    for v in order:
        for e in range(G.row_ptr[v], G.row_ptr[v + 1]):
            u = int(G.col_idx[e])
            if u in idx and idx[v] < idx[u]:
                edges.append((idx[v], idx[u]))
                ws.append(float(G.w[e]))
    S = gg.from_edge_list(len(order), edges, ws)
    par, k = gg.CATERPILLAR10, 10
    col = O.colors(S.n, k, 4, 0)
    tot, maps, bg = O.brute(S, par, col, grad=True, limit=2_000_000_000)
    assert maps > 1000
    f, gw = gpu_grad(S, par, k, 4, 1, [1.0])
    say("brute ball", S.n, S.nnz, maps, tot, f[0])
    assert f[0] == pytest.approx(tot, rel=1e-12, abs=1e-9)
    np.testing.assert_allclose(O.fold_undirected(S, gw), O.fold_undirected(S, bg), rtol=1e-10,
                               atol=1e-9)


def test_grad_diff_config_sampled_vs_oracle_and_fd():
    """Chung-Lu n=262,144, mean degree 16, weights U[0.5,1.5), caterpillar10:
    the GPU gradient at 64 random edges against the oracle's reverse mode and
    against central differences (step 1e-3) of the GPU FP64 forward."""
    G = gg.chung_lu_262k_weighted()
    par, k, seed = gg.CATERPILLAR10, 10, 3
    f, gw = gpu_grad(G, par, k, seed, 1, [1.0])
    say("diff config forward", f[0])
    fo, go = O.grad(G, par, k, O.colors(G.n, k, seed, 0))
    assert f[0] == pytest.approx(fo, rel=1e-12)
    rng = np.random.default_rng(0)
    sample = rng.choice(G.nnz, 64, replace=False)
    np.testing.assert_allclose(gw[sample], go[sample], rtol=1e-10,
                               atol=1e-12 * np.abs(go).max())
    # central differences of the undirected weight (both entries moved)
    gu = O.fold_undirected(G, gw)
    rows = np.repeat(np.arange(G.n), np.diff(G.row_ptr))
    p = sg.Plan(par, k)
    h = 1e-3
    for e in sample:
        i, j = int(rows[e]), int(G.col_idx[e])
        rev = int(G.row_ptr[j] + np.searchsorted(G.col_idx[G.row_ptr[j]:G.row_ptr[j + 1]], i))
        vals = []
        for d in (h, -h):
            w = G.w.astype(np.float64).copy()
            w[e] += d
            w[rev] += d
            g = sg.Graph(G.n, G.row_ptr, G.col_idx, w.astype(np.float32))
            # float32 weights cannot hold w +- 1e-3 exactly: use the rounded step
            dw = float(np.float32(w[e])) - float(G.w[e])
            vals.append((sg.count(p, g, sg.Colorings(g, k, seed, 1), "fp64")["colorful"][0], dw))
        fd = (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])
        assert fd == pytest.approx(gu[e], rel=1e-6, abs=1e-9 * abs(f[0]))


@pytest.mark.parametrize("mode", ["fp64", "fp32s"])
def test_autograd_function(mode):
    import torch
    G = gg.chung_lu(2000, 6.0, 2.1, seed=5, weighted=True)
    par, k = gg.PATH5, 5
    rp = torch.as_tensor(G.row_ptr, device="cuda")
    ci = torch.as_tensor(G.col_idx, device="cuda")
    w = torch.as_tensor(G.w, device="cuda").requires_grad_(True)
    out = sg.SubgraphCount.apply(w, sg.Plan(par, k), rp, ci, 8, 2, mode)
    (out * torch.tensor([1.0, 3.0], dtype=torch.float64, device="cuda")).sum().backward()
    ref = np.zeros(G.nnz)
    for j, a in enumerate((1.0, 3.0)):
        _, go = O.grad(G, par, k, O.colors(G.n, k, 8, j))
        ref += a * go
    # w is float32: the gradient is returned in w's dtype
    np.testing.assert_allclose(w.grad.double().cpu().numpy(), ref, rtol=1e-6 if mode == "fp64" else 2e-5,
                               atol=0 if mode == "fp64" else 2e-5 * np.abs(ref).max())


def test_grad_fp32s_diff_config_sampled_vs_oracle():
    """The differentiation workload (Chung-Lu n=262,144, mean degree 16,
    weights U[0.5,1.5), caterpillar10) in FP32S: 256 sampled entries against
    the oracle's reverse mode."""
    G = gg.chung_lu_262k_weighted()
    par, k, seed = gg.CATERPILLAR10, 10, 3
    g = sg.Graph(G.n, G.row_ptr, G.col_idx, G.w)
    c = sg.Colorings(g, k, seed, 1)
    gw = sg.count_grad(sg.Plan(par, k), g, c, [1.0], "fp32s").cpu().numpy()
    _, go = O.grad(G, par, k, O.colors(G.n, k, seed, 0))
    sample = np.random.default_rng(1).choice(G.nnz, 256, replace=False)
    say("diff config fp32s")
    np.testing.assert_allclose(gw[sample], go[sample], rtol=2e-5, atol=2e-5 * np.abs(go).max())


def test_grad_rejects_u64():
    G = gg.tiny_er()
    g = sg.Graph.from_csr(G)
    p = sg.Plan(gg.PATH5, 5)
    c = sg.Colorings(g, 5, 1, 1)
    with pytest.raises(sg.Sg2vError) as e:
        sg.count_grad(p, g, c, [1.0], "u64")
    assert e.value.status == -1


def _fp32s_vs(go, gw32, rtol=2e-5):
    """FP32S gradient against a reference: relative per entry, with an
    absolute floor of rtol times the largest entry (FP32 frame scaling keeps
    relative accuracy for entries near the table maxima)."""
    np.testing.assert_allclose(gw32, go, rtol=rtol, atol=rtol * np.abs(go).max())


def test_grad_fp32s_small_graphs_vs_oracle():
    rng = np.random.default_rng(7)
    for trial in range(6):
        n = int(rng.integers(20, 60))
        edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.15]
        G = gg.from_edge_list(n, edges, rng.uniform(0.5, 1.5, len(edges)))
        t = int(rng.integers(2, 8))
        par = random_tree(t, rng)
        say("grad fp32s small", trial, par)
        g = sg.Graph(G.n, G.row_ptr, G.col_idx, G.w)
        c = sg.Colorings(g, t, 3, 1)
        gw = sg.count_grad(sg.Plan(par, t), g, c, [1.0], "fp32s").cpu().numpy()
        _, go = O.grad(G, par, t, O.colors(G.n, t, 3, 0))
        _fp32s_vs(go, gw)


def test_grad_fp32s_colourings_and_signs():
    """FP32S adjoint over three colourings weighted 0.5, -2, 1.25 (the sign
    of a colouring's weight carries through its scaled tables)."""
    G = gg.chung_lu(3000, 8.0, 2.1, seed=11, weighted=True)
    par, k = gg.CATERPILLAR10, 10
    gc = [0.5, -2.0, 1.25]
    g = sg.Graph(G.n, G.row_ptr, G.col_idx, G.w)
    c = sg.Colorings(g, k, 9, 3)
    gw = sg.count_grad(sg.Plan(par, k), g, c, gc, "fp32s").cpu().numpy()
    ref = np.zeros(G.nnz)
    for j, a in enumerate(gc):
        _, go = O.grad(G, par, k, O.colors(G.n, k, 9, j))
        ref += a * go
    _fp32s_vs(ref, gw)


@pytest.mark.parametrize("par,k", [(gg.BINTREE7, 7), (gg.PATH8, 8), (gg.CATERPILLAR10, 11)])
def test_grad_fp32s_matches_fp64_on_rmat(par, k):
    """RMAT scale 14 with 800,000 entries (a row of 5228 neighbours is split
    over tasks), unweighted: the FP32S adjoint against the FP64 adjoint of the
    same colouring."""
    G = gg.rmat(14, 400_000, seed=17)
    g = sg.Graph.from_csr(G)
    c = sg.Colorings(g, k, 2, 1)
    p = sg.Plan(par, k)
    say("grad fp32s rmat14", par, k)
    g64 = sg.count_grad(p, g, c, [1.0], "fp64").cpu().numpy()
    g32 = sg.count_grad(p, g, c, [1.0], "fp32s").cpu().numpy()
    _fp32s_vs(g64, g32)


@pytest.mark.parametrize("par,k", [([-1, 0], 2), ([-1, 0, 0, 0], 4), (gg.PATH5, 7), ([-1, 0, 1, 1, 0, 4], 8)])
def test_grad_fp32s_shapes(par, k):
    """FP32S adjoint on an edge, a star (one-vertex passives only), k > t,
    and a small tree with k > t, against the oracle's reverse mode."""
    rng = np.random.default_rng(len(par) * 10 + k)
    n = 50
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.2]
    G = gg.from_edge_list(n, edges, rng.uniform(0.5, 1.5, len(edges)))
    g = sg.Graph(G.n, G.row_ptr, G.col_idx, G.w)
    c = sg.Colorings(g, k, 5, 2)
    say("grad fp32s shape", par, k)
    gw = sg.count_grad(sg.Plan(par, k), g, c, [1.0, 0.25], "fp32s").cpu().numpy()
    ref = np.zeros(G.nnz)
    for j, a in enumerate((1.0, 0.25)):
        _, go = O.grad(G, par, k, O.colors(G.n, k, 5, j))
        ref += a * go
    _fp32s_vs(ref, gw)


@pytest.mark.parametrize("mode", ["fp64", "fp32s"])
def test_grad_checkpointed_equals_recomputed(mode):
    """Forward tables kept from one pass per colouring (checkpointing, the
    default when they fit) and recomputed up to each split give the same
    gradients bit for bit, and both match the oracle's reverse mode."""
    G = gg.chung_lu(5000, 12.0, 2.1, seed=14, weighted=True)
    par, k, seed = gg.CATERPILLAR10, 10, 2
    g = sg.Graph.from_csr(G)
    c = sg.Colorings(g, k, seed, 2)
    p = sg.Plan(par, k)
    gcol = [1.0, -0.5]
    say("grad checkpointed", mode)
    kept = sg.count_grad(p, g, c, gcol, mode).cpu().numpy()
    with sg.tuned(flags=sg.TUNE_GRAD_RECOMPUTE):
        say("grad recomputed", mode)
        rec = sg.count_grad(p, g, c, gcol, mode).cpu().numpy()
    np.testing.assert_array_equal(kept, rec)
    ref = np.zeros(G.nnz)
    for j, gj in enumerate(gcol):
        _, gr = O.grad(G, par, k, O.colors(G.n, k, seed, j))
        ref += gj * gr
    scale = np.abs(ref).max()
    tol = 1e-10 if mode == "fp64" else 2e-5
    np.testing.assert_allclose(kept, ref, rtol=tol, atol=tol * scale)
