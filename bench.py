#!/usr/bin/env python3
"""Benchmark: colourings/s of the FP32 (per-column scaled) count of
the 15-vertex complete binary tree on an RMAT graph with 2^20 vertices and
200,000,000 directed edges (k = 15, 4 colourings per step), next to the plain
one-colouring-per-pass FP64 path and the CPU oracle.

One step = colour the graph 4 times and run the whole dynamic programme
(neighbour-colour histogram, SpMMs, multiply-adds, root reduction) for all 4
colourings; inputs are resident in HBM when the timed region starts.

Prints one JSON line.  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "colorings/s batched FP32 vs plain FP64, RMAT-1M 15-vertex tree; HBM GB/s"
HBM_PEAK_GBPS = 8000.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_2009_11665_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmm_traffic_bintree15_rmat20.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def oracle_work(parent, k, n, nnz):
    """Inner-loop iterations of the oracle for one colouring: for every split
    of its (non-deduplicated, last-child) partition, n * C(k,m) * 2^m sub-mask
    steps and nnz * C(k, m_p) neighbour additions."""
    t = len(parent)
    ch = [[] for _ in range(t)]
    root = parent.index(-1)
    for v, p in enumerate(parent):
        if p >= 0:
            ch[p].append(v)

    def size(v):
        return 1 + sum(size(c) for c in ch[v])

    work = 0

    def walk(v, kept):
        nonlocal work
        if kept == 0:
            return 1
        m_a = walk(v, kept - 1)
        tau = ch[v][kept - 1]
        m_p = walk(tau, len(ch[tau]))
        m = m_a + m_p
        work += n * math.comb(k, m) * (1 << m) + nnz * math.comb(k, m_p)
        return m

    walk(root, len(ch[root]))
    return work


def kernel_sha():
    """Hash of the SpMM kernel source (the text between its BEGIN/END marks)."""
    with open(KERNEL_SOURCE) as f:
        src = f.read()
    body = src[src.index("// BEGIN k_spmm"):src.index("// END k_spmm")]
    return hashlib.sha256(body.encode()).hexdigest()[:16]


def load_traffic(launches_per_colouring, relabel):
    """HBM bytes per SpMM launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source with the same launches per
    colouring (the launch configuration)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        d = json.load(f)
    if d.get("kernel_source_sha") != kernel_sha():
        return None
    if d.get("spmm_launches_per_colouring") != launches_per_colouring:
        return None
    if int(d.get("graph_relabel", 0)) != relabel:
        return None
    return d.get("hbm_bytes_per_launch")


def pmc_per_dispatch(db, counter):
    """(kernel name, value) per dispatch of one counter from a rocprofv3 rocpd
    database (table counters_collection)."""
    import sqlite3
    con = sqlite3.connect(db)
    try:
        rows = con.execute("select dispatch_id, kernel_name, value from counters_collection "
                           "where counter_name = ? order by dispatch_id", (counter,)).fetchall()
    finally:
        con.close()
    return [(r[1], float(r[2])) for r in rows]


def write_traffic(spmm_fetch, spmm_write, copy_fetch, copy_write, gather_fetch, gather_write,
                  mib, relabel):
    """HBM-side bytes per SpMM launch from rocprofv3 --pmc FETCH_SIZE and
    WRITE_SIZE runs (KiB per dispatch).  Reads are scaled by what FETCH_SIZE
    reads for a gather of known size (random 256-byte rows of a table of
    `mib` MiB, each row read once: the SpMM's access pattern), writes by what
    WRITE_SIZE reads for a linear device copy of `mib` MiB.  FETCH_SIZE counts
    L2 read misses, Infinity Cache hits included: an upper bound on HBM reads."""
    def mean_of(db, counter, pick):
        v = [x for name, x in pmc_per_dispatch(db, counter) if pick(name)]
        if not v:
            raise SystemExit(f"no matching dispatches of {counter} in {db}")
        return sum(v) / len(v), len(v)

    is_spmm = lambda name: "k_spmm<float" in name  # noqa: E731
    is_copy = lambda name: "copyBuffer" in name  # noqa: E731
    is_gather = lambda name: "gather" in name.lower()  # noqa: E731
    nbytes = mib * (1 << 20)
    cf, _ = mean_of(copy_fetch, "FETCH_SIZE", is_copy)
    cw, _ = mean_of(copy_write, "WRITE_SIZE", is_copy)
    gf, _ = mean_of(gather_fetch, "FETCH_SIZE", is_gather)
    gw, _ = mean_of(gather_write, "WRITE_SIZE", is_gather)
    f_fetch_lin, f_write = nbytes / (cf * 1024.0), nbytes / (cw * 1024.0)
    # a gather dispatch reads exactly the rows it writes (linearly): its read
    # bytes are its WRITE_SIZE scaled by the copy's write factor
    gather_bytes = gw * 1024.0 * f_write
    f_fetch = gather_bytes / (gf * 1024.0)
    sf, nf = mean_of(spmm_fetch, "FETCH_SIZE", is_spmm)
    sw, nw = mean_of(spmm_write, "WRITE_SIZE", is_spmm)
    rd, wr = sf * 1024.0 * f_fetch, sw * 1024.0 * f_write
    out = {"kernel": "k_spmm<float,...>", "kernel_source_sha": kernel_sha(),
           "graph_relabel": relabel,
           "spmm_launches_per_colouring": nf,
           "hbm_bytes_per_launch": rd + wr, "read_bytes_per_launch": rd, "write_bytes_per_launch": wr,
           "read_bytes_per_launch_linear_calibration": sf * 1024.0 * f_fetch_lin,
           "launches": [nf, nw], "fetch_size_kib_per_launch": sf, "write_size_kib_per_launch": sw,
           "calibration": {"copy_bytes": nbytes, "gather_bytes_per_dispatch": gather_bytes,
                           "fetch_factor_gather": f_fetch, "fetch_factor_linear_copy": f_fetch_lin,
                           "write_factor_linear_copy": f_write},
           "note": "FETCH_SIZE counts L2 read misses including Infinity Cache hits: the read "
                   "bytes are an upper bound on HBM reads",
           "runs": ["rocprofv3 --pmc FETCH_SIZE -- python3 bench.py --steps 1 --warmup 0 "
                    f"--no-cpu-baseline --no-fp64 --no-batch-workload --colorings 1 --relabel {relabel}",
                    "rocprofv3 --pmc WRITE_SIZE -- (same)",
                    f"rocprofv3 --pmc FETCH_SIZE -- python3 bench.py --calibrate-copy {mib}",
                    f"rocprofv3 --pmc WRITE_SIZE -- python3 bench.py --calibrate-copy {mib}",
                    f"rocprofv3 --pmc FETCH_SIZE -- python3 bench.py --calibrate-gather {mib}",
                    f"rocprofv3 --pmc WRITE_SIZE -- python3 bench.py --calibrate-gather {mib}"]}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def treelet_workload(sg, gg, torch, G=None, ncol=8, reps=2):
    """Treelet distribution: the 47 non-isomorphic nine-vertex trees (k = 9)
    x ncol colourings on Chung-Lu n = 500,000, mean degree 20, gamma 2.1 (a
    synthetic stand-in for the paper's protein networks), FP32 with per-column
    exponents: one sg2v_count_multi call sharing isomorphic sub-templates
    across the 47 trees, against the same counts template by template."""
    G = G if G is not None else gg.chung_lu_500k()
    g = sg.Graph.from_csr(G)
    trees = sg.trees(9)
    multi = sg.Plan.multi(trees, 9)
    plans = [sg.Plan(p, 9) for p in trees]
    c = sg.Colorings(g, 9, 6, ncol)
    res = sg.count_multi(multi, g, c, "fp32s")  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = sg.count_multi(multi, g, c, "fp32s")
    torch.cuda.synchronize()
    t_multi = (time.perf_counter() - t0) / reps
    for p in plans:
        sg.count(p, g, c, "fp32s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sep = [sg.count(p, g, c, "fp32s") for p in plans]
    torch.cuda.synchronize()
    t_sep = time.perf_counter() - t0
    diff = max(float(np.max(np.abs(r["colorful"] - res["colorful"][i]) / np.abs(res["colorful"][i])))
               for i, r in enumerate(sep))
    info = multi.info()
    return {
        "workload": f"chung-lu n=500000 d=20 gamma=2.1; all 47 nine-vertex trees, k=9, {ncol} colourings, fp32s",
        "template_colorings_per_s": len(trees) * ncol / t_multi,
        "ms_one_call_shared": t_multi * 1e3,
        "ms_template_by_template": t_sep * 1e3,
        "nodes_shared": info.n_nodes,
        "nodes_unshared": sum(p.info().n_nodes for p in plans),
        "max_rel_diff_shared_vs_separate": diff,
        "frequency": [float(x) for x in res["frequency"]],
    }


def batch_workload(sg, gg, torch, reps=3):
    """Three templates of uneven size (bintree7, path8, caterpillar10, k = t)
    x 16 colourings on Chung-Lu n = 500,000, mean degree 20, each template
    re-rooted by sg2v_template_reroot (same counts, cheaper decomposition):
    all passes of all templates recorded as one HIP graph (sg2v_count_batch,
    replayed; the templates are parallel branches of the graph), against the
    graph with the templates in sequence, one persistent kernel running every
    template's recorded launches (and the graph with that kernel's forced
    kernel choices), the same counts run template by template, colouring
    included, and the templates rooted as given.  Tuning from the autotuner
    on the widest template."""
    G = gg.chung_lu_500k()
    g = sg.Graph.from_csr(G)
    given = (gg.BINTREE7, gg.PATH8, gg.CATERPILLAR10)
    pars = [sg.reroot(p, len(p), 0.05)[0] for p in given]
    plans = [sg.Plan(p) for p in pars]
    ncol, seed = 16, 4
    old = sg.get_tuning()

    def graph_ms(pl):
        sg.count_batch(pl, g, seed, ncol, "fp32s")  # records and caches the graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            cf, _ = sg.count_batch(pl, g, seed, ncol, "fp32s")
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, cf

    try:
        tuned = sg.autotune(plans[2], g, "fp32s", ncol)  # probe with the workload's colourings per template
        t_given, cf_given = graph_ms([sg.Plan(p) for p in given])
        t_graph, cf = graph_ms(plans)
        cur = sg.get_tuning()
        serial = sg.get_tuning()
        serial.flags |= sg.TUNE_BATCH_SERIAL
        sg.restore_tuning(serial)
        t_serial, _ = graph_ms(plans)
        # one persistent kernel over every template's launches, and the graph
        # with the kernel choices that schedule forces (general multiply-add,
        # vertex-order root) for a like-for-like comparison
        pers = sg.get_tuning()
        pers.flags = (cur.flags | sg.TUNE_BATCH_PERSISTENT) & ~sg.TUNE_SPMM_PANEL
        sg.restore_tuning(pers)
        t_pers, cf_pers = graph_ms(plans)
        same = sg.get_tuning()
        same.flags = (cur.flags | sg.TUNE_NO_COLOR_EMA | sg.TUNE_ROOT_ROWS) & ~sg.TUNE_SPMM_PANEL
        sg.restore_tuning(same)
        t_same, _ = graph_ms(plans)
        sg.restore_tuning(cur)
        for p, par in zip(plans, pars):  # warm
            sg.count(p, g, sg.Colorings(g, len(par), seed, ncol), "fp32s")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for p, par in zip(plans, pars):
                sg.count(p, g, sg.Colorings(g, len(par), seed, ncol), "fp32s")
        torch.cuda.synchronize()
        t_seq = (time.perf_counter() - t0) / reps
    finally:
        sg.restore_tuning(old)
    return {
        "workload": "chung-lu n=500000 d=20 gamma=2.1; bintree7, path8, caterpillar10 (k=t, re-rooted) x 16 colourings, fp32s",
        "template_colorings_per_s": 3 * ncol / t_graph,
        "ms_one_graph_launch": t_graph * 1e3,
        "ms_one_graph_launch_templates_in_sequence": t_serial * 1e3,
        "ms_template_by_template": t_seq * 1e3,
        "ms_one_graph_launch_given_roots": t_given * 1e3,
        "ms_one_persistent_kernel": t_pers * 1e3,
        "ms_one_graph_launch_persistent_kernel_choices": t_same * 1e3,
        "persistent_vs_graph_max_rel_diff": float(max(abs(a - b) / abs(b) for a, b in zip(cf_pers.ravel(), cf.ravel()))),
        "rerooted_vs_given_max_rel_diff": float(max(abs(a - b) / abs(b) for a, b in zip(cf.ravel(), cf_given.ravel()))),
        "parents": pars,
        "tuning": {"spmm_width": tuned.spmm_width, "ema_rows": tuned.ema_rows, "batch": tuned.batch,
                   "flags": tuned.flags},
    }


def adjoint_workload(sg, gg, torch, reps=2):
    """The differentiation workload: Chung-Lu n = 262,144, mean degree 16,
    gamma 2.1, edge weights U[0.5, 1.5); caterpillar10, k = 10; one colouring:
    weighted FP64 count and its adjoint (d count / d w_e for every CSR entry,
    sub-template tables recomputed)."""
    G = gg.chung_lu_262k_weighted()
    g = sg.Graph.from_csr(G)
    p = sg.Plan(gg.CATERPILLAR10, 10)
    c = sg.Colorings(g, 10, 3, 1)
    sg.count(p, g, c, "fp64")
    sg.count_grad(p, g, c, [1.0], "fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sg.count(p, g, c, "fp64")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        g64 = sg.count_grad(p, g, c, [1.0], "fp64")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sg.count(p, g, c, "fp32s")
    sg.count_grad(p, g, c, [1.0], "fp32s")
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for _ in range(reps):
        sg.count(p, g, c, "fp32s")
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(reps):
        g32 = sg.count_grad(p, g, c, [1.0], "fp32s")
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    d = (g32 - g64).abs()
    # the adjoint with every split's forward tables recomputed instead of kept
    with sg.tuned(flags=sg.get_tuning().flags | sg.TUNE_GRAD_RECOMPUTE):
        sg.count_grad(p, g, c, [1.0], "fp64")
        torch.cuda.synchronize()
        t6 = time.perf_counter()
        for _ in range(reps):
            g64r = sg.count_grad(p, g, c, [1.0], "fp64")
        torch.cuda.synchronize()
        t7 = time.perf_counter()
    same = bool(torch.equal(g64r, g64))
    return {"workload": "chung-lu n=262144 d=16 gamma=2.1 weighted; caterpillar10 k=10; 1 colouring",
            "ms_forward": (t1 - t0) / reps * 1e3, "ms_adjoint": (t2 - t1) / reps * 1e3,
            "ms_adjoint_recompute_per_split": (t7 - t6) / reps * 1e3,
            "checkpointed_equals_recomputed": same,
            "ms_forward_fp32s": (t4 - t3) / reps * 1e3, "ms_adjoint_fp32s": (t5 - t4) / reps * 1e3,
            "fp32s_vs_fp64_grad_max_abs_err_over_max": float(d.max() / g64.abs().max()),
            "entries": G.nnz}


def host_facts():
    """CPU model and memory of the host, from /proc."""
    model, mem_gb = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    mem_gb = int(line.split()[1]) / (1 << 20)
                    break
    except OSError:
        pass
    return model, mem_gb


def cpu_baseline(parent, k, scale, seed, full_n, full_nnz):
    """The oracle (FP64, OpenMP over vertices) on a bounded sample: one
    colouring of the same template and colouring rule on an RMAT graph of
    2^scale vertices with the full graph's average degree, timed here; the
    rate is scaled to the full graph by the oracle's inner-loop count."""
    import graphgen as gg
    import oracle as O

    avg = full_nnz / full_n
    m = int(round(avg / 2 * (1 << scale)))
    model, mem_gb = host_facts()
    # the oracle's FP64 tables: about 40 GB at scale 18 (measured 5 GB at scale 15)
    need_gb = 5.0 * (1 << scale) / (1 << 15)
    while mem_gb is not None and scale > 14 and need_gb > 0.6 * mem_gb:
        scale -= 1
        m = int(round(avg / 2 * (1 << scale)))
        need_gb /= 2
    G = gg.rmat(scale, m, seed=seed)
    col = O.colors(G.n, k, seed, 0)
    log(f"cpu baseline: oracle on RMAT scale {scale} (n={G.n}, nnz={G.nnz}), {O.num_threads()} threads")
    t0 = time.perf_counter()
    O.count(G, parent, k, col)
    dt = time.perf_counter() - t0
    ratio = oracle_work(parent, k, full_n, full_nnz) / oracle_work(parent, k, G.n, G.nnz)
    return {
        "value": 1.0 / (dt * ratio),
        "unit": "colorings/s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": (f"measured: 1 colouring of bintree15 (k={k}, FP64) on RMAT scale {scale} "
                   f"(n={G.n}, nnz={G.nnz}, the full graph's average degree) took {dt:.1f} s on "
                   f"{O.num_threads()} threads; value = that rate scaled by the oracle's "
                   f"inner-loop count to the full graph (x{ratio:.2f})"),
        "sample_seconds": dt,
        "sample_colorings_per_s": 1.0 / dt,
        "sample_scale": scale,
        "host_cpu": model,
        "host_mem_gb": mem_gb,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--colorings", type=int, default=4)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--edges", type=int, default=100_000_000, help="undirected edges")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--cpu-scale", type=int, default=18)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--relabel", type=int, default=1, choices=(0, 1),
                    help="register the graph with SG2V_GRAPH_RELABEL (vertices by degree, dealt "
                         "round-robin to the XCD neighbour ranges); counts are identical")
    ap.add_argument("--tune-flags", type=int, default=0,
                    help="extra sg2v tuning flags for the timed FP32 steps (e.g. 1024: row-panel SpMM)")
    ap.add_argument("--spmm-width", type=int, default=0, help="SpMM chunk columns (0: automatic)")
    ap.add_argument("--xsplit-min", type=int, default=0,
                    help="neighbour-range split task threshold (0: automatic, 512)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batch-workload", action="store_true",
                    help="skip the multi-template batch and adjoint measurements")
    ap.add_argument("--batch-only", choices=("graph", "graph-same", "persistent"), default=None,
                    help="only run the batch workload's count twice in one mode (graph: the HIP "
                         "graph with 128-column chunks; graph-same: the same with the persistent "
                         "schedule's kernel choices; persistent: the persistent kernel) and exit "
                         "(for profiling)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (calibrates the "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE counters) and exit")
    ap.add_argument("--calibrate-gather", type=int, default=0, metavar="MIB",
                    help="only gather every 256-byte row of a MIB MiB table once in random "
                         "order (3 times; calibrates FETCH_SIZE for row gathers) and exit")
    ap.add_argument("--traffic-from", nargs=6,
                    metavar=("SPMM_FETCH", "SPMM_WRITE", "COPY_FETCH", "COPY_WRITE", "GATHER_FETCH",
                             "GATHER_WRITE"),
                    help="write the SpMM traffic file from six rocprofv3 --pmc databases "
                         "(--calibrate-copy gives the calibration size, default 1024 MiB) and exit")
    args = ap.parse_args()

    if args.traffic_from:
        write_traffic(*args.traffic_from, args.calibrate_copy or 1024, args.relabel)
        return

    if args.batch_only:
        import torch
        import graphgen as gg
        import paper_2009_11665_amd as sg
        G = gg.chung_lu_500k()
        g = sg.Graph.from_csr(G)
        plans = [sg.Plan(sg.reroot(p, len(p), 0.05)[0]) for p in (gg.BINTREE7, gg.PATH8, gg.CATERPILLAR10)]
        flags = sg.TUNE_NO_COLOR_SKIP
        if args.batch_only != "graph":
            flags |= sg.TUNE_NO_COLOR_EMA | sg.TUNE_ROOT_ROWS
        if args.batch_only == "persistent":
            flags |= sg.TUNE_BATCH_PERSISTENT
        with sg.tuned(flags=flags, spmm_width=128):
            for _ in range(2):
                sg.count_batch(plans, g, 4, 16, "fp32s")
        torch.cuda.synchronize()
        print(json.dumps({"batch_only": args.batch_only, "runs": 2}))
        return

    if args.calibrate_gather:
        import torch
        rows = args.calibrate_gather * (1 << 20) // 256
        table = torch.rand(rows, 64, dtype=torch.float32, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(1)
        idx = torch.randperm(rows, device="cuda", generator=g)
        out = torch.empty_like(table)
        for _ in range(3):
            torch.index_select(table, 0, idx, out=out)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_gather_bytes": rows * 256, "gathers": 3}))
        return

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "copies": 5}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU "
                          "sharding of the count is described, not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import graphgen as gg
    import paper_2009_11665_amd as sg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    parent, k, ncol = gg.BINTREE15, 15, args.colorings

    t0 = time.perf_counter()
    G = gg.rmat(args.scale, args.edges, seed=args.seed)
    log(f"graph: RMAT scale {args.scale}, n={G.n}, nnz={G.nnz}, max deg {int(G.degrees().max())} "
        f"({time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    g = sg.Graph.from_csr(G, relabel=bool(args.relabel))
    log(f"graph registered (relabel={args.relabel}, {time.perf_counter() - t0:.1f} s)")
    plan = sg.Plan(parent, k)
    info = plan.info()
    torch.cuda.synchronize()

    def step(mode, first):
        c = sg.Colorings(g, k, args.seed, ncol, first=first)
        return sg.count(plan, g, c, mode)

    # FP32 with per-column exponents
    if args.tune_flags or args.spmm_width or args.xsplit_min:
        cur = sg.get_tuning()
        cur.flags |= args.tune_flags
        cur.spmm_width = args.spmm_width
        cur.xsplit_min = args.xsplit_min
        sg.restore_tuning(cur)
    for w in range(args.warmup):
        step("fp32s", 1000 + w * ncol)
        log(f"warmup step {w} done")
    torch.cuda.synchronize()
    sg.profile_start()
    t0 = time.perf_counter()
    res32 = None
    for s in range(args.steps):
        res32 = step("fp32s", s * ncol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sg.profile_stop()
    log(f"timed {args.steps} fp32s steps: {(t1 - t0) / args.steps * 1e3:.1f} ms/step")
    ms_step = (t1 - t0) / args.steps * 1e3
    value = ncol * args.steps / (t1 - t0)

    # plain per-colouring FP64 on the colourings of the last timed step
    fp64 = None
    err = None
    if not args.no_fp64:
        old = sg.get_tuning()
        one = sg.get_tuning()
        one.batch = 1
        sg.restore_tuning(one)
        try:
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            r64 = None
            for s in range(args.fp64_steps):
                r64 = step("fp64", (args.steps - 1) * ncol)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
        finally:
            sg.restore_tuning(old)
        fp64 = {"value": ncol * args.fp64_steps / (t3 - t2), "unit": "colorings/s",
                "ms_per_step": (t3 - t2) / args.fp64_steps * 1e3}
        err = max(abs(a - b) / abs(b) for a, b in zip(res32["colorful"], r64["colorful"]) if b)
        log(f"fp64 plain: {fp64['ms_per_step']:.1f} ms/step, fp32s rel err {err:.2e}")

    sp = prof["spmm"]
    # one neighbour-colour histogram per pass (bintree15 has one single-vertex passive child)
    passes = prof["hist"]["launches"] // args.steps if args.steps else 0
    achieved = sp["bytes"] / (sp["ms"] * 1e-3) / 1e9 if sp["ms"] > 0 else 0.0
    # measured HBM bytes per SpMM launch (rocprofv3 counters)
    traffic = load_traffic(sp["launches"] // (args.steps * ncol) if sp["launches"] % (args.steps * ncol) == 0
                           else None, args.relabel)
    total_bytes = sum(v["bytes"] for v in prof.values())
    kernels = {kk: {"launches": v["launches"], "ms_per_step": v["ms"] / args.steps,
                    "model_GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] else 0.0}
               for kk, v in prof.items() if v["launches"]}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "colorings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"rmat-s{args.scale}-m{args.edges}-bintree15-k15-{ncol}colorings"),
            "graph": {"generator": "rmat", "scale": args.scale, "a_b_c": list(gg.RMAT_ABC),
                      "n": G.n, "nnz": G.nnz, "seed": args.seed},
            "template": "bintree15", "k": k, "colorings_per_step": ncol,
            "relabel": bool(args.relabel),
            "tune_flags": args.tune_flags,
            "spmm_width": args.spmm_width,
            "xsplit_min": args.xsplit_min,
            "passes_per_step": passes,
            "colorings_per_pass": ncol / passes if passes else None,
            "mode": ("fp32 mantissa + per-column exponent; one colouring per pass (a single "
                     "colouring's 6435-column table already fills 101 SpMM column chunks, so "
                     "colourings are not concatenated as columns here)"
                     if passes == ncol else
                     f"fp32 mantissa + per-column exponent; {ncol // max(passes, 1)} colourings "
                     "concatenated as table columns per pass"),
        },
        "fp64_plain": fp64,
        "speedup_vs_fp64_plain": (value / fp64["value"]) if fp64 else None,
        "fp32_vs_fp64_max_rel_err": err,
        "updates_per_s": (sp["work"] / (sp["ms"] * 1e-3)) if sp["ms"] else None,
        "hbm_GBps_model_step": total_bytes / (ms_step * 1e-3 * args.steps) / 1e9,
        "estimate_mean": res32["mean_estimate"],
        "plan": {"splits": info.n_splits, "spmm_columns": info.spmm_columns,
                 "pairs_per_vertex": info.pairs_per_vertex, "alpha": info.alpha},
        "kernels": kernels,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_spmm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "traffic_over_algorithmic": (traffic / (sp["bytes"] / sp["launches"])) if traffic else None,
            "launches_per_step": sp["launches"] / args.steps,
            "avg_launch_ms": sp["ms"] / sp["launches"] if sp["launches"] else None,
            "gather_model_GBps": (sp["work"] * 4 / (sp["ms"] * 1e-3) / 1e9) if sp["ms"] else None,
        },
        "cpu_baseline": None,
        "batch_workload": None,
        "adjoint_workload": None,
        "treelet_workload": None,
    }
    if not args.no_batch_workload:
        log("batch workload (3 templates x 16 colourings) ...")
        out["batch_workload"] = batch_workload(sg, gg, torch)
        log("adjoint workload ...")
        out["adjoint_workload"] = adjoint_workload(sg, gg, torch)
        log("treelet workload (47 nine-vertex trees) ...")
        out["treelet_workload"] = treelet_workload(sg, gg, torch)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(parent, k, args.cpu_scale, args.seed, G.n, G.nnz)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
