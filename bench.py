#!/usr/bin/env python3
"""Benchmark: uncompressed edges/s of the compressed product y = A x on a
web-like graph (n = 2^20, mean out-degree 20), against the same-GPU CSR
product, plus PageRank seconds to L1 residual 1e-6 (compressed vs CSR).

One step = one compressed product over the whole graph (FP32 vectors,
two-sum compensated accumulation).  Each timed launch follows a 1 GiB device
write, so the layout and x come from HBM, not from the L2s or the 256 MB
MALL; back-to-back (cache-warm) times are reported beside, labelled
mall_warm.  Prints one JSON line.  Single GPU only."""
import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# the device code and the layout it reads: the sources that decide a kernel's
# HBM traffic (host scheduling in bvmv_api.cpp does not)
KERNEL_SOURCES = ["paper_1708_07271_amd/csrc/bv_kernels.hip", "paper_1708_07271_amd/csrc/kernels.hpp",
                  "paper_1708_07271_amd/csrc/bv_layout.cpp", "paper_1708_07271_amd/csrc/bv_layout.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get("%s|%s" % (kernel, workload))
        if e and e.get("kernel_hash") == kernel_hash():
            return e.get("bytes_per_launch")
    except (OSError, ValueError):
        pass
    return None


def time_launches(fn, steps, warmup, torch):
    """Back-to-back launches between two HIP events on the current stream (the
    stream the library launches on): ms per launch with the working set left
    in L2 / the 256 MB MALL by the previous launch (cache-warm)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps   # ms per launch


class Flusher:
    """Writes a 1 GiB device buffer (4x the MALL, far beyond the L2s) so that
    the next launch reads its inputs from HBM."""

    def __init__(self, torch, dev, nbytes=1 << 30):
        self.buf = torch.empty(nbytes // 4, dtype=torch.int32, device=dev)
        self.k = 0

    def __call__(self):
        self.k += 1
        self.buf.fill_(self.k)


class ReadFlusher:
    """Reads a 1 GiB device buffer (a row-wise max into 1 MiB), so that the
    caches hold clean unrelated lines: the next launch reads its inputs from
    HBM without first writing back the dirty lines a write flush leaves."""

    def __init__(self, torch, dev, nbytes=1 << 30):
        self.torch = torch
        self.buf = torch.ones(nbytes // 4, dtype=torch.int32, device=dev).view(-1, 1024)
        self.out = torch.empty(self.buf.shape[0], dtype=torch.int32, device=dev)

    def __call__(self):
        self.torch.amax(self.buf, dim=1, out=self.out)


def pr_median(fn, runs, torch):
    """One untimed run (graph capture), then the median and minimum of
    `runs` whole runs, each bracketed by device synchronisations."""
    fn()
    ts = []
    for _ in range(runs):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return res, float(statistics.median(ts)), min(ts)


def bench_pr_sizes(args, B, P, np, torch, dev):
    """PageRank (FP32 two-sum, uniform teleport, L1 1e-6) of the workload's
    recipe at several sizes, compressed and CSR, with the blocks of each
    layout: where the fold inside the next launch and the finish kernel
    cross over."""
    rows = []
    for n in [int(float(v)) for v in args.pagerank_sizes.split(",") if v]:
        g = B.workload_graph(args.workload, n)
        G = P.bvmv_load(B.encode(g).data, keep_lists=1)
        C = P.bvmv_csr_create(G)
        p = torch.empty(g.n, dtype=torch.float32, device=dev)
        ((it, ok, _),), ms, mn = pr_median(lambda: P.bvmv_pagerank(G, p, prec=P.BVMV_F32_COMP), args.pr_runs, torch)
        (itc, okc, _), msc, mnc = pr_median(lambda: P.bvmv_csr_pagerank(C, p, prec=P.BVMV_F32_COMP), args.pr_runs,
                                           torch)
        row = {"n": g.n, "m": g.m, "blocks": P.bvmv_get_info(G)["ntiles"] // 4, "iterations": it,
               "converged": bool(ok), "ms": 1e3 * ms, "min_ms": 1e3 * mn, "csr_iterations": itc, "csr_ms": 1e3 * msc,
               "csr_min_ms": 1e3 * mnc}
        log("n %d: %d blocks, pagerank %.4f ms (%d it), csr %.4f ms (%d it)" % (g.n, row["blocks"], row["ms"], it,
                                                                                row["csr_ms"], itc))
        rows.append(row)
        del G, C
    print(json.dumps({"mode": "pagerank-sizes", "workload": args.workload, "runs": args.pr_runs,
                      "fused": os.environ.get("BVMV_PR_FUSED", "auto"), "rows": rows}), flush=True)


def time_flushed(fn, steps, warmup, flush, torch):
    """ms per launch with cold caches.  `steps` rounds of (flush, launch) and
    `steps` rounds of the flush alone are each timed between two HIP events on
    the current stream (the stream the library launches on); the launch time
    is the difference of the two means, so neither the flush nor per-launch
    event overhead is counted (this is the figure the profiler's per-kernel
    average agrees with).  Also returns the mean of per-launch event pairs
    recorded around each launch of a third sequence, which adds each event's
    own overhead (reported beside).  Returns (ms per launch, ms per flush,
    per-launch event ms)."""
    for _ in range(warmup):
        flush()
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(s)
    for _ in range(steps):
        flush()
        fn()
    ev[1].record(s)
    ev[2].record(s)
    for _ in range(steps):
        flush()
    ev[3].record(s)
    e0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    e1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for k in range(steps):
        flush()
        e0[k].record(s)
        fn()
        e1[k].record(s)
    torch.cuda.synchronize()
    both = ev[0].elapsed_time(ev[1]) / steps
    alone = ev[2].elapsed_time(ev[3]) / steps
    per = [a.elapsed_time(b) for a, b in zip(e0, e1)]
    return both - alone, alone, sum(per) / len(per)


def cpu_baseline(g, x64, budget_s):
    """The oracle's product (numpy, float64) timed on the host."""
    from oracle import product
    reps, t0 = 0, time.perf_counter()
    while True:
        product.matvec(g.rowptr, g.col, x64)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    try:
        host = len(os.sched_getaffinity(0))
    except AttributeError:
        host = os.cpu_count()
    return {"value": reps * g.m / el, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "%d full products of the %d-edge graph (oracle.product.matvec, numpy float64, one thread; "
                      "%d host cores available)" % (reps, g.m, host)}


def bench_batch(args, B, P, np, torch, dev):
    """K personalized PageRanks (teleport sets of 16 random seeds, seed 104):
    one batched launch sequence against K single-vector runs, plus the
    K-vector product against K single products."""
    K = args.batch
    wl = args.workload if args.workload != "web-n2p20-d20" else "web-n8e6-d25"
    t0 = time.perf_counter()
    g = B.workload_graph(wl)
    enc = B.encode(g)
    log("graph %s n=%d m=%d (%.1fs)" % (wl, g.n, g.m, time.perf_counter() - t0))
    G = P.bvmv_load(enc.data, tile_rows=args.tile_rows, window_cap=args.window_cap, stage_bytes=args.stage_bytes,
                    interval_mode=args.interval_mode)
    info = G.info()
    del enc
    prec = P.BVMV_F32_COMP
    # each right-hand side is one contiguous vector: row c of a (K, n) tensor
    V = torch.from_numpy(np.ascontiguousarray(B.teleport_sets(g.n, K, 16, seed=104).T).reshape(-1)).to(dev)
    X = torch.from_numpy(np.random.default_rng(105).random((K, g.n), dtype=np.float32)).to(dev)
    Y = torch.empty_like(X)
    ms_batch = time_launches(lambda: P.bvmv_multiply_batch(G, X, Y, prec), max(args.steps // 10, 5),
                             max(args.warmup // 10, 2), torch)
    x1 = X[0].contiguous()
    y1 = torch.empty_like(x1)
    ms_one = time_launches(lambda: P.bvmv_multiply(G, x1, y1, prec), args.steps, args.warmup, torch)
    log("product: %d-vector %.3f ms, single %.4f ms" % (K, ms_batch, ms_one))
    p = torch.empty(g.n * K, dtype=torch.float32, device=dev)
    P.bvmv_pagerank(G, p, teleport=V, prec=prec, k=K)  # warm (capture)
    torch.cuda.synchronize()
    t = time.perf_counter()
    res = P.bvmv_pagerank(G, p, teleport=V, prec=prec, k=K)
    torch.cuda.synchronize()
    s_batch = time.perf_counter() - t
    Vc = V.view(K, g.n)
    p1 = torch.empty(g.n, dtype=torch.float32, device=dev)
    cols = [Vc[c].contiguous() for c in range(K)]
    P.bvmv_pagerank(G, p1, teleport=cols[0], prec=prec)
    torch.cuda.synchronize()
    t = time.perf_counter()
    it_single = []
    for c in range(K):
        (it, ok, r), = P.bvmv_pagerank(G, p1, teleport=cols[c], prec=prec)
        it_single.append(it)
    torch.cuda.synchronize()
    s_single = time.perf_counter() - t
    log("pagerank: batched %.3f s, %d single runs %.3f s" % (s_batch, K, s_single))
    out = {"mode": "batched-personalized-pagerank", "workload": wl, "n": g.n, "m": g.m, "k": K,
           "layout_bytes": info["layout_bytes"], "dtype": "f32",
           "product_ms": {"batched": ms_batch, "single": ms_one, "speedup_vs_k_singles": K * ms_one / ms_batch,
                          "edges_per_s_batched": K * g.m / (ms_batch * 1e-3)},
           "pagerank_s": {"batched": s_batch, "k_single_runs": s_single, "speedup": s_single / s_batch},
           "iterations": {"batched": [r[0] for r in res], "single": it_single},
           "converged": all(r[1] for r in res)}
    print(json.dumps(out), flush=True)


def bench_social(args, B, P, np, torch, dev):
    """Social-like workload social-n4e6-d40 (n = 4e6, out-degree from a
    truncated shifted power law with exponent 2.1, mean 40, max 50000, weak
    copying, BFS order; x uniform[0,1) float32, seed 103): per-entry relative
    error of the two-sum compensated and the naive FP32 products against the
    FP64 oracle on the same float32 x (max, 99th percentile, median), and the
    compressed product against the CSR baseline on this GPU."""
    from oracle import product as _oracle_product  # the FP64 reference of the error columns
    t0 = time.perf_counter()
    g = B.workload_graph("social-n4e6-d40")
    enc = B.encode(g)
    log("social: n %d, m %d, %.2f bits/edge (%.1fs)" % (g.n, g.m, 8.0 * enc.data.size / g.m, time.perf_counter() - t0))
    G = P.bvmv_load(enc.data, keep_lists=1)
    C = P.bvmv_csr_create(G)
    info = P.bvmv_get_info(G)
    x32 = B.uniform_x(g.n, 103, np.float32)
    ref = _oracle_product.matvec(g.rowptr, g.col, x32.astype(np.float64))
    nz = ref != 0
    x = torch.from_numpy(x32).to(dev)
    y = torch.empty_like(x)
    err = {}
    for name, prec in (("f32_two_sum", P.BVMV_F32_COMP), ("f32_naive", P.BVMV_F32)):
        P.bvmv_multiply(G, x, y, prec)
        torch.cuda.synchronize()
        rel = np.abs(y.cpu().numpy().astype(np.float64)[nz] - ref[nz]) / np.abs(ref[nz])
        err[name] = {"max": float(rel.max()), "p99": float(np.percentile(rel, 99)), "median": float(np.median(rel))}
        log("%s: max rel err %.3e, p99 %.3e" % (name, err[name]["max"], err[name]["p99"]))
    ms_bv = time_launches(lambda: P.bvmv_multiply(G, x, y), args.steps, args.warmup, torch)
    ms_csr = time_launches(lambda: P.bvmv_csr_multiply(C, x, y), args.steps, args.warmup, torch)
    alg = info["layout_bytes"] + 8 * g.n
    out = {"mode": "social", "workload": "social-n4e6-d40", "n": g.n, "m": g.m,
           "bitstream_bits_per_edge": 8.0 * enc.data.size / g.m, "layout_bytes": info["layout_bytes"],
           "layout_bytes_per_edge": info["layout_bytes"] / g.m, "m_over_m_prime": g.m / max(info["m_prime"], 1),
           "long_rows": info["long_rows"], "escapes": info["escapes"], "rel_error_vs_f64_oracle": err,
           "compressed": {"ms": ms_bv, "edges_per_s": g.m / (ms_bv * 1e-3), "alg_GBs": alg / (ms_bv * 1e-3) / 1e9},
           "csr": {"ms": ms_csr, "edges_per_s": g.m / (ms_csr * 1e-3), "bytes": C.bytes() + 8 * g.n,
                   "alg_GBs": (C.bytes() + 8 * g.n) / (ms_csr * 1e-3) / 1e9},
           "speedup_compressed_vs_csr": ms_csr / ms_bv}
    print(json.dumps(out), flush=True)


def bench_formats(args, B, P, np, torch, dev):
    """One product y = A x (FP32 x uniform[0,1), seed 102, two-sum mode) on
    a workload in three formats on this GPU: the BV-style compressed layout,
    the biclique decomposition mined from the same graph (Section "Final
    Remarks"), and plain CSR.  Each launch is timed from HBM (after a 1 GiB
    device write) and back to back (cache-warm); algorithmic bytes are each
    layout's bytes plus 8 bytes per node (x read once, y written once)."""
    wl = args.workload
    t0 = time.perf_counter()
    g = B.workload_graph(wl)
    enc = B.encode(g)
    G = P.bvmv_load(enc.data, keep_lists=1)
    del enc
    C = P.bvmv_csr_create(G)
    t1 = time.perf_counter()
    bic = B.biclique_mine(g)
    t_mine = time.perf_counter() - t1
    H = P.bvmv_biclique_load(bic)
    log("formats %s: n=%d m=%d, bicliques %d (%.1fs mining), setup %.1fs" % (
        wl, g.n, g.m, bic.nbic, t_mine, time.perf_counter() - t0))
    x = torch.from_numpy(B.uniform_x(g.n, 102, np.float32)).to(dev)
    y = torch.empty_like(x)
    prec = P.BVMV_F32_COMP
    flush = Flusher(torch, dev)
    info, binfo = G.info(), H.info()
    rows = {}
    for name, fn, nbytes in (("bv", lambda: P.bvmv_multiply(G, x, y, prec), info["layout_bytes"]),
                             ("biclique", lambda: P.bvmv_biclique_multiply(H, x, y, prec), binfo["layout_bytes"]),
                             ("csr", lambda: P.bvmv_csr_multiply(C, x, y, prec), C.bytes())):
        ms, _, _ = time_flushed(fn, args.steps, args.warmup, flush, torch)
        warm = time_launches(fn, args.steps, args.warmup, torch)
        alg = nbytes + 8 * g.n
        rows[name] = {"layout_bytes": nbytes, "bytes_per_edge": nbytes / g.m, "ms": ms,
                      "edges_per_s": g.m / (ms * 1e-3), "alg_GBs": alg / (ms * 1e-3) / 1e9,
                      "frac_hbm": alg / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, "mall_warm_ms": warm}
        log("%s: %.4f ms from HBM (%.0f GB/s), %.4f ms warm" % (name, ms, rows[name]["alg_GBs"], warm))
    # the left product y = x A: on the loaded rows (no transposed graph), and
    # as the paper runs it, a right product with the transposed graph
    Gt = P.bvmv_load(B.encode(g.transpose()).data)
    tinfo = Gt.info()
    P.bvmv_multiply_left(G, x, y, prec)  # builds the column-wise layout once
    for name, fn, nbytes in (("left_on_rows", lambda: P.bvmv_multiply_left(G, x, y, prec), None),
                             ("left_as_transposed", lambda: P.bvmv_multiply(Gt, x, y, prec), tinfo["layout_bytes"])):
        ms, _, _ = time_flushed(fn, args.steps, args.warmup, flush, torch)
        warm = time_launches(fn, args.steps, args.warmup, torch)
        rows[name] = {"ms": ms, "edges_per_s": g.m / (ms * 1e-3), "mall_warm_ms": warm}
        if nbytes is not None:
            rows[name]["layout_bytes"] = nbytes
        log("%s: %.4f ms from HBM, %.4f ms warm" % (name, ms, warm))
    out = {"mode": "formats", "workload": wl, "n": g.n, "m": g.m, "dtype": "f32 two-sum compensated",
           "timing": "each launch after a 1 GiB device write; mall_warm_ms back to back",
           "bv_m_over_m_prime": g.m / max(info["m_prime"], 1),
           "biclique": {"bicliques": bic.nbic, "s_ids": binfo["s_ids"], "c_ids": binfo["c_ids"],
                        "residual": binfo["residual"], "words": binfo["words"],
                        "m_over_words": g.m / max(binfo["words"], 1), "mining_seconds": t_mine},
           **rows,
           "speedup_bv_vs_csr": rows["csr"]["ms"] / rows["bv"]["ms"],
           "speedup_biclique_vs_csr": rows["csr"]["ms"] / rows["biclique"]["ms"]}
    print(json.dumps(out), flush=True)


def bench_sweep(args, B, P, np, torch, dev):
    """The paper's proposed improvements of the BV method (Section "Final
    Remarks"): the reference window W (with chain bound R), and splitting
    the matrix into column blocks compressed apart.  For each setting: bits
    per edge of the stream, m / m', layout bytes, and one FP32 two-sum
    product timed from HBM (after a 1 GiB device write) and cache-warm."""
    wl = args.workload
    t0 = time.perf_counter()
    g = B.workload_graph(wl)
    log("sweep %s: n=%d m=%d (%.1fs)" % (wl, g.n, g.m, time.perf_counter() - t0))
    x = torch.from_numpy(B.uniform_x(g.n, 102, np.float32)).to(dev)
    y = torch.empty_like(x)
    prec = P.BVMV_F32_COMP
    flush = Flusher(torch, dev)
    steps, warmup = max(args.steps // 5, 20), max(args.warmup // 5, 5)

    def timed(fn):
        ms, _, _ = time_flushed(fn, steps, warmup, flush, torch)
        return ms, time_launches(fn, steps, warmup, torch)

    windows = []
    for W, R in (((1, 1), (3, 3), (7, 3), (7, 7), (15, 3), (15, 15)) if args.sweep_what != "blocks" else ()):
        enc = B.encode(g, W=W, R=R)
        G = P.bvmv_load(enc.data)
        info = G.info()
        ms, warm = timed(lambda: P.bvmv_multiply(G, x, y, prec))
        windows.append({"W": W, "R": R, "bits_per_edge": enc.data.size * 8.0 / g.m,
                        "m_over_m_prime": g.m / max(info["m_prime"], 1), "layout_bytes": info["layout_bytes"],
                        "escapes": info["escapes"], "ms": ms, "mall_warm_ms": warm,
                        "edges_per_s": g.m / (ms * 1e-3)})
        log("W=%d R=%d: %.3f bits/edge, m/m' %.3f, %.4f ms (warm %.4f)" % (
            W, R, windows[-1]["bits_per_edge"], windows[-1]["m_over_m_prime"], ms, warm))
        del G, enc
    blocks = []
    for nb in ([int(v) for v in args.sweep_blocks.split(",")] if args.sweep_what != "windows" else []):
        bounds, parts = B.column_blocks(g, nb)
        encs = [B.encode(p_) for p_ in parts]
        Gs = [P.bvmv_load(e.data) for e in encs]
        H = P.bvmv_colblocks_create(Gs)
        infos = [G_.info() for G_ in Gs]
        mp = sum(i["m_prime"] for i in infos)
        lb = sum(i["layout_bytes"] for i in infos)
        ms, warm = timed(lambda: P.bvmv_colblocks_multiply(H, x, y, prec))
        blocks.append({"blocks": nb, "bits_per_edge": sum(e.data.size for e in encs) * 8.0 / g.m,
                       "m_over_m_prime": g.m / max(mp, 1), "layout_bytes": lb,
                       "escapes": sum(i["escapes"] for i in infos), "ms": ms, "mall_warm_ms": warm,
                       "edges_per_s": g.m / (ms * 1e-3), "alg_GBs": (lb + 4 * g.n * (nb + 1)) / (ms * 1e-3) / 1e9})
        log("%d column blocks: %.3f bits/edge, m/m' %.3f, layout %.1f MB, %.4f ms (warm %.4f)" % (
            nb, blocks[-1]["bits_per_edge"], blocks[-1]["m_over_m_prime"], lb / 1e6, ms, warm))
        del H, Gs, encs, parts
    out = {"mode": "window-and-column-block-sweep", "workload": wl, "n": g.n, "m": g.m,
           "dtype": "f32 two-sum compensated", "timing": "each launch after a 1 GiB device write",
           "windows": windows, "column_blocks": blocks}
    print(json.dumps(out), flush=True)


def bench_structural_start(args, B, P, np, torch, dev):
    """The first warm-start design, kept as a control: a start vector
    predicted from structure alone.  The network (12 -> 64 -> 64 -> 1) sees
    the 8 structural inputs (the trajectory inputs 8..11 held at 0) and is
    trained on the target log(n p*) of the method's own FP64 PageRank (to
    1e-12) of the same generated graphs as the learned restarts (n
    log-uniform in [1e5, 1e6], mean degree 20, seeds 2000 + i); the start is
    p0 = exp(s) / sum exp(s), kept only if its first step's residual beats the
    uniform start's (the one-step fallback).  On the unseen n = 5e6 graph
    (seed 3000) it is run beside the uniform start and an in-degree
    proportional start (p0 = (indeg + 1) / sum, a non-learned control).
    The start vectors are formed with torch here (a bench-side control, not a
    library path); seconds are reported for PageRank alone and with the
    inputs, the network and the start."""
    rng = np.random.default_rng(2000)
    sizes = np.round(10 ** rng.uniform(5, 6, args.warm_graphs)).astype(np.int64)
    Fs, Ts = [], []
    t0 = time.perf_counter()
    for i, n in enumerate(sizes):
        g = B.web_graph(int(n), 20.0, 2000 + i)
        G = P.bvmv_load(B.encode(g).data)
        ps = torch.empty(g.n, dtype=torch.float64, device=dev)
        P.bvmv_pagerank(G, ps, tol=1e-12, max_iter=5000, prec=P.BVMV_F64)
        F = torch.zeros(g.n, P.NFEAT, device=dev)
        P.bvmv_features(G, F)
        F[:, 8:] = 0.0
        Fs.append(F)
        Ts.append(torch.log(g.n * ps).float())
        del G, g
        if i % 20 == 0:
            log("structural data: graph %d/%d (%.1fs)" % (i, len(sizes), time.perf_counter() - t0))
    F = torch.cat(Fs)
    T = torch.cat(Ts).contiguous()
    del Fs, Ts
    t_data = time.perf_counter() - t0
    m = P.bvmv_mlp_create(B.mlp_init_params(4000))
    loss = torch.empty(1, device=dev)
    gen = torch.Generator(device=dev).manual_seed(4000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for it in range(args.warm_steps):
        lr = 3e-3 * (0.5 * (1 + math.cos(math.pi * it / args.warm_steps)) + 0.01)
        idx = torch.randint(0, F.shape[0], (8192,), device=dev, generator=gen)
        P.bvmv_mlp_train_step(m, F[idx].contiguous(), T[idx].contiguous(), lr, loss)
        if it % max(1, args.warm_steps // 10) == 0 or it == args.warm_steps - 1:
            losses.append(float(loss.item()))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log("structural training: %d steps in %.2fs, loss %s" % (args.warm_steps, t_train, ["%.4f" % v for v in losses]))
    del F, T
    g = B.web_graph(args.warm_test_n, 20.0, 3000)
    G = P.bvmv_load(B.encode(g).data)
    n = g.n
    p = torch.empty(n, device=dev)

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t

    def learned_start():
        Ft = torch.zeros(n, P.NFEAT, device=dev)
        P.bvmv_features(G, Ft)
        Ft[:, 8:] = 0.0
        sv = torch.empty(n, device=dev)
        P.bvmv_mlp_forward(m, Ft, sv)
        return torch.softmax(sv, 0)

    P.bvmv_pagerank(G, p)  # graph capture
    p0_learned, t_start = timed(learned_start)
    indeg = torch.from_numpy(np.bincount(g.col.astype(np.int64), minlength=n).astype(np.float32)).to(dev)
    p0_degree = (indeg + 1.0) / float((indeg + 1.0).sum())
    runs = {}
    for name, start in (("uniform", None), ("structural_learned", p0_learned), ("indegree", p0_degree)):
        ts = []
        for _ in range(3):
            (r,), t = timed(lambda: P.bvmv_pagerank_detail(G, p, start=start, fallback_check=1 if start is not None
                                                             else 0))
            ts.append(t)
        runs[name] = dict(iters=r["iters"], used_start=r["used_start"], converged=bool(r["converged"]),
                          seconds=float(np.median(ts)))
        log("structural start %s: %s" % (name, runs[name]))
    runs["structural_learned"]["seconds_with_start"] = runs["structural_learned"]["seconds"] + t_start
    out = {"mode": "structural-start-control", "train_graphs": len(sizes), "train_nodes": int(sizes.sum()),
           "train_steps": args.warm_steps, "train_seconds": t_train, "data_seconds": t_data, "loss_trace": losses,
           "test_n": n, "test_m": g.m, "dtype": "f32 two-sum compensated", "start_seconds": t_start, **runs}
    print(json.dumps(out), flush=True)


def ragged_encs(B, np):
    """The 48 ragged web-like graphs: n_g = round(10^(4 + 2 u_g)), u_g uniform
    from seed 999, mean out-degree 20, graph seeds 1000 + g (bitstreams)."""
    rng = np.random.default_rng(999)
    sizes = np.round(10 ** (4 + 2 * rng.random(48))).astype(np.int64)
    t0 = time.perf_counter()
    encs = [B.encode(B.web_graph(int(n), 20.0, 1000 + i)).data for i, n in enumerate(sizes)]
    log("ragged: %d graphs, n in [%d, %d], sum n %d (%.1fs)" % (len(sizes), sizes.min(), sizes.max(), sizes.sum(),
                                                                 time.perf_counter() - t0))
    return sizes, encs


def bench_ragged(args, B, P, np, torch, dev):
    """Ragged batch: 48 web-like graphs, n_g = round(10^(4 + 2 u_g)) with u_g
    uniform from seed 999, mean out-degree 20, graph seeds 1000 + g.  Global
    PageRank (beta 0.85, uniform teleport, L1 1e-6) of every graph, timed as
    48 separate calls and as one group (one launch sequence for all members),
    each with the fixed default layout and with autotuned layouts; plus one
    product over the whole group.  Median of 3 after a warm-up call."""
    sizes, encs = ragged_encs(B, np)
    t0 = time.perf_counter()
    fixed = [P.bvmv_load(e) for e in encs]
    t_fixed = time.perf_counter() - t0
    t0 = time.perf_counter()
    auto = [P.bvmv_load(e, autotune=1) for e in encs]
    t_auto = time.perf_counter() - t0
    picks = {}
    for G in auto:
        info = P.bvmv_get_info(G)
        key = "%dx%d" % (info["tile_rows"], info["window_cap"])
        picks[key] = picks.get(key, 0) + 1
    log("load: fixed %.2fs, autotuned %.2fs, picks %s" % (t_fixed, t_auto, picks))
    m_total = sum(P.bvmv_get_info(G)["m"] for G in fixed)

    def timed(fn, reps=3):
        fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return r, float(np.median(ts))

    outs = [torch.empty(int(n), device=dev) for n in sizes]

    def solo(Gs):
        return [P.bvmv_pagerank_detail(G, o)[0] for G, o in zip(Gs, outs)]

    res = {}
    for name, Gs in (("fixed", fixed), ("autotuned", auto)):
        r, t = timed(lambda: solo(Gs))
        res["solo_" + name] = {"seconds": t, "max_iters": max(x["iters"] for x in r),
                               "converged": all(x["converged"] for x in r)}
        grp = P.bvmv_group(Gs)
        pg = torch.empty(int(sizes.sum()), device=dev)
        r, t = timed(lambda: P.bvmv_pagerank_detail(grp, pg))
        offs = P.bvmv_group_offsets(grp)
        solo(Gs)
        diff = max(float((pg[offs[i]:offs[i + 1]] - outs[i]).abs().max()) for i in range(len(Gs)))
        x = torch.rand(int(sizes.sum()), device=dev, generator=torch.Generator(device=dev).manual_seed(5))
        y = torch.empty_like(x)
        ms = time_launches(lambda: P.bvmv_multiply(grp, x, y), 50, 5, torch)
        res["group_" + name] = {"seconds": t, "max_iters": max(x_["iters"] for x_ in r),
                                "converged": all(x_["converged"] for x_ in r), "max_abs_diff_vs_solo": diff,
                                "product_ms": ms, "product_edges_per_s": m_total / (ms * 1e-3)}
        log("%s: solo %.4fs, group %.4fs (diff %.2e), group product %.4f ms"
            % (name, res["solo_" + name]["seconds"], t, diff, ms))
    out = {"mode": "ragged-batch", "graphs": len(sizes), "sum_n": int(sizes.sum()), "sum_m": int(m_total),
           "n_min": int(sizes.min()), "n_max": int(sizes.max()), "dtype": "f32 two-sum compensated",
           "load_seconds_fixed": t_fixed, "load_seconds_autotuned": t_auto, "autotune_picks": picks, **res,
           "speedup_group_vs_solo_fixed": res["solo_fixed"]["seconds"] / res["group_fixed"]["seconds"],
           "speedup_group_autotuned_vs_solo_fixed": res["solo_fixed"]["seconds"] / res["group_autotuned"]["seconds"]}
    print(json.dumps(out), flush=True)


def bench_warm(args, B, P, np, torch, dev):
    """Learned warm restarts: restart samples (the 12 inputs after K = 10 plain
    iterations from the uniform vector, and the target n (p* - p_K) / delta
    from the method's own FP64 PageRank) of generated web-like graphs (n
    log-uniform in [1e5, 1e6], mean degree 20, graph seeds 2000 + i), the
    network trained on the device (Adam, batches of 8192 nodes, network seed
    4000, cosine learning rate), then PageRank of an unseen graph (seed 3000)
    to L1 1e-6: plain, with learned restarts (every 10 iterations, at most 2),
    and with a zero network (every restart accepted and the identity: the
    restart overhead alone).  Each PageRank is timed end to end, median of 3;
    the learned run's first call, which also computes the structural inputs
    once for the graph, is reported apart.  The same three runs then cover the
    ragged group of 48 graphs (one launch sequence for all members)."""
    K = 10
    rng = np.random.default_rng(2000)
    sizes = np.round(10 ** rng.uniform(5, 6, args.warm_graphs)).astype(np.int64)
    Fs, Ts = [], []
    t0 = time.perf_counter()
    for i, n in enumerate(sizes):
        g = B.web_graph(int(n), 20.0, 2000 + i)
        G = P.bvmv_load(B.encode(g).data)
        ps = torch.empty(g.n, dtype=torch.float64, device=dev)
        P.bvmv_pagerank(G, ps, tol=1e-12, max_iter=5000, prec=P.BVMV_F64)
        F = torch.empty(g.n, P.NFEAT, device=dev)
        T = torch.empty(g.n, device=dev)
        P.bvmv_restart_sample(G, K, F, T, ps.float())
        Fs.append(F)
        Ts.append(T)
        del G, g
        if i % 20 == 0:
            log("training data: graph %d/%d (%.1fs)" % (i, len(sizes), time.perf_counter() - t0))
    F = torch.cat(Fs)
    T = torch.cat(Ts).contiguous()
    del Fs, Ts
    t_data = time.perf_counter() - t0
    log("training data: %d graphs, %d nodes (%.1fs)" % (len(sizes), F.shape[0], t_data))
    m = P.bvmv_mlp_create(B.mlp_init_params(4000))
    loss = torch.empty(1, device=dev)
    gen = torch.Generator(device=dev).manual_seed(4000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for it in range(args.warm_steps):
        lr = 3e-3 * (0.5 * (1 + math.cos(math.pi * it / args.warm_steps)) + 0.01)
        idx = torch.randint(0, F.shape[0], (8192,), device=dev, generator=gen)
        P.bvmv_mlp_train_step(m, F[idx].contiguous(), T[idx].contiguous(), lr, loss)
        if it % max(1, args.warm_steps // 10) == 0 or it == args.warm_steps - 1:
            losses.append(float(loss.item()))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log("training: %d steps in %.2fs, loss %s" % (args.warm_steps, t_train, ["%.4f" % v for v in losses]))
    del F, T
    g = B.web_graph(args.warm_test_n, 20.0, 3000)
    G = P.bvmv_load(B.encode(g).data)
    n = g.n
    p = torch.empty(n, device=dev)
    zero = P.bvmv_mlp_create(np.zeros(P.MLP_PARAMS, dtype=np.float32))

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t

    P.bvmv_pagerank(G, p)  # graph capture
    (rf,), s_first = timed(lambda: P.bvmv_pagerank_detail(G, p, mlp=m))
    runs = {}
    for name, kw in (("plain", {}), ("learned", {"mlp": m}), ("zero_network", {"mlp": zero})):
        ts = []
        for _ in range(3):
            (r,), t = timed(lambda: P.bvmv_pagerank_detail(G, p, **kw))
            ts.append(t)
        runs[name] = dict(iters=r["iters"], products=r["products"], accepted=r["restarts_accepted"],
                          rejected=r["restarts_rejected"], converged=bool(r["converged"]),
                          seconds=float(np.median(ts)))
        log("pagerank n=%d %s: %s" % (n, name, runs[name]))
    # the same network on the ragged group of 48 graphs (one launch sequence)
    _, encs = ragged_encs(B, np)
    members = [P.bvmv_load(e) for e in encs]
    grp = P.bvmv_group(members)
    pg = torch.empty(grp.n, device=dev)
    P.bvmv_pagerank(grp, pg)  # graph capture
    timed(lambda: P.bvmv_pagerank_detail(grp, pg, mlp=m))  # structural inputs, once
    group = {}
    for name, kw in (("plain", {}), ("learned", {"mlp": m}), ("zero_network", {"mlp": zero})):
        ts = []
        for _ in range(3):
            rs, t = timed(lambda: P.bvmv_pagerank_detail(grp, pg, **kw))
            ts.append(t)
        group[name] = dict(max_iters=max(r["iters"] for r in rs), products=sum(r["products"] for r in rs),
                           members_accepting=sum(1 for r in rs if r["restarts_accepted"] > 0),
                           members_rejecting=sum(1 for r in rs if r["restarts_rejected"] > 0),
                           converged=all(r["converged"] for r in rs), seconds=float(np.median(ts)))
        log("pagerank ragged group (%d graphs, n=%d) %s: %s" % (len(members), grp.n, name, group[name]))
    group["speedup_learned_vs_plain"] = group["plain"]["seconds"] / group["learned"]["seconds"]
    out = {"mode": "learned-warm-restart", "train_graphs": len(sizes), "train_nodes": int(sizes.sum()),
           "restart_every": K, "train_steps": args.warm_steps, "train_seconds": t_train, "data_seconds": t_data,
           "loss_trace": losses, "test_n": n, "test_m": g.m, "dtype": "f32 two-sum compensated",
           "first_learned_call_seconds": s_first, **runs,
           "speedup_learned_vs_plain": runs["plain"]["seconds"] / runs["learned"]["seconds"],
           "product_ratio_learned_vs_plain": runs["learned"]["products"] / runs["plain"]["products"],
           "ragged_group": {"graphs": len(members), "n": grp.n, **group}}
    print(json.dumps(out), flush=True)


def build_parser():
    """The command line of bench.py (the profiles quote commands in it)."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="web-n2p20-d20")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-pagerank", action="store_true")
    ap.add_argument("--pr-runs", type=int, default=20, help="timed PageRank runs (the median is reported)")
    ap.add_argument("--pagerank-sizes", default="", metavar="N1,N2,...",
                    help="only PageRank (median of --pr-runs whole runs) of --workload's recipe at each size n, "
                         "compressed and CSR; BVMV_PR_FUSED=0/1 forces the finish-kernel or the fused form")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--only", choices=["bv", "csr", "all"], default="all",
                    help="restrict the timed kernels (profiling runs)")
    ap.add_argument("--timing", choices=["both", "flushed", "warm"], default="both",
                    help="time launches from HBM (after a 1 GiB write), back to back, or both (profiling runs "
                         "take one, so that the profiler's per-kernel average is that figure)")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--window-cap", type=int, default=0)
    ap.add_argument("--stage-bytes", type=int, default=0)
    ap.add_argument("--interval-mode", type=int, default=0)
    ap.add_argument("--batch", type=int, default=0, metavar="K",
                    help="batched personalized PageRank with K teleport sets of 16 seeds (workload "
                         "web-n8e6-d25 unless --workload is given) instead of the single-vector metric")
    ap.add_argument("--warm-start", action="store_true",
                    help="learned warm restarts: train the network on generated graphs, then PageRank of an "
                         "unseen graph with restarts against the plain method")
    ap.add_argument("--social", action="store_true",
                    help="social-like workload (n = 4e6): FP32 error against the FP64 oracle, compressed vs CSR")
    ap.add_argument("--ragged", action="store_true",
                    help="ragged batch of 48 graphs: solo against grouped PageRank, fixed against autotuned layouts")
    ap.add_argument("--formats", action="store_true",
                    help="one product of --workload in three formats: BV compressed, mined bicliques, CSR "
                         "(flushed and cache-warm)")
    ap.add_argument("--sweep", action="store_true",
                    help="reference window W (and chain bound R) sweep and column-block splitting of --workload")
    ap.add_argument("--sweep-what", choices=["both", "windows", "blocks"], default="both")
    ap.add_argument("--sweep-blocks", default="1,2,4,8", help="column-block counts of --sweep")
    ap.add_argument("--structural-start", action="store_true",
                    help="control: a start vector predicted from structure alone (the first warm-start design) "
                         "against the uniform and an in-degree start")
    ap.add_argument("--warm-graphs", type=int, default=200)
    ap.add_argument("--warm-steps", type=int, default=3000)
    ap.add_argument("--warm-test-n", type=int, default=5_000_000)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run torch copies of MIB MiB (the calibration kernel for HBM byte counters)")
    return ap


def main():
    args = build_parser().parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the compressed product and PageRank here are single-GPU "
              "kernels; independent graphs or right-hand sides would go one set per GPU", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    if args.copy_probe:
        # a plain device copy of known size: FETCH_SIZE / WRITE_SIZE of this
        # kernel calibrate the counters read on the product kernels
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n, "launches": args.steps}), flush=True)
        return

    import bvinputs as B
    import paper_1708_07271_amd as P

    if args.pagerank_sizes:
        return bench_pr_sizes(args, B, P, np, torch, dev)
    if args.batch:
        return bench_batch(args, B, P, np, torch, dev)
    if args.warm_start:
        return bench_warm(args, B, P, np, torch, dev)
    if args.structural_start:
        return bench_structural_start(args, B, P, np, torch, dev)
    if args.ragged:
        return bench_ragged(args, B, P, np, torch, dev)
    if args.social:
        return bench_social(args, B, P, np, torch, dev)
    if args.formats:
        return bench_formats(args, B, P, np, torch, dev)
    if args.sweep:
        return bench_sweep(args, B, P, np, torch, dev)
    t0 = time.perf_counter()
    g = B.workload_graph(args.workload)
    enc = B.encode(g)
    log("graph n=%d m=%d bitstream %.1f MB (%.2f bits/edge) in %.1fs" % (
        g.n, g.m, enc.data.size / 1e6, enc.data.size * 8 / g.m, time.perf_counter() - t0))
    G = P.bvmv_load(enc.data, keep_lists=1, tile_rows=args.tile_rows, window_cap=args.window_cap,
                    stage_bytes=args.stage_bytes, interval_mode=args.interval_mode)
    info = G.info()
    C = P.bvmv_csr_create(G)
    log("layout %.1f MB, units %d, m' %d, escapes %d, long rows %d; csr %.1f MB" % (
        info["layout_bytes"] / 1e6, info["units"], info["m_prime"], info["escapes"], info["long_rows"],
        C.bytes() / 1e6))
    x32 = B.uniform_x(g.n, 102, np.float32)
    x = torch.from_numpy(x32).to(dev)
    y = torch.empty_like(x)
    y2 = torch.empty_like(x)
    prec = P.BVMV_F32_COMP

    flush = Flusher(torch, dev)
    ms_bv = ms_csr = warm_bv = warm_csr = ms_flush = None
    per_launch = {}

    def both(fn, name):
        ms = fl = warm = None
        if args.timing in ("both", "flushed"):
            ms, fl, per_launch[name] = time_flushed(fn, args.steps, args.warmup, flush, torch)
        if args.timing in ("both", "warm"):
            warm = time_launches(fn, args.steps, args.warmup, torch)
        return ms if ms is not None else warm, fl, warm if warm is not None else ms

    if args.only in ("bv", "all"):
        ms_bv, ms_flush, warm_bv = both(lambda: P.bvmv_multiply(G, x, y, prec), "bv")
        log("compressed product: %.4f ms from HBM (flush %s ms), %.4f ms cache-warm" % (ms_bv, ms_flush, warm_bv))
    if args.only in ("csr", "all"):
        ms_csr, ms_flush, warm_csr = both(lambda: P.bvmv_csr_multiply(C, x, y2, prec), "csr")
        log("csr product: %.4f ms from HBM, %.4f ms cache-warm" % (ms_csr, warm_csr))
    # the same bytes as the compressed product's (layout + x + y) moved by a
    # plain device copy, timed the same way: what HBM delivers at this size
    copy_floor = None
    if args.only in ("bv", "all") and args.timing != "warm":
        nfl = (info["layout_bytes"] + 8 * g.n) // 8
        ca = torch.ones(nfl, dtype=torch.float32, device=dev)
        cb = torch.empty_like(ca)
        ms_c, _, _ = time_flushed(lambda: cb.copy_(ca), args.steps, args.warmup, flush, torch)
        warm_c = time_launches(lambda: cb.copy_(ca), args.steps, args.warmup, torch)
        copy_floor = {"bytes_moved": 8 * nfl, "ms": ms_c, "GBps": 8 * nfl / (ms_c * 1e-3) / 1e9,
                      "mall_warm_ms": warm_c, "product_over_copy": ms_bv / ms_c}
        log("device copy of the same bytes: %.4f ms from HBM (%.0f GB/s), %.4f ms cache-warm; product / copy %.2f"
            % (ms_c, copy_floor["GBps"], warm_c, ms_bv / ms_c))
        # the same product and copy after a read flush instead (reported beside
        # the headline, which keeps the write flush)
        rflush = ReadFlusher(torch, dev)
        ms_rb, ms_rf, _ = time_flushed(lambda: P.bvmv_multiply(G, x, y, prec), args.steps, args.warmup, rflush, torch)
        ms_rc, _, _ = time_flushed(lambda: cb.copy_(ca), args.steps, args.warmup, rflush, torch)
        copy_floor["read_flush"] = {
            "product_ms": ms_rb, "copy_ms": ms_rc, "flush_ms": ms_rf, "product_over_copy": ms_rb / ms_rc,
            "achieved_GBs": (info["layout_bytes"] + 8 * g.n) / (ms_rb * 1e-3) / 1e9,
            "note": "each launch after a 1 GiB read instead of a 1 GiB write: the caches hold clean lines, so the "
                    "launch does not pay for writing back the flush's dirty lines"}
        log("after a read flush: product %.4f ms, copy %.4f ms (flush %.3f ms)" % (ms_rb, ms_rc, ms_rf))
        del rflush
        del ca, cb
    del flush
    if ms_bv is None:
        ms_bv, warm_bv = ms_csr, warm_csr

    pr = None
    if not args.no_pagerank and args.only == "all":
        p = torch.empty(g.n, dtype=torch.float32, device=dev)

        # each run from the uniform start
        ((it, ok, r),), pr_s, pr_min = pr_median(lambda: P.bvmv_pagerank(G, p, prec=prec), args.pr_runs, torch)
        (it_c, ok_c, r_c), pr_csr_s, pr_csr_min = pr_median(lambda: P.bvmv_csr_pagerank(C, p, prec=prec),
                                                            args.pr_runs, torch)
        pr = {"seconds_to_1e-6": pr_s, "iterations": it, "converged": ok, "residual": r,
              "csr_seconds_to_1e-6": pr_csr_s, "csr_iterations": it_c, "speedup_vs_csr": pr_csr_s / pr_s,
              "runs": args.pr_runs, "statistic": "median of whole runs (min %.6f s, csr min %.6f s)" % (
                  pr_min, pr_csr_min)}
        log("pagerank: %.4f s (%d it, median of %d runs) vs csr %.4f s (%d it)" % (pr_s, it, args.pr_runs,
                                                                                   pr_csr_s, it_c))

    alg_bytes = info["layout_bytes"] + 4 * g.n + 4 * g.n     # layout + read x once + write y once
    achieved = alg_bytes / (ms_bv * 1e-3) / 1e9
    csr_bytes = C.bytes() + 8 * g.n
    result = {
        "metric": "uncompressed edges/s: compressed A·x vs CSR SpMV; PageRank s to L1 1e-6",
        "value": g.m / (ms_bv * 1e-3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_bv,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "precision": "f32 two-sum compensated",
                   "x": "uniform[0,1) float32, seed 102",
                   "timing": ("each launch after a 1 GiB device write (L2 and MALL flushed): inputs read from HBM; "
                              "mean of (flush + launch) less mean of flush alone, HIP events on the library's "
                              "stream" if args.timing != "warm" else "back-to-back launches (cache-warm)"),
                   "per_launch_event_ms": per_launch.get("bv")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": load_traffic("bv_wave_kernel", args.workload),
                     "kernel": "bv_wave_kernel", "alg_bytes_per_launch": alg_bytes,
                     "caches": "flushed" if args.timing != "warm" else "warm"},
        "copy_same_bytes": copy_floor,
        "mall_warm": {"ms": warm_bv, "edges_per_s": g.m / (warm_bv * 1e-3),
                      "achieved_GBs": alg_bytes / (warm_bv * 1e-3) / 1e9,
                      "frac": alg_bytes / (warm_bv * 1e-3) / 1e9 / PEAK_HBM_GBS,
                      "note": "back-to-back launches; the working set stays in the 256 MB MALL"},
        "layout": {"bytes": info["layout_bytes"], "bytes_per_edge": info["layout_bytes"] / g.m,
                   "m_prime": info["m_prime"], "m_over_m_prime": g.m / max(info["m_prime"], 1),
                   "units": info["units"], "escapes": info["escapes"], "long_rows": info["long_rows"],
                   "singles": info["n_singles"], "wide": info["n_wide"], "interval_pairs": info["n_intervals"],
                   "tiles": info["ntiles"], "bitstream_bits_per_edge": enc.data.size * 8 / g.m},
    }
    if ms_csr is not None:
        result["csr"] = {"edges_per_s": g.m / (ms_csr * 1e-3), "ms": ms_csr, "bytes": csr_bytes,
                         "achieved_GBs": csr_bytes / (ms_csr * 1e-3) / 1e9,
                         "speedup_compressed_vs_csr": ms_csr / ms_bv,
                         "mall_warm_ms": warm_csr, "mall_warm_edges_per_s": g.m / (warm_csr * 1e-3)}
    if pr is not None:
        result["pagerank"] = pr
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(g, x32.astype(np.float64), args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
