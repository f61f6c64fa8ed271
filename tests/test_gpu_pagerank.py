"""GPU parity of PageRank (power method, Eq. (1) of the paper) against the
CPU oracle: closed forms, iteration-matched oracle runs, degenerate cases,
personalized teleport, warm start, groups (ragged batch) and the CSR path.

The loaded rows are in-link lists; dangling mass goes to the teleport vector;
the stopping test is ||p_t - p_{t-1}||_1 < tol accumulated in double."""
import numpy as np
import pytest

import bvinputs as B
from oracle import pagerank
from tests import tolerances as TOL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1708_07271_amd as mod
    mod.load_library()
    return mod


def _rel(a, b):
    """Largest per-entry relative error of a against the oracle's b; entries
    where b is 0 must be exactly 0."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.abs(a - b)
    z = b == 0
    assert np.all(d[z] == 0), "nonzero result where the oracle gives 0"
    return float(np.max(d[~z] / np.abs(b[~z]))) if np.any(~z) else 0.0


def _pers(p, p_ref, prec_name):
    """Per-entry check of a personalized PageRank vector: relative tol plus
    the floor of tolerances.py (a few roundings of the largest entry)."""
    tol = TOL.F64 if prec_name == "f64" else TOL.F32C
    ratio, rel_big = TOL.within(p, p_ref, tol, TOL.FLOOR[prec_name])
    print("personalized %s: ratio %.3g, relative error on entries above the floor %.3g" % (prec_name, ratio, rel_big),
          flush=True)
    return ratio <= 1.0 and rel_big < tol


def _in_links(g):
    return g.transpose()


def _pr(P, G, n, prec, **kw):
    dt = torch.float64 if prec == P.BVMV_F64 else torch.float32
    p = torch.empty(n, dtype=dt, device=DEV)
    for key in ("teleport", "start"):
        if key in kw and kw[key] is not None:
            kw[key] = torch.from_numpy(np.ascontiguousarray(kw[key]).astype(np.float64 if dt == torch.float64
                                                                              else np.float32)).to(DEV)
    res = P.bvmv_pagerank(G, p, prec=prec, **kw)
    torch.cuda.synchronize()
    return p.cpu().numpy().astype(np.float64), res


def test_closed_forms(P):
    beta = 0.85
    n = 17
    cases = [(B.complete_graph(n), None), (B.cycle_graph(n), None)]
    for kind, pc in (("both", ((1 - beta) / n + beta) / (1 + beta)),
                     ("in", (1 + (n - 1) * beta) / (n + (n - 1) * beta)),
                     ("out", 1.0 / (n + beta))):
        cases.append((B.star_graph(n, 0, kind), pc))
    for ci, (g, pc) in enumerate(cases):
        bt = _in_links(g)
        G = P.bvmv_load(B.encode(bt).data)
        # tol 1e-13: the L1 contraction bound puts p within 0.85/0.15 * 1e-13 of the fixed point
        p, ((it, ok, r),) = _pr(P, G, n, P.BVMV_F64, tol=1e-13, max_iter=1000)
        print("case", ci, it, ok, r, flush=True)
        assert ok
        if pc is None:
            assert np.max(np.abs(p - 1.0 / n)) < 1e-14
        else:
            assert abs(p[0] - pc) < 1e-12
            assert np.max(np.abs(p[1:] - (1 - pc) / (n - 1))) < 1e-12


@pytest.mark.parametrize("prec_name,tol", [("f64", TOL.F64), ("f32c", TOL.F32C), ("f32", TOL.F32_NAIVE)])
def test_iteration_matched(P, prec_name, tol):
    prec = P.PREC_NAMES[prec_name]
    g = B.web_graph(40_000, 15.0, 77)          # rows read as in-link lists, as loaded
    G = P.bvmv_load(B.encode(g).data)
    p, ((it, ok, r),) = _pr(P, G, g.n, prec)
    assert ok and r < 1e-6
    _, t_or, _, ok_or = pagerank.pagerank(g.rowptr, g.col, 0.85, tol=1e-6)
    assert ok_or and abs(it - t_or) <= 1
    p_ref = pagerank.pagerank(g.rowptr, g.col, 0.85, iters=it)[0]
    assert _rel(p, p_ref) < tol
    assert abs(p.sum() - 1.0) < (1e-12 if prec == P.BVMV_F64 else 1e-5)


def test_personalized_start_and_limits(P):
    g = B.web_graph(20_000, 12.0, 78)
    G = P.bvmv_load(B.encode(g).data)
    v = np.zeros(g.n)
    seeds = np.random.default_rng(1).choice(g.n, 16, replace=False)
    v[seeds] = 1.0 / 16
    p, ((it, ok, r),) = _pr(P, G, g.n, P.BVMV_F64, teleport=v)
    p_ref = pagerank.pagerank(g.rowptr, g.col, 0.85, teleport=v, iters=it)[0]
    assert ok and _pers(p, p_ref, "f64")
    # warm start from the converged vector: stops almost at once
    p2, ((it2, ok2, r2),) = _pr(P, G, g.n, P.BVMV_F64, teleport=v, start=p)
    assert ok2 and it2 <= 2
    # iteration limit: NOT_CONVERGED status, outputs still written
    p3, ((it3, ok3, r3),) = _pr(P, G, g.n, P.BVMV_F64, teleport=v, max_iter=3)
    assert not ok3 and it3 == 3
    assert _pers(p3, pagerank.pagerank(g.rowptr, g.col, 0.85, teleport=v, iters=3)[0], "f64")
    # beta = 0: p = v
    p4, _ = _pr(P, G, g.n, P.BVMV_F64, teleport=v, damping=0.0)
    assert np.max(np.abs(p4 - v)) < 1e-16


@pytest.mark.parametrize("prec_name", ["f64", "f32c"])
def test_fallback_check_keeps_better_start(P, prec_name):
    """fallback_check: one probe iteration from `start` and one from the
    teleport vector; `start` is kept only if its residual is the smaller.  A
    start near the fixed point is kept (and converges at once); a start with
    all mass on one node is rejected, and the run is then the plain run from
    the teleport vector, bit for bit, probes not counted."""
    prec = P.PREC_NAMES[prec_name]
    dt = torch.float64 if prec == P.BVMV_F64 else torch.float32
    g = B.web_graph(20_000, 12.0, 83)
    G = P.bvmv_load(B.encode(g).data)
    plain = torch.empty(g.n, dtype=dt, device=DEV)
    (rp,) = P.bvmv_pagerank_detail(G, plain, prec=prec)
    good = plain.clone()
    out = torch.empty_like(plain)
    (rg,) = P.bvmv_pagerank_detail(G, out, start=good, prec=prec, fallback_check=1)
    torch.cuda.synchronize()
    assert rg["used_start"] == 1 and rg["converged"] and rg["iters"] <= 2
    bad = torch.zeros_like(plain)
    bad[0] = 1.0
    (rb,) = P.bvmv_pagerank_detail(G, out, start=bad, prec=prec, fallback_check=1)
    torch.cuda.synchronize()
    assert rb["used_start"] == 0 and rb["iters"] == rp["iters"] and rb["products"] == rp["products"]
    assert torch.equal(out, plain)
    # without the check the bad start is used as given
    (rn,) = P.bvmv_pagerank_detail(G, out, start=bad, prec=prec)
    assert rn["used_start"] == 1


def _pr_k(P, G, n, k, prec, V=None, start=None, **kw):
    """k personalized PageRanks at once.  V, start and the result are (n, k)
    host arrays; on the device each right-hand side is one contiguous
    vector (column-major n x k)."""
    dt = torch.float64 if prec == P.BVMV_F64 else torch.float32
    nd = np.float64 if dt == torch.float64 else np.float32
    p = torch.empty(n * k, dtype=dt, device=DEV)
    tv = torch.from_numpy(np.ascontiguousarray(V.T, dtype=nd).reshape(-1)).to(DEV) if V is not None else None
    sv = torch.from_numpy(np.ascontiguousarray(start.T, dtype=nd).reshape(-1)).to(DEV) if start is not None else None
    res = P.bvmv_pagerank(G, p, teleport=tv, start=sv, prec=prec, k=k, **kw)
    torch.cuda.synchronize()
    return p.cpu().numpy().astype(np.float64).reshape(k, n).T, res


@pytest.mark.parametrize("prec_name,tol", [("f64", TOL.F64), ("f32c", TOL.F32C)])
def test_batched_personalized(P, prec_name, tol):
    """k teleport sets in one launch sequence: each column is the oracle's
    personalized PageRank (iteration-matched), columns stop independently."""
    prec = P.PREC_NAMES[prec_name]
    g = B.web_graph(30_000, 15.0, 81)
    G = P.bvmv_load(B.encode(g).data)
    k = 6
    V = B.teleport_sets(g.n, k, 16, seed=7).astype(np.float64)
    p, res = _pr_k(P, G, g.n, k, prec, V)
    assert len(res) == k
    iters = set()
    for c in range(k):
        it, ok, r = res[c]
        assert ok and r < 1e-6
        _, t_or, _, ok_or = pagerank.pagerank(g.rowptr, g.col, 0.85, teleport=V[:, c], tol=1e-6)
        assert ok_or and abs(it - t_or) <= 1
        p_ref = pagerank.pagerank(g.rowptr, g.col, 0.85, teleport=V[:, c], iters=it)[0]
        assert _pers(p[:, c], p_ref, prec_name), c
        assert abs(p[:, c].sum() - 1.0) < (1e-12 if prec == P.BVMV_F64 else 1e-5)
        iters.add(it)
    # deterministic
    p2, res2 = _pr_k(P, G, g.n, k, prec, V)
    assert np.array_equal(p, p2) and res == res2


def test_batched_uniform_and_limits(P):
    """Uniform teleport in every column equals the single-vector run; an
    iteration limit stops every column at max_iter with NOT_CONVERGED."""
    g = B.web_graph(20_000, 12.0, 82)
    G = P.bvmv_load(B.encode(g).data)
    k = 3
    p, res = _pr_k(P, G, g.n, k, P.BVMV_F64)
    p1, ((it1, ok1, r1),) = _pr(P, G, g.n, P.BVMV_F64)
    for c in range(k):
        assert abs(res[c][0] - it1) <= 1 and res[c][1]
        ref = pagerank.pagerank(g.rowptr, g.col, 0.85, iters=res[c][0])[0]
        assert _rel(p[:, c], ref) < TOL.F64
    V = B.teleport_sets(g.n, k, 16, seed=9).astype(np.float64)
    p3, res3 = _pr_k(P, G, g.n, k, P.BVMV_F64, V, max_iter=4)
    for c in range(k):
        assert res3[c][0] == 4 and not res3[c][1]
        ref = pagerank.pagerank(g.rowptr, g.col, 0.85, teleport=V[:, c], iters=4)[0]
        assert _pers(p3[:, c], ref, "f64")
    # warm start from the converged columns: done almost at once
    p4, _ = _pr_k(P, G, g.n, k, P.BVMV_F64, V)
    p5, res5 = _pr_k(P, G, g.n, k, P.BVMV_F64, V, start=p4)
    assert all(r[0] <= 2 and r[1] for r in res5)


def test_batched_64_columns_equal_single_runs(P):
    """The largest batch (k = 64, one column per lane of the epilogue's
    state): every column is bit-identical to the single-vector run with its
    teleport vector, with the same iteration count, although the columns stop
    at different iterations."""
    g = B.web_graph(12_000, 10.0, 85)
    G = P.bvmv_load(B.encode(g).data)
    k = 64
    V = B.teleport_sets(g.n, k, 16, seed=11).astype(np.float32)
    p, res = _pr_k(P, G, g.n, k, P.BVMV_F32_COMP, V)
    assert len({r[0] for r in res}) > 1
    for c in range(0, k, 9):
        print("column", c, flush=True)
        pc, ((it, ok, r),) = _pr(P, G, g.n, P.BVMV_F32_COMP, teleport=V[:, c].astype(np.float64))
        assert ok and res[c][1] and res[c][0] == it
        assert np.array_equal(p[:, c], pc)


def test_edgeless_and_determinism(P):
    G = P.bvmv_load(B.encode(B.empty_graph(500)).data)
    p, ((it, ok, r),) = _pr(P, G, 500, P.BVMV_F32_COMP)
    assert ok and it == 1 and np.allclose(p, 1 / 500, rtol=1e-6)
    g = B.web_graph(30_000, 15.0, 79)
    G = P.bvmv_load(B.encode(g).data)
    a, ra = _pr(P, G, g.n, P.BVMV_F32_COMP)
    b, rb = _pr(P, G, g.n, P.BVMV_F32_COMP)
    assert ra == rb and np.array_equal(a, b)



def test_fused_iteration_own_fold(P, monkeypatch):
    """Iterations without a finish kernel: the first block of each member
    publishes the dangling mass; a wave that does not see it in time folds the
    same partials itself.  Forcing every wave to fold itself
    (BVMV_FOLD_POLLS=-1), or to fold whenever its first read finds nothing
    (0), must give the same iterates bit for bit, for a single graph in both
    precisions and the CSR baseline.  (Groups keep a finish kernel per
    iteration; test_group_equals_solo checks that both forms agree bit for
    bit.)"""
    g = B.web_graph(40_000, 14.0, 91)
    G = P.bvmv_load(B.encode(g).data, keep_lists=1)
    C = P.bvmv_csr_create(G)

    def runs():
        out = []
        for prec in (P.BVMV_F64, P.BVMV_F32_COMP):
            out.append(_pr(P, G, g.n, prec))
        p = torch.empty(g.n, dtype=torch.float32, device=DEV)
        res = P.bvmv_csr_pagerank(C, p)
        torch.cuda.synchronize()
        out.append((p.cpu().numpy().astype(np.float64), res))
        return out

    base = runs()
    for polls in ("-1", "0"):
        monkeypatch.setenv("BVMV_FOLD_POLLS", polls)
        other = runs()
        for (a, ra), (b, rb) in zip(base, other):
            assert ra == rb, polls
            assert np.array_equal(a, b), polls
    monkeypatch.delenv("BVMV_FOLD_POLLS")
    p_ref = pagerank.pagerank(g.rowptr, g.col, 0.85, iters=base[1][1][0][0])[0]
    assert _rel(base[1][0], p_ref) < TOL.F32C

def test_fused_and_finish_forms_identical(P, monkeypatch):
    """The fold inside the next launch (BVMV_PR_FUSED=1, also for a group)
    and a finish kernel between launches (BVMV_PR_FUSED=0) give the same
    iterates bit for bit: a single graph in both precisions, a group and the
    CSR baseline."""
    g = B.web_graph(40_000, 14.0, 97)
    G = P.bvmv_load(B.encode(g).data, keep_lists=1)
    C = P.bvmv_csr_create(G)
    gs = [B.web_graph(n, 12.0, 310 + i) for i, n in enumerate((5000, 900, 17_000))]
    grp = P.bvmv_group([P.bvmv_load(B.encode(h).data) for h in gs])
    offs = P.bvmv_group_offsets(grp)

    def runs():
        out = [_pr(P, G, g.n, prec) for prec in (P.BVMV_F64, P.BVMV_F32_COMP)]
        out.append(_pr(P, grp, offs[-1], P.BVMV_F32_COMP))
        p = torch.empty(g.n, dtype=torch.float32, device=DEV)
        res = P.bvmv_csr_pagerank(C, p)
        torch.cuda.synchronize()
        out.append((p.cpu().numpy().astype(np.float64), res))
        return out

    forms = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("BVMV_PR_FUSED", mode)
        forms[mode] = runs()
    monkeypatch.delenv("BVMV_PR_FUSED")
    for (a, ra), (b, rb) in zip(forms["0"], forms["1"]):
        assert ra == rb
        assert np.array_equal(a, b)
    assert forms["1"][1][1][0][1]


def test_group_equals_solo(P):
    sizes = [3000, 800, 12_000, 5000, 200]
    gs = [B.web_graph(n, 10.0 + i, 200 + i) for i, n in enumerate(sizes)]
    Gs = [P.bvmv_load(B.encode(g).data) for g in gs]
    grp = P.bvmv_group(Gs)
    offs = P.bvmv_group_offsets(grp)
    pg, res = _pr(P, grp, offs[-1], P.BVMV_F32_COMP)
    assert len(res) == len(gs)
    for i, g in enumerate(gs):
        ps, ((it, ok, r),) = _pr(P, Gs[i], g.n, P.BVMV_F32_COMP)
        assert res[i][0] == it and res[i][1] == ok
        assert np.array_equal(pg[offs[i]:offs[i + 1]], ps)
        p_ref = pagerank.pagerank(g.rowptr, g.col, 0.85, iters=it)[0]
        assert _rel(ps, p_ref) < TOL.F32C


def test_csr_pagerank(P):
    g = B.web_graph(30_000, 15.0, 80)
    G = P.bvmv_load(B.encode(g).data, keep_lists=1)
    C = P.bvmv_csr_create(G)
    p = torch.empty(g.n, dtype=torch.float32, device=DEV)
    it, ok, r = P.bvmv_csr_pagerank(C, p)
    torch.cuda.synchronize()
    p_ref = pagerank.pagerank(g.rowptr, g.col, 0.85, iters=it)[0]
    assert ok and _rel(p.cpu().numpy(), p_ref) < TOL.F32C
    pc, ((itc, okc, rc),) = _pr(P, G, g.n, P.BVMV_F32_COMP)
    assert abs(itc - it) <= 1


@pytest.mark.slow
def test_full_size_pagerank_finish_kernel_path(P):
    """More than 12,288 blocks of tiles (n = 3.3e6, about as many edges as
    the 2^20 graph): each iteration's partials are folded by a finish kernel
    between launches instead of inside the next launch, for the compressed
    layout and for the CSR baseline.  Iteration-matched parity with the
    oracle."""
    g = B.web_graph(3_300_000, 6.0, 61)
    G = P.bvmv_load(B.encode(g).data, keep_lists=1)
    assert P.bvmv_get_info(G)["ntiles"] // 4 > 12288
    p, ((it, ok, r),) = _pr(P, G, g.n, P.BVMV_F32_COMP)
    assert ok
    p_ref, t_or, _, _ = pagerank.pagerank(g.rowptr, g.col, 0.85, tol=1e-6)
    assert abs(it - t_or) <= 1
    p_ref = pagerank.pagerank(g.rowptr, g.col, 0.85, iters=it)[0]
    assert _rel(p, p_ref) < TOL.F32C
    C = P.bvmv_csr_create(G)
    pc = torch.empty(g.n, dtype=torch.float32, device=DEV)
    itc, okc, rc = P.bvmv_csr_pagerank(C, pc)
    torch.cuda.synchronize()
    assert okc and abs(itc - t_or) <= 1
    pc_ref = p_ref if itc == it else pagerank.pagerank(g.rowptr, g.col, 0.85, iters=itc)[0]
    assert _rel(pc.cpu().numpy(), pc_ref) < TOL.F32C


def test_full_size_pagerank_2p20(P):
    g = B.workload_graph("web-n2p20-d20")
    G = P.bvmv_load(B.encode(g).data)
    p, ((it, ok, r),) = _pr(P, G, g.n, P.BVMV_F32_COMP)
    assert ok
    p_ref, t_or, _, _ = pagerank.pagerank(g.rowptr, g.col, 0.85, tol=1e-6)
    assert abs(it - t_or) <= 1
    p_ref = pagerank.pagerank(g.rowptr, g.col, 0.85, iters=it)[0]
    assert _rel(p, p_ref) < TOL.F32C
    assert abs(p.sum() - 1.0) < 1e-5
