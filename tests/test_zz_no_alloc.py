"""The allocation-free PageRank entry point (bvmv_pagerank_noalloc), through
the C ABI, against bvmv_pagerank on the same inputs: identical results (the
same kernels and fold order) on two calls in a row, the second on a
smaller graph, for the double and the two-sum float modes, with a
personalized teleport vector and a start vector too; a graph whose working
set does not fit the fixed array is refused before any device work."""
import numpy as np
import pytest

import bvinputs as B

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


def _both(P, G, n, prec, **kw):
    dt = torch.float64 if prec == P.BVMV_F64 else torch.float32
    a = torch.empty(n, dtype=dt, device=DEV)
    b = torch.full((n,), float("nan"), dtype=dt, device=DEV)
    (ra,) = P.bvmv_pagerank_detail(G, a, prec=prec, **kw)
    rb = P.bvmv_pagerank_noalloc(G, b, prec=prec, **kw)
    torch.cuda.synchronize()
    return a.cpu().numpy(), ra, b.cpu().numpy(), rb


@pytest.mark.parametrize("prec_name", ["f64", "f32c"])
def test_noalloc_equals_pagerank(P, prec_name):
    prec = P.PREC_NAMES[prec_name]
    nd = np.float64 if prec == P.BVMV_F64 else np.float32
    # a larger graph, then a smaller one: the second call reuses the array
    for n, seed in ((60_000, 91), (7_000, 92)):
        print("noalloc %s n=%d seed=%d" % (prec_name, n, seed), flush=True)
        g = B.web_graph(n, 14.0, seed)
        G = P.bvmv_load(B.encode(g).data)
        a, ra, b, rb = _both(P, G, n, prec)
        assert ra["converged"] and rb["converged"]
        assert (rb["iters"], rb["residual"], rb["products"]) == (ra["iters"], ra["residual"], ra["products"])
        assert np.array_equal(a, b)
        # personalized teleport, a start vector and an iteration limit
        v = np.zeros(n, dtype=nd)
        v[np.random.default_rng(seed).choice(n, 16, replace=False)] = 1.0 / 16
        tv = torch.from_numpy(v).to(DEV)
        start = torch.from_numpy(np.full(n, 1.0 / n, dtype=nd)).to(DEV)
        a, ra, b, rb = _both(P, G, n, prec, teleport=tv, start=start, max_iter=7, chunk=4)
        assert not ra["converged"] and ra["iters"] == 7 and rb == ra
        assert np.array_equal(a, b)
        del G


def test_noalloc_equals_pagerank_past_the_fold_threshold(P):
    """32-row tiles on n = 2e6: 15,625 blocks, past the 12,288 up to which
    bvmv_pagerank folds each iteration's partials inside the next launch; it
    then runs a finish kernel per iteration while the allocation-free call
    stays fused.  The fold order is the same, so the results are identical."""
    n = 2_000_000
    print("noalloc f32c n=%d 32-row tiles" % n, flush=True)
    g = B.web_graph(n, 6.0, 94)
    G = P.bvmv_load(B.encode(g).data, tile_rows=32, stage_bytes=2048)
    assert P.bvmv_get_info(G)["ntiles"] // 4 > 12288
    a, ra, b, rb = _both(P, G, n, P.BVMV_F32_COMP)
    assert ra["converged"] and rb == ra
    assert np.array_equal(a, b)
    del G


def test_noalloc_limit(P):
    """n = 2^21 + 2^18 float nodes (four vectors of 9 MiB) need more than the
    fixed array: BVMV_EINVAL with a message, and the library stays usable."""
    n = (1 << 21) + (1 << 18)
    edgeless = B.Graph(np.zeros(n + 1, dtype=np.uint64), np.zeros(0, dtype=np.uint32))
    G = P.bvmv_load(B.encode(edgeless).data)
    p = torch.empty(n, dtype=torch.float32, device=DEV)
    with pytest.raises(P.BvmvError) as e:
        P.bvmv_pagerank_noalloc(G, p)
    assert e.value.code == P.BVMV_EINVAL and "too large" in str(e.value)
    g = B.web_graph(3000, 10.0, 93)
    G2 = P.bvmv_load(B.encode(g).data)
    a, ra, b, rb = _both(P, G2, g.n, P.BVMV_F32_COMP)
    assert rb == ra and np.array_equal(a, b)
