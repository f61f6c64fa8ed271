"""GPU parity of the biclique-format product (paper, Section "Final
Remarks": c_r = sum of x over C_r, added to every row of S_r, plus the
residual edges) against the CPU oracle: planted and mined decompositions in
every precision, integer x bit-exact, edge cases (no bicliques, no residual,
empty sets, long lists on both passes, ids at the ragged end), and the mined
web-like workload at full size on sampled rows."""
import numpy as np
import pytest

import bvinputs as B
from oracle import biclique as bic
from oracle import product
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
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.abs(a - b)
    z = b == 0
    assert np.all(d[z] == 0), "nonzero result where the oracle gives 0"
    return float(np.max(d[~z] / np.abs(b[~z]))) if np.any(~z) else 0.0


def _mul(P, H, x, prec):
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    yd = torch.full_like(xd, float("nan"))
    P.bvmv_biclique_multiply(H, xd, yd, prec)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def _check_all(P, b, tag):
    print("biclique case", tag, "n=%d bicliques=%d" % (b.n, b.nbic), flush=True)
    H = P.bvmv_biclique_load(b)
    rp, col = bic.lists(b)
    info = H.info()
    assert info["m"] == int(rp[-1]) and info["words"] == b.words() and info["nbic"] == b.nbic
    xi = B.integer_x(b.n, 5, 1000)
    want = product.matvec(rp, col, xi)
    assert np.array_equal(_mul(P, H, xi, P.BVMV_F64), want)
    for prec in (P.BVMV_F32, P.BVMV_F32_COMP):
        assert np.array_equal(_mul(P, H, xi.astype(np.float32), prec), want), prec
    x = B.uniform_x(b.n, 6)
    assert _rel(_mul(P, H, x, P.BVMV_F64), product.matvec_exact(rp, col, x)) < TOL.F64
    x32 = x.astype(np.float32)
    ref32 = product.matvec_exact(rp, col, x32.astype(np.float64))
    assert _rel(_mul(P, H, x32, P.BVMV_F32_COMP), ref32) < TOL.F32C
    assert _rel(_mul(P, H, x32, P.BVMV_F32), ref32) < TOL.F32_NAIVE
    # the paper's own two-step order gives the same result within rounding
    assert _rel(bic.paper_product(b, x), product.matvec_exact(rp, col, x)) < 1e-14
    return H


@pytest.mark.parametrize("n,nb,seed", [(3000, 400, 1), (9999, 1500, 2), (257, 60, 3)])
def test_planted(P, n, nb, seed):
    g, b = B.planted_bicliques(n, nb, seed=seed)
    _check_all(P, b, "planted n=%d seed=%d" % (n, seed))


def test_mined_web(P):
    g = B.web_graph(40_000, 15.0, 31)
    b = B.biclique_mine(g)
    H = _check_all(P, b, "mined web n=40000")
    assert H.info()["m"] == g.m


def test_edge_cases(P):
    n = 5000
    rng = np.random.default_rng(8)
    # no bicliques: the residual alone (a plain CSR product)
    g = B.web_graph(n, 10.0, 9)
    _check_all(P, B.Bicliques(n, np.zeros(1, np.uint64), np.zeros(0, np.uint32), np.zeros(1, np.uint64),
                              np.zeros(0, np.uint32), g.rowptr.copy(), g.col.copy()), "residual only")
    # no residual; an empty S, an empty C; a C list of 3000 ids (a long row of
    # the first pass) and a node in 700 bicliques (a long row of the second);
    # ids at n - 1
    S_l, C_l = [], []
    for r in range(700):
        S_l.append(np.array(sorted({0, int(rng.integers(1, n))}), np.uint32))
        C_l.append(np.array([r * 7 % (n - 1) + 1], np.uint32) if r % 2 else np.array([n - 1 - r], np.uint32))
    S_l.append(np.array([], np.uint32))
    C_l.append(np.array([1, 2, 3], np.uint32))
    S_l.append(np.array([5, n - 1], np.uint32))
    C_l.append(np.array([], np.uint32))
    S_l.append(np.array([n - 2, n - 1], np.uint32))
    C_l.append(np.arange(1000, 4000, dtype=np.uint32))
    cnt = lambda L: np.concatenate([[0], np.cumsum([len(x) for x in L])]).astype(np.uint64)
    b = B.Bicliques(n, cnt(S_l), np.concatenate(S_l).astype(np.uint32), cnt(C_l),
                    np.concatenate(C_l).astype(np.uint32), np.zeros(n + 1, np.uint64), np.zeros(0, np.uint32))
    A = bic.dense(b)
    assert set(np.unique(A).tolist()) <= {0.0, 1.0}
    _check_all(P, b, "edge cases")


def test_errors_and_determinism(P):
    g, b = B.planted_bicliques(2000, 200, seed=4)
    H = P.bvmv_biclique_load(b)
    x = torch.from_numpy(B.uniform_x(g.n, 1).astype(np.float32)).to(DEV)
    with pytest.raises(P.BvmvError) as e:
        P.bvmv_biclique_multiply(H, x, x)
    assert e.value.code == P.BVMV_EINVAL
    y1 = torch.empty_like(x)
    y2 = torch.empty_like(x)
    P.bvmv_biclique_multiply(H, x, y1)
    P.bvmv_biclique_multiply(H, x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)


@pytest.mark.slow
def test_full_size_mined_web_2p20(P):
    """The mined n = 2^20 web-like workload: degrees exactly (x = 1) and
    sampled rows against the correctly rounded oracle."""
    g = B.workload_graph("web-n2p20-d20")
    b = B.biclique_mine(g)
    H = P.bvmv_biclique_load(b)
    assert H.info()["m"] == g.m
    ones = np.ones(g.n, dtype=np.float32)
    assert np.array_equal(_mul(P, H, ones, P.BVMV_F32_COMP), np.diff(g.rowptr.astype(np.int64)).astype(np.float32))
    x32 = B.uniform_x(g.n, 102, np.float32)
    y = _mul(P, H, x32, P.BVMV_F32_COMP)
    rows = np.random.default_rng(0).choice(g.n, 20_000, replace=False)
    rows = np.concatenate([rows, np.arange(g.n - 64, g.n)])
    ref = product.matvec_rows(g.rowptr, g.col, x32.astype(np.float64), rows)
    assert _rel(y[rows], ref) < TOL.F32C
