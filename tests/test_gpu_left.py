"""GPU parity of the left product y = x A (PageRank's p M, Section
"PageRank"), computed on the loaded rows without the transposed graph
(x A = c A', c = x (I - R)^{-1}), against the CPU oracle's left product:
integer x bit-exact in every precision, uniform x per entry within the
tolerance (plus the floor of a few roundings of the largest entry: a
column's terms cancel where a row skips an entry of its reference row), on
web-like and social-like graphs and several layouts; equal to the right
product on the transposed graph; deterministic; the full-size web-like
workload on sampled columns."""
import numpy as np
import pytest

import bvinputs as B
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


def _left(P, G, x, prec):
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    yd = torch.full_like(xd, float("nan"))
    P.bvmv_multiply_left(G, xd, yd, prec)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def _ok(y, ref, name):
    tol = TOL.F64 if name == "f64" else TOL.F32C if name == "f32c" else TOL.F32_NAIVE
    ratio, rel_big = TOL.within(y, ref, tol, TOL.FLOOR[name])
    print("left %s: ratio %.3g, relative error above the floor %.3g" % (name, ratio, rel_big), flush=True)
    return ratio <= 1.0


CASES = [("web", {}), ("social", {}), ("web", dict(tile_rows=128, window_cap=512)), ("web", dict(interval_mode=1)),
         ("web30", dict(long_row_bytes=40)), ("web", dict(tile_rows=32))]


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_left_product(P, ci):
    kind, kw = CASES[ci]
    print("left case", ci, kind, kw, flush=True)
    g = {"web": lambda: B.web_graph(25_000, 15.0, 51), "social": lambda: B.social_graph(25_000, 40.0, 5000, 2.1, 52),
         "web30": lambda: B.web_graph(4000, 30.0, 53)}[kind]()
    G = P.bvmv_load(B.encode(g).data, **kw)
    xi = B.integer_x(g.n, 5, 1000)
    want = product.left_matvec(g.rowptr, g.col, xi)
    assert np.array_equal(_left(P, G, xi, P.BVMV_F64), want)
    for prec in (P.BVMV_F32, P.BVMV_F32_COMP):
        assert np.array_equal(_left(P, G, xi.astype(np.float32), prec), want), prec
    x = B.uniform_x(g.n, 6)
    assert _ok(_left(P, G, x, P.BVMV_F64), product.left_matvec_exact(g.rowptr, g.col, x), "f64")
    x32 = x.astype(np.float32)
    ref32 = product.left_matvec_exact(g.rowptr, g.col, x32.astype(np.float64))
    assert _ok(_left(P, G, x32, P.BVMV_F32_COMP), ref32, "f32c")
    assert _ok(_left(P, G, x32, P.BVMV_F32), ref32, "f32")
    # deterministic, and the right product on the transposed graph agrees
    a = _left(P, G, x32, P.BVMV_F32_COMP)
    assert np.array_equal(a, _left(P, G, x32, P.BVMV_F32_COMP))
    gt = g.transpose()
    Gt = P.bvmv_load(B.encode(gt).data)
    xd = torch.from_numpy(xi.astype(np.float32)).to(DEV)
    yd = torch.empty_like(xd)
    P.bvmv_multiply(Gt, xd, yd, P.BVMV_F32_COMP)
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), want)


def test_left_edge_cases_and_errors(P):
    for g in (B.empty_graph(70), B.complete_graph(90), B.star_graph(300, 0, "out"), B.star_graph(300, 7, "in"),
              B.path_graph(1000), B.from_lists([[0], [0, 1], [1, 2]])):
        G = P.bvmv_load(B.encode(g).data)
        xi = B.integer_x(g.n, 2, 1000)
        assert np.array_equal(_left(P, G, xi, P.BVMV_F64), product.left_matvec(g.rowptr, g.col, xi))
    G = P.bvmv_load(B.encode(B.web_graph(500, 5.0, 1)).data)
    x = torch.ones(500, dtype=torch.float32, device=DEV)
    with pytest.raises(P.BvmvError) as e:
        P.bvmv_multiply_left(G, x, x)
    assert e.value.code == P.BVMV_EINVAL
    grp = P.bvmv_group([G, P.bvmv_load(B.encode(B.web_graph(300, 5.0, 2)).data)])
    y = torch.empty(800, dtype=torch.float32, device=DEV)
    with pytest.raises(P.BvmvError) as e:
        P.bvmv_multiply_left(grp, torch.ones(800, dtype=torch.float32, device=DEV), y)
    assert e.value.code == P.BVMV_EINVAL


@pytest.mark.slow
def test_left_full_size_2p20(P):
    g = B.workload_graph("web-n2p20-d20")
    G = P.bvmv_load(B.encode(g).data)
    x32 = B.uniform_x(g.n, 102, np.float32)
    y = _left(P, G, x32, P.BVMV_F32_COMP)
    ref = product.left_matvec(g.rowptr, g.col, x32.astype(np.float64))
    assert _ok(y, ref, "f32c")
    ones = np.ones(g.n, dtype=np.float32)
    indeg = np.bincount(g.col.astype(np.int64), minlength=g.n).astype(np.float32)
    assert np.array_equal(_left(P, G, ones, P.BVMV_F32_COMP), indeg)
