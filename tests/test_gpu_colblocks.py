"""GPU parity of the column-block product (paper, Section "Final Remarks":
the matrix split into submatrices of consecutive columns, each compressed
with references of its own): y = sum of the blocks' products equals the
oracle on the whole graph, bit-exact for integer x, within the per-entry
tolerances otherwise; blocks encoded with different reference windows."""
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
    P.bvmv_colblocks_multiply(H, xd, yd, prec)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


@pytest.mark.parametrize("kind,nblocks,W", [("web", 1, 7), ("web", 3, 7), ("social", 4, 7), ("web", 5, 15),
                                            ("social", 2, 1)])
def test_column_blocks(P, kind, nblocks, W):
    print("colblocks", kind, nblocks, W, flush=True)
    g = B.web_graph(30_000, 15.0, 41) if kind == "web" else B.social_graph(30_000, 40.0, 5000, 2.1, 42)
    bounds, parts = B.column_blocks(g, nblocks)
    assert sum(p.m for p in parts) == g.m
    Gs = [P.bvmv_load(B.encode(p, W=W).data) for p in parts]
    H = P.bvmv_colblocks_create(Gs)
    xi = B.integer_x(g.n, 5, 1000)
    want = product.matvec(g.rowptr, g.col, xi)
    assert np.array_equal(_mul(P, H, xi, P.BVMV_F64), want)
    for prec in (P.BVMV_F32, P.BVMV_F32_COMP):
        assert np.array_equal(_mul(P, H, xi.astype(np.float32), prec), want), prec
    x = B.uniform_x(g.n, 6)
    assert _rel(_mul(P, H, x, P.BVMV_F64), product.matvec_exact(g.rowptr, g.col, x)) < TOL.F64
    x32 = x.astype(np.float32)
    ref32 = product.matvec_exact(g.rowptr, g.col, x32.astype(np.float64))
    assert _rel(_mul(P, H, x32, P.BVMV_F32_COMP), ref32) < TOL.F32C
    assert _rel(_mul(P, H, x32, P.BVMV_F32), ref32) < TOL.F32_NAIVE
    # one block is the plain product, bit for bit
    if nblocks == 1:
        xd = torch.from_numpy(x32).to(DEV)
        y1 = torch.empty_like(xd)
        P.bvmv_multiply(Gs[0], xd, y1, P.BVMV_F32_COMP)
        torch.cuda.synchronize()
        assert np.array_equal(y1.cpu().numpy(), _mul(P, H, x32, P.BVMV_F32_COMP))


def test_column_block_errors(P):
    a = P.bvmv_load(B.encode(B.web_graph(1000, 5.0, 1)).data)
    b = P.bvmv_load(B.encode(B.web_graph(999, 5.0, 2)).data)
    with pytest.raises(P.BvmvError) as e:
        P.bvmv_colblocks_create([a, b])
    assert e.value.code == P.BVMV_EINVAL
