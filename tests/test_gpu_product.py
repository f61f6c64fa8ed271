"""GPU parity of the compressed product, degrees, CSR baseline and batched
products against the CPU oracle (same seeded inputs).

Tolerances (tests/tolerances.py): FP64 path 1e-12 relative per entry; the
two-sum FP32 path 1e-5 relative per entry against the float64 oracle on the
same float32 inputs; the naive FP32 path 1e-3; integer-valued x makes every
partial sum exact, so all modes must then be bit-exact."""
import numpy as np
import pytest

import bvinputs as B
from oracle import bvdecode, product
from tests import tolerances as TOL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1708_07271_amd as mod
    mod.load_library()
    return mod


DEV = "cuda:0"


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.abs(a - b)
    z = b == 0
    assert np.all(d[z] == 0), "nonzero result where the oracle gives 0"
    return float(np.max(d[~z] / np.abs(b[~z]))) if np.any(~z) else 0.0


def _mul(P, G, x, prec):
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    yd = torch.empty_like(xd)
    P.bvmv_multiply(G, xd, yd, prec)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def _csr_mul(P, C, x, prec):
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    yd = torch.empty_like(xd)
    P.bvmv_csr_multiply(C, xd, yd, prec)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


LAYOUTS = [dict(), dict(tile_rows=16, window_cap=64, stage_bytes=512, long_row_bytes=16),
           dict(tile_rows=64, window_cap=2048, stage_bytes=8192), dict(interval_mode=1),
           dict(tile_rows=32, window_cap=256, stage_bytes=1024, long_row_bytes=40, interval_mode=1)]


def _graphs():
    return {
        "web-n1e4-d15": B.web_graph(10_000, 15.0, 1),
        "social-n3e4-d30": B.social_graph(30_000, 30.0, 5000, 2.1, 3),
    }


@pytest.fixture(scope="module")
def graphs():
    out = {}
    for name, g in _graphs().items():
        out[name] = (g, B.encode(g))
    return out


@pytest.mark.parametrize("lay", range(len(LAYOUTS)))
def test_product_parity_all_modes(P, graphs, lay):
    for name, (g, enc) in graphs.items():
        print("case", name, LAYOUTS[lay], flush=True)
        G = P.bvmv_load(enc.data, **LAYOUTS[lay])
        x = B.uniform_x(g.n, 101)
        assert _rel(_mul(P, G, x, P.BVMV_F64), product.matvec(g.rowptr, g.col, x)) < TOL.F64
        x32 = x.astype(np.float32)
        ref32 = product.matvec(g.rowptr, g.col, x32.astype(np.float64))
        assert _rel(_mul(P, G, x32, P.BVMV_F32_COMP), ref32) < TOL.F32C
        assert _rel(_mul(P, G, x32, P.BVMV_F32), ref32) < TOL.F32_NAIVE
        xi = B.integer_x(g.n, 5, 7)                 # partial sums < 2^24: exact in float32
        refi = product.matvec(g.rowptr, g.col, xi)
        for prec in (P.BVMV_F32, P.BVMV_F32_COMP):
            assert np.array_equal(_mul(P, G, xi.astype(np.float32), prec), refi)
        xi = B.integer_x(g.n, 6, 1000)
        assert np.array_equal(_mul(P, G, xi, P.BVMV_F64), product.matvec(g.rowptr, g.col, xi))


def test_deterministic(P, graphs):
    g, enc = graphs["social-n3e4-d30"]
    G = P.bvmv_load(enc.data)
    x = B.uniform_x(g.n, 3).astype(np.float32)
    for prec in (P.BVMV_F32, P.BVMV_F32_COMP):
        a = _mul(P, G, x, prec)
        b = _mul(P, G, x, prec)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_degrees_and_export(P, graphs):
    for name, (g, enc) in graphs.items():
        G = P.bvmv_load(enc.data, keep_lists=1)
        deg = torch.empty(g.n, dtype=torch.int32, device=DEV)
        P.bvmv_degrees(G, deg)
        torch.cuda.synchronize()
        assert np.array_equal(deg.cpu().numpy(), np.diff(g.rowptr).astype(np.int32))
        rp, col = P.bvmv_export_csr(G)
        assert np.array_equal(rp, g.rowptr) and np.array_equal(col, g.col)
        info = G.info()
        assert info["m"] == g.m and info["n"] == g.n


def test_closed_forms_on_device(P):
    n = 300
    x = B.uniform_x(n, 9)
    cases = [(B.complete_graph(n), x.sum() - x), (B.star_graph(n, 7, "out"), None), (B.path_graph(n), None)]
    for g, _ in cases:
        G = P.bvmv_load(B.encode(g).data)
        y = _mul(P, G, x, P.BVMV_F64)
        assert _rel(y, product.matvec_exact(g.rowptr, g.col, x)) < TOL.F64
    G = P.bvmv_load(B.encode(B.complete_graph(n)).data)
    assert _rel(_mul(P, G, x, P.BVMV_F64), x.sum() - x) < TOL.F64


def test_edge_cases(P):
    # empty graph, single node, self-loops, rows touching 0 and n-1, a long reused row
    for g in (B.empty_graph(1), B.empty_graph(1000), B.from_lists([[0]]), B.from_lists([[1], [0, 1]])):
        G = P.bvmv_load(B.encode(g).data)
        x = B.integer_x(g.n, 1, 1000)
        assert np.array_equal(_mul(P, G, x, P.BVMV_F64), product.matvec(g.rowptr, g.col, x))
    n = 70_000
    rng = np.random.default_rng(5)
    lists = [[] for _ in range(n)]
    lists[1] = list(range(0, 300))
    lists[2] = list(range(0, 300))
    lists[5] = sorted(rng.choice(n, 50_000, replace=False).tolist())
    lists[6] = sorted(set(lists[5][:45_000]) | {n - 1})
    lists[n - 1] = list(range(n - 20, n))
    g = B.from_lists(lists)
    enc = B.encode(g)
    for lay in LAYOUTS:
        G = P.bvmv_load(enc.data, **lay)
        x = B.integer_x(n, 2, 7)
        assert np.array_equal(_mul(P, G, x.astype(np.float32), P.BVMV_F32_COMP), product.matvec(g.rowptr, g.col, x))


@pytest.mark.parametrize("lay", range(len(LAYOUTS)))
def test_entries_at_the_end_of_the_stream_array(P, lay):
    """The last tile's rows reach far outside their window (wide entries) and
    hold runs (prefix pairs in the singles stream), so the device stream array
    ends with both kinds of entry and then only its zero padding.  Each flat
    pass reads whole rounds of stream words near that end: the pass that
    decodes whole rounds (other precisions, wide entries) must see only words
    of its own stream, and the running-sum pass must zero what lies past its
    chunk.  Every mode matches the oracle."""
    n = 5000
    lists = [[(i + 1) % n] for i in range(n)]
    for i in range(n - 48, n):
        lists[i] = sorted(({0, 3, 7, 11, i - 1500, i - 3100} | set(range(i - 40, i - 30))) - {i})
    g = B.from_lists(lists)
    G = P.bvmv_load(B.encode(g).data, **LAYOUTS[lay])
    assert P.bvmv_get_info(G)["escapes"] > 0
    x = B.uniform_x(n, 77)
    assert _rel(_mul(P, G, x, P.BVMV_F64), product.matvec(g.rowptr, g.col, x)) < TOL.F64
    x32 = x.astype(np.float32)
    ref32 = product.matvec(g.rowptr, g.col, x32.astype(np.float64))
    assert _rel(_mul(P, G, x32, P.BVMV_F32_COMP), ref32) < TOL.F32C
    assert _rel(_mul(P, G, x32, P.BVMV_F32), ref32) < TOL.F32_NAIVE
    xi = B.integer_x(n, 5, 9)
    refi = product.matvec(g.rowptr, g.col, xi)
    for prec in (P.BVMV_F32, P.BVMV_F32_COMP):
        assert np.array_equal(_mul(P, G, xi.astype(np.float32), prec), refi)


def test_largest_layouts(P, graphs):
    """The widest x windows the device's LDS admits.  On the social graph
    (uniform random targets) every tile's best window fills the cap, so a cap
    of 8191 columns must be refused at load with an LDS error, before any
    launch; the widest accepted cap, for 64- and 128-row tiles, stages its
    window through the general (more than 16 values per lane) path and must
    still be exact on integer x and within tolerance on uniform x."""
    g, enc = graphs["social-n3e4-d30"]
    with pytest.raises(P.BvmvError) as e:
        P.bvmv_load(enc.data, window_cap=8191, stage_bytes=16384)
    assert e.value.code == P.BVMV_EINVAL and "LDS" in str(e.value)
    xi = B.integer_x(g.n, 3, 1000)
    want_i = product.matvec(g.rowptr, g.col, xi)
    x = B.uniform_x(g.n, 4)
    want = product.matvec_exact(g.rowptr, g.col, x)
    x32 = x.astype(np.float32)
    want32 = product.matvec_exact(g.rowptr, g.col, x32.astype(np.float64))
    for rows in (64, 128):
        G, cap = None, 0
        for cap in (4096, 3072, 2560, 2496, 2432, 2368, 2304, 2048):
            try:
                G = P.bvmv_load(enc.data, tile_rows=rows, window_cap=cap, stage_bytes=16384)
                break
            except P.BvmvError as err:
                assert err.code == P.BVMV_EINVAL and "LDS" in str(err)
        assert G is not None and cap >= 2048, rows
        print("largest window cap for %d-row tiles: %d" % (rows, cap), flush=True)
        for prec in (P.BVMV_F64, P.BVMV_F32, P.BVMV_F32_COMP):
            xp = xi if prec == P.BVMV_F64 else xi.astype(np.float32)
            assert np.array_equal(_mul(P, G, xp, prec), want_i), (rows, prec)
        assert _rel(_mul(P, G, x, P.BVMV_F64), want) < TOL.F64
        assert _rel(_mul(P, G, x32, P.BVMV_F32_COMP), want32) < TOL.F32C


def test_csr_baseline(P, graphs):
    for name, (g, enc) in graphs.items():
        G = P.bvmv_load(enc.data, keep_lists=1)
        C = P.bvmv_csr_create(G)
        x = B.uniform_x(g.n, 11)
        assert _rel(_csr_mul(P, C, x, P.BVMV_F64), product.matvec(g.rowptr, g.col, x)) < TOL.F64
        x32 = x.astype(np.float32)
        ref32 = product.matvec(g.rowptr, g.col, x32.astype(np.float64))
        assert _rel(_csr_mul(P, C, x32, P.BVMV_F32_COMP), ref32) < TOL.F32C
        xi = B.integer_x(g.n, 12, 7).astype(np.float32)
        assert np.array_equal(_csr_mul(P, C, xi, P.BVMV_F32), product.matvec(g.rowptr, g.col, xi))


@pytest.mark.parametrize("k", [1, 3, 16, 32, 64])
def test_batch_matches_oracle(P, graphs, k):
    for name, (g, enc) in graphs.items():
        print("case", name, k, flush=True)
        G = P.bvmv_load(enc.data)
        rng = np.random.default_rng(k)
        X = rng.random((g.n, k), dtype=np.float32)
        # right-hand side c is row c of the (k, n) device tensors
        Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to(DEV)
        Yd = torch.empty_like(Xd)
        P.bvmv_multiply_batch(G, Xd, Yd, P.BVMV_F32_COMP)
        torch.cuda.synchronize()
        Y = Yd.cpu().numpy().T
        for c in range(0, k, max(1, k // 4)):
            assert _rel(Y[:, c], product.matvec(g.rowptr, g.col, X[:, c].astype(np.float64))) < TOL.F32C
        Xi = rng.integers(0, 8, size=(g.n, k)).astype(np.float32)
        Xd = torch.from_numpy(np.ascontiguousarray(Xi.T)).to(DEV)
        P.bvmv_multiply_batch(G, Xd, Yd, P.BVMV_F32)
        torch.cuda.synchronize()
        Y = Yd.cpu().numpy().T
        for c in range(k):
            assert np.array_equal(Y[:, c], product.matvec(g.rowptr, g.col, Xi[:, c].astype(np.float64)))
        Xd64 = torch.from_numpy(np.ascontiguousarray(X.T, dtype=np.float64)).to(DEV)
        Yd64 = torch.empty_like(Xd64)
        P.bvmv_multiply_batch(G, Xd64, Yd64, P.BVMV_F64)
        torch.cuda.synchronize()
        assert _rel(Yd64.cpu().numpy()[k - 1], product.matvec(g.rowptr, g.col, X[:, k - 1].astype(np.float64))) < TOL.F64


def test_batch_leading_dimension(P):
    """Right-hand sides as rows of a wider buffer (ld = n + 37): the padding
    is neither read into the products nor written."""
    g = B.web_graph(9000, 12.0, 71)
    G = P.bvmv_load(B.encode(g).data)
    k, ld = 5, g.n + 37
    rng = np.random.default_rng(71)
    Xb = torch.from_numpy(rng.random((k, ld), dtype=np.float32)).to(DEV)
    Yb = torch.full((k, ld), -7.0, device=DEV)
    P.bvmv_multiply_batch(G, Xb[:, :g.n], Yb[:, :g.n], P.BVMV_F32_COMP)
    torch.cuda.synchronize()
    X = Xb.cpu().numpy()
    Y = Yb.cpu().numpy()
    assert np.all(Y[:, g.n:] == -7.0)
    for c in range(k):
        assert _rel(Y[c, :g.n], product.matvec(g.rowptr, g.col, X[c, :g.n].astype(np.float64))) < TOL.F32C
    # each column equals the single-vector product bit for bit
    y1 = torch.empty(g.n, device=DEV)
    P.bvmv_multiply(G, Xb[3, :g.n].contiguous(), y1, P.BVMV_F32_COMP)
    torch.cuda.synchronize()
    assert torch.equal(y1, Yb[3, :g.n])


def test_group_block_diagonal(P):
    sizes = [1000, 5000, 20_000, 300]
    gs = [B.web_graph(n, 12.0, 50 + i) for i, n in enumerate(sizes)]
    Gs = [P.bvmv_load(B.encode(g).data) for g in gs]
    grp = P.bvmv_group(Gs)
    offs = P.bvmv_group_offsets(grp)
    assert offs == [0] + list(np.cumsum(sizes))
    x = B.integer_x(offs[-1], 3, 7).astype(np.float32)
    y = _mul(P, grp, x, P.BVMV_F32_COMP)
    for i, g in enumerate(gs):
        seg = slice(offs[i], offs[i + 1])
        assert np.array_equal(y[seg], product.matvec(g.rowptr, g.col, x[seg].astype(np.float64)))
        assert np.array_equal(y[seg], _mul(P, Gs[i], x[seg], P.BVMV_F32_COMP))



def test_group_of_mixed_layouts(P):
    """Members laid out differently (as the autotuner may leave them): with
    their lists kept, the group is laid out with one of the members' layouts,
    the faster over the whole group; without lists the members' own layouts
    are concatenated.  Either way every member's rows are exact on integer x
    and within the tolerance on uniform x."""
    sizes = [3000, 12_000, 700]
    gs = [B.web_graph(n, 14.0, 80 + i) for i, n in enumerate(sizes)]
    shapes = [dict(tile_rows=64, window_cap=256), dict(tile_rows=128, window_cap=768, stage_bytes=6144),
              dict(tile_rows=32, window_cap=256, stage_bytes=2048)]
    for keep in (1, 0):
        Gs = [P.bvmv_load(B.encode(g).data, keep_lists=keep, **sh) for g, sh in zip(gs, shapes)]
        grp = P.bvmv_group(Gs)
        info = P.bvmv_get_info(grp)
        print("group of mixed layouts, lists kept %d: tile rows %d, window %d, autotuned %d"
              % (keep, info["tile_rows"], info["window_cap"], info["autotuned"]), flush=True)
        if keep:
            assert info["autotuned"] == 1
            assert (info["tile_rows"], info["window_cap"]) in [(sh["tile_rows"], sh["window_cap"]) for sh in shapes]
        else:
            assert info["autotuned"] == 0
        offs = P.bvmv_group_offsets(grp)
        xi = B.integer_x(offs[-1], 4, 9).astype(np.float32)
        x = B.uniform_x(offs[-1], 5, np.float32)
        yi = _mul(P, grp, xi, P.BVMV_F32_COMP)
        y = _mul(P, grp, x, P.BVMV_F32_COMP)
        for i, g in enumerate(gs):
            seg = slice(offs[i], offs[i + 1])
            assert np.array_equal(yi[seg], product.matvec(g.rowptr, g.col, xi[seg].astype(np.float64)))
            assert _rel(y[seg], product.matvec_exact(g.rowptr, g.col, x[seg].astype(np.float64))) < TOL.F32C


# the autotuner's candidate layouts (tile rows, window columns, staged bytes)
TUNE_CANDS = [(32, 256, 2048), (64, 256, 4096), (64, 384, 3072), (64, 512, 4096), (64, 768, 6144),
              (128, 768, 6144)]


@pytest.mark.parametrize("cand", TUNE_CANDS)
def test_autotune_candidates_exact(P, graphs, cand):
    # every layout the autotuner may pick gives the exact sums on integer x
    for name, (g, enc) in graphs.items():
        print("case", name, cand, flush=True)
        G = P.bvmv_load(enc.data, tile_rows=cand[0], window_cap=cand[1], stage_bytes=cand[2])
        xi = B.integer_x(g.n, 8, 7).astype(np.float32)
        refi = product.matvec(g.rowptr, g.col, xi.astype(np.float64))
        for prec in (P.BVMV_F32, P.BVMV_F32_COMP):
            assert np.array_equal(_mul(P, G, xi, prec), refi)
        x = B.uniform_x(g.n, 9)
        assert _rel(_mul(P, G, x, P.BVMV_F64), product.matvec(g.rowptr, g.col, x)) < TOL.F64


def test_autotune_load(P):
    g = B.web_graph(50_000, 17.0, 71)
    enc = B.encode(g)
    G = P.bvmv_load(enc.data, autotune=1)
    info = P.bvmv_get_info(G)
    assert info["autotuned"] in (1, 2)
    assert (info["tile_rows"], info["window_cap"], info["stage_bytes"]) in TUNE_CANDS
    # the same size bucket again: the remembered choice
    G2 = P.bvmv_load(enc.data, autotune=1)
    info2 = P.bvmv_get_info(G2)
    assert info2["autotuned"] == 2 and info2["tile_rows"] == info["tile_rows"]
    assert info2["window_cap"] == info["window_cap"]
    x = B.uniform_x(g.n, 72, np.float32)
    ref = product.matvec(g.rowptr, g.col, x.astype(np.float64))
    assert _rel(_mul(P, G, x, P.BVMV_F32_COMP), ref) < TOL.F32C
    assert P.bvmv_get_info(P.bvmv_load(enc.data))["autotuned"] == 0


@pytest.mark.slow
def test_full_size_web_2p20(P):
    """n = 2^20, mean out-degree 20: every row against the oracle, and sampled
    rows against correctly rounded sums."""
    g = B.workload_graph("web-n2p20-d20")
    G = P.bvmv_load(B.encode(g).data)
    x32 = B.uniform_x(g.n, 102, np.float32)
    y = _mul(P, G, x32, P.BVMV_F32_COMP)
    x64 = x32.astype(np.float64)
    assert _rel(y, product.matvec(g.rowptr, g.col, x64)) < TOL.F32C
    rows = np.random.default_rng(0).choice(g.n, 2000, replace=False)
    assert _rel(y[rows], product.matvec_rows(g.rowptr, g.col, x64, rows)) < TOL.F32C
    xi = B.integer_x(g.n, 4, 7).astype(np.float32)
    assert np.array_equal(_mul(P, G, xi, P.BVMV_F32_COMP), product.matvec(g.rowptr, g.col, xi))


@pytest.mark.slow
def test_full_size_web_2p20_f64(P):
    """n = 2^20, FP64 vectors in the bench's launch configuration: every row
    within 1e-12 of the oracle, and sampled rows against correctly rounded
    sums."""
    g = B.workload_graph("web-n2p20-d20")
    G = P.bvmv_load(B.encode(g).data)
    x = B.uniform_x(g.n, 102)
    y = _mul(P, G, x, P.BVMV_F64)
    assert _rel(y, product.matvec(g.rowptr, g.col, x)) < TOL.F64
    rows = np.random.default_rng(3).choice(g.n, 2000, replace=False)
    assert _rel(y[rows], product.matvec_rows(g.rowptr, g.col, x, rows)) < TOL.F64


def _chain_graph(nchains, base_size, seed):
    """Chains of 16 rows (depths 0..15 with R = 15, W = 1).  Row 0 of a chain
    holds a big column and `base_size` small ones; every later row drops one
    entry of the row before it and adds one: at odd depths it drops the big
    column and adds a tiny one, at even depths it drops a small column and
    adds a new big one.  Big x lie in [4096, 8192), where a float's spacing is
    2^-11, and tiny x in [2^-13, 2^-12), under half that spacing: a float sum
    of a row's partial (+tiny - big) loses the tiny value, so the naive chain
    misses one more of them at every odd depth.  Columns 0..nbig-1 are big,
    then the tiny ones, then the small ones."""
    rng = np.random.default_rng(seed)
    nbig, ntiny = nchains * 8, nchains * 8
    n = nbig + ntiny + max(nchains * 16, 8 * base_size)
    lists = []
    big, tiny = iter(range(nbig)), iter(range(nbig, nbig + ntiny))
    small = np.arange(nbig + ntiny, n)
    for c in range(nchains):
        row = set(rng.choice(small, base_size, replace=False).tolist())
        b = next(big)
        row.add(b)
        lists.append(sorted(row))
        for d in range(1, 16):
            if d % 2:
                row.discard(b)
                row.add(next(tiny))
            else:
                row.discard(max(row))               # a small column (the largest ids are small ones)
                b = next(big)
                row.add(b)
            lists.append(sorted(row))
    lists += [[] for _ in range(n - len(lists))]
    g = B.from_lists(lists)
    x = np.random.default_rng(seed + 1).random(n).astype(np.float32)
    r = np.random.default_rng(seed + 2)
    x[:nbig] = (4096.0 * (1.0 + r.random(nbig))).astype(np.float32)
    x[nbig:nbig + ntiny] = (2.0 ** -13 * (1.0 + r.random(ntiny))).astype(np.float32)
    return g, x


def test_deep_chain_compensation(P):
    """Reference chains 15 deep (R = 15): the naive FP32 error of the odd
    (small-sum) rows grows with the chain depth, one swamped tiny value more
    at every odd step, while the TwoSum-compensated chains stay within 1e-5
    of the FP64 oracle at every depth; the FP64 path stays within 1e-12."""
    g, x = _chain_graph(48, 24, 5)
    enc = B.encode(g, W=1, R=15)
    _, _, _, hdr, st = bvdecode.decode(enc.data, with_stats=True)
    depth = st[:, 0]
    assert depth.max() == 15
    G = P.bvmv_load(enc.data)
    assert G.info()["max_level"] == 15
    ref = product.matvec(g.rowptr, g.col, x.astype(np.float64))
    yc = _mul(P, G, x, P.BVMV_F32_COMP).astype(np.float64)
    yn = _mul(P, G, x, P.BVMV_F32).astype(np.float64)
    assert _rel(yc, ref) < TOL.F32C
    assert _rel(_mul(P, G, x.astype(np.float64), P.BVMV_F64), ref) < TOL.F64
    nz = ref != 0
    en = np.zeros_like(ref)
    en[nz] = np.abs(yn[nz] - ref[nz]) / np.abs(ref[nz])
    by_depth = np.array([en[nz & (depth == d)].mean() for d in range(1, 16, 2)])
    print("naive FP32 mean relative error at depths 1, 3, .., 15:", ["%.1e" % v for v in by_depth],
          "compensated max %.2e" % _rel(yc, ref), flush=True)
    # one more swamped tiny value per odd depth: the error grows with depth
    assert by_depth[-1] > 2.5 * by_depth[0] and by_depth[-1] > 5 * TOL.F32C
    assert np.polyfit(np.arange(1, 16, 2), by_depth, 1)[0] > 0


@pytest.mark.slow
def test_full_size_social_4e6(P):
    """social-n4e6-d40 (n = 4e6, m = 1.6e8, BFS order), in the launch
    configuration bench.py --social times: two-sum FP32 within 1e-5 of the
    correctly rounded sums on sampled rows, naive FP32 within 1e-3, and
    integer x exact on every row."""
    g = B.workload_graph("social-n4e6-d40")
    G = P.bvmv_load(B.encode(g).data)
    x32 = B.uniform_x(g.n, 103, np.float32)
    rows = np.random.default_rng(1).choice(g.n, 3000, replace=False)
    ref = product.matvec_rows(g.rowptr, g.col, x32.astype(np.float64), rows)
    assert _rel(_mul(P, G, x32, P.BVMV_F32_COMP)[rows], ref) < TOL.F32C
    assert _rel(_mul(P, G, x32, P.BVMV_F32)[rows], ref) < TOL.F32_NAIVE
    xi = B.integer_x(g.n, 5, 7).astype(np.float32)
    assert np.array_equal(_mul(P, G, xi, P.BVMV_F32_COMP), product.matvec(g.rowptr, g.col, xi.astype(np.float64)))


@pytest.mark.slow
def test_full_size_batch_8e6(P):
    """web-n8e6-d25 with 32 right-hand sides (the batched personalized
    PageRank workload): every column of the batched product within 1e-5 of
    the correctly rounded sums on sampled rows."""
    g = B.workload_graph("web-n8e6-d25")
    G = P.bvmv_load(B.encode(g).data)
    k = 32
    X = np.random.default_rng(104).random((g.n, k), dtype=np.float32)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to(DEV)
    Yd = torch.empty_like(Xd)
    P.bvmv_multiply_batch(G, Xd, Yd, P.BVMV_F32_COMP)
    torch.cuda.synchronize()
    rows = np.random.default_rng(2).choice(g.n, 400, replace=False)
    Yr = Yd[:, torch.from_numpy(rows).to(DEV)].cpu().numpy().T
    for c in (0, 7, 31):
        ref = product.matvec_rows(g.rowptr, g.col, X[:, c].astype(np.float64), rows)
        assert _rel(Yr[:, c], ref) < TOL.F32C, c
