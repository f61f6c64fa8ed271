"""Pins of the CPU oracle against facts fixed outside it: hand-written code
tables and bitstreams, dense brute force, closed forms, invariants, and the
paper's own sequential algorithm.  All CPU-only."""
import math

import numpy as np
import pytest

import bvinputs as B
from oracle import bvdecode, pagerank, product
from tests.golden_io import pack_stream, read_codes, read_tiny_stream


# ------------------------------------------------------------------ codes
def test_codes_golden():
    for kind, k, x, bits in read_codes():
        data = np.frombuffer(int(bits + "0" * ((-len(bits)) % 8), 2).to_bytes((len(bits) + 7) // 8, "big"),
                             dtype=np.uint8)
        br = bvdecode.BitReader(data.tobytes(), len(bits))
        got = {"unary": br.unary, "gamma": br.gamma, "zeta": lambda: br.zeta(k)}[kind]()
        assert got == x, (kind, k, bits)
        assert br.pos == len(bits), (kind, k, bits)


def test_nu_inverse():
    for z in range(-50, 51):
        u = 2 * z if z >= 0 else 2 * (-z) - 1
        assert bvdecode.nu_inv(u) == z


# ------------------------------------------------------------- bitstream
def test_tiny_stream_golden():
    data, lists, refs = read_tiny_stream()
    rowptr, col, got_refs, hdr = bvdecode.decode(data)
    assert hdr["n"] == 6 and hdr["m"] == 16
    for i, L in enumerate(lists):
        assert col[int(rowptr[i]):int(rowptr[i + 1])].tolist() == L
    assert got_refs.tolist() == refs


def _roundtrip(g, **kw):
    enc = B.encode(g, **kw)
    rowptr, col, refs, hdr = bvdecode.decode(enc.data)
    assert np.array_equal(rowptr, g.rowptr)
    assert np.array_equal(col, g.col)
    assert np.array_equal(refs, enc.refs)
    assert hdr["m"] == g.m
    return refs


def test_roundtrip_web():
    g = B.web_graph(3000, 15.0, 11)
    refs = _roundtrip(g)
    assert (refs > 0).mean() > 0.5          # the copying model is referenced heavily


def test_roundtrip_social():
    _roundtrip(B.social_graph(3000, 12.0, 400, 2.1, 12))


@pytest.mark.parametrize("W,R,Lmin,zk", [(7, 3, 4, 3), (1, 1, 2, 1), (0, 0, 3, 2), (15, 15, 8, 5)])
def test_roundtrip_params(W, R, Lmin, zk):
    _roundtrip(B.web_graph(1500, 12.0, 5), W=W, R=R, Lmin=Lmin, zeta_k=zk, stride=0 if W * R == 0 else W * R + 1)


def test_roundtrip_crafted():
    n = 200
    lists = [[] for _ in range(n)]
    lists[1] = list(range(0, 10))                 # interval touching 0
    lists[2] = list(range(0, 10))                 # identical to its reference
    lists[3] = [150]                              # reference fully skipped
    lists[4] = [3, 4, 150, 199]                   # self-loop at 4, id n-1
    lists[5] = list(range(190, 200))              # interval touching n-1
    lists[6] = list(range(0, 200, 2))             # long strided row
    lists[7] = list(range(0, 200))                # complete row incl. self
    for i in range(8, 40):                        # a deep chain of near-identical rows
        lists[i] = sorted(set(lists[i - 1] if i > 8 else range(20, 60)) ^ {60 + i, 20 + (i % 7)})
    g = B.from_lists(lists)
    for W, R in [(7, 3), (3, 1), (7, 15)]:
        _roundtrip(g, W=W, R=R, stride=W * R + 1)


def test_roundtrip_long_row():
    n = 60000
    rng = np.random.default_rng(3)
    lists = [[] for _ in range(n)]
    lists[10] = sorted(rng.choice(n, 50000, replace=False).tolist())
    lists[11] = sorted(set(lists[10][:40000]) | {5, 6, 7, 8})
    g = B.from_lists(lists)
    _roundtrip(g)


def test_corrupt_streams():
    g = B.web_graph(500, 10.0, 7)
    data = B.encode(g).data
    bad = data.copy(); bad[0] = ord("X")
    with pytest.raises(bvdecode.FormatError):
        bvdecode.decode(bad)
    with pytest.raises(bvdecode.FormatError):
        bvdecode.decode(data[: len(data) // 2])
    bad = data.copy(); bad[16] ^= 1               # edge count in the header
    with pytest.raises(bvdecode.FormatError):
        bvdecode.decode(bad)
    # a reference outside the window: node 1 claiming g=2
    bits = "010" + "1" + "110" + "010" + "001"   # node0 [..]; node1 d=1 g=2
    with pytest.raises(bvdecode.FormatError):
        bvdecode.decode(pack_stream(2, 2, 7, 3, 4, 3, bits))


# --------------------------------------------------------------- product
def _csr(g):
    return g.rowptr, g.col


def test_product_dense_bruteforce():
    for seed in range(3):
        g = B.web_graph(800, 12.0, 100 + seed)
        x = B.uniform_x(g.n, seed)
        y = product.matvec_exact(*_csr(g), x)
        yd = product.matvec_dense(*_csr(g), x)
        assert np.allclose(y, yd, rtol=1e-14, atol=0)
        assert np.allclose(product.matvec(*_csr(g), x), y, rtol=1e-14, atol=0)
        rows = np.array([0, 1, 17, 400, g.n - 2, g.n - 1])
        assert np.allclose(product.matvec_rows(*_csr(g), x, rows), yd[rows], rtol=1e-14, atol=0)


def test_product_closed_forms():
    n = 37
    x = B.uniform_x(n, 9)
    y = product.matvec_exact(*_csr(B.complete_graph(n)), x)
    assert np.allclose(y, x.sum() - x, rtol=1e-14)
    y = product.matvec_exact(*_csr(B.path_graph(n)), x)
    assert np.array_equal(y[:-1], x[1:]) and y[-1] == 0.0
    y = product.matvec_exact(*_csr(B.star_graph(n, 3, "out")), x)
    assert math.isclose(y[3], x.sum() - x[3], rel_tol=1e-14) and np.all(np.delete(y, 3) == 0)
    y = product.matvec_exact(*_csr(B.star_graph(n, 3, "in")), x)
    assert y[3] == 0 and np.all(np.delete(y, 3) == x[3])


def test_product_indicator_and_ones():
    g = B.web_graph(2000, 15.0, 21)
    deg = np.diff(g.rowptr).astype(np.float64)
    assert np.array_equal(product.matvec(*_csr(g), np.ones(g.n)), deg)
    for j in (0, 777, g.n - 1):
        e = np.zeros(g.n); e[j] = 1.0
        colj = np.zeros(g.n)
        for i in range(g.n):
            if j in set(g.row(i).tolist()):
                colj[i] = 1.0
        assert np.array_equal(product.matvec(*_csr(g), e), colj)


def test_product_integer_exact_and_invariants():
    g = B.web_graph(3000, 15.0, 22)
    x = B.integer_x(g.n, 5, 1000)
    y = product.matvec(*_csr(g), x)
    assert np.array_equal(y, product.matvec_exact(*_csr(g), x))
    indeg = np.bincount(g.col, minlength=g.n).astype(np.float64)
    assert y.sum() == float(np.dot(indeg, x))
    x2 = B.integer_x(g.n, 6, 1000)
    assert np.array_equal(product.matvec(*_csr(g), x + x2), y + product.matvec(*_csr(g), x2))


def test_proposition_reuse_equals_plain():
    """A x = A' x + w, computed by the paper's sequential algorithm."""
    g = B.web_graph(3000, 15.0, 23)
    enc = B.encode(g)
    r, plus, minus, m_prime = product.difference_form(g.rowptr, g.col, enc.refs)
    assert m_prime < g.m                           # the copying model compresses
    xi = B.integer_x(g.n, 1, 1000)
    assert np.array_equal(product.reuse_product(r, plus, minus, xi), product.matvec(*_csr(g), xi))
    x = B.uniform_x(g.n, 2)
    y0 = product.matvec_exact(*_csr(g), x)
    y1 = product.reuse_product(r, plus, minus, x)
    assert np.max(np.abs(y1 - y0) / np.maximum(np.abs(y0), 1e-300)) < 1e-12


def test_difference_form_rule():
    """Rows whose difference is not smaller than themselves keep v_i."""
    g = B.from_lists([[1, 2, 3, 4], [9], [1, 2, 3, 5]])
    r, plus, minus, mp = product.difference_form(g.rowptr, g.col, np.array([0, 1, 2], dtype=np.uint8))
    assert r.tolist() == [-1, -1, 0]              # row 1 vs row 0: |diff| = 5 >= 1 -> keep
    assert plus[2] == [5] and minus[2] == [4] and mp == 4 + 1 + 2


# -------------------------------------------------------------- pagerank
def _in_links(g):
    return g.transpose()


def _dense(g):
    A = np.zeros((g.n, g.n))
    for i in range(g.n):
        A[i, g.row(i)] = 1.0
    return A


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pagerank_dense_solve(seed):
    rng = np.random.default_rng(seed)
    n = 60
    lists = [sorted(set(rng.choice(n, rng.integers(0, 6), replace=False).tolist()) - {i}) for i in range(n)]
    lists[5] = []                                  # make sure dangling nodes exist
    g = B.from_lists(lists)
    bt = _in_links(g)
    for tele in (None, rng.dirichlet(np.ones(n))):
        pstar = pagerank.pagerank_dense(_dense(g), 0.85, tele)
        p, t, r, ok = pagerank.pagerank(bt.rowptr, bt.col, 0.85, iters=300, teleport=tele)
        assert np.max(np.abs(p - pstar)) < 1e-13
        p, t, r, ok = pagerank.pagerank(bt.rowptr, bt.col, 0.85, tol=1e-6, teleport=tele)
        assert ok and r < 1e-6
        assert np.abs(p - pstar).sum() <= 0.85 / 0.15 * r * (1 + 1e-9)


def test_pagerank_closed_forms():
    beta = 0.85
    for n in (2, 5, 17):
        for g in (B.complete_graph(n), B.cycle_graph(n)):
            bt = _in_links(g)
            p = pagerank.pagerank(bt.rowptr, bt.col, beta, iters=400)[0]
            assert np.allclose(p, 1.0 / n, rtol=0, atol=1e-14)
        c = 0
        cases = {
            "both": ((1 - beta) / n + beta) / (1 + beta),
            "in": (1 + (n - 1) * beta) / (n + (n - 1) * beta),
            "out": 1.0 / (n + beta),
        }
        for kind, pc in cases.items():
            g = B.star_graph(n, c, kind)
            bt = _in_links(g)
            p = pagerank.pagerank(bt.rowptr, bt.col, beta, iters=400)[0]
            assert abs(p[c] - pc) < 1e-13, kind
            assert np.allclose(np.delete(p, c), (1 - pc) / (n - 1), atol=1e-13)
            assert abs(pagerank.pagerank_dense(_dense(g), beta)[c] - pc) < 1e-13


def test_pagerank_degenerate():
    g = B.empty_graph(10)
    bt = _in_links(g)
    p, t, r, ok = pagerank.pagerank(bt.rowptr, bt.col, 0.85)
    assert ok and t == 1 and np.allclose(p, 0.1, atol=1e-16)
    h = B.web_graph(300, 8.0, 3).transpose()
    v = np.random.default_rng(0).dirichlet(np.ones(300))
    p, t, r, ok = pagerank.pagerank(h.rowptr, h.col, 0.0, teleport=v)
    assert np.allclose(p, v, atol=1e-16)


def test_pagerank_mass_conserved():
    g = B.web_graph(2000, 10.0, 8).transpose()
    for it in (1, 5, 30):
        p = pagerank.pagerank(g.rowptr, g.col, 0.85, iters=it)[0]
        assert abs(p.sum() - 1.0) < 1e-12


# ------------------------------------------------------------ warm-start oracle
from oracle import features as feat  # noqa: E402
from oracle import mlp  # noqa: E402


def test_bf16_rounding_values():
    # exact values stay; halfway cases go to the even neighbour; above half rounds up
    cases = [(1.0, 1.0), (-2.5, -2.5), (0.0, 0.0),
             (1 + 2 ** -8, 1.0),                       # halfway between 1 and 1 + 2^-7 (odd): to 1
             (1 + 3 * 2 ** -8, 1 + 2 ** -6),           # halfway between 1 + 2^-7 (odd) and 1 + 2^-6: up
             (1 + 2 ** -8 + 2 ** -20, 1 + 2 ** -7),    # above half: up
             (1 + 2 ** -8 - 2 ** -20, 1.0),            # below half: down
             (3.0 * 2 ** 100, 3.0 * 2 ** 100), (0.1, 0.10009765625)]
    for a, want in cases:
        assert mlp.bf16(np.array([a]))[0] == want, a


def test_gelu_identities():
    z = np.linspace(-6, 6, 49)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert np.max(np.abs(mlp.gelu(z) - mlp.gelu(-z) - z)) < 1e-14       # sigma(u) + sigma(-u) = 1
    # the sigmoid form stays within 0.021 of the exact z Phi(z) (erf from the standard library)
    zz = np.linspace(-8, 8, 3201)
    exact = np.array([t * 0.5 * (1.0 + math.erf(t / math.sqrt(2.0))) for t in zz])
    err = np.abs(mlp.gelu(zz) - exact)
    assert err.max() < 0.021 and err[np.abs(zz) > 6].max() < 3e-4
    # logistic at a point: 1 / (1 + e^-1.702) through the standard library's exp
    assert abs(mlp.gelu(np.array([1.0]))[0] - 1.0 / (1.0 + math.exp(-1.702))) < 1e-15
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(z))) < 1e-8


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(5)
    theta = mlp.init_params(3) + rng.normal(0, 0.05, mlp.NPARAM)   # nonzero biases too
    X = rng.normal(0, 1, (7, mlp.NIN))
    t = rng.normal(0, 1, 7)
    L, g = mlp.grad(theta, X, t, quantize=False)
    assert abs(L - mlp.loss(theta, X, t, quantize=False)) < 1e-15
    idx = np.concatenate([rng.choice(768, 40, replace=False), 768 + np.arange(64)[::7],
                          832 + rng.choice(4096, 60, replace=False), 4928 + np.arange(64)[::5],
                          4992 + np.arange(64)[::3], [5056]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss(theta + e, X, t, False) - mlp.loss(theta - e, X, t, False)) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(g[i])), i


def test_mlp_quantized_close_to_exact():
    rng = np.random.default_rng(6)
    theta = mlp.init_params(4)
    X = rng.normal(0, 1, (50, mlp.NIN))
    t = rng.normal(0, 1, 50)
    s_q, _ = mlp.forward(theta, X, True)
    s_e, _ = mlp.forward(mlp.pack(mlp.weights_bf16(theta)), X, False)
    assert np.max(np.abs(s_q - s_e)) < 0.05 * max(1.0, np.max(np.abs(s_e)))
    _, gq = mlp.grad(theta, X, t, True)
    _, ge = mlp.grad(mlp.pack(mlp.weights_bf16(theta)), X, t, False)
    assert np.linalg.norm(gq - ge) < 0.05 * np.linalg.norm(ge)


def _bf16_spacing(a):
    """Distance between consecutive BF16 values around |a| (8 significant bits)."""
    return 2.0 ** (np.floor(np.log2(np.abs(a))) - 7)


def test_mlp_inputs_enter_as_bf16():
    # the first product takes bf(x): inputs that round to the same BF16 value
    # give bit-identical outputs and gradients, while the unrounded network
    # tells them apart
    rng = np.random.default_rng(8)
    theta = mlp.init_params(5) + rng.normal(0, 0.05, mlp.NPARAM)
    X = mlp.bf16(rng.normal(0, 1.5, (64, mlp.NIN)))
    assert np.all(X != 0)
    Xp = X + 0.25 * _bf16_spacing(X) * rng.choice([-1.0, 1.0], X.shape)   # a quarter step: same BF16 value
    t = rng.normal(0, 1, 64)
    s0, _ = mlp.forward(theta, X)
    s1, _ = mlp.forward(theta, Xp)
    assert np.array_equal(s0, s1)
    assert np.array_equal(mlp.grad(theta, X, t)[1], mlp.grad(theta, Xp, t)[1])
    assert not np.array_equal(mlp.forward(theta, X, False)[0], mlp.forward(theta, Xp, False)[0])


def test_mlp_weights_enter_as_bf16():
    # the network uses BF16 copies of W1, W2 and w3: master weights moved
    # within their BF16 cell give the same outputs; biases are used as given
    rng = np.random.default_rng(9)
    theta = mlp.init_params(7) + rng.normal(0, 0.05, mlp.NPARAM)
    p = mlp.unpack(theta)
    for k in mlp.WEIGHTS:
        p[k] = mlp.bf16(p[k])
        p[k][p[k] == 0] = 2.0 ** -20
    q = {k: v.copy() for k, v in p.items()}
    for k in mlp.WEIGHTS:
        q[k] = p[k] + 0.25 * _bf16_spacing(p[k]) * rng.choice([-1.0, 1.0], p[k].shape)
    X = rng.normal(0, 1.5, (32, mlp.NIN))
    assert np.array_equal(mlp.forward(mlp.pack(p), X)[0], mlp.forward(mlp.pack(q), X)[0])
    q["b2"] = p["b2"] + 0.25 * _bf16_spacing(p["b2"] + 1e-3)
    assert not np.array_equal(mlp.forward(mlp.pack(p), X)[0], mlp.forward(mlp.pack(q), X)[0])


def _saturated_theta(seed):
    """A network whose first layer sits at z1 = 8 + (small input term): every
    h1 = gelu(z1) lies in [7.98, 8.02] and rounds to the BF16 value 8.0
    (spacing 1/32 below 8, 1/16 above)."""
    rng = np.random.default_rng(seed)
    p = mlp.unpack(mlp.init_params(seed) + rng.normal(0, 0.05, mlp.NPARAM))
    p["W1"] = 2.0 ** -10 * np.where(rng.random((mlp.NH, mlp.NIN)) < 0.5, -1.0, 1.0)
    p["b1"] = np.full(mlp.NH, 8.0)
    return mlp.pack(p)


def test_mlp_hidden_layer_enters_as_bf16():
    # the second product takes bf(h1): with every h1 rounding to 8.0 the output
    # is one value for all rows, although z1 and h1 differ from row to row
    theta = _saturated_theta(10)
    X = np.random.default_rng(11).uniform(-1, 1, (40, mlp.NIN))
    s, c = mlp.forward(theta, X)
    assert np.ptp(c["z1"]) > 1e-3
    assert np.all(c["h1q"] == 8.0)
    assert np.all(s == s[0])
    assert np.ptp(mlp.forward(theta, X, False)[0]) > 1e-6


def test_mlp_backward_operands_are_bf16():
    # one row: the weight gradients are products of BF16-rounded deltas with
    # the layer inputs, the bias gradients the unrounded deltas.  With h1q = 8
    # (saturated first layer): dW2[i, j] = 8 bf(db2[i]).  With a one-hot input
    # x = e_3: dW1[:, 3] = bf(db1) and the other columns are zero.
    theta = _saturated_theta(12)
    rng = np.random.default_rng(13)
    x = rng.uniform(-1, 1, (1, mlp.NIN))
    _, g = mlp.grad(theta, x, np.array([-3.0]))
    d = mlp.unpack(g)
    assert np.any(mlp.bf16(d["b2"]) != d["b2"])
    assert np.array_equal(d["W2"], 8.0 * np.repeat(mlp.bf16(d["b2"])[:, None], mlp.NH, axis=1))
    theta = mlp.init_params(14) + rng.normal(0, 0.05, mlp.NPARAM)
    e3 = np.zeros((1, mlp.NIN))
    e3[0, 3] = 1.0
    _, g = mlp.grad(theta, e3, np.array([2.0]))
    d = mlp.unpack(g)
    assert np.any(mlp.bf16(d["b1"]) != d["b1"])
    assert np.array_equal(d["W1"][:, 3], mlp.bf16(d["b1"]))
    assert np.all(np.delete(d["W1"], 3, axis=1) == 0.0)


def test_bvinputs_init_equals_oracle_init():
    # the benchmark's seeded starting parameters (bvinputs) and the oracle's
    # own copy of the same recipe agree value for value
    for seed in (0, 4000):
        a = B.mlp_init_params(seed).astype(np.float64)
        b = mlp.init_params(seed)
        assert a.shape == (mlp.NPARAM,) and np.array_equal(a, b)


def test_adam_first_step_closed_form():
    # after one step mhat = g and vhat = g^2, so theta moves by lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th0 = np.array([1.0, 2.0, 3.0, 4.0])
    opt = mlp.Adam(4, lr=0.01)
    th1 = opt.step(th0, g)
    assert np.allclose(th1, th0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_row_stats_match_lists():
    g = B.web_graph(3000, 12.0, 21)
    enc = B.encode(g)
    rowptr, col, refs, hdr, st = bvdecode.decode(enc.data, with_stats=True)
    want = feat.row_stats_from_lists(rowptr, col, refs, hdr["Lmin"])
    assert np.array_equal(st, want)
    assert st[:, 0].max() <= hdr["R"] and st[:, 2].sum() > 0 and st[:, 1].sum() > 0


def test_structural_closed_forms_star():
    # loaded rows: row 0 lists every other node (all of them link to 0); other rows empty
    n = 40
    g = B.from_lists([list(range(1, n))] + [[] for _ in range(n - 1)])
    rowptr, col, refs, hdr, st = bvdecode.decode(B.encode(g).data, with_stats=True)
    F = feat.structural(rowptr, col, st, hdr["R"])
    assert F.shape == (n, 8)
    assert np.allclose(F[0, :4], [math.log1p(n - 1), 0.0, 0.0, 1.0])
    assert np.allclose(F[1:, :4], [0.0, math.log(2.0), 0.0, 0.0])
    assert np.allclose(F[0, 4:6], [math.log(2.0), 0.0])          # one interval 1..n-1, no residual
    # in-neighbours of 0 have out-degree 1 and in-degree 0
    assert np.allclose(F[0, 6:8], [math.log(2.0), 0.0])
    assert np.allclose(F[1:, 4:8], 0.0)


def _cycle2_iterates(beta, s0, ks):
    """Iterates of the oracle power method on the 2-cycle from s0."""
    g = B.from_lists([[1], [0]])
    return [pagerank.pagerank(g.rowptr, g.col, beta, start=s0, iters=k)[0] if k else np.array(s0) for k in ks]


def test_trajectory_and_target_single_mode():
    # On the 2-cycle the error of the power method is one eigenmode: e_k =
    # (-beta)^k e_0, p* = (1/2, 1/2).  Then p_K - p_{K-1} = e_K (1 + 1/beta),
    # so the remaining correction p* - p_K = -e_K is the last step times
    # beta / (1 + beta) with a minus sign, and each older step is the newer one
    # divided by -beta.
    beta, K = 0.85, 6
    pK3, pK2, pK1, pK = _cycle2_iterates(beta, [0.9, 0.1], [K - 3, K - 2, K - 1, K])
    Tr, delta = feat.trajectory(pK, pK1, pK2, pK3)
    e = 0.4 * beta ** K
    assert abs(delta - 2 * e * (1 + 1 / beta)) < 1e-15
    assert np.allclose(Tr[:, 0], np.log(2 * pK), rtol=0, atol=1e-15)
    assert np.allclose(Tr[:, 1], [1.0, -1.0], rtol=0, atol=1e-12)      # K even: p_K above 1/2 at node 0
    assert np.allclose(Tr[:, 2], Tr[:, 1] / -beta, rtol=0, atol=1e-12)
    assert np.allclose(Tr[:, 3], Tr[:, 1] / beta ** 2, rtol=0, atol=1e-12)
    t = feat.target([0.5, 0.5], pK, delta)
    assert np.allclose(t, -Tr[:, 1] * beta / (1 + beta), rtol=0, atol=1e-12)


def test_restart_vector_perfect_and_floor():
    rng = np.random.default_rng(5)
    ps = rng.uniform(0.5, 1.5, 30)
    ps /= ps.sum()
    pK = ps * rng.uniform(0.9, 1.1, 30)
    pK /= pK.sum()
    delta = 0.037
    # the target as prediction restores p* exactly
    assert np.allclose(feat.restart_vector(pK, feat.target(ps, pK, delta), delta), ps, rtol=0, atol=1e-16)
    # zero prediction keeps p_K; a very negative one floors every entry, which normalises back to p_K
    assert np.allclose(feat.restart_vector(pK, np.zeros(30), delta), pK, rtol=0, atol=1e-16)
    assert np.allclose(feat.restart_vector(pK, np.full(30, -1e12), delta), pK, rtol=0, atol=1e-16)
    # partial floor: entries below p_K / 1000 are raised to it
    s = np.zeros(30)
    s[3] = -1e12
    q = np.maximum(pK + s * delta / 30, pK / 1000)
    assert q[3] == pK[3] / 1000
    assert np.allclose(feat.restart_vector(pK, s, delta), q / q.sum(), rtol=0, atol=1e-16)


def _small_web():
    g = B.web_graph(3000, 10.0, 17)
    rowptr, col, refs, hdr, st = bvdecode.decode(B.encode(g).data, with_stats=True)
    return rowptr, col, feat.structural(rowptr, col, st, hdr["R"])


def test_restarted_zero_and_rejected_predictions_follow_plain_method():
    from oracle import restart
    rowptr, col, Fs = _small_web()
    p0, t0, r0, ok0 = pagerank.pagerank(rowptr, col, 0.85, tol=1e-8)
    # zero prediction: each restart is p_K itself (up to the sum's rounding), accepted
    p, t, r, ok, info = restart.pagerank_restarted(rowptr, col, lambda F: np.zeros(len(F)), Fs, tol=1e-8)
    assert ok and t == t0 and info["accepted"] == 2 and info["rejected"] == 0
    assert np.max(np.abs(p - p0)) < 1e-15
    # a wild prediction is rejected once, costs one product, the rest is the plain run
    p, t, r, ok, info = restart.pagerank_restarted(rowptr, col, lambda F: np.full(len(F), 1e9), Fs, tol=1e-8)
    assert ok and t == t0 and info == dict(products=t0 + 1, accepted=0, rejected=1)
    assert np.array_equal(p, p0)


def test_restarted_perfect_prediction_converges_after_restart():
    from oracle import restart
    rowptr, col, Fs = _small_web()
    n = len(rowptr) - 1
    ps = pagerank.pagerank(rowptr, col, 0.85, tol=1e-15, max_iter=5000)[0]
    K = 8
    pK = pagerank.pagerank(rowptr, col, 0.85, iters=K)[0]
    pK1 = pagerank.pagerank(rowptr, col, 0.85, iters=K - 1)[0]
    delta = np.abs(pK - pK1).sum()
    p, t, r, ok, info = restart.pagerank_restarted(rowptr, col, lambda F: feat.target(ps, pK, delta), Fs,
                                                   tol=1e-8, K=K)
    assert ok and t == K + 1 and info == dict(products=K + 1, accepted=1, rejected=0)
    assert np.abs(p - ps).sum() < 1e-12


def test_restarted_matches_dense_fixed_point():
    from oracle import restart
    # a noisy predictor still ends at the unique fixed point within the plain method's bound
    g = B.web_graph(400, 6.0, 3)
    rowptr, col, refs, hdr, st = bvdecode.decode(B.encode(g).data, with_stats=True)
    Fs = feat.structural(rowptr, col, st, hdr["R"])
    n = len(rowptr) - 1
    A = np.zeros((n, n))
    for v in range(n):
        A[col[int(rowptr[v]):int(rowptr[v + 1])], v] = 1.0      # row v lists u -> v
    exact = pagerank.pagerank_dense(A, 0.85)
    rng = np.random.default_rng(9)
    p, t, r, ok, info = restart.pagerank_restarted(rowptr, col, lambda F: F[:, 9] + rng.normal(0, 0.5, len(F)),
                                                   Fs, tol=1e-9, K=5)
    assert ok and abs(p.sum() - 1.0) < 1e-12
    assert np.abs(p - exact).sum() <= r * 0.85 / 0.15 + 1e-13


def test_restart_kept_only_under_the_contraction_bound():
    """The probe keeps a restart only when its step is below beta times the
    step it replaces: beta bounds the plain method's L1 contraction, so a kept
    restart never converges slower than not restarting.  The probe's ratio
    rho = ||q - p'||_1 / ||p_K - p_{K-1}||_1 is computed here through the
    plain power method (started from p_K and from the restart vector p') and
    the pinned restart-vector function; restarts with rho below beta, between
    beta and 1, and between 1 and 2 must be kept, dropped and dropped."""
    from oracle import restart
    rowptr, col, Fs = _small_web()
    beta, K = 0.85, 10
    ps = pagerank.pagerank(rowptr, col, beta, tol=1e-15, max_iter=5000)[0]
    pK = pagerank.pagerank(rowptr, col, beta, iters=K)[0]
    pK1 = pagerank.pagerank(rowptr, col, beta, iters=K - 1)[0]
    delta = np.abs(pK - pK1).sum()
    t_true = feat.target(ps, pK, delta)

    def rho(c):
        q0 = feat.restart_vector(pK, c * t_true, delta)
        r = pagerank.pagerank(rowptr, col, beta, start=q0, iters=1)[2]
        return r / delta

    cs = np.linspace(-4.0, 6.0, 201)
    rs = np.array([rho(c) for c in cs])
    windows = {"keep": (0.0, 0.97 * beta), "drop_beta": (1.03 * beta, 0.97), "drop_one": (1.03, 1.97)}
    for name, (lo, hi) in windows.items():
        inside = np.flatnonzero((rs > lo) & (rs < hi))
        assert inside.size, name
        c = float(cs[inside[0]])
        p, t, r, ok, info = restart.pagerank_restarted(rowptr, col, lambda F: c * t_true, Fs, beta=beta, tol=1e-8,
                                                       K=K, max_restarts=1)
        want = (1, 0) if name == "keep" else (0, 1)
        assert (info["accepted"], info["rejected"]) == want, (name, c, rs[inside[0]])


def test_structural_depth_input_is_normalised():
    """Input 2 is the row's reference-chain depth over R: on a copying-model
    graph whose chains reach the bound R it takes the values 0, 1/R, ..., 1,
    reaches 1, and is 0 exactly on rows coded without a reference."""
    g = B.web_graph(3000, 10.0, 17)
    for R in (1, 3, 5):
        rowptr, col, refs, hdr, st = bvdecode.decode(B.encode(g, R=R).data, with_stats=True)
        F = feat.structural(rowptr, col, st, hdr["R"])
        k = F[:, 2] * R
        assert np.allclose(k, np.round(k), atol=1e-12) and k.min() == 0.0 and k.max() == R
        assert np.array_equal(F[:, 2] == 0.0, refs == 0)


# ------------------------------------------------------------ biclique format
from oracle import biclique as bic  # noqa: E402


def _one_biclique(n, S, C, res=None):
    """A decomposition of one biclique S x C plus the given residual lists."""
    res = res or [[] for _ in range(n)]
    rp = np.zeros(n + 1, dtype=np.uint64)
    rp[1:] = np.cumsum([len(r) for r in res])
    cat = [j for r in res for j in sorted(r)]
    return B.Bicliques(n, np.array([0, len(S)], np.uint64), np.asarray(S, np.uint32),
                       np.array([0, len(C)], np.uint64), np.asarray(C, np.uint32), rp,
                       np.asarray(cat, np.uint32))


def test_biclique_closed_form_complete_bipartite():
    """K_{|S|,|C|}: y_i = sum_{j in C} x_j for i in S and 0 elsewhere; with
    residual edges added, each row also gains its residual targets' x."""
    n = 40
    S, C = [3, 4, 9, 20, 21], [0, 5, 6, 7, 30, 39]
    x = B.integer_x(n, 1, 1000)
    want = np.zeros(n)
    want[S] = x[C].sum()
    b = _one_biclique(n, S, C)
    assert np.array_equal(bic.paper_product(b, x), want)
    rp, col = bic.lists(b)
    assert np.array_equal(product.matvec(rp, col, x), want)
    res = [[] for _ in range(n)]
    res[3], res[10], res[39] = [1, 2], [0], [38]
    b2 = _one_biclique(n, S, C, res)
    want2 = want.copy()
    want2[3] += x[1] + x[2]
    want2[10] += x[0]
    want2[39] += x[38]
    assert np.array_equal(bic.paper_product(b2, x), want2)
    assert np.array_equal(product.matvec(*bic.lists(b2), x), want2)


def test_biclique_dense_bruteforce_and_lists():
    """A planted decomposition: its dense matrix is 0/1 (a partition of the
    edges) and equals the generator's graph; the paper's two-step product and
    the per-row sums over the written-out lists equal A @ x."""
    for seed in (0, 1, 2):
        g, b = B.planted_bicliques(300, 40, seed=seed)
        A = bic.dense(b)
        assert set(np.unique(A).tolist()) <= {0.0, 1.0}
        rp, col = bic.lists(b)
        assert np.array_equal(rp, g.rowptr) and np.array_equal(col, g.col)
        Ag = np.zeros_like(A)
        for i in range(g.n):
            Ag[i, g.row(i).astype(np.int64)] = 1.0
        assert np.array_equal(A, Ag)
        x = B.uniform_x(g.n, 7 + seed)
        ref = A @ x
        for y in (bic.paper_product(b, x), product.matvec(rp, col, x)):
            assert np.max(np.abs(y - ref) / np.maximum(np.abs(ref), 1e-300)) < 1e-14
        xi = B.integer_x(g.n, 3, 1000)
        assert np.array_equal(bic.paper_product(b, xi), A @ xi)


def test_biclique_indicator_and_ones():
    """x = 1 gives the out-degrees; x = e_j gives column j of A, exactly."""
    g, b = B.planted_bicliques(200, 30, seed=5)
    deg = np.diff(g.rowptr.astype(np.int64)).astype(np.float64)
    assert np.array_equal(bic.paper_product(b, np.ones(g.n)), deg)
    A = bic.dense(b)
    for j in (0, 17, 199):
        e = np.zeros(g.n)
        e[j] = 1.0
        assert np.array_equal(bic.paper_product(b, e), A[:, j])


def test_biclique_miner_partitions_the_edges():
    """The miner's decomposition of a web-like graph stands for exactly that
    graph, every biclique is one (each of S_r's rows lists all of C_r), and
    it stores fewer ids than edges."""
    g = B.web_graph(5000, 12.0, 21)
    b = B.biclique_mine(g)
    rp, col = bic.lists(b)
    assert np.array_equal(rp, g.rowptr) and np.array_equal(col, g.col)
    for r in range(0, b.nbic, 97):
        S, C = b.biclique(r)
        assert S.size >= 2 and C.size >= 2
        for i in S.tolist():
            assert np.all(np.isin(C, g.row(i)))
    assert b.words() < g.m
    xi = B.integer_x(g.n, 4, 1000)
    assert np.array_equal(bic.paper_product(b, xi), product.matvec(g.rowptr, g.col, xi))


# --------------------------------------------------------------- left product
def test_left_product_dense_and_closed_forms():
    """y = x A against numpy's x @ A on the dense matrix; closed forms: the
    complete graph gives sum(x) - x_j, the out-star (centre -> leaves) gives
    x_c on every leaf and 0 at the centre, the in-star gives the leaves' sum
    at the centre, the path i -> i+1 gives x_{j-1}; x = 1 gives the
    in-degrees exactly."""
    for seed in (0, 1):
        g = B.web_graph(400, 8.0, 30 + seed)
        A = np.zeros((g.n, g.n))
        for i in range(g.n):
            A[i, g.row(i).astype(np.int64)] = 1.0
        x = B.uniform_x(g.n, 5 + seed)
        ref = x @ A
        for y in (product.left_matvec(g.rowptr, g.col, x), product.left_matvec_exact(g.rowptr, g.col, x)):
            assert np.max(np.abs(y - ref) / np.maximum(np.abs(ref), 1e-300)) < 1e-14
        indeg = np.bincount(g.col.astype(np.int64), minlength=g.n).astype(np.float64)
        assert np.array_equal(product.left_matvec(g.rowptr, g.col, np.ones(g.n)), indeg)
    n = 12
    x = B.integer_x(n, 2, 1000)
    g = B.complete_graph(n)
    assert np.array_equal(product.left_matvec(g.rowptr, g.col, x), x.sum() - x)
    g = B.star_graph(n, 0, "out")
    want = np.full(n, x[0])
    want[0] = 0.0
    assert np.array_equal(product.left_matvec(g.rowptr, g.col, x), want)
    g = B.star_graph(n, 0, "in")
    want = np.zeros(n)
    want[0] = x[1:].sum()
    assert np.array_equal(product.left_matvec(g.rowptr, g.col, x), want)
    g = B.path_graph(n)
    want = np.concatenate([[0.0], x[:-1]])
    assert np.array_equal(product.left_matvec(g.rowptr, g.col, x), want)


def test_left_product_through_the_difference_form():
    """x A = c A' with c = x (I - R)^{-1}: exact for integer x, within
    rounding otherwise; equals x A of the transposed lists' product."""
    g = B.web_graph(3000, 12.0, 33)
    enc = B.encode(g)
    rowptr, col, refs, _ = bvdecode.decode(enc.data)
    r, plus, minus, _ = product.difference_form(rowptr, col, refs)
    xi = B.integer_x(g.n, 3, 1000)
    want = product.left_matvec(g.rowptr, g.col, xi)
    assert np.array_equal(product.left_reuse_product(r, plus, minus, xi), want)
    gt = g.transpose()
    assert np.array_equal(product.matvec(gt.rowptr, gt.col, xi), want)
    x = B.uniform_x(g.n, 4)
    ex = product.left_matvec_exact(g.rowptr, g.col, x)
    nz = ex != 0
    assert np.max(np.abs(product.left_reuse_product(r, plus, minus, x)[nz] - ex[nz]) / ex[nz]) < 1e-12
