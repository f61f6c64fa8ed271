"""Learned warm start on the device against the CPU oracle: features, the MLP
forward and gradient (MFMA kernels), Adam, the start vector, and end to end
PageRank from a trained network with the fallback check."""
import numpy as np
import pytest
import torch

import bvinputs as B
from oracle import bvdecode, mlp, pagerank
from oracle import features as feat

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def P():
    import paper_1708_07271_amd as P
    return P


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _theta(seed):
    rng = np.random.default_rng(seed)
    return (mlp.init_params(seed) + rng.normal(0, 0.05, mlp.NPARAM)).astype(np.float32).astype(np.float64)


def test_features_match_oracle(P):
    g = B.web_graph(20_000, 15.0, 31)
    enc = B.encode(g)
    G = P.bvmv_load(enc.data)
    F = torch.empty(g.n, P.NFEAT, device=DEV)
    P.bvmv_features(G, F)
    torch.cuda.synchronize()
    rowptr, col, refs, hdr, st = bvdecode.decode(enc.data, with_stats=True)
    Fo = feat.features(rowptr, col, st, hdr["R"])
    Fg = F.cpu().numpy().astype(np.float64)
    # integer-derived features agree to float32 rounding of the logarithm; the
    # three product features to the product's FP32 tolerance
    assert np.max(np.abs(Fg[:, :8] - Fo[:, :8])) < 2e-6
    assert np.max(np.abs(Fg[:, 8:11] - Fo[:, 8:11]) / (1 + np.abs(Fo[:, 8:11]))) < 2e-5
    assert np.max(np.abs(Fg[:, 11] - Fo[:, 11])) < 2e-6


@pytest.mark.parametrize("n", [32, 1000, 4099])
def test_mlp_forward_matches_oracle(P, n):
    theta = _theta(11)
    X = np.random.default_rng(n).normal(0, 1.5, (n, mlp.NIN))
    m = P.bvmv_mlp_create(theta)
    s = torch.empty(n, device=DEV)
    P.bvmv_mlp_forward(m, _dev(X), s)
    torch.cuda.synchronize()
    so, _ = mlp.forward(theta, X.astype(np.float32), quantize=True)
    sg = s.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(sg - so) / (1 + np.abs(so))) < 1e-3
    # deterministic
    s2 = torch.empty(n, device=DEV)
    P.bvmv_mlp_forward(m, _dev(X), s2)
    assert torch.equal(s, s2)


@pytest.mark.parametrize("n", [32, 777, 5000])
def test_mlp_gradient_matches_oracle(P, n):
    theta = _theta(12)
    rng = np.random.default_rng(100 + n)
    X = rng.normal(0, 1.5, (n, mlp.NIN)).astype(np.float32)
    t = rng.normal(0, 1, n).astype(np.float32)
    m = P.bvmv_mlp_create(theta)
    gd = torch.empty(P.MLP_PARAMS + 1, device=DEV)
    P.bvmv_mlp_gradient(m, _dev(X), _dev(t), gd)
    torch.cuda.synchronize()
    gg = gd.cpu().numpy().astype(np.float64)
    L, go = mlp.grad(theta, X, t, quantize=True)
    assert abs(gg[-1] - L) < 1e-4 * L
    offs = np.cumsum([0] + [int(np.prod(sh)) for _, sh in mlp.SIZES])
    for (name, _), a, b in zip(mlp.SIZES, offs[:-1], offs[1:]):
        ref = go[a:b]
        err = np.linalg.norm(gg[a:b] - ref) / max(np.linalg.norm(ref), 1e-12)
        assert err < 1e-2, (name, err)
    # deterministic
    gd2 = torch.empty_like(gd)
    P.bvmv_mlp_gradient(m, _dev(X), _dev(t), gd2)
    assert torch.equal(gd, gd2)


def test_adam_step_matches_oracle(P):
    theta = _theta(13)
    rng = np.random.default_rng(7)
    n = 3000
    X, t = _dev(rng.normal(0, 1, (n, mlp.NIN))), _dev(rng.normal(0, 1, n))
    m = P.bvmv_mlp_create(theta)
    opt = mlp.Adam(mlp.NPARAM, lr=1e-2)
    th = theta.copy()
    gd = torch.empty(P.MLP_PARAMS + 1, device=DEV)
    for _ in range(3):
        P.bvmv_mlp_gradient(m, X, t, gd)
        g = gd.cpu().numpy().astype(np.float64)[:-1]
        P.bvmv_mlp_train_step(m, X, t, 1e-2)
        th = opt.step(th, g)
        got = P.bvmv_mlp_params(m).astype(np.float64)
        assert np.max(np.abs(got - th)) < 2e-6
        th = got  # follow the device's FP32 state
    # the BF16 copies follow the master weights: forward equals the oracle on them
    s = torch.empty(n, device=DEV)
    P.bvmv_mlp_forward(m, X, s)
    so, _ = mlp.forward(th, X.cpu().numpy(), quantize=True)
    assert np.max(np.abs(s.cpu().numpy() - so) / (1 + np.abs(so))) < 1e-3


def _train(P, graphs, steps, seed=1):
    """Train on (features, log(n p*)) of the given loaded graphs."""
    Fs, Ts = [], []
    for G, n in graphs:
        F = torch.empty(n, P.NFEAT, device=DEV)
        P.bvmv_features(G, F)
        p = torch.empty(n, device=DEV)
        P.bvmv_pagerank(G, p)
        Fs.append(F)
        Ts.append(torch.log(p * n))
    F = torch.cat(Fs)
    T = torch.cat(Ts).contiguous()
    m = P.bvmv_mlp_create(mlp.init_params(seed))
    loss = torch.empty(1, device=DEV)
    gen = torch.Generator(device=DEV).manual_seed(seed)
    first = None
    for it in range(steps):
        idx = torch.randint(0, F.shape[0], (8192,), device=DEV, generator=gen)
        P.bvmv_mlp_train_step(m, F[idx].contiguous(), T[idx].contiguous(), 3e-3, loss)
        if it == 0:
            first = float(loss.item())
    return m, first, float(loss.item())


def test_warm_start_end_to_end(P):
    train = [B.web_graph(n, 15.0, 40 + i) for i, n in enumerate((30_000, 50_000, 40_000))]
    Gs = [(P.bvmv_load(B.encode(g).data), g.n) for g in train]
    m, l0, l1 = _train(P, Gs, 400)
    assert l1 < 0.5 * l0
    g = B.web_graph(60_000, 15.0, 77)
    G = P.bvmv_load(B.encode(g).data)
    p0 = torch.empty(g.n, device=DEV)
    P.bvmv_warm_start(G, m, p0)
    torch.cuda.synchronize()
    assert abs(float(p0.double().sum()) - 1.0) < 1e-5 and float(p0.min()) > 0
    pu = torch.empty(g.n, device=DEV)
    (iu, oku, ru), = P.bvmv_pagerank(G, pu)
    pw = torch.empty(g.n, device=DEV)
    rw = P.bvmv_pagerank_detail(G, pw, start=p0, fallback_check=1)[0]
    assert oku and rw["converged"] and rw["used_start"] == 1
    assert rw["iters"] < iu
    # same fixed point within the L1 contraction bound (beta / (1 - beta)) * tol, twice
    assert float((pw.double() - pu.double()).abs().sum()) < 2 * (0.85 / 0.15) * 1e-6 + 1e-5
    # against the oracle started from the same warm vector, iteration-matched
    p_ref = pagerank.pagerank(g.rowptr, g.col, 0.85, start=p0.cpu().numpy().astype(np.float64),
                              iters=rw["iters"])[0]
    assert np.max(np.abs(pw.cpu().numpy() - p_ref) / p_ref) < 1e-5
    # a bad start is rejected by the fallback check
    bad = torch.zeros(g.n, device=DEV)
    bad[0] = 1.0
    rb = P.bvmv_pagerank_detail(G, pw, start=bad, fallback_check=1)[0]
    assert rb["used_start"] == 0 and rb["iters"] == iu
