"""Learned warm restarts on the device against the CPU oracle: structural
inputs, restart samples (trajectory inputs and targets), the MLP forward and
gradient (MFMA kernels), Adam, and PageRank with restarts: exact agreement
with the plain method for a zero network and for a rejected restart, parity
with the oracle's restarted run, and the gain of a trained network."""
import numpy as np
import pytest
import torch

import bvinputs as B
from oracle import bvdecode, mlp, pagerank, restart
from oracle import features as feat

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
F64, F32C = 0, 2


@pytest.fixture(scope="module")
def P():
    import paper_1708_07271_amd as P
    return P


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _theta(seed):
    rng = np.random.default_rng(seed)
    return (mlp.init_params(seed) + rng.normal(0, 0.05, mlp.NPARAM)).astype(np.float32).astype(np.float64)


def _decoded(enc):
    rowptr, col, refs, hdr, st = bvdecode.decode(enc.data, with_stats=True)
    return rowptr, col, feat.structural(rowptr, col, st, hdr["R"])


def test_features_match_oracle(P):
    g = B.web_graph(20_000, 15.0, 31)
    enc = B.encode(g)
    G = P.bvmv_load(enc.data)
    F = torch.full((g.n, P.NFEAT), 7.0, device=DEV)
    P.bvmv_features(G, F)
    torch.cuda.synchronize()
    _, _, Fo = _decoded(enc)
    Fg = F.cpu().numpy().astype(np.float64)
    # integer-derived inputs agree to float32 rounding of the logarithm; the two
    # product inputs to the product's FP32 tolerance; columns 8..11 untouched
    assert np.max(np.abs(Fg[:, :6] - Fo[:, :6])) < 2e-6
    assert np.max(np.abs(Fg[:, 6:8] - Fo[:, 6:8]) / (1 + np.abs(Fo[:, 6:8]))) < 2e-5
    assert np.all(Fg[:, 8:] == 7.0)


@pytest.mark.parametrize("prec,K", [(F64, 6), (F64, 7), (F64, 10), (F32C, 10)])
def test_restart_sample_matches_oracle(P, prec, K):
    g = B.web_graph(30_000, 15.0, 32)
    enc = B.encode(g)
    G = P.bvmv_load(enc.data)
    rowptr, col, Fs = _decoded(enc)
    its = [pagerank.pagerank(rowptr, col, 0.85, iters=k)[0] for k in (K - 3, K - 2, K - 1, K)]
    Tr, delta = feat.trajectory(its[3], its[2], its[1], its[0])
    ps = pagerank.pagerank(rowptr, col, 0.85, tol=1e-13, max_iter=5000)[0]
    dt = torch.float64 if prec == F64 else torch.float32
    F = torch.empty(g.n, P.NFEAT, device=DEV)
    T = torch.empty(g.n, device=DEV)
    d = P.bvmv_restart_sample(G, K, F, T, torch.from_numpy(ps).to(dt).to(DEV), prec=prec)
    torch.cuda.synchronize()
    Fg = F.cpu().numpy().astype(np.float64)
    Tg = T.cpu().numpy().astype(np.float64)
    To = feat.target(ps, its[3], delta)
    if prec == F64:
        assert abs(d - delta) < 1e-12 * delta
        assert np.max(np.abs(Fg[:, 8:] - Tr) / (1 + np.abs(Tr))) < 2e-6    # FP32 storage of the inputs
        assert np.max(np.abs(Tg - To) / (1 + np.abs(To))) < 2e-6
    else:
        # FP32 iterates: delta to 1e-5, the step differences to what FP32
        # rounding of p (~6e-8 relative) leaves of a step that is ~1e-3 of p
        assert abs(d - delta) < 1e-5 * delta
        assert np.max(np.abs(Fg[:, 8] - Tr[:, 0])) < 1e-5
        assert np.max(np.abs(Fg[:, 9:] - Tr[:, 1:]) / (1 + np.abs(Tr[:, 1:]))) < 5e-3
        assert np.max(np.abs(Tg - To) / (1 + np.abs(To))) < 5e-3
    assert np.max(np.abs(Fg[:, :6] - Fs[:, :6])) < 2e-6


def test_restart_sample_rejects_converged(P):
    # uniform is the fixed point of the complete graph: converged at once
    G = P.bvmv_load(B.encode(B.complete_graph(50)).data)
    F = torch.empty(50, P.NFEAT, device=DEV)
    with pytest.raises(P.BvmvError):
        P.bvmv_restart_sample(G, 5, F)

def _forward_bound(theta, X):
    """Per-row bound on |s_device - s_oracle| for the network's forward pass,
    from the oracle's own intermediates, and the rows where a BF16 rounding
    of h1 may go the other way on the device.

    The device takes the same BF16 operands (x, W1, W2, w3 exactly as here),
    forms the products exactly and sums them in FP32 (12 and 64 terms), and
    evaluates GELU in FP32 with a hardware exponential and reciprocal.  An
    FP32 sum of k terms errs by at most k u sum|terms| (u = 2^-24), GELU by a
    few u relative, so, with S = 1 + sum_k |w3_k| (|h2_k| + 1.1 (sum_j
    |W2_kj h1q_j| + |b2_k|)) the sum of magnitudes the output is built from,
    |ds| <= 64 u S (1 + 1.1) + 12 u-terms < 1e-5 S, as long as every bf(h1)
    is the oracle's.  h1 itself comes with an FP32 error below e_j = 2 (4 u
    |h1_j| + |gelu'(z1_j)| 13 u (sum_i |W1_ji x_i| + |b1_j|)): twice the worst
    case of its 13-term sum carried through GELU, plus GELU's own few
    roundings; a value of h1 closer than e_j to a BF16 rounding boundary may round
    the other way, which moves s by at most |ds/dh1q_j| times one BF16 step.
    Returns (s, FP32 bound, bound with the flips, near-tie rows)."""
    s, c = mlp.forward(theta, X)
    p = c["p"]
    u = 2.0 ** -24
    z2_mag = np.abs(c["h1q"]) @ np.abs(p["W2"]).T + np.abs(p["b2"])
    S = 1.0 + (np.abs(c["h2"]) + 1.1 * z2_mag) @ np.abs(p["w3"]) + abs(p["b3"][0])
    bound = 4 * 64 * u * S
    h1 = mlp.gelu(c["z1"])
    z1_mag = np.abs(c["xq"]) @ np.abs(p["W1"]).T + np.abs(p["b1"])
    e = 2.0 * (4 * u * np.abs(h1) + np.abs(mlp.gelu_grad(c["z1"])) * 13 * u * z1_mag)
    near = (mlp.bf16(h1 + e) != c["h1q"]) | (mlp.bf16(h1 - e) != c["h1q"])
    # ds/dh1q_j = sum_k w3_k gelu'(z2_k) W2_kj; one BF16 step of h1 at j
    ds = (mlp.gelu_grad(c["z2"]) * p["w3"]) @ p["W2"]
    step = 2.0 ** (np.floor(np.log2(np.maximum(np.abs(h1) + e, 1e-30))) - 7)
    flip = np.sum(np.where(near, np.abs(ds) * step, 0.0), axis=1)
    return s, bound, bound + flip, near.any(axis=1)


@pytest.mark.parametrize("n", [32, 1000, 4099])
def test_mlp_forward_matches_oracle(P, n):
    theta = _theta(11)
    X = np.random.default_rng(n).normal(0, 1.5, (n, mlp.NIN)).astype(np.float32)
    m = P.bvmv_mlp_create(theta)
    s = torch.empty(n, device=DEV)
    P.bvmv_mlp_forward(m, _dev(X), s)
    torch.cuda.synchronize()
    so, b32, bound, near = _forward_bound(theta, X)
    sg = s.cpu().numpy().astype(np.float64)
    err = np.abs(sg - so)
    # every row within its bound: FP32 sums and GELU, plus one BF16 step for
    # each h1 next to a rounding boundary; rows with no such h1 within the
    # FP32 part alone; and a rounding that does go the other way is rare
    assert np.all(err <= bound), (np.max(err / bound), int(np.argmax(err / bound)))
    assert np.all(err[~near] <= b32[~near])
    assert np.mean(err > b32) < 0.05
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
    so, _, bound, _ = _forward_bound(th, X.cpu().numpy())
    assert np.all(np.abs(s.cpu().numpy().astype(np.float64) - so) <= bound)


def _zero_theta():
    return np.zeros(mlp.NPARAM)


def _const_theta(b3):
    th = np.zeros(mlp.NPARAM)
    th[-1] = b3
    return th


@pytest.mark.parametrize("prec", [F64, F32C])
def test_learned_zero_network_follows_plain(P, prec):
    g = B.web_graph(40_000, 15.0, 51)
    G = P.bvmv_load(B.encode(g).data)
    dt = torch.float64 if prec == F64 else torch.float32
    pp = torch.empty(g.n, dtype=dt, device=DEV)
    rp = P.bvmv_pagerank_detail(G, pp, prec=prec)[0]
    m = P.bvmv_mlp_create(_zero_theta())
    pl = torch.empty(g.n, dtype=dt, device=DEV)
    rl = P.bvmv_pagerank_detail(G, pl, prec=prec, mlp=m)[0]
    # s = 0: each restart is p_K divided by its own sum, accepted
    assert rl["converged"] and rl["restarts_accepted"] == 2 and rl["restarts_rejected"] == 0
    assert abs(rl["iters"] - rp["iters"]) <= (0 if prec == F64 else 1)
    assert rl["products"] == rl["iters"]
    tol = 1e-12 if prec == F64 else 2e-6
    assert float(((pl.double() - pp.double()).abs() / pp.double()).max()) < tol


@pytest.mark.parametrize("prec,K", [(F64, 10), (F32C, 10), (F32C, 7)])
def test_learned_rejected_restart_is_plain_run(P, prec, K):
    """K = 10: the phase runs fused iterations (no finish kernel between
    products); K = 7 ends on an odd iterate, so the phase has a finish kernel
    per iteration and the rest is fused.  Either way the run is the plain
    run bit for bit."""
    g = B.web_graph(40_000, 15.0, 52)
    G = P.bvmv_load(B.encode(g).data)
    dt = torch.float64 if prec == F64 else torch.float32
    pp = torch.empty(g.n, dtype=dt, device=DEV)
    rp = P.bvmv_pagerank_detail(G, pp, prec=prec)[0]
    m = P.bvmv_mlp_create(_const_theta(1e6))
    pl = torch.empty(g.n, dtype=dt, device=DEV)
    rl = P.bvmv_pagerank_detail(G, pl, prec=prec, mlp=m, restart_every=K)[0]
    # a wild correction fails the probe once; the run resumes from p_K itself
    assert rl["restarts_accepted"] == 0 and rl["restarts_rejected"] == 1
    assert rl["iters"] == rp["iters"] and rl["products"] == rp["iters"] + 1
    assert torch.equal(pl, pp)


def test_learned_argument_errors(P):
    g = B.web_graph(5000, 10.0, 53)
    G = P.bvmv_load(B.encode(g).data)
    m = P.bvmv_mlp_create(_zero_theta())
    p = torch.empty(g.n, device=DEV)
    with pytest.raises(P.BvmvError):
        P.bvmv_pagerank_detail(G, p, mlp=m, restart_every=2)
    with pytest.raises(P.BvmvError):
        P.bvmv_pagerank_detail(G, p, mlp=m, start=torch.full((g.n,), 1.0 / g.n, device=DEV))
    with pytest.raises(P.BvmvError):
        P.bvmv_pagerank_detail(G, p, mlp=m, teleport=torch.full((g.n,), 1.0 / g.n, device=DEV))
    with pytest.raises(P.BvmvError):
        P.bvmv_pagerank_detail(G, torch.empty(g.n * 2, device=DEV), mlp=m, k=2)
    # input rows off a 16-byte boundary are refused (the kernels read them as
    # 16-byte vectors)
    Fb = torch.zeros(100 * 12 + 1, device=DEV)
    with pytest.raises(P.BvmvError):
        P.bvmv_mlp_forward(m, Fb[1:], torch.empty(100, device=DEV))
    with pytest.raises(P.BvmvError):
        P.bvmv_features(G, torch.zeros(g.n * 12 + 1, device=DEV)[1:])
    # a group whose members were coded with different R has no depth input
    G4 = P.bvmv_load(B.encode(g, R=4).data)
    grp = P.bvmv_group([G, G4])
    with pytest.raises(P.BvmvError):
        P.bvmv_pagerank_detail(grp, torch.empty(2 * g.n, device=DEV), mlp=m)


def test_learned_edge_cases(P):
    m = P.bvmv_mlp_create(_const_theta(1e6))
    # converges before the first restart: the plain run, no probe
    g = B.complete_graph(60)
    G = P.bvmv_load(B.encode(g).data)
    p = torch.empty(g.n, dtype=torch.float64, device=DEV)
    r = P.bvmv_pagerank_detail(G, p, prec=F64, mlp=m)[0]
    assert r["converged"] and r["iters"] == 1 and r["products"] == 1 and r["restarts_rejected"] == 0
    assert torch.allclose(p, torch.full_like(p, 1.0 / g.n), rtol=0, atol=1e-15)
    # max_iter below K: no restart, the plain run's state at max_iter
    g = B.web_graph(20_000, 12.0, 54)
    G = P.bvmv_load(B.encode(g).data)
    pp = torch.empty(g.n, dtype=torch.float64, device=DEV)
    rp = P.bvmv_pagerank_detail(G, pp, prec=F64, max_iter=6)[0]
    pl = torch.empty(g.n, dtype=torch.float64, device=DEV)
    rl = P.bvmv_pagerank_detail(G, pl, prec=F64, max_iter=6, mlp=m)[0]
    assert not rp["converged"] and not rl["converged"]
    assert rl["iters"] == rp["iters"] == 6 and rl["products"] == 6
    assert torch.equal(pl, pp)
    # restart_every = 3 (the smallest): still the plain fixed point within the bound
    pw = torch.empty(g.n, dtype=torch.float64, device=DEV)
    rw = P.bvmv_pagerank_detail(G, pw, prec=F64, mlp=P.bvmv_mlp_create(_zero_theta()), restart_every=3)[0]
    pu = torch.empty(g.n, dtype=torch.float64, device=DEV)
    ru = P.bvmv_pagerank_detail(G, pu, prec=F64)[0]
    assert rw["converged"] and rw["restarts_accepted"] == 2
    assert float((pw - pu).abs().sum()) < 2 * (0.85 / 0.15) * 1e-6


# ---------------------------------------------------------------- groups
# Learned restarts on a group (block-diagonal union of graphs): every member
# is restarted at the same phase boundary while all are active, and each
# keeps or rejects its restart on its own probe.

def _group_members():
    return [B.web_graph(15_000, 15.0, 81), B.web_graph(30_000, 6.0, 82), B.web_graph(20_000, 30.0, 83)]


def _group_run(P, gs, prec, **kw):
    Gs = [P.bvmv_load(B.encode(g).data) for g in gs]
    grp = P.bvmv_group(Gs)
    dt = torch.float64 if prec == F64 else torch.float32
    n = sum(g.n for g in gs)
    pg = torch.empty(n, dtype=dt, device=DEV)
    rg = P.bvmv_pagerank_detail(grp, pg, prec=prec, **kw)
    solo = []
    for G, g in zip(Gs, gs):
        ps = torch.empty(g.n, dtype=dt, device=DEV)
        solo.append((ps, P.bvmv_pagerank_detail(G, ps, prec=prec, **kw)[0]))
    offs = np.cumsum([0] + [g.n for g in gs])
    return pg, rg, solo, offs


@pytest.mark.parametrize("prec", [F64, F32C])
def test_group_learned_zero_network_matches_solo_runs(P, prec):
    """Zero network: every member keeps both restarts, exactly as alone."""
    gs = _group_members()
    pg, rg, solo, offs = _group_run(P, gs, prec, mlp=P.bvmv_mlp_create(_zero_theta()))
    for i, (ps, rs) in enumerate(solo):
        print("member", i, rg[i], flush=True)
        assert rg[i] == rs and rg[i]["restarts_accepted"] == 2 and rg[i]["converged"]
        assert torch.equal(pg[offs[i]:offs[i + 1]], ps)


@pytest.mark.parametrize("prec", [F64, F32C])
def test_group_learned_mixed_decisions(P, prec):
    """A constant correction of 1.75 deltas fails the probe of the first two
    members and passes the third's (decided by the oracle's restarted run).
    With one restart the group's members are exactly their solo runs, and
    their decisions and fixed points are the oracle's."""
    gs = _group_members()
    m = P.bvmv_mlp_create(_const_theta(1.75))
    pg, rg, solo, offs = _group_run(P, gs, prec, mlp=m, max_restarts=1)
    assert [r["restarts_accepted"] for r in rg] == [0, 0, 1]
    assert [r["restarts_rejected"] for r in rg] == [1, 1, 0]
    for i, (g, (ps, rs)) in enumerate(zip(gs, solo)):
        assert rg[i] == rs
        assert torch.equal(pg[offs[i]:offs[i + 1]], ps)
        rowptr, col, Fs = _decoded(B.encode(g))
        po, to, ro, oko, info = restart.pagerank_restarted(rowptr, col, lambda F: np.full(F.shape[0], 1.75), Fs,
                                                           max_restarts=1)
        assert oko and (rg[i]["restarts_accepted"], rg[i]["restarts_rejected"]) == (info["accepted"], info["rejected"])
        assert abs(rg[i]["iters"] - to) <= 1
        assert float(np.abs(ps.double().cpu().numpy() - po).sum()) < 2 * (0.85 / 0.15) * 1e-6


def test_group_learned_rejection_ends_restarts(P):
    """After a member rejects, no member is restarted again: with the default
    two restarts, the accepting member of the mixed group is restarted once."""
    gs = _group_members()
    pg, rg, solo, offs = _group_run(P, gs, F64, mlp=P.bvmv_mlp_create(_const_theta(1.75)))
    assert [(r["restarts_accepted"], r["restarts_rejected"]) for r in rg] == [(0, 1), (0, 1), (1, 0)]
    assert all(r["converged"] for r in rg)
    # the rejecting members are their plain runs (one extra product each)
    Gs = [P.bvmv_load(B.encode(g).data) for g in gs[:2]]
    for i, G in enumerate(Gs):
        pp = torch.empty(gs[i].n, dtype=torch.float64, device=DEV)
        rp = P.bvmv_pagerank_detail(G, pp, prec=F64)[0]
        assert rg[i]["iters"] == rp["iters"] and rg[i]["products"] == rp["iters"] + 1
        assert torch.equal(pg[offs[i]:offs[i + 1]], pp)


def test_group_learned_no_restart_once_a_member_is_done(P):
    """A member that converges within the first phase (a complete graph, one
    iteration) holds every restart back: the group's run is its plain run."""
    gs = [B.complete_graph(60), B.web_graph(20_000, 12.0, 84)]
    Gs = [P.bvmv_load(B.encode(g).data) for g in gs]
    grp = P.bvmv_group(Gs)
    n = sum(g.n for g in gs)
    pl = torch.empty(n, dtype=torch.float64, device=DEV)
    rl = P.bvmv_pagerank_detail(grp, pl, prec=F64, mlp=P.bvmv_mlp_create(_zero_theta()))
    pp = torch.empty(n, dtype=torch.float64, device=DEV)
    rp = P.bvmv_pagerank_detail(grp, pp, prec=F64)
    for a, b in zip(rl, rp):
        assert a["restarts_accepted"] == a["restarts_rejected"] == 0
        assert a["iters"] == b["iters"] and a["products"] == b["iters"]
    assert torch.equal(pl, pp)


def _train(P, graphs, steps, K=10, seed=1):
    """Train on restart samples (inputs after K plain iterations, targets from
    the method's own converged PageRank in FP64) of the given loaded graphs."""
    Fs, Ts = [], []
    for G, n in graphs:
        ps = torch.empty(n, dtype=torch.float64, device=DEV)
        P.bvmv_pagerank(G, ps, tol=1e-12, max_iter=5000, prec=F64)
        F = torch.empty(n, P.NFEAT, device=DEV)
        T = torch.empty(n, device=DEV)
        P.bvmv_restart_sample(G, K, F, T, ps.float(), prec=F32C)
        Fs.append(F)
        Ts.append(T)
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


@pytest.fixture(scope="module")
def trained(P):
    train = [B.web_graph(n, 15.0, 40 + i) for i, n in enumerate((60_000, 90_000, 75_000, 50_000))]
    Gs = [(P.bvmv_load(B.encode(g).data), g.n) for g in train]
    return _train(P, Gs, 1500)


def test_training_reduces_loss(P, trained):
    m, l0, l1 = trained
    assert l1 < 0.3 * l0


def test_learned_matches_oracle_restarted_run(P, trained):
    m = trained[0]
    theta = P.bvmv_mlp_params(m).astype(np.float64)
    g = B.web_graph(20_000, 15.0, 61)
    enc = B.encode(g)
    G = P.bvmv_load(enc.data)
    rowptr, col, Fs = _decoded(enc)
    pl = torch.empty(g.n, dtype=torch.float64, device=DEV)
    rl = P.bvmv_pagerank_detail(G, pl, prec=F64, mlp=m)[0]
    po, to, ro, oko, info = restart.pagerank_restarted(
        rowptr, col, lambda F: mlp.forward(theta, F.astype(np.float32), quantize=True)[0], Fs)
    assert rl["converged"] and oko
    # the decisions agree; the BF16 network's order of summation may move the
    # stopping iteration by one
    assert (rl["restarts_accepted"], rl["restarts_rejected"]) == (info["accepted"], info["rejected"])
    assert abs(rl["iters"] - to) <= 1
    assert float(np.abs(pl.cpu().numpy() - po).sum()) < 2 * (0.85 / 0.15) * 1e-6


def test_learned_restarts_gain(P, trained):
    m = trained[0]
    g = B.web_graph(200_000, 15.0, 77)
    G = P.bvmv_load(B.encode(g).data)
    pu = torch.empty(g.n, device=DEV)
    ru = P.bvmv_pagerank_detail(G, pu)[0]
    pw = torch.empty(g.n, device=DEV)
    rw = P.bvmv_pagerank_detail(G, pw, mlp=m)[0]
    assert ru["converged"] and rw["converged"] and rw["restarts_accepted"] >= 1
    # at least 15% fewer products than the plain method, same fixed point
    assert rw["products"] <= 0.85 * ru["products"], (rw, ru)
    assert float((pw.double() - pu.double()).abs().sum()) < 2 * (0.85 / 0.15) * 1e-6 + 1e-5
