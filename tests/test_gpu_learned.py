"""Learned swap proposal on the device: static features vs the oracle, exact
stationarity of the q-corrected chains, and the harvest of accepted moves."""
import itertools
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1210_5128_amd import datagen

pytestmark = pytest.mark.gpu

N_PARAM = 17793


@pytest.fixture(scope="module")
def bnos():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_5128_amd import bnos as b
    return b


@pytest.fixture(scope="module")
def prior20(bnos):
    w = datagen.WORKLOADS["prior20"]
    net, prior = datagen.make(w)
    t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior)
    orc = oracle.build_table(net.data, net.arities, w.K, prior=prior)
    yield w, net, prior, t, orc
    t.free()


def test_static_node_features_match_oracle(bnos, prior20):
    w, net, prior, t, orc = prior20
    got = t.node_features()
    pn = oracle.prior_nats(prior, w.n)
    np.testing.assert_allclose(got[:, 0], pn.sum(axis=1), rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(got[:, 1], pn.sum(axis=0), rtol=1e-12, atol=1e-9)
    st = oracle.table_stats(orc, w.K, round_f32=True)
    np.testing.assert_allclose(got[:, 2:], st, rtol=1e-9)


def test_learned_chains_sample_the_exact_posterior(bnos):
    # the asymmetric network of the oracle's stationarity test: without the
    # reverse-q factor the visiting frequencies would miss by TV 0.1-0.2
    n, K = 4, 3
    arities = [2, 2, 3, 2]
    rng = np.random.default_rng(12)
    data = np.stack([rng.integers(0, a, size=8) for a in arities], axis=1).astype(np.int8)
    t = bnos.build_score_table(data, arities, K)
    orc = oracle.build_table(data, arities, K)
    orders = list(itertools.permutations(range(n)))
    sc = np.array([oracle.score_order(orc, K, o)[0] for o in orders])
    post = np.exp(sc - sc.max())
    post /= post.sum()
    prm = datagen.mlp_params(7, scale=1.0)
    prm[1:8 * 128:8] *= 6.0
    mu = np.zeros(8, np.float32)
    mu[1] = np.float32(np.mean(sc) / n)
    sd = np.array([0.3, 1.0, 1.0, 1.0, 1.0, 30.0, 30.0, 5.0], np.float32)
    m = bnos.Mlp()
    m.set_params(prm.astype(np.float32), mu, sd)
    C = 32768
    st = t.new_chain_state(C, 300, trace_every=300)
    t.run_chains(st, 300, seed=55, mlp=m, eps=0.1, trace_every=300)
    fin = st["orders"].cpu().numpy()
    idx = {o: k for k, o in enumerate(orders)}
    freq = np.zeros(24)
    for row in fin:
        freq[idx[tuple(int(v) for v in row)]] += 1
    freq /= C
    tv = 0.5 * np.abs(freq - post).sum()
    assert tv < 0.03, tv
    acc = st["accepted"].cpu().numpy().sum() / (C * 300)
    assert 0.05 < acc < 0.99
    m.free()
    t.free()


def test_harvest_records_the_order_before_each_accepted_move(bnos, prior20):
    w, net, prior, t, orc = prior20
    C, iters, cap = 4, 300, 64
    st = t.new_chain_state(C, iters, trace_every=1, flags=True, harvest_cap=cap)
    t.run_chains(st, iters, seed=71)
    feats = st["harvest_feats"].cpu().numpy()
    pairs = st["harvest_pairs"].cpu().numpy()
    cnt = st["harvest_count"].cpu().numpy()
    acc = st["accepted"].cpu().numpy()
    static = t.node_features()
    assert np.all(cnt == np.minimum(acc, cap)) and cnt.min() > 3
    for c in range(C):
        orders = []
        for k in range(int(cnt[c])):
            f = feats[c, k]
            order = np.argsort(f[:, 0]).astype(np.int32)         # position / n gives the order
            assert np.allclose(np.sort(f[:, 0]), np.arange(w.n) / w.n)
            l, mx, best, nl, nb, ns = oracle.score_order(orc, w.K, order)
            np.testing.assert_allclose(f[:, 1], nb, rtol=1e-6)
            gap = np.where(np.isinf(ns), 0.0, nb - ns)
            np.testing.assert_allclose(f[:, 2], gap, rtol=1e-4, atol=1e-2)
            np.testing.assert_allclose(f[:, 3:], static, rtol=1e-6, atol=1e-5)
            orders.append(order)
        for k in range(len(orders) - 1):
            a, b = (int(x) for x in pairs[c, k])
            nxt = orders[k].copy()
            pa, pb = int(np.nonzero(nxt == a)[0][0]), int(np.nonzero(nxt == b)[0][0])
            nxt[pa], nxt[pb] = nxt[pb], nxt[pa]
            assert np.array_equal(nxt, orders[k + 1]), (c, k)


def test_uniform_chains_unchanged_by_harvest(bnos, prior20):
    w, net, prior, t, orc = prior20
    a = t.new_chain_state(3, 200, trace_every=1, flags=True)
    t.run_chains(a, 200, seed=3)
    b = t.new_chain_state(3, 200, trace_every=1, flags=True, harvest_cap=16)
    t.run_chains(b, 200, seed=3)
    for k in ("orders", "scores", "best_graphs", "best_scores", "accepted", "trace", "accept_flags"):
        assert torch.equal(a[k], b[k]), k


def dyadic_position_network(seed):
    """Parameters whose forward pass is exact in BF16/FP32 and FP64 alike when
    the only nonzero first-layer column is the position feature p/n with n = 8:
    all weights are small dyadic rationals, so both sides get identical logits."""
    rng = np.random.default_rng(seed)
    H = 128
    W1 = np.zeros((H, 8))
    W1[:, 0] = rng.choice([-1.0, -0.5, 0.5, 1.0], size=H)
    b1 = rng.integers(-2, 3, size=H) / 4.0
    W2 = rng.choice([-0.25, 0.0, 0.0, 0.25], size=(H, H))
    b2 = rng.integers(-2, 3, size=H) / 8.0
    w3 = rng.choice([-0.5, 0.0, 0.5], size=H)
    prm = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [0.0]])
    assert np.array_equal(prm.astype(np.float32).astype(np.float64), prm)
    return prm


def oracle_learned_step(orc, K, seed, chain, t, res, prm, stats, eps, target):
    """The oracle's (ln u, log MH ratio) at iteration t of its own learned chain `res`."""
    n = orc.shape[0]
    zeros, ones = np.zeros(8), np.ones(8)

    def logits_of(order):
        l, m, best, nl, nb, ns = oracle.score_order(orc, K, order, round_f32=True)
        return oracle.mlp_forward(prm, (oracle.features(order, nb, ns, None, stats) - zeros) / ones), l, m

    cur = list(oracle.initial_order(seed, chain, n))
    for s in range(1, t + 1):
        lc, _, _ = logits_of(cur)
        pa, pb = oracle.learned_pair(seed, chain, s, lc, cur, eps)
        prop = list(cur)
        prop[pa], prop[pb] = prop[pb], prop[pa]
        if s < t:
            if res["acc"][s - 1]:
                cur = prop
            continue
        lp, l, m = logits_of(prop)
        a, b = cur[pa], cur[pb]
        new = l if target == 0 else m
        ratio = new - res["trace"][t - 1] + oracle.pair_logq(lp, a, b, eps) - oracle.pair_logq(lc, a, b, eps)
        return math.log(oracle.accept_uniform(seed, chain, t)), ratio


@pytest.mark.parametrize("target", [0, 1])
def test_learned_chains_match_oracle_in_lockstep(bnos, target):
    # same proposals (the logits agree exactly, the pair sampler is FP64 on
    # both sides) and the same decisions except within TAU of the threshold
    TAU, REL = 1e-3, 1e-5
    w = datagen.WORKLOADS["tiny8"]
    net, _ = datagen.make(w)
    t = bnos.build_score_table(net.data, net.arities, w.K)
    orc = oracle.build_table(net.data, net.arities, w.K)
    stats = oracle.table_stats(orc, w.K, round_f32=True)
    prm = dyadic_position_network(31 + target)
    m = bnos.Mlp()
    m.set_params(prm.astype(np.float32), np.zeros(8, np.float32), np.ones(8, np.float32))
    C, iters, seed, eps = 10, 400, 77 + target, 0.25
    st = t.new_chain_state(C, iters, trace_every=1, flags=True)
    t.run_chains(st, iters, seed=seed, target=target, mlp=m, eps=eps, trace_every=1)
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in st.items()}
    full = 0
    for c in range(C):
        res = oracle.run_chain_learned(orc, w.K, seed, c, iters, prm, np.zeros(8), np.ones(8), None, stats,
                                       eps=eps, target=target)
        flags = g["accept_flags"][c, :iters].astype(bool)
        mism = np.nonzero(flags != res["acc"].astype(bool))[0]
        if len(mism):
            k = int(mism[0]) + 1
            lu, ratio = oracle_learned_step(orc, w.K, seed, c, k, res, prm, stats, eps, target)
            assert abs(lu - ratio) <= TAU, (c, k, lu, ratio)
            np.testing.assert_allclose(g["trace"][c, :k], res["trace"][:k], rtol=REL)
            continue
        full += 1
        np.testing.assert_allclose(g["trace"][c, :iters + 1], res["trace"], rtol=REL, atol=1e-6)
        assert list(g["orders"][c]) == list(res["order"]), c
        assert [int(x) for x in g["best_graphs"][c].view(np.uint64)] == [int(x) for x in res["best_graph"]], c
        assert int(g["accepted"][c]) == res["accepted"]
    assert full >= C - 1
    acc = g["accepted"].sum() / (C * iters)
    assert 0.02 < acc < 0.98
    m.free()
    t.free()


def test_trained_network_gains_over_uniform_swaps(bnos):
    # harvest accepted moves from uniform chains, train on the device, then
    # resume the same chains under both proposals: the trained proposal must
    # fit the harvest better than uniform pairs and raise acceptance and the
    # effective sample size per iteration
    from paper_1210_5128_amd import ess as E
    w = datagen.WORKLOADS["mixed40"]
    net, prior = datagen.make(w)
    t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior)
    C, harvest_iters, iters = 128, 4000, 2000
    st = t.new_chain_state(C, 1, trace_every=0, harvest_cap=1024)
    t.run_chains(st, harvest_iters, 11, trace_every=0)
    cnt = st["harvest_count"].cpu().numpy()
    feats = torch.cat([st["harvest_feats"][c, :int(cnt[c])] for c in range(C)])
    pairs = torch.cat([st["harvest_pairs"][c, :int(cnt[c])] for c in range(C)])
    m = bnos.Mlp()
    m.set_params(datagen.mlp_params(5, scale=0.5).astype(np.float32))
    m.fit_norm(feats)
    m.train(feats, pairs, epochs=12, batch=1024, lr=2e-3, seed=3)
    g = torch.empty(N_PARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    m.grad(feats, pairs, g, loss)
    uniform_loss = np.log(w.n * (w.n - 1) / 2)
    assert loss.item() < uniform_loss - 0.1, (loss.item(), uniform_loss)
    res = {}
    for label, mlp in (("uniform", None), ("learned", m)):
        s2 = {k: st[k].clone() for k in ("orders", "scores", "best_graphs", "best_scores", "accepted")}
        s2["trace"] = torch.zeros((C, iters + 1), dtype=torch.float64, device="cuda")
        a0 = s2["accepted"].clone()
        t.run_chains(s2, iters, 21, first_iteration=harvest_iters, mlp=mlp, eps=0.1)
        tr = s2["trace"].cpu().numpy()
        res[label] = dict(acc=float((s2["accepted"] - a0).sum().item()) / (C * iters), ess=E.ess(tr))
    # measured: acceptance 0.304 vs 0.189, ESS 1,819 vs 1,236, loss 6.44 vs 6.66 nats
    assert res["learned"]["acc"] > 1.3 * res["uniform"]["acc"], res
    assert res["learned"]["ess"] > 1.05 * res["uniform"]["ess"], res
    m.free()
    t.free()


def test_network_trained_across_datasets(bnos):
    # one network trained on the accepted moves of two datasets of different size
    # (n=20 and n=28): the loss on each harvest falls below that of uniform pairs,
    # and the network then drives exact chains on a third, unseen size (n=4)
    sets = [datagen.WORKLOADS["prior20"], datagen.Workload("x28", 28, 1500, (2, 3), 3, 4, 31, None)]
    C, iters, cap = 64, 4000, 512
    feats, pairs = [], []
    for k, w in enumerate(sets):
        net, prior = datagen.make(w)
        t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior)
        st = t.new_chain_state(C, 1, trace_every=0, harvest_cap=cap)
        t.run_chains(st, iters, 40 + k, trace_every=0)
        cnt = st["harvest_count"].cpu().numpy()
        assert cnt.min() > 0
        feats.append(torch.cat([st["harvest_feats"][c, :int(min(cnt[c], cap))] for c in range(C)]))
        pairs.append(torch.cat([st["harvest_pairs"][c, :int(min(cnt[c], cap))] for c in range(C)]))
        t.free()
    m = bnos.Mlp()
    m.set_params(datagen.mlp_params(9, scale=0.5).astype(np.float32))
    m.fit_norm(torch.cat([f.reshape(-1, 8) for f in feats]).contiguous())
    g = torch.empty(N_PARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")

    def losses():
        out = []
        for f, p in zip(feats, pairs):
            m.grad(f, p, g, loss)
            out.append(loss.item())
        return out

    before = losses()
    for ep in range(10):
        for k in range(len(sets)):
            m.train(feats[k], pairs[k], epochs=1, batch=512, lr=2e-3, seed=100 * ep + k)
    after = losses()
    for w, b, a in zip(sets, before, after):
        uniform_loss = np.log(w.n * (w.n - 1) / 2)
        assert a < b, (w.name, b, a)
        assert a < uniform_loss - 0.05, (w.name, a, uniform_loss)
    # exactness on an unseen size: the visiting frequencies of the q-corrected
    # chains match the exact order posterior
    n, K = 4, 3
    arities = [2, 3, 2, 2]
    rng = np.random.default_rng(21)
    data = np.stack([rng.integers(0, a, size=10) for a in arities], axis=1).astype(np.int8)
    t = bnos.build_score_table(data, arities, K)
    orc = oracle.build_table(data, arities, K)
    orders = list(itertools.permutations(range(n)))
    sc = np.array([oracle.score_order(orc, K, o)[0] for o in orders])
    post = np.exp(sc - sc.max())
    post /= post.sum()
    C2 = 32768
    st = t.new_chain_state(C2, 300, trace_every=300)
    t.run_chains(st, 300, seed=77, mlp=m, eps=0.1, trace_every=300)
    fin = st["orders"].cpu().numpy()
    idx = {o: k for k, o in enumerate(orders)}
    freq = np.zeros(len(orders))
    for row in fin:
        freq[idx[tuple(int(v) for v in row)]] += 1
    freq /= C2
    tv = 0.5 * np.abs(freq - post).sum()
    assert tv < 0.03, tv
    m.free()
    t.free()
