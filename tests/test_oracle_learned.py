"""Pins for the oracle's learned proposal: finite differences, normalisation of
q, the sampler against q, and exact stationarity of the corrected chain."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1210_5128_amd import datagen


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    n = 6
    prm = datagen.mlp_params(3)
    z = rng.standard_normal((n, 8))
    eps = 0.1
    loss, g = oracle.mlp_loss_grad(prm, z, 1, 4, eps)
    assert loss == pytest.approx(-oracle.pair_logq(oracle.mlp_forward(prm, z), 1, 4, eps), rel=1e-14)
    idx = np.concatenate([rng.choice(prm.size, 300, replace=False), np.arange(prm.size - 129, prm.size)])
    h = 1e-6
    for k in idx:
        p1 = prm.copy(); p1[k] += h
        p2 = prm.copy(); p2[k] -= h
        l1, _ = oracle.mlp_loss_grad(p1, z, 1, 4, eps)
        l2, _ = oracle.mlp_loss_grad(p2, z, 1, 4, eps)
        fd = (l1 - l2) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-7), k


def test_pair_distribution_sums_to_one_and_matches_sampler():
    rng = np.random.default_rng(1)
    n = 5
    logits = rng.standard_normal(n) * 1.5
    eps = 0.1
    tot = sum(math.exp(oracle.pair_logq(logits, a, b, eps)) for a, b in itertools.combinations(range(n), 2))
    assert tot == pytest.approx(1.0, abs=1e-12)
    # uniform limit
    assert math.exp(oracle.pair_logq(np.zeros(n), 0, 1, 0.0)) == pytest.approx(2 / (n * (n - 1)))
    order = np.array([3, 0, 4, 1, 2], dtype=np.int32)
    counts = {}
    T = 60000
    for t in range(1, T + 1):
        pa, pb = oracle.learned_pair(11, 2, t, logits, order, eps)
        assert pa != pb
        key = tuple(sorted((int(order[pa]), int(order[pb]))))
        counts[key] = counts.get(key, 0) + 1
    chi2 = 0.0
    for a, b in itertools.combinations(range(n), 2):
        e = T * math.exp(oracle.pair_logq(logits, a, b, eps))
        chi2 += (counts.get((a, b), 0) - e) ** 2 / e
    assert chi2 < 35            # 9 dof


def test_features_definition():
    n = 5
    order = np.array([2, 4, 0, 1, 3], dtype=np.int32)
    nb = np.array([-1.0, -2.0, -3.0, -4.0, -5.0])
    ns = np.array([-1.5, -np.inf, -3.25, -4.0, -6.0])
    pn = np.arange(25, dtype=np.float64).reshape(5, 5)
    np.fill_diagonal(pn, 0)
    st = np.arange(15, dtype=np.float64).reshape(5, 3)
    f = oracle.features(order, nb, ns, pn, st)
    assert list(f[:, 0]) == [2 / 5, 3 / 5, 0.0, 4 / 5, 1 / 5]
    assert list(f[:, 1]) == list(nb)
    assert list(f[:, 2]) == [0.5, 0.0, 0.25, 0.0, 1.0]
    assert list(f[:, 3]) == list(pn.sum(axis=1))
    assert list(f[:, 4]) == list(pn.sum(axis=0))
    assert np.array_equal(f[:, 5:], st)


def test_table_stats_by_definition():
    rng = np.random.default_rng(4)
    data = np.stack([rng.integers(0, 3, 40) for _ in range(5)], axis=1).astype(np.int8)
    t = oracle.build_table(data, [3] * 5, 2)
    st = oracle.table_stats(t, 2, round_f32=False)
    assert np.allclose(st[:, 0], t.max(axis=1), rtol=0, atol=0)
    assert np.allclose(st[:, 1], t.mean(axis=1), rtol=1e-14)
    assert np.allclose(st[:, 2], t.std(axis=1), rtol=1e-12)


@pytest.mark.parametrize("target,N,scale,w_best", [(0, 8, 1.0, 6.0), (0, 12, 1.5, 3.0), (1, 12, 1.0, 3.0)])
def test_learned_chain_is_stationary_at_exact_posterior(target, N, scale, w_best):
    # The network weights the best-score feature heavily, so the proposal is
    # strongly asymmetric between an order and its swap; without the
    # q(new)/q(old) factor this chain's visiting frequencies miss the posterior
    # by a total variation of about 0.1-0.2 at these settings.
    n, K = 4, 3
    arities = [2, 2, 3, 2]
    rng = np.random.default_rng(12)
    data = np.stack([rng.integers(0, a, size=N) for a in arities], axis=1).astype(np.int8)
    table = oracle.build_table(data, arities, K)
    orders = list(itertools.permutations(range(n)))
    sc = np.array([oracle.score_order(table, K, o, round_f32=False)[target] for o in orders])
    post = np.exp(sc - sc.max())
    post /= post.sum()
    prm = datagen.mlp_params(7, scale=scale)
    prm[1:8 * 128:8] *= w_best                       # column of W1 for the best-score feature
    stats = oracle.table_stats(table, K, round_f32=False)
    mu = np.zeros(8)
    mu[1] = float(np.mean(sc) / n)
    sd = np.array([0.3, 1.0, 1.0, 1.0, 1.0, 30.0, 30.0, 5.0])
    iters = 200000
    res = oracle.run_chain_learned(table, K, 31, 0, iters, prm, mu, sd, None, stats, eps=0.1, target=target,
                                   round_f32=False)
    # replay the visited orders from the proposals the chain drew and its decisions
    cur = list(oracle.initial_order(31, 0, n))
    freq = np.zeros(len(orders))
    idx = {o: k for k, o in enumerate(orders)}
    l, m, b, nl, nb, ns = oracle.score_order(table, K, cur, round_f32=False)
    logits = oracle.mlp_forward(prm, (oracle.features(cur, nb, ns, None, stats) - mu) / sd)
    for t in range(1, iters + 1):
        pa, pb = oracle.learned_pair(31, 0, t, logits, cur, 0.1)
        if res["acc"][t - 1]:
            cur[pa], cur[pb] = cur[pb], cur[pa]
            l, m, b, nl, nb, ns = oracle.score_order(table, K, cur, round_f32=False)
            logits = oracle.mlp_forward(prm, (oracle.features(cur, nb, ns, None, stats) - mu) / sd)
        if t > 2000:
            freq[idx[tuple(cur)]] += 1
    assert tuple(cur) == tuple(res["order"])
    freq /= freq.sum()
    tv = 0.5 * np.abs(freq - post).sum()
    assert tv < 0.04, tv
    # the proposal really is far from uniform over the six pairs
    qs = [math.exp(oracle.pair_logq(logits, a, b, 0.1)) for a, b in itertools.combinations(range(n), 2)]
    assert max(qs) / min(qs) > 3.0
