"""GPU Metropolis-Hastings chains against the oracle chain on the same RNG stream.

The two sides take every accept decision from their own scores; a decision
may legitimately differ only where the oracle's |ln u - delta| is within
TAU of the threshold (the FP32 table and FP32 sums move delta by ~1e-5).
"""
import itertools
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1210_5128_amd import datagen

pytestmark = pytest.mark.gpu

TAU = 1e-3
REL = 1e-5


@pytest.fixture(scope="module")
def bnos():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_5128_amd import bnos as b
    return b


def gpu_chains(table, chains, iters, seed, target=0, sweep_len=0, chain_offset=0, topk=0):
    st = table.new_chain_state(chains, iters, trace_every=1, flags=True, topk=topk)
    table.run_chains(st, iters, seed, target=target, sweep_len=sweep_len, chain_offset=chain_offset)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in st.items()}


def oracle_replay_delta(orc, K, seed, chain, t, res, target):
    """The oracle's (ln u, delta) at iteration t of its own chain `res`."""
    n = orc.shape[0]
    cur = list(oracle.initial_order(seed, chain, n))
    for s in range(1, t):
        if res["acc"][s - 1]:
            a, b = oracle.swap_pair(seed, chain, n, s)
            cur[a], cur[b] = cur[b], cur[a]
    a, b = oracle.swap_pair(seed, chain, n, t)
    prop = list(cur)
    prop[a], prop[b] = prop[b], prop[a]
    l, m, *_ = oracle.score_order(orc, K, prop, round_f32=True)
    new = l if target == 0 else m
    return math.log(oracle.accept_uniform(seed, chain, t)), new - res["trace"][t - 1]


def compare_topk(gg, gs, gc, og, os_, full_record):
    """GPU best-graph record vs the oracle's: equal scores (REL) position by
    position; equal graphs, except that records whose scores are near-tied (the
    two sides sum FP32 scores that differ in the last bits) may swap places
    within their tie group, and a tie group at the cut of a full record may
    hold different members."""
    cnt = int(gc)
    assert cnt == len(os_)
    np.testing.assert_allclose(gs[:cnt], os_, rtol=REL)
    tol = 1e-4 + REL * np.abs(os_)
    r = 0
    while r < cnt:
        e = r
        while e + 1 < cnt and abs(os_[e + 1] - os_[e]) <= tol[e]:
            e += 1
        at_cut = full_record and e == cnt - 1
        if not at_cut:
            a = sorted(tuple(int(x) for x in gg[q].view(np.uint64)) for q in range(r, e + 1))
            b = sorted(tuple(int(x) for x in og[q]) for q in range(r, e + 1))
            assert a == b, (r, e)
        r = e + 1


def compare_chains(g, orc, K, seed, iters, target, chain_offset=0, topk=0):
    full = 0
    C = g["orders"].shape[0]
    for c in range(C):
        chain = chain_offset + c
        res = oracle.run_chain(orc, K, seed, chain, iters, target=target, round_f32=True, topk=topk)
        flags = g["accept_flags"][c, :iters].astype(bool)
        mism = np.nonzero(flags != res["acc"].astype(bool))[0]
        if len(mism):
            t = int(mism[0]) + 1
            lu, d = oracle_replay_delta(orc, K, seed, chain, t, res, target)
            assert abs(lu - d) <= TAU, (c, t, lu, d)
            np.testing.assert_allclose(g["trace"][c, :t], res["trace"][:t], rtol=REL)
            continue
        full += 1
        np.testing.assert_allclose(g["trace"][c, :iters + 1], res["trace"], rtol=REL, atol=1e-6)
        assert list(g["orders"][c]) == list(res["order"]), c
        assert [int(x) for x in g["best_graphs"][c].view(np.uint64)] == [int(x) for x in res["best_graph"]], c
        assert abs(g["best_scores"][c] - res["best_score"]) <= REL * max(1.0, abs(res["best_score"]))
        assert int(g["accepted"][c]) == res["accepted"]
        assert abs(g["scores"][c] - res["trace"][-1]) <= REL * max(1.0, abs(res["trace"][-1]))
        if topk:
            compare_topk(g["top_graphs"][c], g["top_scores"][c], g["top_count"][c], res["top_graphs"],
                         res["top_scores"], int(g["top_count"][c]) == topk)
            assert [int(x) for x in g["top_graphs"][c, 0].view(np.uint64)] == \
                [int(x) for x in g["best_graphs"][c].view(np.uint64)]
    return full


@pytest.fixture(scope="module")
def tiny8(bnos):
    w = datagen.WORKLOADS["tiny8"]
    net, prior = datagen.make(w)
    t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior)
    orc = oracle.build_table(net.data, net.arities, w.K, prior=prior)
    yield w, t, orc
    t.free()


@pytest.fixture(scope="module")
def prior20(bnos):
    w = datagen.WORKLOADS["prior20"]
    net, prior = datagen.make(w)
    t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior)
    orc = oracle.build_table(net.data, net.arities, w.K, prior=prior)
    yield w, t, orc
    t.free()


def test_chains_match_oracle_tiny8_lse(bnos, tiny8):
    w, t, orc = tiny8
    iters, C = 2000, 12
    g = gpu_chains(t, C, iters, seed=100)
    full = compare_chains(g, orc, w.K, 100, iters, 0)
    assert full >= C - 1


def test_chains_match_oracle_prior20_max_target(bnos, prior20):
    w, t, orc = prior20
    iters, C = 400, 6
    g = gpu_chains(t, C, iters, seed=101, target=1, chain_offset=7)
    full = compare_chains(g, orc, w.K, 101, iters, 1, chain_offset=7)
    assert full >= C - 1


@pytest.mark.parametrize("wname,topk,target", [("tiny8", 6, 0), ("prior20", 10, 1), ("prior20", 64, 0)])
def test_best_graph_record_matches_oracle(bnos, wname, topk, target, request):
    w, t, orc = request.getfixturevalue(wname)
    iters, C = (1500, 8) if wname == "tiny8" else (400, 5)
    g = gpu_chains(t, C, iters, seed=130 + topk, target=target, topk=topk)
    full = compare_chains(g, orc, w.K, 130 + topk, iters, target, topk=topk)
    assert full >= C - 1
    assert g["top_count"].max() >= min(topk, 5)
    # records are distinct and sorted
    for c in range(C):
        k = int(g["top_count"][c])
        sc = g["top_scores"][c, :k]
        assert np.all(np.diff(sc) <= 0)
        assert len({tuple(r) for r in g["top_graphs"][c, :k].tolist()}) == k


def test_best_graph_record_resumes(bnos, tiny8):
    w, t, orc = tiny8
    C, topk = 6, 5
    ref = gpu_chains(t, C, 300, seed=9, topk=topk)
    st = t.new_chain_state(C, 100, trace_every=1, topk=topk)
    t.run_chains(st, 100, 9)
    st["trace"] = torch.zeros((C, 201), dtype=torch.float64, device="cuda")
    t.run_chains(st, 200, 9, first_iteration=100)
    torch.cuda.synchronize()
    for k in ("top_graphs", "top_scores", "top_count", "best_graphs"):
        assert np.array_equal(st[k].cpu().numpy(), ref[k]), k


def test_chains_prior20_lse(bnos, prior20):
    w, t, orc = prior20
    iters, C = 600, 5
    g = gpu_chains(t, C, iters, seed=102)
    assert compare_chains(g, orc, w.K, 102, iters, 0) >= C - 1


def test_resume_and_graph_shapes_are_bitwise_identical(bnos, tiny8):
    w, t, orc = tiny8
    C, iters = 9, 301
    ref = gpu_chains(t, C, iters, seed=5, sweep_len=0)
    for sl in (1, 7, 1000):
        g = gpu_chains(t, C, iters, seed=5, sweep_len=sl)
        for k in ("orders", "scores", "best_graphs", "best_scores", "accepted", "trace", "accept_flags"):
            assert np.array_equal(g[k], ref[k]), (sl, k)
    # resume: 120 iterations, then 181 more from the saved state
    st = t.new_chain_state(C, 120, trace_every=1, flags=True)
    t.run_chains(st, 120, 5)
    st2 = dict(st)
    st2["trace"] = torch.zeros((C, 182), dtype=torch.float64, device="cuda")
    st2["accept_flags"] = torch.zeros((C, 181), dtype=torch.uint8, device="cuda")
    t.run_chains(st2, 181, 5, first_iteration=120)
    torch.cuda.synchronize()
    for k in ("orders", "scores", "best_graphs", "best_scores", "accepted"):
        assert np.array_equal(st2[k].cpu().numpy(), ref[k]), k
    assert np.array_equal(st["accept_flags"].cpu().numpy()[:, :120], ref["accept_flags"][:, :120])
    assert np.array_equal(st2["accept_flags"].cpu().numpy(), ref["accept_flags"][:, 120:301])
    assert np.array_equal(st2["trace"].cpu().numpy(), ref["trace"][:, 120:302])


def test_gpu_chains_sample_the_exact_order_posterior(bnos):
    # n = 4: 24 orders; many short independent chains, final states vs exact P(order)
    rng = np.random.default_rng(12)
    arities = [2, 2, 3, 2]
    data = np.stack([rng.integers(0, a, size=12) for a in arities], axis=1).astype(np.int8)
    K = 3
    t = bnos.build_score_table(data, arities, K)
    orc = oracle.build_table(data, arities, K)
    for target in (0, 1):
        orders = list(itertools.permutations(range(4)))
        sc = np.array([oracle.score_order(orc, K, o)[target] for o in orders])
        post = np.exp(sc - sc.max())
        post /= post.sum()
        C = 32768
        st = t.new_chain_state(C, 200, trace_every=200)
        t.run_chains(st, 200, seed=77 + target, target=target, trace_every=200)
        fin = st["orders"].cpu().numpy()
        idx = {o: k for k, o in enumerate(orders)}
        freq = np.zeros(24)
        for row in fin:
            freq[idx[tuple(int(v) for v in row)]] += 1
        freq /= C
        tv = 0.5 * np.abs(freq - post).sum()
        assert tv < 0.03, (target, tv)
    t.free()


def test_chain_validation(bnos, tiny8):
    w, t, orc = tiny8
    st = t.new_chain_state(2, 10)
    with pytest.raises(bnos.BnosError) as e:
        t.run_chains(st, 10, 1, target=3)
    assert e.value.status == bnos.E_INVALID
    with pytest.raises(bnos.BnosError) as e:
        t.run_chains(st, -1, 1)
    assert e.value.status == bnos.E_RANGE
    with pytest.raises(bnos.BnosError) as e:
        t.run_chains(t.new_chain_state(2, 10, topk=65), 10, 1)
    assert e.value.status == bnos.E_RANGE
    with pytest.raises(bnos.BnosError) as e:
        t.run_chains(t.new_chain_state(2, 10, edges=[(1, 0), (w.n, 2)]), 10, 1)
    assert e.value.status == bnos.E_RANGE
    with pytest.raises(bnos.BnosError) as e:
        t.run_chains(t.new_chain_state(2, 10, edges=[(3, 3)]), 10, 1)
    assert e.value.status == bnos.E_RANGE


def test_mixed60_chain_properties(bnos):
    w = datagen.WORKLOADS["mixed60"]
    net, prior = datagen.make(w)
    t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior)
    C, iters = 16, 60
    st = t.new_chain_state(C, iters, trace_every=1, flags=True)
    t.run_chains(st, iters, seed=9)
    g = {k: v.cpu().numpy() for k, v in st.items() if v is not None}
    for c in range(C):
        assert sorted(g["orders"][c]) == list(range(60))
        l, m, best = t.score_order(g["orders"][c])
        assert abs(l - g["scores"][c]) <= REL * abs(l)
        assert int(g["accepted"][c]) == int(g["accept_flags"][c].sum())
        # the record starts at the initial order's max score and never decreases
        init = oracle.initial_order(9, c, 60)
        l0, m0, _ = t.score_order(init)
        assert abs(l0 - g["trace"][c, 0]) <= REL * abs(l0)
        assert g["best_scores"][c] >= m0
    t.free()


def test_uneven_datasets_in_one_launch_match_one_at_a_time(bnos):
    ws = [datagen.uneven_workload(d) for d in range(5)]
    ws = [datagen.Workload(w.name, w.n, min(w.N, 1500), w.arity_choices, w.dmax, 3, w.data_seed, None)
          for w in ws]                                     # K=3 keeps the test short
    tabs = []
    for w in ws:
        net, _ = datagen.make(w)
        tabs.append(bnos.build_score_table(net.data, net.arities, w.K))
    C, iters, seed = 6, 150, 33
    states = [t.new_chain_state(C, iters, trace_every=1, flags=True) for t in tabs]
    bnos.run_chains_multi(tabs, states, iters, seed, chain_offset=11)
    torch.cuda.synchronize()
    for k, t in enumerate(tabs):
        ref = t.new_chain_state(C, iters, trace_every=1, flags=True)
        t.run_chains(ref, iters, seed, chain_offset=11 + k * C)
        torch.cuda.synchronize()
        for key in ("orders", "scores", "best_graphs", "best_scores", "accepted", "trace", "accept_flags"):
            assert torch.equal(states[k][key], ref[key]), (k, key)
    for t in tabs:
        t.free()


def test_edge_trace_matches_oracle_replay(bnos, tiny8):
    # the traced edge bits are the greedy graph of each chain's current order,
    # replayed on the oracle from its own accept decisions
    w, t, orc = tiny8
    n, K = w.n, w.K
    edges = [(1, 0), (2, 5), (3, 1), (7, 6), (4, 2), (0, 3), (5, 7)]
    C, iters, seed, every = 6, 300, 41, 3
    st = t.new_chain_state(C, iters, trace_every=every, flags=True, edges=edges)
    t.run_chains(st, iters, seed, trace_every=every)
    et = st["edge_trace"].cpu().numpy().view(np.uint32)
    flags = st["accept_flags"].cpu().numpy()
    compared = 0
    for c in range(C):
        res = oracle.run_chain(orc, K, seed, c, iters, target=0, round_f32=True)
        if not np.array_equal(flags[c, :iters].astype(bool), res["acc"].astype(bool)):
            continue                       # a near-tie decision went the other way
        compared += 1
        cur = list(oracle.initial_order(seed, c, n))
        for it in range(iters + 1):
            if it > 0 and res["acc"][it - 1]:
                a, b = oracle.swap_pair(seed, c, n, it)
                cur[a], cur[b] = cur[b], cur[a]
            if it % every:
                continue
            best = oracle.score_order(orc, K, cur, round_f32=True)[2]
            want = sum(1 << e for e, (ch, pa) in enumerate(edges) if (int(best[ch]) >> pa) & 1)
            assert int(et[c, it // every]) == want, (c, it)
    assert compared >= C - 1
    # resumed runs continue the same trace
    a = t.new_chain_state(C, 120, trace_every=every, edges=edges)
    t.run_chains(a, 120, seed, trace_every=every)
    b = dict(a)
    b["trace"] = torch.zeros((C, 180 // every + 1), dtype=torch.float64, device="cuda")
    b["edge_trace"] = torch.zeros((C, 180 // every + 1), dtype=torch.int32, device="cuda")
    t.run_chains(b, 180, seed, first_iteration=120, trace_every=every)
    torch.cuda.synchronize()
    whole = et
    assert np.array_equal(a["edge_trace"].cpu().numpy().view(np.uint32), whole[:, :120 // every + 1])
    assert np.array_equal(b["edge_trace"].cpu().numpy().view(np.uint32), whole[:, 120 // every:])


@pytest.mark.parametrize("bt", [2, 8])
def test_chains_match_oracle_other_block_shapes(bnos, tiny8, bt):
    """Chain sweeps with 2 or 8 chains per scoring block (4 is the default)."""
    w, t, orc = tiny8
    iters, C = 1000, 12
    t.set_launch(C, orders_per_block=bt)
    try:
        g = gpu_chains(t, C, iters, seed=103)
    finally:
        t.set_launch(C)
    assert compare_chains(g, orc, w.K, 103, iters, 0) >= C - 1


def test_mixed40_chains_match_oracle_golden(bnos):
    # 4 oracle chains x 200 iterations on the 40-node table (stored by a script that
    # calls only the oracle), replayed inside a launch of 256 chains -- the batched
    # benchmark's shape -- on the same random-number streams
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mixed40_chains.json")) as f:
        gold = json.load(f)
    w = datagen.WORKLOADS[gold["workload"]]
    assert (w.n, w.K, w.N) == (gold["n"], gold["K"], gold["N"])
    net, prior = datagen.make(w)
    t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior)
    iters, seed = gold["iterations"], gold["seed"]
    g = gpu_chains(t, 256, iters, seed=seed)
    t.free()
    for rec in gold["chains"]:
        c = rec["chain"]
        flags = g["accept_flags"][c, :iters].astype(bool)
        mism = np.nonzero(flags != np.asarray(rec["acc"], dtype=bool))[0]
        if len(mism):
            # a decision may differ only where the oracle's |ln u - delta| is within TAU
            k = int(mism[0])
            assert rec["margin"][k] <= TAU, (c, k + 1, rec["margin"][k])
            np.testing.assert_allclose(g["trace"][c, :k + 1], rec["trace"][:k + 1], rtol=REL)
            continue
        np.testing.assert_allclose(g["trace"][c, :iters + 1], rec["trace"], rtol=REL)
        assert list(g["orders"][c]) == rec["order"], c
        assert [int(x) for x in g["best_graphs"][c].view(np.uint64)] == rec["best_graph"], c
        assert abs(g["best_scores"][c] - rec["best_score"]) <= REL * abs(rec["best_score"])
        assert int(g["accepted"][c]) == rec["accepted"]


def test_chain_sweep_autotune_picks_a_shape_and_keeps_the_chain(bnos, prior20):
    # the tuner times real sweeps (from a copy of burned-in chains) and stores the
    # fastest shape for this chain count; the tuned sweep takes the same decisions
    w, t, orc = prior20
    C, burn, iters = 32, 200, 150
    st = t.new_chain_state(C, burn, trace_every=burn)
    t.run_chains(st, burn, seed=5, trace_every=burn)
    before = {k: st[k].clone() for k in ("orders", "scores", "best_graphs", "best_scores", "accepted")}
    cs, bt, ms = t.chains_autotune(C, 32, seed=6, state=st, first_iteration=burn, reps=1)
    torch.cuda.synchronize()
    for k, v in before.items():               # the caller's state is not written
        assert torch.equal(st[k], v), k
    assert cs in (1, 2, 4, 8, 16) and bt in (1, 2, 4, 8) and ms > 0
    runs = []
    for shape in ("tuned", "default"):
        if shape == "default":
            t.chains_set_launch(C, 0, 0)
        s2 = {k: v.clone() for k, v in before.items()}
        s2["trace"] = torch.zeros((C, iters + 1), dtype=torch.float64, device="cuda")
        s2["accept_flags"] = torch.zeros((C, iters), dtype=torch.uint8, device="cuda")
        t.run_chains(s2, iters, seed=7, first_iteration=burn)
        torch.cuda.synchronize()
        runs.append({k: v.cpu().numpy() for k, v in s2.items()})
    a, b = runs
    assert np.array_equal(a["accept_flags"], b["accept_flags"])
    assert np.array_equal(a["orders"], b["orders"])
    assert np.array_equal(a["best_graphs"], b["best_graphs"])
    np.testing.assert_allclose(a["trace"], b["trace"], rtol=REL)


@pytest.mark.parametrize("bt", [1, 4, 8])
def test_score_bound_leaves_chain_sweeps_unchanged(bnos, bt):
    # 128 chains x 150 iterations on the 40-node table with and without the score
    # bound, for several chains per block: the same decisions, orders, best graphs
    # and (bitwise) the same traced scores
    w = datagen.WORKLOADS["mixed40"]
    net, prior = datagen.make(w)
    t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior)
    C, iters = 128, 150
    runs = []
    try:
        t.chains_set_launch(C, 0, bt)
        for on in (False, True):
            t.score_bound(on)
            st = t.new_chain_state(C, iters, trace_every=1, flags=True)
            t.run_chains(st, iters, seed=31)
            torch.cuda.synchronize()
            runs.append({k: v.cpu().numpy() for k, v in st.items() if v is not None})
    finally:
        t.score_bound(True)
        t.free()
    a, b = runs
    for k in ("accept_flags", "orders", "best_graphs", "best_scores", "accepted", "scores", "trace"):
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k
