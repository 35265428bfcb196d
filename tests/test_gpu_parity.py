"""GPU parity: the HIP library against the CPU oracle on the same seeded inputs.

Bars: counts and argmax parent sets bit-exact; stored FP32 scores within
2 ulp of the oracle's FP64 value; log-scores within 1e-5 relative.  The
oracle takes its argmax on its own scores rounded to FP32, the precision in
which the library stores scores and decides the argmax.
"""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1210_5128_amd import datagen

pytestmark = pytest.mark.gpu

REL = 1e-5
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def bnos():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_5128_amd import bnos as b
    return b


def ulp32(x):
    x = np.abs(np.asarray(x, dtype=np.float64)).astype(np.float32)
    return np.spacing(x).astype(np.float64)


def dev_score(table, orders, want_nodes=True):
    dev = torch.device("cuda")
    B, n = orders.shape
    o = torch.from_numpy(np.ascontiguousarray(orders, dtype=np.int32)).to(dev)
    lse = torch.empty(B, dtype=torch.float64, device=dev)
    mx = torch.empty(B, dtype=torch.float64, device=dev)
    best = torch.empty((B, n), dtype=torch.int64, device=dev)
    nl = torch.empty((B, n), dtype=torch.float64, device=dev) if want_nodes else None
    ns = torch.empty((B, n), dtype=torch.float32, device=dev) if want_nodes else None
    table.score_orders(o, lse, mx, best, nl, ns)
    torch.cuda.synchronize()
    out = dict(lse=lse.cpu().numpy(), max=mx.cpu().numpy(),
               best=best.cpu().numpy().view(np.uint64))
    if want_nodes:
        out["node_lse"] = nl.cpu().numpy()
        out["node_second"] = ns.cpu().numpy()
    return out


def check_orders_against_oracle(got, orc_table, K, orders):
    ulp_ties = 0
    for b in range(orders.shape[0]):
        wl, wm, wb, wnl, wnb, wns = oracle.score_order(orc_table, K, orders[b], round_f32=True)
        assert abs(got["lse"][b] - wl) <= REL * max(1.0, abs(wl)), (b, got["lse"][b], wl)
        assert abs(got["max"][b] - wm) <= REL * max(1.0, abs(wm)), (b, got["max"][b], wm)
        for i in range(orders.shape[1]):
            if int(got["best"][b, i]) != int(wb[i]):
                # allowed only when the oracle's FP64 scores of the two picks are within 2 ulp32
                from oracle import rank
                a = orc_table[i, rank(orders.shape[1], K, i, int(got["best"][b, i]))]
                c = orc_table[i, rank(orders.shape[1], K, i, int(wb[i]))]
                assert abs(a - c) <= 2 * ulp32(c), (b, i, got["best"][b, i], wb[i], a, c)
                ulp_ties += 1
        if "node_lse" in got:
            np.testing.assert_allclose(got["node_lse"][b], wnl, rtol=REL, atol=1e-6)
            sec = got["node_second"][b].astype(np.float64)
            fin = np.isfinite(wns)
            assert np.array_equal(np.isfinite(sec), fin)
            np.testing.assert_allclose(sec[fin], wns[fin], rtol=0, atol=0)
            assert math.isclose(got["node_lse"][b].sum(), got["lse"][b], rel_tol=1e-12, abs_tol=1e-9)
    return ulp_ties


# ------------------------------------------------------------------ fixtures per workload

def make_tables(bnos, wname, with_oracle=True):
    w = datagen.WORKLOADS[wname]
    net, prior = datagen.make(w)
    t = bnos.build_score_table(net.data, net.arities, w.K, ess=w.ess, prior=prior)
    orc = oracle.build_table(net.data, net.arities, w.K, ess=w.ess, prior=prior) if with_oracle else None
    return w, net, prior, t, orc


@pytest.fixture(scope="module")
def tiny8(bnos):
    r = make_tables(bnos, "tiny8")
    yield r
    r[3].free()


@pytest.fixture(scope="module")
def prior20(bnos):
    r = make_tables(bnos, "prior20")
    yield r
    r[3].free()


# ------------------------------------------------------------------ counts

@pytest.mark.parametrize("wname", ["tiny8", "prior20"])
def test_counts_bit_exact(bnos, wname, request):
    # every (node, parent set) family of the table: 512 at n=8, K=3 and 100,720 at
    # n=20, K=4 (20.5M count cells), from the default build's joint histograms
    w, net, prior, t, orc = request.getfixturevalue(wname)
    S = oracle.num_sets(w.n - 1, w.K)
    nodes, masks = [], []
    for i in range(w.n):
        for r in range(S):
            nodes.append(i)
            masks.append(oracle.unrank(w.n, w.K, i, r))
    got = t.counts(nodes, masks, net.arities)
    assert len(got) == w.n * S
    for i, m, g in zip(nodes, masks, got):
        want = oracle.counts(net.data, net.arities, i, m)
        assert np.array_equal(g, want), (i, m)


def test_counts_per_family_path_bit_exact(bnos):
    # a table built with one histogram per family answers count queries with that code
    w = datagen.WORKLOADS["prior20"]
    net, prior = datagen.make(w)
    t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior, count_mode=1)
    rng = np.random.default_rng(4)
    S = oracle.num_sets(w.n - 1, w.K)
    nodes = [int(rng.integers(w.n)) for _ in range(2000)]
    masks = [oracle.unrank(w.n, w.K, i, int(rng.integers(S))) for i in nodes]
    got = t.counts(nodes, masks, net.arities)
    t.free()
    for i, m, g in zip(nodes, masks, got):
        assert np.array_equal(g, oracle.counts(net.data, net.arities, i, m)), (i, m)


# ------------------------------------------------------------------ table

@pytest.mark.parametrize("wname", ["tiny8", "prior20"])
def test_table_entries_and_scores(bnos, wname, request):
    w, net, prior, t, orc = request.getfixturevalue(wname)
    info = t.info()
    S = oracle.num_sets(w.n - 1, w.K)
    assert info["entries_per_node"] == S and info["n"] == w.n and info["K"] == w.K
    not_rne = 0
    for i in range(w.n):
        masks, scores = t.export(i)
        # every parent set of size <= K over the other nodes, once, ascending after removing bit i
        slot = [(int(m) & ((1 << i) - 1)) | ((int(m) >> (i + 1)) << i) for m in masks]
        assert slot == sorted(slot) and len(set(slot)) == S
        assert all(not (int(m) >> i) & 1 and bin(int(m)).count("1") <= w.K for m in masks)
        ranks = np.array([oracle.rank(w.n, w.K, i, int(m)) for m in masks])
        want = orc[i, ranks]
        diff = np.abs(scores.astype(np.float64) - want)
        assert np.all(diff <= 2 * ulp32(want)), (i, diff.max())
        not_rne += int(np.sum(scores != want.astype(np.float32)))
    assert not_rne <= max(2, S * w.n // 10000)


# ------------------------------------------------------------------ order scoring

@pytest.mark.parametrize("B", [1, 2, 3, 4, 5, 64])
def test_score_orders_tiny8(bnos, tiny8, B):
    w, net, prior, t, orc = tiny8
    orders = datagen.random_orders(w.n, B, seed=100 + B)
    got = dev_score(t, orders)
    assert check_orders_against_oracle(got, orc, w.K, orders) == 0


@pytest.mark.parametrize("B", [1, 7, 32])
def test_score_orders_prior20(bnos, prior20, B):
    w, net, prior, t, orc = prior20
    orders = datagen.random_orders(w.n, B, seed=200 + B)
    got = dev_score(t, orders)
    assert check_orders_against_oracle(got, orc, w.K, orders) == 0


def test_host_score_order_and_determinism(bnos, prior20):
    w, net, prior, t, orc = prior20
    orders = datagen.random_orders(w.n, 16, seed=5)
    a = dev_score(t, orders)
    b = dev_score(t, orders)
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k
    # the host entry point is the one-order launch: bitwise equal to B = 1, and
    # within FP32 summation-order noise of the 16-order launch (another chunk length)
    one = dev_score(t, orders[3:4])
    l, m, best = t.score_order(orders[3])
    assert l == one["lse"][0] and m == one["max"][0]
    assert np.array_equal(best, one["best"][0]) and np.array_equal(best, a["best"][3])
    assert abs(l - a["lse"][3]) <= 1e-9 * abs(l) and m == a["max"][3]


def test_invalid_orders(bnos, tiny8):
    w, net, prior, t, orc = tiny8
    orders = datagen.random_orders(w.n, 4, seed=9)
    orders[1, 2] = orders[1, 5]          # duplicate id
    orders[2, 0] = w.n + 3               # out of range
    got = dev_score(t, orders)
    assert np.isnan(got["lse"][1]) and np.isnan(got["max"][2])
    assert np.all(got["best"][1] == 0) and np.all(got["best"][2] == 0)
    ok = check_orders_against_oracle({k: v[[0, 3]] for k, v in got.items()}, orc, w.K, orders[[0, 3]])
    assert ok == 0
    with pytest.raises(bnos.BnosError) as e:
        t.score_order(orders[1])
    assert e.value.status == bnos.E_INVALID


# ------------------------------------------------------------------ edge cases

def test_empty_data_closed_form(bnos):
    for n, K in [(8, 3), (20, 4)]:
        data = np.zeros((0, n), dtype=np.int8)
        t = bnos.build_score_table(data, [2] * n, K)
        orders = datagen.random_orders(n, 3, seed=n)
        got = dev_score(t, orders)
        closed = sum(math.log(oracle.num_sets(p, K)) for p in range(n))
        np.testing.assert_allclose(got["lse"], closed, rtol=REL)
        assert np.all(got["max"] == 0.0) and np.all(got["best"] == 0)
        t.free()


@pytest.mark.parametrize("n,K,N,arities", [
    (1, 0, 50, (3,)),            # single node, only the empty set
    (6, 0, 100, (2, 3)),         # K = 0
    (5, 4, 37, (2, 3, 4)),       # K = n - 1, N not a multiple of 4
    (64, 2, 129, (2,)),          # the largest n, bit 63 in use
    (12, 3, 1, (4,)),            # one sample
    (9, 6, 200, (2,)),           # the largest K
    (10, 4, 300, (5, 6)),        # tables of up to 7,776 cells: one wavefront per block
])
def test_edge_shapes(bnos, n, K, N, arities):
    net = datagen.random_network(n, N, arities, min(3, n - 1), seed=n * 31 + K)
    t = bnos.build_score_table(net.data, net.arities, K)
    orc = oracle.build_table(net.data, net.arities, K)
    orders = datagen.random_orders(n, 5, seed=N)
    got = dev_score(t, orders)
    assert check_orders_against_oracle(got, orc, K, orders) == 0
    t.free()


def test_constant_data_and_log_gamma(bnos):
    n, K = 7, 3
    data = np.ones((300, n), dtype=np.int8)
    ar = [2, 3, 2, 2, 4, 2, 3]
    t = bnos.build_score_table(data, ar, K, log_gamma=-0.5, prior=np.full((n, n), 0.9, np.float32),
                               prior_mode=1)
    orc = oracle.build_table(data, ar, K, log_gamma=-0.5, prior=np.full((n, n), 0.9, np.float32),
                             prior_mode=1)
    orders = datagen.random_orders(n, 6, seed=1)
    got = dev_score(t, orders)
    assert check_orders_against_oracle(got, orc, K, orders) == 0
    t.free()


def test_build_validation_errors(bnos):
    data = np.zeros((4, 3), dtype=np.int8)
    with pytest.raises(bnos.BnosError) as e:
        bnos.build_score_table(data, [2, 2, 2], 3)            # K > n - 1
    assert e.value.status == bnos.E_RANGE
    bad = data.copy()
    bad[2, 1] = 2
    with pytest.raises(bnos.BnosError) as e:
        bnos.build_score_table(bad, [2, 2, 2], 1)             # state >= arity
    assert e.value.status == bnos.E_INVALID
    with pytest.raises(bnos.BnosError) as e:
        bnos.build_score_table(data, [2, 2, 2], 1, ess=0.0)
    assert e.value.status == bnos.E_INVALID
    with pytest.raises(bnos.BnosError) as e:
        bnos.build_score_table(data, [2, 2, 2], 1, prior=np.full((3, 3), np.nan, np.float32))
    assert e.value.status == bnos.E_INVALID


# ------------------------------------------------------------------ full-size spot checks

@pytest.fixture(scope="module")
def mixed60(bnos):
    w = datagen.WORKLOADS["mixed60"]
    net, prior = datagen.make(w)
    t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior)
    yield w, net, prior, t
    t.free()


def test_mixed60_counts_and_scores_sampled(bnos, mixed60):
    # 10^4 random (node, parent set) entries of the 60-node table: the counts of
    # the default build's joint-histogram path bit-exact, the stored scores
    # within 2 ulp(FP32) of the oracle's FP64 local score
    w, net, prior, t = mixed60
    rng = np.random.default_rng(60)
    S = oracle.num_sets(w.n - 1, w.K)
    assert t.info()["entries_per_node"] == S == 489406
    Q = 10000
    nodes = rng.integers(0, w.n, size=Q)
    idx = rng.integers(0, S, size=Q)
    exported = {i: t.export(i) for i in range(w.n)}
    masks = [int(exported[int(i)][0][int(e)]) for i, e in zip(nodes, idx)]
    got = t.counts(nodes, masks, net.arities)
    bad = [k for k in range(Q) if not np.array_equal(got[k], oracle.counts(net.data, net.arities, int(nodes[k]),
                                                                          masks[k]))]
    assert not bad, (len(bad), bad[:5])
    for i, m, e in zip(nodes[:2000], masks[:2000], idx[:2000]):
        ls = oracle.local_score(net.data, net.arities, int(i), m, prior=prior)
        assert abs(float(exported[int(i)][1][int(e)]) - ls) <= 2 * ulp32(ls), (i, m)


def mixed60_golden():
    with open(os.path.join(GOLDEN, "mixed60_orders.json")) as f:
        return json.load(f)


def check_against_golden(got, rows, idx, net, w, prior):
    """Full orders vs the oracle's enumeration on its own FP64 table (golden file):
    per-order log-sum-exp and max within 1e-5 relative; every node's log-sum-exp
    within 1e-5; best parent sets bit-exact except ulp-ties (the oracle's FP64
    scores of the two picks within 2 ulp(FP32), counted); second best within
    2 ulp(FP32)."""
    ties = 0
    for b, r in zip(idx, rows):
        assert abs(got["lse"][b] - r["lse"]) <= REL * abs(r["lse"]), (b, got["lse"][b], r["lse"])
        assert abs(got["max"][b] - r["max"]) <= REL * abs(r["max"]), (b, got["max"][b], r["max"])
        np.testing.assert_allclose(got["node_lse"][b], r["node_lse"], rtol=REL, atol=1e-6)
        for i in range(w.n):
            gm, om = int(got["best"][b, i]), int(r["best"][i])
            if gm != om:
                a = oracle.local_score(net.data, net.arities, i, gm, prior=prior)
                c = oracle.local_score(net.data, net.arities, i, om, prior=prior)
                assert abs(a - c) <= 2 * ulp32(c), (b, i, gm, om, a, c)
                ties += 1
            sec, osec = float(got["node_second"][b, i]), r["node_second"][i]
            if math.isinf(osec):
                assert math.isinf(sec) and sec < 0, (b, i)
            else:
                assert abs(sec - osec) <= 2 * ulp32(osec), (b, i, sec, osec)
    return ties


@pytest.mark.parametrize("shape", ["bench_b1", "default_b1", "batched256"])
def test_mixed60_full_orders_against_oracle(bnos, mixed60, shape):
    # every node of 8 random 60-node orders against the oracle's enumeration, at
    # one order per launch with the launch the benchmark times (16-step chunks,
    # one order per block, computed masks, tile skipping) and with the build's
    # default chunk, and inside one launch of 256 orders (16-step chunks, 4 orders
    # per block, stored masks)
    w, net, prior, t = mixed60
    g = mixed60_golden()
    assert (g["n"], g["K"], g["N"]) == (w.n, w.K, w.N)
    rows = g["orders"]
    orders = np.array([r["order"] for r in rows], dtype=np.int32)
    try:
        if shape == "batched256":
            t.set_launch(256, chunk_steps=16, orders_per_block=4)
            batch = datagen.random_orders(w.n, 256, seed=62)
            idx = [0, 37, 74, 111, 148, 185, 222, 255]
            batch[idx] = orders
            got = dev_score(t, batch)
            # the argmax and max order score do not depend on the launch shape
            one = dev_score(t, batch[100:101])
            assert np.array_equal(one["best"][0], got["best"][100])
            assert one["max"][0] == got["max"][100]
        else:
            t.set_launch(1, chunk_steps=16 if shape == "bench_b1" else 0, orders_per_block=1)
            parts = [dev_score(t, orders[b:b + 1]) for b in range(len(rows))]
            got = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
            idx = list(range(len(rows)))
        ties = check_against_golden(got, rows, idx, net, w, prior)
        assert ties == 0, ties
    finally:
        t.set_launch(1)
        t.set_launch(256)


def test_mixed60_orders_against_direct_oracle(bnos, mixed60):
    w, net, prior, t = mixed60
    orders = datagen.random_orders(w.n, 8, seed=61)
    got = dev_score(t, orders)
    # global properties at any size
    assert np.all(got["lse"] >= got["max"])
    np.testing.assert_allclose(got["node_lse"].sum(axis=1), got["lse"], rtol=1e-12)
    # per-node spot checks against scoring straight from the data
    checks = [(0, 12), (1, 20), (2, 27), (5, 59)]     # (order, position)
    for b, p in checks:
        node = int(orders[b, p])
        pred = 0
        for v in orders[b, :p]:
            pred |= 1 << int(v)
        l, best, bm, sec = oracle.score_node_direct(net.data, net.arities, w.K, node, pred,
                                                    prior=prior, round_f32=True)
        assert abs(got["node_lse"][b, node] - l) <= REL * max(1.0, abs(l))
        assert int(got["best"][b, node]) == bm
        assert float(got["node_second"][b, node]) == sec


@pytest.mark.parametrize("B", [1, 3, 8, 20])
def test_tile_skipping_is_bitwise_identical(bnos, mixed60, B):
    w, net, prior, t = mixed60
    orders = datagen.random_orders(w.n, B, seed=90 + B)
    t.tile_skip(False)
    full = dev_score(t, orders)
    t.tile_skip(True)
    skip = dev_score(t, orders)
    loaded, per_pass = t.count_tiles(torch.from_numpy(orders).cuda())
    for k in full:
        assert np.array_equal(full[k].view(np.uint8), skip[k].view(np.uint8)), k
    passes = -(-B // (4 if B >= 4 else (2 if B >= 2 else 1)))    # orders per block without tuning
    assert 0 < loaded < passes * per_pass


def test_tile_skipping_small_tables(bnos, prior20):
    w, net, prior, t, orc = prior20
    orders = datagen.random_orders(w.n, 9, seed=3)
    t.tile_skip(False)
    full = dev_score(t, orders)
    t.tile_skip(True)
    skip = dev_score(t, orders)
    for k in full:
        assert np.array_equal(full[k].view(np.uint8), skip[k].view(np.uint8)), k
    assert check_orders_against_oracle(skip, orc, w.K, orders) == 0


@pytest.mark.parametrize("chunk_steps", [1, 2, 4, 16])
def test_chunk_length_option_matches_oracle(bnos, prior20, chunk_steps):
    # every chunk length (and the row padding it implies) gives the oracle's result
    w, net, prior, t0, orc = prior20
    t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior, chunk_steps=chunk_steps)
    try:
        orders = datagen.random_orders(w.n, 11, seed=40 + chunk_steps)
        got = dev_score(t, orders)
        assert check_orders_against_oracle(got, orc, w.K, orders) == 0
        ref = dev_score(t0, orders)
        assert np.array_equal(got["best"], ref["best"])
        assert np.array_equal(got["node_second"].view(np.uint32), ref["node_second"].view(np.uint32))
    finally:
        t.free()


def test_autotune_is_per_batch_bucket(bnos, mixed60):
    w, net, prior, t = mixed60
    o1 = torch.from_numpy(datagen.random_orders(w.n, 1, seed=70)).cuda()
    o20 = torch.from_numpy(datagen.random_orders(w.n, 20, seed=71)).cuda()
    before = dev_score(t, o20.cpu().numpy())
    cs1, bt1, g1, ms1 = t.autotune(o1, reps=2)
    assert cs1 in (1, 2, 4, 8, 16) and bt1 == 1 and g1 in (0, 1) and ms1 > 0
    single = dev_score(t, o1.cpu().numpy())
    cs20, bt20, g20, ms20 = t.autotune(o20, reps=2)
    assert cs20 in (1, 2, 4, 8, 16) and bt20 in (1, 2, 4, 8) and g20 in (0, 1) and ms20 > 0
    # tuning the 16+ bucket leaves the single-order launch as it was
    again = dev_score(t, o1.cpu().numpy())
    for k in single:
        assert np.array_equal(single[k].view(np.uint8), again[k].view(np.uint8)), k
    after = dev_score(t, o20.cpu().numpy())
    assert np.array_equal(after["best"], before["best"])
    assert np.array_equal(after["node_second"].view(np.uint32), before["node_second"].view(np.uint32))
    # another chunk length adds the FP32 partial sums in another order: ln s of
    # each node moves by a few 1e-7, the per-order sum of 60 nodes by ~1e-6
    np.testing.assert_allclose(after["node_lse"], before["node_lse"], rtol=0, atol=2e-6)
    np.testing.assert_allclose(after["lse"], before["lse"], rtol=0, atol=2e-5)


@pytest.mark.parametrize("n,K,N,arities,with_prior", [
    (8, 3, 200, (2,), False),
    (20, 4, 1000, (3,), True),
    (9, 6, 200, (2,), False),
    (10, 4, 300, (5, 6), True),
    (64, 2, 129, (2,), False),
    (1, 0, 50, (3,), False),
])
def test_joint_and_family_histograms_give_the_same_table(bnos, n, K, N, arities, with_prior):
    net = datagen.random_network(n, N, arities, min(3, n - 1), seed=n + 7 * K)
    prior = datagen.random_prior(n, seed=n) if with_prior else None
    a = bnos.build_score_table(net.data, net.arities, K, prior=prior, count_mode=0)
    b = bnos.build_score_table(net.data, net.arities, K, prior=prior, count_mode=1)
    try:
        for i in range(n):
            ma, sa = a.export(i)
            mb, sb = b.export(i)
            assert np.array_equal(ma, mb), i
            assert np.array_equal(sa.view(np.uint32), sb.view(np.uint32)), i
        orders = datagen.random_orders(n, 4, seed=3)
        ga, gb = dev_score(a, orders), dev_score(b, orders)
        for k in ga:
            assert np.array_equal(ga[k].view(np.uint8), gb[k].view(np.uint8)), k
    finally:
        a.free()
        b.free()


@pytest.mark.parametrize("n,K,N,arities", [
    (8, 3, 200, (2,)), (20, 4, 1000, (3,)), (64, 2, 129, (2,)), (7, 1, 60, (2, 3)), (5, 0, 40, (2,)),
])
def test_gather_pass_matches_streaming_and_oracle(bnos, n, K, N, arities):
    net = datagen.random_network(n, N, arities, min(3, n - 1), seed=3 * n + K)
    t = bnos.build_score_table(net.data, net.arities, K)
    orc = oracle.build_table(net.data, net.arities, K)
    try:
        orders = datagen.random_orders(n, 6, seed=11 + n)
        stream = dev_score(t, orders)
        t.set_launch(6, gather=True)
        got = dev_score(t, orders)
        assert check_orders_against_oracle(got, orc, K, orders) == 0
        assert np.array_equal(got["best"], stream["best"])
        assert np.array_equal(got["node_second"].view(np.uint32), stream["node_second"].view(np.uint32))
        np.testing.assert_allclose(got["lse"], stream["lse"], rtol=1e-9)
        again = dev_score(t, orders)                     # deterministic
        for k in got:
            assert np.array_equal(got[k].view(np.uint8), again[k].view(np.uint8)), k
        bad = orders.copy()
        bad[2, 0] = bad[2, 1]                             # not a permutation
        b = dev_score(t, bad)
        assert np.isnan(b["lse"][2]) and np.all(b["best"][2] == 0)
        assert np.array_equal(b["best"][[0, 1, 3, 4, 5]], got["best"][[0, 1, 3, 4, 5]])
    finally:
        t.free()


def test_gather_pass_on_the_60_node_table(bnos, mixed60):
    w, net, prior, t = mixed60
    orders = datagen.random_orders(w.n, 3, seed=77)
    t.set_launch(3, gather=False)
    stream = dev_score(t, orders)
    t.set_launch(3, gather=True)
    got = dev_score(t, orders)
    t.set_launch(3, gather=False)
    assert np.array_equal(got["best"], stream["best"])
    np.testing.assert_allclose(got["node_lse"], stream["node_lse"], rtol=1e-9)
    assert np.array_equal(got["node_second"].view(np.uint32), stream["node_second"].view(np.uint32))


def test_gather_needs_small_K(bnos):
    net = datagen.random_network(8, 50, (2,), 3, seed=1)
    t = bnos.build_score_table(net.data, net.arities, 5)
    with pytest.raises(bnos.BnosError) as e:
        t.set_launch(1, gather=True)
    assert e.value.status == bnos.E_RANGE
    t.free()


# ------------------------------------------------------------------ computed masks (one order per block)

def same_bits(a, b):
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k


@pytest.mark.parametrize("n,K,N,arities", [
    (8, 3, 200, (2,)), (20, 4, 1000, (3,)), (64, 2, 129, (2,)), (64, 1, 60, (2,)), (1, 0, 50, (3,)),
    (12, 0, 40, (2,)), (9, 6, 200, (2,)), (33, 5, 80, (2,)), (63, 2, 100, (2,)), (61, 1, 80, (2,)),
    (62, 1, 80, (2,)),
])
def test_computed_masks_are_bitwise_the_stored_ones(bnos, n, K, N, arities):
    net = datagen.random_network(n, N, arities, min(3, n - 1), seed=7 * n + K)
    t = bnos.build_score_table(net.data, net.arities, K)
    orc = oracle.build_table(net.data, net.arities, K) if n <= 20 else None
    try:
        B = 7
        orders = datagen.random_orders(n, B, seed=13 + n + K)
        if n > 1:
            orders[4, 0] = orders[4, 1]                   # not a permutation
        t.set_launch(B, orders_per_block=1)
        for skip in (True, False):
            t.tile_skip(skip)
            t.computed_masks(False)
            stored = dev_score(t, orders)
            t.computed_masks(True)
            got = dev_score(t, orders)
            same_bits(got, stored)
        t.tile_skip(True)
        ok = [b for b in range(B) if len(set(orders[b])) == n]
        if orc is not None:
            check_orders_against_oracle({k: v[ok] for k, v in got.items()}, orc, K, orders[ok])
        for b in set(range(B)) - set(ok):
            assert np.isnan(got["lse"][b]) and np.all(got["best"][b] == 0)
    finally:
        t.free()


def test_computed_masks_on_the_60_node_table(bnos, mixed60):
    w, net, prior, t = mixed60
    orders = datagen.random_orders(w.n, 4, seed=123)
    for cs in (1, 8, 16):
        t.set_launch(1, chunk_steps=cs)
        for b in range(4):
            t.computed_masks(False)
            stored = dev_score(t, orders[b:b + 1])
            t.computed_masks(True)
            same_bits(dev_score(t, orders[b:b + 1]), stored)
    t.set_launch(1)


def test_kernel_timing_samples_and_ring(bnos, prior20):
    w, net, prior, t, *_ = prior20
    o = torch.from_numpy(datagen.random_orders(w.n, 1, seed=3)).cuda()
    lse = torch.empty(1, dtype=torch.float64, device="cuda")
    mx = torch.empty_like(lse)
    best = torch.empty((1, w.n), dtype=torch.int64, device="cuda")
    t.set_launch(1, orders_per_block=1)
    t.timing(True, every=4)
    for _ in range(10):
        t.score_orders(o, lse, mx, best)
    ms, launches, passes = t.timing_read()
    assert launches == 3 and passes == 3 and ms > 0          # launches 0, 4 and 8
    t.timing(True)                                            # every launch; more than the 256-pair ring
    for _ in range(300):
        t.score_orders(o, lse, mx, best)
    ms2, launches2, passes2 = t.timing_read()
    assert launches2 == 300 and passes2 == 300 and ms2 > 0
    t.timing(False)
    with pytest.raises(bnos.BnosError) as e:
        bnos._check(bnos._lib.bnos_table_timing(t._h, -1))
    assert e.value.status == bnos.E_RANGE
    t.set_launch(1)


def test_maximum_size_64_nodes_K4(bnos):
    """The largest table the masks allow: n = 64, K = 4 (637,393 entries per node),
    spot-checked per node against scoring straight from the data, one order per launch
    (computed masks) and four per launch (stored masks)."""
    net = datagen.random_network(64, 2000, (2, 3, 4), 3, seed=64)
    K = 4
    t = bnos.build_score_table(net.data, net.arities, K)
    try:
        assert t.info()["entries_per_node"] == oracle.num_sets(63, K) == 637393
        orders = datagen.random_orders(64, 4, seed=65)
        t.set_launch(1, orders_per_block=1)
        singles = [dev_score(t, orders[b:b + 1]) for b in range(4)]
        t.computed_masks(False)
        stored = [dev_score(t, orders[b:b + 1]) for b in range(4)]
        t.computed_masks(True)
        for a, b in zip(singles, stored):
            same_bits(a, b)
        batch = dev_score(t, orders)
        for b in range(4):
            one = singles[b]
            assert one["lse"][0] >= one["max"][0]
            np.testing.assert_allclose(one["node_lse"].sum(), one["lse"][0], rtol=1e-12)
            np.testing.assert_allclose(batch["lse"][b], one["lse"][0], rtol=1e-9)
            assert np.array_equal(batch["best"][b], one["best"][0])
        for b, p in [(0, 0), (1, 14), (2, 27), (3, 33)]:
            node = int(orders[b, p])
            pred = 0
            for v in orders[b, :p]:
                pred |= 1 << int(v)
            l, best, bm, sec = oracle.score_node_direct(net.data, net.arities, K, node, pred, round_f32=True)
            for got, row in ((singles[b], 0), (batch, b)):
                assert abs(got["node_lse"][row, node] - l) <= REL * max(1.0, abs(l))
                assert int(got["best"][row, node]) == bm
                assert float(got["node_second"][row, node]) == sec
    finally:
        t.set_launch(1)
        t.free()


@pytest.mark.parametrize("bt", [2, 8])
def test_batched_block_shapes_match_oracle(bnos, prior20, bt):
    """Scoring launches with 2 or 8 orders per block (4 is the default for 4+ orders)."""
    w, net, prior, t, orc = prior20
    orders = datagen.random_orders(w.n, 11, seed=40 + bt)
    t.set_launch(11, orders_per_block=bt)
    try:
        got = dev_score(t, orders)
    finally:
        t.set_launch(11)
    check_orders_against_oracle(got, orc, w.K, orders)


def test_score_bound_is_bitwise_identical_on_the_60_node_table(bnos, mixed60):
    # one order per launch: random orders, the generating DAG's topological order
    # (every node's best parent sets usable: the bound leaves out most tiles) and
    # its reverse (no parent usable: the bound is weak); every output bitwise equal
    # to tile skipping without the bound, and never more tiles read
    w, net, prior, t = mixed60
    topo = np.asarray(net.perm, dtype=np.int32)
    orders = np.concatenate([datagen.random_orders(w.n, 10, seed=501), topo[None], topo[::-1][None]])
    t.set_launch(1, chunk_steps=16)
    fewer = 0
    try:
        for b in range(orders.shape[0]):
            o = orders[b:b + 1]
            t.score_bound(False)
            plain = dev_score(t, o)
            n_plain, _ = t.count_tiles(torch.from_numpy(o).cuda())
            t.score_bound(True)
            got = dev_score(t, o)
            n_bound, _ = t.count_tiles(torch.from_numpy(o).cuda())
            same_bits(got, plain)
            assert n_bound <= n_plain
            fewer += n_bound < n_plain
        # the topological order: most of the table is left out
        o = topo[None]
        t.score_bound(False)
        n_plain, _ = t.count_tiles(torch.from_numpy(o).cuda())
        t.score_bound(True)
        n_bound, _ = t.count_tiles(torch.from_numpy(o).cuda())
        assert n_bound < 0.2 * n_plain, (n_bound, n_plain)
        assert fewer >= 8
    finally:
        t.score_bound(True)
        t.set_launch(1)


@pytest.mark.parametrize("n,K,N,arities", [
    (8, 3, 200, (2,)), (20, 4, 1000, (3,)), (64, 2, 129, (2,)), (1, 0, 50, (3,)), (12, 0, 40, (2,)),
    (9, 6, 200, (2,)), (33, 5, 80, (2,)), (61, 1, 80, (2,)), (40, 4, 3000, (2, 3, 4)),
])
def test_score_bound_edge_shapes(bnos, n, K, N, arities):
    # bound on vs off, one order per block, several chunk lengths: bitwise equal,
    # and equal to the oracle where it is small enough to build
    net = datagen.random_network(n, N, arities, min(4, n - 1), seed=11 * n + K)
    t = bnos.build_score_table(net.data, net.arities, K)
    orc = oracle.build_table(net.data, net.arities, K) if n <= 20 else None
    try:
        orders = datagen.random_orders(n, 6, seed=17 + n)
        orders = np.concatenate([orders, np.asarray(net.perm, dtype=np.int32)[None]])
        for cs in (1, 4, 16):
            try:
                t.set_launch(orders.shape[0], chunk_steps=cs, orders_per_block=1)
            except bnos.BnosError:       # longer than this table's row padding
                continue
            t.score_bound(False)
            plain = dev_score(t, orders)
            t.score_bound(True)
            got = dev_score(t, orders)
            same_bits(got, plain)
        if orc is not None:
            assert check_orders_against_oracle(got, orc, K, orders) == 0
    finally:
        t.free()


@pytest.mark.parametrize("bt", [2, 4, 8])
def test_score_bound_several_orders_per_block(bnos, mixed60, bt):
    # a block of several orders reads a tile if any of its orders needs it and each
    # order folds only its own: bitwise the same as without the bound, fewer tiles
    w, net, prior, t = mixed60
    B = 16
    orders = datagen.random_orders(w.n, B, seed=700 + bt)
    orders[3] = np.asarray(net.perm, dtype=np.int32)
    t.set_launch(B, orders_per_block=bt)
    try:
        t.score_bound(False)
        plain = dev_score(t, orders)
        n_plain, _ = t.count_tiles(torch.from_numpy(orders).cuda())
        t.score_bound(True)
        got = dev_score(t, orders)
        n_bound, _ = t.count_tiles(torch.from_numpy(orders).cuda())
        same_bits(got, plain)
        assert n_bound < n_plain, (n_bound, n_plain)
    finally:
        t.score_bound(True)
        t.set_launch(B)


def test_build_from_device_data_matches_host_data(bnos):
    # the same rows handed over as a device tensor give the same table, bit for
    # bit; an out-of-range state in device data is rejected like host data
    w = datagen.WORKLOADS["prior20"]
    net, prior = datagen.make(w)
    th = bnos.build_score_table(net.data, net.arities, w.K, prior=prior)
    dd = torch.from_numpy(np.ascontiguousarray(net.data, dtype=np.int8)).cuda()
    td = bnos.build_score_table(dd, net.arities, w.K, prior=prior)
    try:
        for v in (0, 7, w.n - 1):
            mh, sh = th.export(v)
            md, sd = td.export(v)
            assert np.array_equal(mh, md) and np.array_equal(sh.view(np.uint32), sd.view(np.uint32))
        bad = dd.clone()
        bad[5, 3] = int(net.arities[3])
        with pytest.raises(bnos.BnosError) as e:
            bnos.build_score_table(bad, net.arities, w.K)
        assert e.value.status == bnos.E_INVALID
    finally:
        th.free()
        td.free()


@pytest.mark.parametrize("log_gamma,prior_mode", [(-8.0, 0), (3.0, 0), (0.0, 1)])
def test_score_bound_with_structure_penalty_and_priors(bnos, log_gamma, prior_mode):
    # the bound's candidates and tile maxima follow the stored scores whatever shifts
    # them: a structure penalty per parent (either sign) or the paper's R-form prior
    # with strong entries; bound on vs off bitwise, and against the oracle
    w = datagen.WORKLOADS["prior20"]
    net, prior = datagen.make(w)
    if prior_mode == 1:
        prior = np.clip((1.0 + prior) / 2.0, 0.0, 1.0).astype(np.float32)
        prior[np.abs(prior - 0.5) > 0.3] = 1.0          # a few confident edges
    t = bnos.build_score_table(net.data, net.arities, w.K, prior=prior, prior_mode=prior_mode,
                               log_gamma=log_gamma)
    orc = oracle.build_table(net.data, net.arities, w.K, prior=prior, prior_mode=prior_mode,
                             log_gamma=log_gamma)
    try:
        orders = np.concatenate([datagen.random_orders(w.n, 6, seed=41),
                                 np.asarray(net.perm, dtype=np.int32)[None]])
        t.set_launch(orders.shape[0], orders_per_block=1)
        t.score_bound(False)
        plain = dev_score(t, orders)
        t.score_bound(True)
        got = dev_score(t, orders)
        same_bits(got, plain)
        assert check_orders_against_oracle(got, orc, w.K, orders) == 0
    finally:
        t.free()
