"""Benchmark: order scoring on the 60-node, K=4 table (one MI355X).

One step = one pass of the hot path over one batch of synthetic input: B
random orders are scored against the resident local-score table (predecessor
masks, consistency filter, log-sum-exp + argmax + second best per node,
per-order FP64 sums).  The table build (counts + BDeu + prior) happens once
before the timed region and is reported as build_s.

Prints one JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "order-scores/s + HBM GB/s at n=60,K=4; ESS/s learned vs uniform-swap proposal"
HBM_PEAK_GBS = 8000.0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(net, prior, K: int, sample_nodes=(7, 41), seed: int = 3):
    """The CPU oracle scoring orders of the same workload, single-threaded.

    Sample: the oracle builds the FP64 rows of ``sample_nodes`` from the data,
    then scores each sampled node at every position 0..n-1 of random orders by
    enumeration.  Time per order = mean over the sampled nodes of the summed
    per-position time (every node visits every position once per order on
    average); the row build is timed separately per local score.
    """
    import oracle
    n = net.n
    rng = np.random.default_rng(seed)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    rows = {v: oracle.build_row(net.data, net.arities, K, v, prior=prior, threads=threads)
            for v in sample_nodes}
    t_build = time.perf_counter() - t0
    n_local = sum(len(r) for r in rows.values())
    per_node = []
    for v in sample_nodes:
        others = [m for m in range(n) if m != v]
        t = 0.0
        for p in range(n):
            pred_nodes = rng.choice(others, size=p, replace=False)
            pred = 0
            for m in pred_nodes:
                pred |= 1 << int(m)
            s = time.perf_counter()
            oracle.score_node_row(rows[v], n, K, v, pred)
            t += time.perf_counter() - s
        per_node.append(t)
    t_order = float(np.mean(per_node))
    # table build on one core: a slice of one node's row
    t0 = time.perf_counter()
    oracle.build_row(net.data, net.arities, K, sample_nodes[0], prior=prior, threads=1, ranks=(0, 20000))
    build_1core = 20000 / (time.perf_counter() - t0)
    # Metropolis-Hastings on the oracle: one chain on one core, and independent chains on
    # every core (threads; the C calls release the GIL), on the 20-node table of the
    # prior20 workload, whose oracle table builds in about a second
    from paper_1210_5128_amd import datagen
    from concurrent.futures import ThreadPoolExecutor
    w20 = datagen.WORKLOADS["prior20"]
    net20, prior20 = datagen.make(w20)
    tab20 = oracle.build_table(net20.data, net20.arities, w20.K, prior=prior20)
    it1 = 300
    t0 = time.perf_counter()
    oracle.run_chain(tab20, w20.K, 5, 0, it1)
    mh_1core = it1 / (time.perf_counter() - t0)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda c: oracle.run_chain(tab20, w20.K, 5, c, it1), range(threads)))
    mh_all = threads * it1 / (time.perf_counter() - t0)
    return {
        "value": 1.0 / t_order,
        "unit": "order-scores/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle FP64 rows of nodes {list(sample_nodes)} built from the data "
                   f"({n_local} local scores in {t_build:.1f} s on {threads} threads), then each node "
                   f"scored by enumeration on 1 thread at all {n} positions of random orders; "
                   f"seconds per order = mean per-node sum = {t_order:.4f}"),
        "build_local_scores_per_s": n_local / t_build,
        "build_threads": threads,
        "build_local_scores_per_s_1core": build_1core,
        "table_build_s_1core_estimate": n * oracle.num_sets(n - 1, K) / build_1core,
        "mh_iterations_per_s_1core_n60": 1.0 / t_order,
        "mh_note": ("an oracle MH iteration rescores the whole proposed order by enumeration, so at n=60 its "
                    "rate is the order-scoring rate above; measured directly on the 20-node prior20 table:"),
        "mh_iterations_per_s_1core_n20": mh_1core,
        "mh_iterations_per_s_all_cores_n20": mh_all,
        "mh_all_cores_threads": threads,
        "cpu_model": cpu_model(),
        "cpu_count": os.cpu_count(),
        "affinity_cores": len(os.sched_getaffinity(0)),
    }


def measured_traffic(batch: int, mode: str):
    """HBM bytes per k_score launch ("full" scan or tile "skip") from the committed
    rocprofv3 counter runs, or None when the scoring sources changed since they
    were taken or no run matches the batch size."""
    import hashlib
    try:
        recs = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
        h = hashlib.sha256()
        for f in recs["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
    except (OSError, ValueError, KeyError):
        return None
    if h.hexdigest() != recs.get("sources_sha256"):
        return None
    for rec in recs.get("runs", []):
        if rec.get("batch") == batch and rec.get("mode") == mode:
            return float(rec["bytes_per_launch"])
    return None


STATE_KEYS = ("orders", "scores", "best_graphs", "best_scores", "accepted")


def sample_until_mixed(table, state, C, first, block, max_blocks, seed, every, edges=None, mlp=None, eps=0.5,
                       rhat_target=1.05, target=0, done_when=None):
    """Advance burned-in chains (state after `first` iterations) in blocks of `block`
    iterations, tracing the score (and edge indicators) every `every` iterations, until
    the rank-normalised split-R-hat of the pooled trace is below `rhat_target` (or, with
    `done_when`, until done_when(score traces, edge traces) holds) or `max_blocks` blocks
    ran.  Returns (score traces [C][T], edge traces [C][T] or None,
    sampling seconds, iterations, accepted moves)."""
    import torch
    from paper_1210_5128_amd import ess as E
    dev = state["scores"].device
    traces, etr, secs, done = [], [], 0.0, 0
    acc0 = state["accepted"].clone()
    for k in range(max_blocks):
        s2 = {key: state[key] for key in STATE_KEYS}
        s2["trace"] = torch.zeros((C, block // every + 1), dtype=torch.float64, device=dev)
        if edges:
            s2["edges"] = np.asarray(edges, dtype=np.int32)
            s2["edge_trace"] = torch.zeros((C, block // every + 1), dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        table.run_chains(s2, block, seed, first_iteration=first + done, trace_every=every, mlp=mlp, eps=eps,
                         target=target)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        done += block
        traces.append(s2["trace"].cpu().numpy()[:, 1:])
        if edges:
            etr.append(s2["edge_trace"].cpu().numpy().view(np.uint32)[:, 1:])
        tr = np.concatenate(traces, axis=1)
        if done_when is not None:
            if done_when(tr, np.concatenate(etr, axis=1) if edges else None):
                break
        elif E.rhat_rank(tr, burn=0.0) < rhat_target:
            break
    acc = float((state["accepted"] - acc0).sum().item())
    return tr, (np.concatenate(etr, axis=1) if edges else None), secs, done, acc


def chain_stats(tr, et, secs, C, iters, acc, n_edges):
    """ESS figures of one sampler's post-burn-in traces: summed per-chain Geyer ESS, the
    rank-normalised multi-chain (bulk) ESS, rank split-R-hat, and per-edge bulk ESS."""
    from paper_1210_5128_amd import ess as E
    out = {"chains": C, "iterations": iters, "seconds": secs, "chain_iterations_per_s": C * iters / secs,
           "accept_rate": acc / (C * iters), "ess_summed": E.ess(tr, burn=0.0), "ess_bulk": E.ess_bulk(tr, burn=0.0),
           "rhat_rank": E.rhat_rank(tr, burn=0.0), "score_mean": float(tr.mean()),
           "score_mcse": E.mcse_mean(tr, burn=0.0)}
    out["ess_bulk_per_s"] = out["ess_bulk"] / secs
    out["ess_summed_per_s"] = out["ess_summed"] / secs
    if et is not None:
        ee = [E.ess_bulk(((et >> np.uint32(k)) & np.uint32(1)).astype(np.float64), burn=0.0) for k in range(n_edges)]
        out["edge_ess_bulk_min"] = float(np.nanmin(ee))
        out["edge_ess_bulk_min_per_s"] = out["edge_ess_bulk_min"] / secs
        out["edge_rhat_max"] = float(np.nanmax([E.rhat_rank(((et >> np.uint32(k)) & np.uint32(1)).astype(np.float64),
                                                            burn=0.0) for k in range(n_edges)]))
    return out


def agreement(tr_a, et_a, tr_b, et_b, n_edges):
    """Posterior mean score and edge frequencies of two samplers within 3 combined MCSE."""
    from paper_1210_5128_amd import ess as E
    d, tol, ok = E.agree_within_mcse(tr_a, tr_b, burn=0.0)
    out = {"score_mean_diff": d, "score_3mcse": tol, "score_agrees": ok}
    if et_a is not None and et_b is not None:
        agree, worst = 0, 0.0
        for k in range(n_edges):
            xa = ((et_a >> np.uint32(k)) & np.uint32(1)).astype(np.float64)
            xb = ((et_b >> np.uint32(k)) & np.uint32(1)).astype(np.float64)
            dk, tk, okk = E.agree_within_mcse(xa, xb, burn=0.0)
            agree += int(okk)
            worst = max(worst, dk)
        out.update(edges=n_edges, edges_agree=agree, edge_freq_max_diff=worst)
    return out


def bench_chains(bnos, datagen, wname: str, chains: int, block: int, burn: int, max_blocks: int,
                 seed: int = 102, every: int = 10):
    """Batched MH chains vs one chain on the same table.  Both burn in for `burn`
    iterations, then sample in blocks of `block` iterations until the rank split-R-hat of
    the score trace is below 1.05 (at most `max_blocks` blocks).  ESS/s uses the
    rank-normalised multi-chain ESS of the sampling phase; 'same_accuracy' states whether
    both reached R-hat < 1.05 and agree on the posterior mean score and on the frequencies
    of the 20 most uncertain edges within 3 MCSE.  The chain sweep's launch shape is
    autotuned on burned-in chains first (tuned vs default chain-iterations/s reported)."""
    import torch
    w = datagen.WORKLOADS[wname]
    net, prior = datagen.make(w)
    table = bnos.build_score_table(net.data, net.arities, w.K, ess=w.ess, prior=prior)
    out = {"workload": f"{w.name}: n={w.n}, K={w.K}, N={w.N}", "burn_in": burn, "trace_every": every}
    res = {}
    for label, C in (("batched", chains), ("single", 1)):
        st = table.new_chain_state(C, burn, trace_every=burn)
        t0 = time.perf_counter()
        table.run_chains(st, burn, seed, trace_every=burn)
        torch.cuda.synchronize()
        burn_s = time.perf_counter() - t0
        if label == "batched":
            # chain-sweep autotuner on copies of the burned-in chains, then tuned vs default
            cs, bt, ms = table.chains_autotune(C, 64, seed + 7, state=st, first_iteration=burn, reps=2)
            tuned = {"chunk_steps": cs, "orders_per_block": bt, "ms_per_iteration": ms}
            rates = {}
            for shape in ("default", "tuned"):
                if shape == "default":
                    table.chains_set_launch(C, 0, 0)
                else:
                    table.chains_set_launch(C, cs, bt)
                s2 = {k: st[k].clone() for k in STATE_KEYS}
                s2["trace"] = None
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                table.run_chains(s2, 2000, seed + 9, first_iteration=burn, trace_every=2000)
                torch.cuda.synchronize()
                rates[shape] = C * 2000 / (time.perf_counter() - t1)
            out["autotune"] = dict(tuned, chain_iterations_per_s_tuned=rates["tuned"],
                                   chain_iterations_per_s_default=rates["default"])
            print(f"# chains autotune: chunk {cs}, {bt} chains/block: {rates['tuned']:.0f} vs default "
                  f"{rates['default']:.0f} chain-it/s", file=sys.stderr, flush=True)
            edges = uncertain_edges(table, st["orders"], w.n)
            out["traced_edges"] = len(edges)
        tr, et, secs, iters, acc = sample_until_mixed(table, st, C, burn, block, max_blocks, seed + 1, every, edges)
        res[label] = (tr, et)
        out[label] = chain_stats(tr, et, secs, C, iters, acc, len(edges))
        out[label]["burn_in_seconds"] = burn_s
        print(f"# chains {label}: {C} x {iters} sampling iterations in {secs:.2f} s, bulk ESS/s "
              f"{out[label]['ess_bulk_per_s']:.1f}, R-hat {out[label]['rhat_rank']:.3f}", file=sys.stderr, flush=True)
    out["agreement"] = agreement(res["batched"][0], res["batched"][1], res["single"][0], res["single"][1], len(edges))
    b, sg = out["batched"], out["single"]
    out["ess_bulk_per_s_ratio_batched_vs_single"] = b["ess_bulk_per_s"] / max(sg["ess_bulk_per_s"], 1e-30)
    out["ess_summed_per_s_ratio_batched_vs_single"] = b["ess_summed_per_s"] / max(sg["ess_summed_per_s"], 1e-30)
    ag = out["agreement"]
    out["same_accuracy"] = bool(b["rhat_rank"] < 1.05 and sg["rhat_rank"] < 1.05 and ag["score_agrees"]
                                and ag.get("edges_agree", 0) == ag.get("edges", 0))
    if not out["same_accuracy"]:
        out["note"] = ("not an equal-accuracy comparison: the batched chains' multi-chain R-hat is "
                       f"{b['rhat_rank']:.2f} (the posterior has separated modes that no chain crosses in this "
                       "budget, which one chain's split-R-hat cannot see); the ESS/s ratio is throughput only")
    table.free()
    return out


def bench_uneven(bnos, datagen, n_datasets: int, chains: int, iters: int, seed: int = 202):
    """Uneven family (n ~ U[20,60], N ~ U[1000,5000], K=4): all datasets' chains in one
    set of launches vs one dataset at a time (chain-iterations/s)."""
    import torch
    tabs, ns = [], []
    t0 = time.perf_counter()
    for d in range(n_datasets):
        w = datagen.uneven_workload(d)
        net, _ = datagen.make(w)
        tabs.append(bnos.build_score_table(net.data, net.arities, w.K))
        ns.append(w.n)
    build_s = time.perf_counter() - t0
    table_bytes = sum(t.info()["device_bytes"] for t in tabs)
    states = [t.new_chain_state(chains, iters, trace_every=max(1, iters)) for t in tabs]
    bnos.run_chains_multi(tabs, states, 20, seed + 1, trace_every=20)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bnos.run_chains_multi(tabs, states, iters, seed, trace_every=iters)
    torch.cuda.synchronize()
    one = time.perf_counter() - t0
    t0 = time.perf_counter()
    for k, t in enumerate(tabs):
        t.run_chains(states[k], iters, seed, trace_every=iters, chain_offset=k * chains)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    total = n_datasets * chains * iters
    for t in tabs:
        t.free()
    print(f"# uneven: one launch {one:.2f} s, one at a time {seq:.2f} s", file=sys.stderr, flush=True)
    return {"datasets": n_datasets, "n": ns, "chains_per_dataset": chains, "iterations": iters,
            "tables_device_bytes": table_bytes, "build_s": build_s,
            "one_launch_s": one, "one_launch_chain_iterations_per_s": total / one,
            "one_at_a_time_s": seq, "one_at_a_time_chain_iterations_per_s": total / seq,
            "speedup": seq / one}


def bench_learned(bnos, datagen, wname: str, chains: int, moves: int, iters: int, epochs: int,
                  eps_list=(0.1,), seed: int = 404, max_blocks: int = 4, every: int = 5, single_blocks: int = 60):
    """Learned swap proposal: harvest `moves` accepted moves from uniform chains
    (which also serves as burn-in), train the network on the device, then resume
    every chain from its harvested state twice, with the uniform and with the
    learned proposal, on the same random-number streams; plus one uniform chain
    alone.  Each run samples in blocks of `iters` iterations until its rank
    split-R-hat is below 1.05 (at most max_blocks blocks); the single chain runs
    until it agrees with the batched uniform chains within 3 MCSE (at most
    single_blocks blocks).  Reported: bulk
    (rank-normalised multi-chain) ESS/s of the log-sum-exp trace and the smallest
    over the indicators of the 20 most uncertain edges, R-hat, acceptance,
    best-graph score, and whether learned and uniform agree within 3 MCSE."""
    import torch
    w = datagen.WORKLOADS[wname]
    net, prior = datagen.make(w)
    table = bnos.build_score_table(net.data, net.arities, w.K, ess=w.ess, prior=prior)
    n = w.n
    out = {"workload": f"{w.name}: n={n}, K={w.K}, N={w.N}", "chains": chains, "iterations": iters}
    # 1. harvest (uniform proposal, fresh start); the chains run until every one
    # has filled its share of the harvest
    cap = -(-moves // chains)
    st = table.new_chain_state(chains, 1, trace_every=0, harvest_cap=cap)
    t0 = time.perf_counter()
    done, block = 0, 2000
    while True:
        table.run_chains(st, block, seed + 1, first_iteration=done, trace_every=0)
        done += block
        torch.cuda.synchronize()
        if int(st["harvest_count"].min().item()) >= cap or done >= 400000:
            break
    cnt = st["harvest_count"].cpu().numpy()
    feats = torch.cat([st["harvest_feats"][c, :int(min(cnt[c], cap))] for c in range(chains)])
    pairs = torch.cat([st["harvest_pairs"][c, :int(min(cnt[c], cap))] for c in range(chains)])
    del st["harvest_feats"], st["harvest_pairs"]
    out["harvest"] = {"moves": int(feats.shape[0]), "iterations_per_chain": done,
                      "accept_rate": float(st["accepted"].sum().item()) / (chains * done),
                      "seconds": time.perf_counter() - t0}
    print(f"# harvest: {feats.shape[0]} moves in {done} iterations per chain, "
          f"{out['harvest']['seconds']:.1f} s", file=sys.stderr, flush=True)
    # 2. train
    m = bnos.Mlp()
    m.set_params(datagen.mlp_params(seed + 2, scale=0.5).astype(np.float32))
    m.fit_norm(feats)
    batch = 1024
    steps = epochs * ((feats.shape[0] + batch - 1) // batch)
    trace = torch.zeros(max(steps, 1), dtype=torch.float32, device=feats.device)
    t0 = time.perf_counter()
    m.train(feats, pairs, epochs=epochs, batch=batch, lr=2e-3, seed=seed + 3, loss_trace=trace)
    torch.cuda.synchronize()
    tr = trace.cpu().numpy()
    out["train"] = {"samples": int(feats.shape[0]), "epochs": epochs, "batch": batch, "steps": int(steps),
                    "seconds": time.perf_counter() - t0,
                    "loss_first": float(tr[:10].mean()), "loss_last": float(tr[-10:].mean()),
                    "uniform_pair_loss": float(np.log(n * (n - 1) / 2))}
    print(f"# train: {steps} steps in {out['train']['seconds']:.1f} s, loss {out['train']['loss_first']:.3f} -> "
          f"{out['train']['loss_last']:.3f} (uniform {out['train']['uniform_pair_loss']:.3f})",
          file=sys.stderr, flush=True)
    del feats, pairs
    # 3. the 20 most uncertain edges: greedy graphs of the chains' current orders,
    # edges whose frequency over chains is closest to 1/2
    edges = uncertain_edges(table, st["orders"], n)
    out["traced_edges"] = len(edges)
    # 4. resume every chain from its harvested state: uniform vs learned, and one uniform chain
    # alone, each sampling in blocks until its rank split-R-hat is below 1.05 (at most
    # max_blocks blocks of `iters` iterations)
    base = {k: v for k, v in st.items() if k in STATE_KEYS}
    runs = [("uniform", None, chains, 0.1)]
    for k, eps in enumerate(eps_list):
        runs.append(("learned" if k == 0 else f"learned_eps{eps:g}", m, chains, eps))
    runs.append(("single_uniform", None, 1, 0.1))
    res = {}
    for label, mlp, C, eps in runs:
        s2 = {k: v[:C].clone() for k, v in base.items()}
        stop, cap = None, max_blocks
        if label == "single_uniform":
            # one chain cannot see its own separated modes (its split-R-hat stays near 1), so it
            # runs until its estimates agree with the converged batched uniform ones within 3 MCSE
            ref_tr, ref_et = res["uniform"]

            def stop(tr_, et_, ref_tr=ref_tr, ref_et=ref_et):
                a_ = agreement(tr_, et_, ref_tr, ref_et, len(edges))
                return a_["score_agrees"] and a_.get("edges_agree", 0) == a_.get("edges", 0)
            cap = single_blocks
        tr, et, secs, its, acc = sample_until_mixed(table, s2, C, done, iters, cap, seed + 5, every,
                                                    edges, mlp=mlp, eps=eps, done_when=stop)
        res[label] = (tr, et)
        out[label] = chain_stats(tr, et, secs, C, its, acc, len(edges))
        out[label].update(eps=eps if mlp is not None else None,
                          best_score_max=float(s2["best_scores"].max().item()),
                          best_score_mean=float(s2["best_scores"].mean().item()))
        print(f"# {label}: {C} x {its} iterations in {secs:.2f} s, bulk ESS/s {out[label]['ess_bulk_per_s']:.1f}, "
              f"min edge bulk ESS/s {out[label].get('edge_ess_bulk_min_per_s')}, R-hat {out[label]['rhat_rank']:.3f}, "
              f"accept {out[label]['accept_rate']:.3f}", file=sys.stderr, flush=True)
    L, U = out["learned"], out["uniform"]
    out["agreement_learned_vs_uniform"] = agreement(res["learned"][0], res["learned"][1], res["uniform"][0],
                                                    res["uniform"][1], len(edges))
    out["ess_bulk_per_s_ratio_learned_vs_uniform"] = L["ess_bulk_per_s"] / max(U["ess_bulk_per_s"], 1e-30)
    out["ess_summed_per_s_ratio_learned_vs_uniform"] = L["ess_summed_per_s"] / max(U["ess_summed_per_s"], 1e-30)
    out["ess_bulk_per_s_ratio_learned_vs_single_uniform"] = (L["ess_bulk_per_s"] /
                                                             max(out["single_uniform"]["ess_bulk_per_s"], 1e-30))
    if edges:
        out["edge_ess_bulk_min_per_s_ratio_learned_vs_uniform"] = (L["edge_ess_bulk_min_per_s"] /
                                                                   max(U["edge_ess_bulk_min_per_s"], 1e-30))
    ag = out["agreement_learned_vs_uniform"]
    out["same_accuracy"] = bool(L["rhat_rank"] < 1.05 and U["rhat_rank"] < 1.05 and ag["score_agrees"]
                                and ag.get("edges_agree", 0) == ag.get("edges", 0)
                                and L["best_score_max"] >= U["best_score_max"])
    # the spec comparisons: the batched uniform chains and the learned chains against the
    # plain single-chain uniform sampler, each at the same accuracy (both R-hat < 1.05, the
    # posterior mean score and every traced edge frequency within 3 MCSE)
    S1 = out["single_uniform"]
    ns = {}
    for label in ("uniform", "learned"):
        agr = agreement(res[label][0], res[label][1], res["single_uniform"][0], res["single_uniform"][1], len(edges))
        X = out[label]
        ns[label + "_vs_single_uniform"] = {
            "ess_bulk_per_s_ratio": X["ess_bulk_per_s"] / max(S1["ess_bulk_per_s"], 1e-30),
            "edge_ess_bulk_min_per_s_ratio": (X["edge_ess_bulk_min_per_s"] / max(S1["edge_ess_bulk_min_per_s"], 1e-30)
                                              if edges else None),
            "agreement": agr,
            "same_accuracy": bool(X["rhat_rank"] < 1.05 and S1["rhat_rank"] < 1.05 and agr["score_agrees"]
                                  and agr.get("edges_agree", 0) == agr.get("edges", 0))}
    ns["single_uniform_blocks_cap"] = single_blocks
    ns["note"] = ("the single chain samples until its score mean and traced edge frequencies agree with the "
                  "converged batched uniform chains within 3 MCSE (its own split-R-hat cannot see modes it has "
                  "not visited); ESS/s uses the rank-normalised bulk ESS of each sampler's sampling phase")
    out["north_star"] = ns
    # the paper's own target (Eq. (6), the max order score): the same burned-in chains resumed
    # with the MAX target, uniform vs learned (the network as trained on the LSE-target harvest)
    for label, mlp in (("uniform_max_target", None), ("learned_max_target", m)):
        s2 = {k: v.clone() for k, v in base.items()}
        tr, et, secs, its, acc = sample_until_mixed(table, s2, chains, done, iters, max_blocks, seed + 7, every,
                                                    edges, mlp=mlp, eps=eps_list[0], target=1)
        res[label] = (tr, et)
        out[label] = chain_stats(tr, et, secs, chains, its, acc, len(edges))
        out[label].update(best_score_max=float(s2["best_scores"].max().item()),
                          best_score_mean=float(s2["best_scores"].mean().item()))
        print(f"# {label}: {chains} x {its} iterations in {secs:.2f} s, bulk ESS/s {out[label]['ess_bulk_per_s']:.1f}, "
              f"R-hat {out[label]['rhat_rank']:.3f}, best {out[label]['best_score_max']:.2f}", file=sys.stderr,
              flush=True)
    LM, UM = out["learned_max_target"], out["uniform_max_target"]
    agm = agreement(res["learned_max_target"][0], res["learned_max_target"][1], res["uniform_max_target"][0],
                    res["uniform_max_target"][1], len(edges))
    out["max_target"] = {"ess_bulk_per_s_ratio_learned_vs_uniform": LM["ess_bulk_per_s"] / max(UM["ess_bulk_per_s"],
                                                                                                1e-30),
                         "best_score_learned_minus_uniform": LM["best_score_max"] - UM["best_score_max"],
                         "agreement": agm,
                         "same_accuracy": bool(LM["rhat_rank"] < 1.05 and UM["rhat_rank"] < 1.05
                                               and agm["score_agrees"]
                                               and agm.get("edges_agree", 0) == agm.get("edges", 0))}
    m.free()
    table.free()
    return out


def uncertain_edges(table, orders, n: int, count: int = 20):
    """(child, parent) pairs whose frequency over the greedy graphs of these
    orders (DEVICE int32 [C][n]) is closest to 1/2, at most `count`."""
    import torch
    B = orders.shape[0]
    lse = torch.empty(B, dtype=torch.float64, device=orders.device)
    mx = torch.empty_like(lse)
    best = torch.empty((B, n), dtype=torch.int64, device=orders.device)
    table.score_orders(orders, lse, mx, best)
    bm = best.cpu().numpy().view(np.uint64)
    cand = []
    for i in range(n):
        for p in range(n):
            f = float(np.mean((bm[:, i] >> np.uint64(p)) & np.uint64(1)))
            if i != p and 0.0 < f < 1.0:
                cand.append((abs(f - 0.5), i, p))
    return [(i, p) for _, i, p in sorted(cand)[:count]]


def bench_generalize(bnos, datagen, train_sets: int, test_sets: int, chains: int = 64, seed: int = 808):
    """Learned proposal across datasets: one network trained on the accepted moves
    of uniform chains on `train_sets` members of the uneven family (n ~ U[20,60]),
    then used on `test_sets` other members (n not seen in training): ESS/s of the
    score trace and the smallest ESS over 20 uncertain edges, learned vs uniform,
    every chain resumed from the same burned-in state on the same random streams."""
    import torch
    from paper_1210_5128_amd import ess as E
    t0 = time.perf_counter()
    feats, pairs, train_n = [], [], []
    for d in range(train_sets):
        w = datagen.uneven_workload(d)
        net, _ = datagen.make(w)
        t = bnos.build_score_table(net.data, net.arities, w.K)
        st = t.new_chain_state(chains, 1, trace_every=0, harvest_cap=1024)
        t.run_chains(st, 6000, seed + d, trace_every=0)
        torch.cuda.synchronize()
        cnt = st["harvest_count"].cpu().numpy()
        feats.append(torch.cat([st["harvest_feats"][c, :int(min(cnt[c], 1024))] for c in range(chains)]))
        pairs.append(torch.cat([st["harvest_pairs"][c, :int(min(cnt[c], 1024))] for c in range(chains)]))
        train_n.append(w.n)
        t.free()
    harvest_s = time.perf_counter() - t0
    m = bnos.Mlp()
    m.set_params(datagen.mlp_params(seed, scale=0.5).astype(np.float32))
    m.fit_norm(torch.cat([f.reshape(-1, 8) for f in feats]).contiguous())
    t0 = time.perf_counter()
    for ep in range(8):
        for d in range(train_sets):
            m.train(feats[d], pairs[d], epochs=1, batch=1024, lr=2e-3, seed=seed + 100 * ep + d)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    moves = int(sum(f.shape[0] for f in feats))
    del feats, pairs
    tests = []
    iters, burn = 2000, 4000
    for d in range(1000, 1000 + test_sets):
        w = datagen.uneven_workload(d)
        net, _ = datagen.make(w)
        t = bnos.build_score_table(net.data, net.arities, w.K)
        st = t.new_chain_state(chains, 1, trace_every=0)
        t.run_chains(st, burn, seed + d, trace_every=0)
        edges = uncertain_edges(t, st["orders"], w.n)
        rec = {"n": w.n, "N": w.N}
        for label, mlp in (("uniform", None), ("learned", m)):
            s2 = {k: st[k].clone() for k in ("orders", "scores", "best_graphs", "best_scores", "accepted")}
            s2["trace"] = torch.zeros((chains, iters + 1), dtype=torch.float64, device=s2["scores"].device)
            if edges:
                s2["edges"] = np.asarray(edges, dtype=np.int32)
                s2["edge_trace"] = torch.zeros((chains, iters + 1), dtype=torch.int32, device=s2["scores"].device)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            t.run_chains(s2, iters, seed + 7 * d, first_iteration=burn, mlp=mlp)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            e = E.ess(s2["trace"].cpu().numpy())
            ee = None
            if edges:
                et = s2["edge_trace"].cpu().numpy().view(np.uint32)
                ee = min(E.ess(((et >> np.uint32(k)) & np.uint32(1)).astype(np.float64)) for k in range(len(edges)))
            rec[label] = {"ess_per_s": e / dt, "edge_ess_min_per_s": None if ee is None else ee / dt}
        rec["ess_per_s_ratio"] = rec["learned"]["ess_per_s"] / max(rec["uniform"]["ess_per_s"], 1e-30)
        if edges:
            rec["edge_ess_min_per_s_ratio"] = (rec["learned"]["edge_ess_min_per_s"] /
                                               max(rec["uniform"]["edge_ess_min_per_s"], 1e-30))
        tests.append(rec)
        t.free()
    m.free()
    out = {"train_datasets": train_sets, "train_n": train_n, "harvested_moves": moves, "harvest_s": harvest_s,
           "train_s": train_s, "chains": chains, "iterations": iters, "tests": tests,
           "geomean_ess_per_s_ratio": float(np.exp(np.mean([np.log(r["ess_per_s_ratio"]) for r in tests]))),
           "geomean_edge_ess_min_per_s_ratio": float(np.exp(np.mean(
               [np.log(r["edge_ess_min_per_s_ratio"]) for r in tests if "edge_ess_min_per_s_ratio" in r])))}
    print(f"# generalize: {train_sets} training sets, {test_sets} unseen: score ESS/s x"
          f"{out['geomean_ess_per_s_ratio']:.2f}, min edge ESS/s x{out['geomean_edge_ess_min_per_s_ratio']:.2f}",
          file=sys.stderr, flush=True)
    return out


def bench_accuracy(bnos, datagen, chains: int, seed: int = 606):
    """Sec. VI's study on a 20-node binary graph with 1,000 samples: the best
    graph's edge TPR/FPR without priors and with the four injected-prior
    settings, at 1,000 and 10,000 iterations, and under bit-flip noise."""
    from paper_1210_5128_amd import accuracy as A
    w = datagen.WORKLOADS["roc20"]
    net, _ = datagen.make(w)
    out = {"workload": f"{w.name}: n={w.n}, K={w.K}, N={w.N}, binary", "chains_per_run": chains,
           "true_edges": int(sum(bin(int(m)).count("1") for m in net.true_parent_masks()))}
    t0 = time.perf_counter()
    for iters in (1000, 10000):
        pts = A.roc_study(bnos, net, w.K, iters, chains, seed)
        out[f"roc_{iters}_iterations"] = [
            {"prior": p["prior"], "tpr": round(p["tpr"], 4), "fpr": round(p["fpr"], 5)} for p in pts]
    out["noise_10000_iterations"] = [
        {"p": p["p"], "tpr": round(p["tpr"], 4), "fpr": round(p["fpr"], 5)}
        for p in A.noise_study(bnos, net, w.K, 10000, chains, seed)]
    out["seconds"] = time.perf_counter() - t0
    print(f"# accuracy: {out['seconds']:.1f} s; no prior, 10k iterations: TPR "
          f"{out['roc_10000_iterations'][0]['tpr']:.3f} FPR {out['roc_10000_iterations'][0]['fpr']:.4f}",
          file=sys.stderr, flush=True)
    return out


def run_only(args, bnos, datagen, dev):
    """One piece of the path alone (for profiler runs): its wall time as JSON."""
    import torch
    out = {"only": args.only}
    if args.only == "mlp":
        R, n = args.mlp_samples, 60
        rng = np.random.default_rng(1)
        feats = torch.from_numpy(rng.standard_normal((R, n, 8)).astype(np.float32)).to(dev)
        pairs = torch.from_numpy(np.stack([rng.choice(n, 2, replace=False) for _ in range(R)]).astype(np.int32)).to(dev)
        m = bnos.Mlp()
        m.set_params(datagen.mlp_params(3, scale=0.5).astype(np.float32))
        m.fit_norm(feats)
        logits = torch.empty((R, n), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.forward(feats, logits)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m.train(feats, pairs, epochs=2, batch=1024, lr=1e-3, seed=1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        m.free()
        out.update(samples=R, n=n, forward_s=t1 - t0, train_2_epochs_s=t2 - t1)
        return out
    w = datagen.WORKLOADS[args.workload]
    net, prior = datagen.make(w)
    t0 = time.perf_counter()
    table = bnos.build_score_table(net.data, net.arities, w.K, ess=w.ess, prior=prior)
    torch.cuda.synchronize()
    out.update(workload=w.name, build_s=time.perf_counter() - t0)
    if args.only == "chains":
        C, iters = max(1, args.chains), args.chain_iters
        st = table.new_chain_state(C, iters, trace_every=iters)
        table.run_chains(st, min(iters, 20), 1, trace_every=min(iters, 20))      # warm-up
        torch.cuda.synchronize()
        st = table.new_chain_state(C, iters, trace_every=iters)
        t0 = time.perf_counter()
        table.run_chains(st, iters, 2, trace_every=iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out.update(chains=C, iterations=iters, seconds=dt, chain_iterations_per_s=C * iters / dt,
                   ms_per_iteration=dt / iters * 1e3)
    table.free()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--batch", type=int, default=1, help="orders scored per step (one table pass each "
                    "for B=1; B orders share each streamed tile otherwise)")
    ap.add_argument("--batched-check", type=int, default=256,
                    help="also time steps of this many orders (0 = skip); reported under 'batched'")
    ap.add_argument("--workload", default="mixed60")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--chunk-steps", type=int, default=0,
                    help="fix the scoring chunk length (x1024 entries) instead of autotuning it")
    ap.add_argument("--passes", choices=("both", "skip", "full"), default="both",
                    help="which scoring passes to time: tile skipping (the headline), full scan, or both; "
                         "one alone keeps a profiler's per-kernel figures unmixed")
    ap.add_argument("--computed-masks", type=int, choices=(0, 1), default=1,
                    help="1: one-order scoring blocks compute the masks from per-4-entry anchors (6 B/entry); "
                         "0: they read the stored masks (12 B/entry)")
    ap.add_argument("--hbm-tables", type=int, default=2,
                    help="also time the one-order pass alternating over this many independently built tables "
                         "(1 = skip)")
    ap.add_argument("--chains", type=int, default=256, help="batched chains on the mixed40 table (0 = skip)")
    ap.add_argument("--chain-iters", type=int, default=20000, help="sampling iterations per block")
    ap.add_argument("--chain-burn", type=int, default=20000, help="burn-in iterations before sampling")
    ap.add_argument("--chain-blocks", type=int, default=4,
                    help="at most this many sampling blocks, stopping once the rank split-R-hat is below 1.05")
    ap.add_argument("--learned", type=int, default=256, metavar="C",
                    help="learned-proposal comparison with C chains on the mixed60 table (0 = skip)")
    ap.add_argument("--learned-iters", type=int, default=4000, help="iterations per sampling block of each "
                    "compared run")
    ap.add_argument("--learned-blocks", type=int, default=10,
                    help="at most this many sampling blocks per run, stopping once the rank split-R-hat is below 1.05")
    ap.add_argument("--learned-moves", type=int, default=1000000, help="accepted moves harvested for training")
    ap.add_argument("--learned-epochs", type=int, default=16)
    ap.add_argument("--learned-eps", default="0.5",
                    help="comma-separated weights of the uniform pair in the learned q; the first is the headline")
    ap.add_argument("--learned-workload", default="mixed60")
    ap.add_argument("--generalize", default="8,4", metavar="TRAIN,TEST",
                    help="learned proposal trained on TRAIN uneven datasets, evaluated on TEST unseen ones "
                         "('0' = skip)")
    ap.add_argument("--accuracy", type=int, default=1, metavar="C",
                    help="structure-recovery study on the roc20 workload with C chains per run (0 = skip)")
    ap.add_argument("--uneven", type=int, default=32, metavar="D",
                    help="uneven family: D datasets x 64 chains in one set of launches vs one at a time (0 = skip)")
    ap.add_argument("--uneven-iters", type=int, default=1000)
    ap.add_argument("--only", choices=("build", "chains", "mlp"), default=None,
                    help="run one piece alone for a profiler and print its own JSON line: the table build of "
                         "--workload; --chains chains x --chain-iters iterations on it; or the network's "
                         "forward and two training epochs on --mlp-samples synthetic n=60 samples")
    ap.add_argument("--mlp-samples", type=int, default=16384)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (scale for HBM byte counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(chains and datasets shard across GPUs with no exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1210_5128_amd import bnos, datagen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}), flush=True)
        return

    if args.only:
        print(json.dumps(run_only(args, bnos, datagen, dev)), flush=True)
        return

    w = datagen.WORKLOADS[args.workload]
    net, prior = datagen.make(w)
    n, K, B = w.n, w.K, args.batch
    print(f"# building table: {w}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    table = bnos.build_score_table(net.data, net.arities, K, ess=w.ess, prior=prior, chunk_steps=args.chunk_steps)
    build_s = time.perf_counter() - t0
    table.computed_masks(bool(args.computed_masks))
    info = table.info()
    S = info["entries_per_node"]
    print(f"# table built in {build_s:.3f} s, S={S}", file=sys.stderr, flush=True)

    def launch_bytes(tab, ords, Bq, skip, eb, passes):
        """Algorithmic bytes of one scoring launch of these orders: with tile skipping the
        64-entry sub-tiles it loads (64 x eb bytes) plus the 8-byte summary of every tile of
        each pass and, with one order per block, the 8-byte summary of every sub-tile, the
        4-byte maximum of every tile and each node's 256 score-bound candidates (12 B);
        without, the full scan."""
        if not skip:
            return eb * n * S * passes
        tl, per_pass = tab.count_tiles(ords)
        one = passes == Bq
        per_launch = passes * (per_pass // 4) * 8
        if one:
            per_launch += passes * (per_pass * 8 + (per_pass // 4) * 4 + n * 256 * 12)
        return tl * 64 * eb + per_launch

    def timed(Bq, steps, warmup, skip=True, tables=None, seed_base=5, computed=None):
        """Time `steps` scoring launches of Bq random orders each, rotating over `tables`
        (launch s uses tables[s % len]); the kernel time comes from HIP events on every
        7th launch of each table (every launch for batches), and the algorithmic bytes
        are those of exactly the launches that carried events."""
        tabs = tables or [table]
        for tb in tabs:
            tb.tile_skip(skip)
        pool = max(8, min(64, steps))
        pool = pool - 1 if pool % 7 == 0 else pool
        orders = torch.from_numpy(datagen.random_orders(n, pool * Bq, seed=seed_base + Bq).reshape(pool, Bq, n)).to(dev)
        lse = torch.empty(Bq, dtype=torch.float64, device=dev)
        mx = torch.empty(Bq, dtype=torch.float64, device=dev)
        best = torch.empty((Bq, n), dtype=torch.int64, device=dev)
        views = [orders[i] for i in range(pool)]      # made once: the loop only launches
        T = len(tabs)
        for s_ in range(warmup):
            tabs[s_ % T].score_orders(views[s_ % pool], lse, mx, best, stream=stream)
        torch.cuda.synchronize()
        every = 7 if Bq < 16 else 1
        for tb in tabs:
            tb.timing(True, every=every)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for s_ in range(steps):
            tabs[s_ % T].score_orders(views[s_ % pool], lse, mx, best, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        total_ms = ev0.elapsed_time(ev1)
        k_ms, k_launches, k_passes = 0.0, 0, 0
        for tb in tabs:
            a, b_, c_ = tb.timing_read()
            tb.timing(False)
            k_ms, k_launches, k_passes = k_ms + a, k_launches + b_, k_passes + c_
        # the launches that carried events: the (s // T)-th launch of table s % T, timed when
        # that count is a multiple of `every`
        timed_s = [s_ for s_ in range(steps) if (s_ // T) % every == 0]
        assert len(timed_s) == k_launches, (len(timed_s), k_launches)
        kernel_avg_ms = k_ms / k_launches
        passes_per_launch = k_passes / k_launches
        # bytes per entry: a one-order block with computed masks reads the score and a quarter
        # of an 8-byte anchor mask (6 B); otherwise mask + score (12 B)
        computed_now = bool(args.computed_masks) if computed is None else computed
        eb = 6 if (computed_now and passes_per_launch == Bq) else 12
        cache = {}
        alg_tot, tiles_tot, per_pass = 0.0, 0, 1
        for s_ in timed_s:
            key = (s_ % T, s_ % pool)
            if key not in cache:
                cache[key] = launch_bytes(tabs[s_ % T], views[s_ % pool], Bq, skip, eb, passes_per_launch)
                if skip:
                    cache[key] = (cache[key], *tabs[s_ % T].count_tiles(views[s_ % pool]))
                else:
                    cache[key] = (cache[key], 0, 1)
            alg_tot += cache[key][0]
            tiles_tot += cache[key][1]
            per_pass = cache[key][2]
        alg = alg_tot / len(timed_s)
        gbs = alg / (kernel_avg_ms / 1e3) / 1e9
        return dict(total_ms=total_ms, ms_per_step=total_ms / steps, value=Bq * steps / (total_ms / 1e3),
                    kernel_avg_ms=kernel_avg_ms, passes_per_launch=passes_per_launch, gbs=gbs, alg_bytes=alg,
                    entry_bytes=eb, timed_launches=len(timed_s),
                    tile_fraction=tiles_tot / max(1, len(timed_s) * passes_per_launch * per_pass) if skip else 1.0)

    stream = torch.cuda.current_stream()
    # launch shape (chunk length, orders per block) tuned per batch size before timing
    tuned = {}
    for Bq in ([] if args.chunk_steps else sorted({B, args.batched_check} - {0})):
        o = torch.from_numpy(datagen.random_orders(n, Bq, seed=900 + Bq)).to(dev)
        cs, bt, g, ms = table.autotune(o, reps=20 if Bq < 64 else 3, stream=stream)
        tuned[str(Bq)] = {"gather": bool(g), "chunk_steps": cs, "orders_per_block": bt, "tune_ms_per_launch": ms}
        print(f"# autotune B={Bq}: " + ("gather pass" if g else f"chunk {cs}x1024 entries, {bt} orders/block") +
              f", {ms * 1e3:.1f} us", file=sys.stderr, flush=True)
    if args.chunk_steps:
        tuned = {"fixed_chunk_steps": args.chunk_steps}
        for Bq in sorted({B, args.batched_check} - {0}):
            table.set_launch(Bq, chunk_steps=args.chunk_steps)
    rf = r = rs = rh = None
    extra_steps = max(args.steps, 140)
    if args.passes != "skip":
        rf = timed(B, args.steps, args.warmup, skip=False)     # full scan of every entry
        print(f"# full scan: {rf['total_ms']:.3f} ms for {args.steps} steps", file=sys.stderr, flush=True)
    if args.passes != "full":
        r = timed(B, args.steps, args.warmup, skip=True)       # with tile summaries (default path)
    else:
        r = rf
    print(f"# timed {args.steps} steps: {r['total_ms']:.3f} ms", file=sys.stderr, flush=True)
    if args.passes == "both" and B == 1:
        # the stored-mask full scan: 12 B x n x S = 352 MB per launch at n = 60, more than the
        # 256 MB Infinity Cache holds, so every launch streams from HBM
        table.computed_masks(False)
        rs = timed(B, extra_steps, args.warmup, skip=False, computed=False)
        table.computed_masks(bool(args.computed_masks))
        print(f"# stored-mask full scan: {rs['kernel_avg_ms'] * 1e3:.1f} us per launch, {rs['gbs']:.0f} GB/s",
              file=sys.stderr, flush=True)
    if args.hbm_tables > 1 and args.passes != "full" and B == 1:
        # the headline pass alternating over independently built tables of the same shape:
        # their combined read set exceeds the Infinity Cache, so launches stream from HBM
        others = []
        for k in range(1, args.hbm_tables):
            w2 = datagen.Workload(f"{w.name}-{k}", w.n, w.N, w.arity_choices, w.dmax, w.K, w.data_seed + 100 * k,
                                  None if w.prior_seed is None else w.prior_seed + 100 * k, w.ess)
            net2, prior2 = datagen.make(w2)
            t2 = bnos.build_score_table(net2.data, net2.arities, K, ess=w.ess, prior=prior2,
                                        chunk_steps=args.chunk_steps)
            t2.computed_masks(bool(args.computed_masks))
            if str(B) in tuned:
                t2.set_launch(B, gather=tuned[str(B)]["gather"], chunk_steps=tuned[str(B)]["chunk_steps"],
                              orders_per_block=tuned[str(B)]["orders_per_block"])
            elif args.chunk_steps:
                t2.set_launch(B, chunk_steps=args.chunk_steps)
            others.append(t2)
        rh = timed(B, extra_steps * args.hbm_tables, args.warmup, skip=True, tables=[table] + others)
        read_set = sum(tb.info()["entries_per_node"] for tb in [table] + others) * n * 6
        for t2 in others:
            t2.free()
        print(f"# {args.hbm_tables} tables alternating: {rh['kernel_avg_ms'] * 1e3:.1f} us per launch, "
              f"{rh['gbs']:.0f} GB/s", file=sys.stderr, flush=True)
    ms_per_step, value = r["ms_per_step"], r["value"]
    kernel_avg_ms, passes_per_launch, achieved_gbs = r["kernel_avg_ms"], r["passes_per_launch"], r["gbs"]
    full_scan = None if rf is None else {
        "order_scores_per_s": rf["value"], "ms_per_step": rf["ms_per_step"],
        "kernel_avg_us": rf["kernel_avg_ms"] * 1e3, "algorithmic_bytes_per_launch": rf["alg_bytes"],
        "effective_GBs": rf["gbs"], "frac": rf["gbs"] / HBM_PEAK_GBS, "bytes_per_entry": rf["entry_bytes"],
        "traffic": measured_traffic(B, "full") if args.workload == "mixed60" else None}
    full_scan_stored = None if rs is None else {
        "kernel": "k_score (full scan, stored masks)", "kernel_avg_us": rs["kernel_avg_ms"] * 1e3,
        "timed_launches": rs["timed_launches"], "algorithmic_bytes_per_launch": rs["alg_bytes"],
        "bytes_per_entry": rs["entry_bytes"], "achieved_GBs": rs["gbs"], "frac": rs["gbs"] / HBM_PEAK_GBS,
        "note": "one launch reads 12 B x n x S, more than the 256 MB Infinity Cache: HBM-resident"}
    hbm_resident = None if rh is None else {
        "tables": args.hbm_tables, "read_set_bytes": read_set, "kernel": "k_score (tile skipping)",
        "kernel_avg_us": rh["kernel_avg_ms"] * 1e3, "timed_launches": rh["timed_launches"],
        "algorithmic_bytes_per_launch": rh["alg_bytes"], "achieved_GBs": rh["gbs"], "frac": rh["gbs"] / HBM_PEAK_GBS,
        "order_scores_per_s": rh["value"],
        "note": "B=1 launches alternating over independently built tables whose scores and anchors together "
                "exceed the 256 MB Infinity Cache"}
    batched = None
    if args.batched_check:
        rb = timed(args.batched_check, 20, 3)
        batched = {"batch": args.batched_check, "order_scores_per_s": rb["value"], "ms_per_step": rb["ms_per_step"],
                   "kernel_avg_us": rb["kernel_avg_ms"] * 1e3, "table_passes_per_launch": rb["passes_per_launch"],
                   "stream_GBs": rb["gbs"]}
        print(f"# batched {args.batched_check}: {rb['value']:.0f} order-scores/s", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "order-scores/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"score_orders on the {w.name} table: n={n}, K={K}, N={w.N}, arities U{{2,3,4}}, "
                         f"BDeu ess={w.ess}, pairwise prior on 10% of ordered pairs; {B} random order(s) per step"),
            "n": n, "K": K, "N": w.N, "batch": B, "entries_per_node": S, "launch_shape": tuned,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": (measured_traffic(B, "full" if args.passes == "full" else "skip")
                        if args.workload == "mixed60" else None),
            "kernel": "k_score (full scan)" if args.passes == "full" else "k_score (tile skipping)",
            "kernel_avg_us": kernel_avg_ms * 1e3,
            "algorithmic_bytes_per_launch": r["alg_bytes"],
            "bytes_per_entry": r["entry_bytes"],
            "tile_fraction_read": r["tile_fraction"] if args.passes != "full" else 1.0,
            "timed_launches": r["timed_launches"],
            "note": ("with tile skipping and the score bound a launch reads ~6% of the table's entries and the "
                     "pass is bound by the latency of its longest wavefronts, not by bandwidth; full_scan "
                     "(every entry, no skipping) is the streaming-bandwidth figure. Effective bandwidth: the "
                     "scores and anchors (176 MB at n=60) fit the 256 MB Infinity Cache between launches; "
                     "hbm_resident and full_scan_stored_masks stream from HBM"),
        },
        "hbm_resident": hbm_resident,
        "full_scan": full_scan,
        "full_scan_stored_masks": full_scan_stored,
        "batched": batched,
        "build_s": build_s,
        "table_device_bytes": info["device_bytes"],
        "paper_context": {"order_scores_per_s_n60": 2.92, "hardware": "Tesla M2090 (Fermi), 2012",
                          "note": "per-iteration time 0.3427 s at n=60, s=4; its data are not described"},
    }
    if args.chains:
        out["chains"] = bench_chains(bnos, datagen, "mixed40", args.chains, args.chain_iters, args.chain_burn,
                                     args.chain_blocks)
    if args.uneven:
        out["uneven"] = bench_uneven(bnos, datagen, args.uneven, 64, args.uneven_iters)
    if args.accuracy:
        out["accuracy"] = bench_accuracy(bnos, datagen, args.accuracy)
    if args.generalize != "0":
        tr, te = (int(x) for x in args.generalize.split(","))
        out["generalize"] = bench_generalize(bnos, datagen, tr, te)
    if args.learned:
        out["learned"] = bench_learned(bnos, datagen, args.learned_workload, args.learned, args.learned_moves,
                                       args.learned_iters, epochs=args.learned_epochs,
                                       eps_list=[float(x) for x in args.learned_eps.split(",")],
                                       max_blocks=args.learned_blocks)
    if not args.no_cpu:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(net, prior, K)
    table.free()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
