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


def bench_chains(bnos, datagen, wname: str, chains: int, iters: int, seed: int = 102):
    """Batched MH chains vs one chain on the same table: iterations/s and ESS/s of the
    log-sum-exp score trace (Geyer initial-monotone ESS after 20% burn-in, summed over chains)."""
    import torch
    from paper_1210_5128_amd import ess as E
    w = datagen.WORKLOADS[wname]
    net, prior = datagen.make(w)
    table = bnos.build_score_table(net.data, net.arities, w.K, ess=w.ess, prior=prior)
    out = {"workload": f"{w.name}: n={w.n}, K={w.K}, N={w.N}", "iterations": iters}
    for label, C in (("batched", chains), ("single", 1)):
        st = table.new_chain_state(C, iters, trace_every=1)
        table.run_chains(st, min(iters, 50), seed + 1000, sweep_len=32)     # warm-up (separate seed)
        torch.cuda.synchronize()
        st = table.new_chain_state(C, iters, trace_every=1)
        t0 = time.perf_counter()
        table.run_chains(st, iters, seed, sweep_len=32)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tr = st["trace"].cpu().numpy()
        e = E.ess(tr)
        out[label] = {"chains": C, "seconds": dt, "chain_iterations_per_s": C * iters / dt,
                      "ess": e, "ess_per_s": e / dt,
                      "accept_rate": float(st["accepted"].sum().item()) / (C * iters),
                      "best_score_max": float(st["best_scores"].max().item()),
                      "split_rhat": E.split_rhat(tr) if C > 1 else None}
        print(f"# chains {label}: {C}x{iters} in {dt:.2f} s, ESS/s {e / dt:.1f}", file=sys.stderr, flush=True)
    out["ess_per_s_ratio_batched_vs_single"] = out["batched"]["ess_per_s"] / max(out["single"]["ess_per_s"], 1e-30)
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
                  eps_list=(0.1,), seed: int = 404):
    """Learned swap proposal: harvest `moves` accepted moves from uniform chains
    (which also serves as burn-in), train the network on the device, then resume
    every chain from its harvested state twice, with the uniform and with the
    learned proposal, on the same random-number streams; plus one uniform chain
    alone.  ESS/s of the log-sum-exp trace and the smallest ESS over the
    indicators of the 20 most uncertain edges, acceptance, best-graph score."""
    import torch
    from paper_1210_5128_amd import ess as E
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
    # 4. resume every chain from its harvested state: uniform vs learned, and one uniform chain alone
    base = {k: v for k, v in st.items() if k in ("orders", "scores", "best_graphs", "best_scores", "accepted")}
    runs = [("uniform", None, chains, 0.1)]
    for k, eps in enumerate(eps_list):
        runs.append(("learned" if k == 0 else f"learned_eps{eps:g}", m, chains, eps))
    runs.append(("single_uniform", None, 1, 0.1))
    for label, mlp, C, eps in runs:
        s2 = {k: v[:C].clone() for k, v in base.items()}
        s2["trace"] = torch.zeros((C, iters + 1), dtype=torch.float64, device=base["scores"].device)
        s2["accept_flags"] = None
        if edges:
            s2["edges"] = np.asarray(edges, dtype=np.int32)
            s2["edge_trace"] = torch.zeros((C, iters + 1), dtype=torch.int32, device=base["scores"].device)
        a0 = s2["accepted"].clone()
        t0 = time.perf_counter()
        table.run_chains(s2, iters, seed + 5, first_iteration=done, mlp=mlp, eps=eps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        trc = s2["trace"].cpu().numpy()
        e = E.ess(trc)
        edge_ess = None
        if edges:
            et = s2["edge_trace"].cpu().numpy().view(np.uint32)
            edge_ess = min(E.ess(((et >> np.uint32(k)) & np.uint32(1)).astype(np.float64))
                           for k in range(len(edges)))
        out[label] = {"chains": C, "eps": eps if mlp is not None else None, "seconds": dt,
                      "chain_iterations_per_s": C * iters / dt,
                      "ess": e, "ess_per_s": e / dt, "ess_per_1k_chain_iterations": 1e3 * e / (C * iters),
                      "edge_ess_min": edge_ess, "edge_ess_min_per_s": None if edge_ess is None else edge_ess / dt,
                      "accept_rate": float((s2["accepted"] - a0).sum().item()) / (C * iters),
                      "best_score_max": float(s2["best_scores"].max().item()),
                      "best_score_mean": float(s2["best_scores"].mean().item()),
                      "score_mean": float(trc.mean()),
                      "split_rhat": E.split_rhat(trc) if C > 1 else None}
        print(f"# {label}: {dt:.2f} s, ESS {e:.0f}, ESS/s {e / dt:.1f}, min edge ESS {edge_ess}, "
              f"accept {out[label]['accept_rate']:.3f}", file=sys.stderr, flush=True)
    out["ess_per_s_ratio_learned_vs_uniform"] = out["learned"]["ess_per_s"] / max(out["uniform"]["ess_per_s"], 1e-30)
    out["ess_per_s_ratio_learned_vs_single_uniform"] = (out["learned"]["ess_per_s"] /
                                                        max(out["single_uniform"]["ess_per_s"], 1e-30))
    out["ess_per_iteration_ratio_learned_vs_uniform"] = (out["learned"]["ess_per_1k_chain_iterations"] /
                                                         max(out["uniform"]["ess_per_1k_chain_iterations"], 1e-30))
    if edges:
        out["edge_ess_min_per_s_ratio_learned_vs_uniform"] = (out["learned"]["edge_ess_min_per_s"] /
                                                              max(out["uniform"]["edge_ess_min_per_s"], 1e-30))
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
    ap.add_argument("--chains", type=int, default=256, help="batched chains on the mixed40 table (0 = skip)")
    ap.add_argument("--chain-iters", type=int, default=20000)
    ap.add_argument("--learned", type=int, default=256, metavar="C",
                    help="learned-proposal comparison with C chains on the mixed60 table (0 = skip)")
    ap.add_argument("--learned-iters", type=int, default=4000, help="iterations of each compared run")
    ap.add_argument("--learned-moves", type=int, default=1000000, help="accepted moves harvested for training")
    ap.add_argument("--learned-epochs", type=int, default=16)
    ap.add_argument("--learned-eps", default="0.5,0.1",
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

    bytes_per_pass = 12 * n * S                           # (u64 mask + f32 score) per entry, one full scan

    def timed(Bq, steps, warmup, skip=True):
        table.tile_skip(skip)
        pool = max(8, min(64, steps))
        pool = pool - 1 if pool % 7 == 0 else pool      # sampled launches visit every order
        orders = torch.from_numpy(datagen.random_orders(n, pool * Bq, seed=5 + Bq).reshape(pool, Bq, n)).to(dev)
        lse = torch.empty(Bq, dtype=torch.float64, device=dev)
        mx = torch.empty(Bq, dtype=torch.float64, device=dev)
        best = torch.empty((Bq, n), dtype=torch.int64, device=dev)
        views = [orders[i] for i in range(pool)]      # made once: the loop only launches
        for s in range(warmup):
            table.score_orders(views[s % pool], lse, mx, best, stream=stream)
        torch.cuda.synchronize()
        # events on 1 launch in 7 for short launches (an event pair costs the host ~15 us
        # per launch, which would make a single-order loop host-bound), spread over the
        # whole timed region and, 7 being prime to the pool size, over every order of the
        # pool (whose sub-tiles the algorithmic bytes count); on every launch for batches
        table.timing(True, every=7 if Bq < 16 else 1)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for s in range(steps):
            table.score_orders(views[s % pool], lse, mx, best, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        total_ms = ev0.elapsed_time(ev1)
        k_ms, k_launches, k_passes = table.timing_read()
        table.timing(False)
        tiles, tiles_per_pass = 0, 1
        if skip:          # tiles the launches read: counted by a separate kernel over the same orders
            for s in range(steps):
                tl, tiles_per_pass = table.count_tiles(orders[s % pool])
                tiles += tl
                if s + 1 == pool:
                    tiles = tiles * steps // pool
                    break
        kernel_avg_ms = k_ms / k_launches
        passes_per_launch = k_passes / k_launches
        # bytes the launch had to read: with tile skipping, the 64-entry sub-tiles it
        # loaded (64 x 12 B) plus the 8-byte summary of every tile of each pass and,
        # with one order per block, of every sub-tile; without, the full scan
        # bytes per entry: a one-order block with computed masks reads the score and a quarter
        # of an 8-byte anchor mask (6 B); otherwise mask + score (12 B)
        eb = 6 if (args.computed_masks and passes_per_launch == Bq) else 12
        if skip:
            sub_summaries = tiles_per_pass if passes_per_launch == Bq else 0
            alg = tiles / steps * 64 * eb + passes_per_launch * (tiles_per_pass // 4 + sub_summaries) * 8
        else:
            alg = eb * n * S * passes_per_launch
        gbs = alg / (kernel_avg_ms / 1e3) / 1e9
        return dict(total_ms=total_ms, ms_per_step=total_ms / steps, value=Bq * steps / (total_ms / 1e3),
                    kernel_avg_ms=kernel_avg_ms, passes_per_launch=passes_per_launch, gbs=gbs, alg_bytes=alg,
                    entry_bytes=eb,
                    tile_fraction=tiles / max(1, steps * passes_per_launch * tiles_per_pass),
                    full_scan_equiv_gbs=bytes_per_pass * passes_per_launch / (kernel_avg_ms / 1e3) / 1e9)

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
    rf = r = None
    if args.passes != "skip":
        rf = timed(B, args.steps, args.warmup, skip=False)     # full scan of every entry
        print(f"# full scan: {rf['total_ms']:.3f} ms for {args.steps} steps", file=sys.stderr, flush=True)
    if args.passes != "full":
        r = timed(B, args.steps, args.warmup, skip=True)       # with tile summaries (default path)
    else:
        r = rf
    print(f"# timed {args.steps} steps: {r['total_ms']:.3f} ms", file=sys.stderr, flush=True)
    ms_per_step, value = r["ms_per_step"], r["value"]
    kernel_avg_ms, passes_per_launch, achieved_gbs = r["kernel_avg_ms"], r["passes_per_launch"], r["gbs"]
    full_scan = None if rf is None else {
        "order_scores_per_s": rf["value"], "ms_per_step": rf["ms_per_step"],
        "kernel_avg_us": rf["kernel_avg_ms"] * 1e3, "algorithmic_bytes_per_launch": rf["alg_bytes"],
        "achieved_GBs": rf["gbs"], "frac": rf["gbs"] / HBM_PEAK_GBS,
        "traffic": measured_traffic(B, "full") if args.workload == "mixed60" else None}
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
            "full_scan_equivalent_GBs": r["full_scan_equiv_gbs"],
        },
        "full_scan": full_scan,
        "batched": batched,
        "build_s": build_s,
        "table_device_bytes": info["device_bytes"],
        "paper_context": {"order_scores_per_s_n60": 2.92, "hardware": "Tesla M2090 (Fermi), 2012",
                          "note": "per-iteration time 0.3427 s at n=60, s=4; its data are not described"},
    }
    if args.chains:
        out["chains"] = bench_chains(bnos, datagen, "mixed40", args.chains, args.chain_iters)
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
                                       eps_list=[float(x) for x in args.learned_eps.split(",")])
    if not args.no_cpu:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(net, prior, K)
    table.free()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
