"""Structure-recovery accuracy of the learned best graph (Sec. VI's ROC study).

The paper measures how close the best graph its sampler finds is to the graph
that generated the data, as true- and false-positive rates of the edges; it
adds pairwise priors on the edges a prior-free run got wrong (Sec. IV's
confidence R: above 0.5 for an edge believed present, below for absent), and
flips the states of binary data at a given rate to test noise tolerance.

Edges are directed (parent m -> child i) and read from per-node parent masks.
TPR = (true edges found) / (true edges); FPR = (edges found that are not in the
true graph) / (ordered pairs i != m that are not true edges).  A reversed edge
counts as one missed and one false edge.

This module only draws the experiment's random inputs (which wrong edges get a
prior, which data values flip) and counts edges; the learning itself is the
library's (table build, chains on the device).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def masks_to_adjacency(masks, n: int) -> np.ndarray:
    """bool [n][n], A[m, i] = True iff m is a parent of i (bit m of masks[i])."""
    a = np.zeros((n, n), dtype=bool)
    for i in range(n):
        m = int(masks[i]) & ((1 << 64) - 1)
        for p in range(n):
            if (m >> p) & 1:
                a[p, i] = True
    return a


@dataclass
class EdgeRates:
    tp: int
    fp: int
    fn: int
    tn: int

    @property
    def tpr(self) -> float:
        return self.tp / max(1, self.tp + self.fn)

    @property
    def fpr(self) -> float:
        return self.fp / max(1, self.fp + self.tn)


def edge_rates(learned_masks, true_masks, n: int) -> EdgeRates:
    """Directed-edge confusion counts of a learned graph against the true one."""
    L = masks_to_adjacency(learned_masks, n)
    T = masks_to_adjacency(true_masks, n)
    off = ~np.eye(n, dtype=bool)
    return EdgeRates(tp=int((L & T & off).sum()), fp=int((L & ~T & off).sum()),
                     fn=int((~L & T & off).sum()), tn=int((~L & ~T & off).sum()))


def injected_prior(true_masks, learned_masks, n: int, r_present: float, r_absent: float, prob: float,
                   seed: int) -> np.ndarray:
    """Confidence matrix R [child][parent] (0.5 = no opinion) for the prior
    injection protocol: every true edge the prior-free result missed gets
    R = r_present with probability `prob`, every edge it added that is not
    true gets R = r_absent with probability `prob`.  Draws: one uniform per
    wrong edge, missed edges first, each list in (child, parent) order."""
    L = masks_to_adjacency(learned_masks, n)
    T = masks_to_adjacency(true_masks, n)
    R = np.full((n, n), 0.5, dtype=np.float32)
    rng = np.random.default_rng(seed)
    missed = [(i, m) for i in range(n) for m in range(n) if m != i and T[m, i] and not L[m, i]]
    added = [(i, m) for i in range(n) for m in range(n) if m != i and L[m, i] and not T[m, i]]
    for (i, m) in missed:
        if rng.random() < prob:
            R[i, m] = np.float32(r_present)
    for (i, m) in added:
        if rng.random() < prob:
            R[i, m] = np.float32(r_absent)
    return R


def flip_states(data: np.ndarray, p: float, seed: int) -> np.ndarray:
    """Binary data with every value flipped (0 <-> 1) independently with probability p."""
    data = np.asarray(data, dtype=np.int8)
    if data.size and data.max() > 1:
        raise ValueError("flip_states expects binary data")
    flip = np.random.default_rng(seed).random(data.shape) < p
    return np.where(flip, 1 - data, data).astype(np.int8)


def learn_best_graph(table, iterations: int, chains: int, seed: int, target: int = 1):
    """Best graph over `chains` uniform-swap chains of `iterations` iterations
    (best-graph record per chain, then the best chain): (parent masks as
    uint64 [n], its max score)."""
    import torch
    st = table.new_chain_state(chains, iterations, trace_every=max(1, iterations))
    table.run_chains(st, iterations, seed, target=target, trace_every=max(1, iterations))
    torch.cuda.synchronize()
    scores = st["best_scores"].cpu().numpy()
    c = int(np.argmax(scores))
    return st["best_graphs"][c].cpu().numpy().view(np.uint64).copy(), float(scores[c])


# the prior settings of the ROC study: (R for a missed edge, R for an added edge, probability)
ROC_PRIORS = [None, (0.7, 0.2, 0.2), (0.7, 0.2, 0.4), (0.8, 0.1, 0.2), (0.8, 0.1, 0.4)]
NOISE_RATES = [0.01, 0.05, 0.06, 0.07, 0.08, 0.10, 0.11, 0.13, 0.15]


def roc_study(bnos, net, K: int, iterations: int, chains: int, seed: int):
    """One ROC curve: the prior-free result, then the four injected-prior settings
    (each built on the prior-free result's mistakes).  Returns a list of dicts."""
    true = net.true_parent_masks()
    t = bnos.build_score_table(net.data, net.arities, K)
    base, base_score = learn_best_graph(t, iterations, chains, seed)
    t.free()
    out = []
    for k, setting in enumerate(ROC_PRIORS):
        if setting is None:
            g, s = base, base_score
        else:
            R = injected_prior(true, base, net.n, setting[0], setting[1], setting[2], seed + 100 + k)
            tp = bnos.build_score_table(net.data, net.arities, K, prior=R, prior_mode=1)
            g, s = learn_best_graph(tp, iterations, chains, seed)
            tp.free()
        r = edge_rates(g, true, net.n)
        out.append(dict(prior=setting, tpr=r.tpr, fpr=r.fpr, tp=r.tp, fp=r.fp, fn=r.fn, score=s))
    return out


def noise_study(bnos, net, K: int, iterations: int, chains: int, seed: int, rates=NOISE_RATES):
    """Rates of the learned graph when every binary value flips with probability p."""
    true = net.true_parent_masks()
    out = []
    for j, p in enumerate(rates):
        data = flip_states(net.data, p, seed + 1000 + j)
        t = bnos.build_score_table(data, net.arities, K)
        g, s = learn_best_graph(t, iterations, chains, seed)
        t.free()
        r = edge_rates(g, true, net.n)
        out.append(dict(p=p, tpr=r.tpr, fpr=r.fpr, tp=r.tp, fp=r.fp, fn=r.fn))
    return out
