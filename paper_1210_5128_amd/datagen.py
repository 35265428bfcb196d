"""Seeded synthetic inputs for order-space structure learning.

This module only draws random inputs: discrete data sampled from a random
Bayesian network, a sparse pairwise-prior weight matrix, and random node
orders.  It holds none of the scoring arithmetic, so both the HIP path and the
CPU oracle can consume what it produces.

Workload recipe (the paper's data are complete multinomial samples of discrete
variables, Sec. II; its timing tables use random graphs of 13-60 nodes with at
most 4 parents, Sec. VI):

1. arities r_v drawn from the given set;
2. a uniform random permutation of the nodes;
3. for the node at permutation position p: in-degree d = min(U{0..dmax}, p),
   parents drawn uniformly without replacement among the p earlier nodes;
4. one Dirichlet(1) row per parent configuration (CPT);
5. N ancestral samples by inverse-CDF on uniforms;
6. stored as int8 [N][n], row-major.

All draws use ``numpy.random.default_rng(seed)`` in exactly that order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np


@dataclass
class Network:
    """A random discrete Bayesian network together with samples drawn from it."""

    n: int
    arities: np.ndarray          # int32 [n]
    perm: np.ndarray             # int64 [n]   topological order used to build the DAG
    parents: list                # list of sorted parent-id lists, indexed by node id
    data: np.ndarray             # int8 [N][n] row-major
    cpts: list = field(repr=False, default_factory=list)

    @property
    def N(self) -> int:
        return int(self.data.shape[0])

    def true_parent_masks(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.uint64)
        for v, ps in enumerate(self.parents):
            m = 0
            for p in ps:
                m |= 1 << int(p)
            out[v] = np.uint64(m)
        return out


def random_network(n: int, N: int, arity_choices: Sequence[int], dmax: int,
                   seed: int) -> Network:
    """Draw a random DAG with CPTs and ``N`` ancestral samples (recipe above)."""
    if n < 1 or n > 64:
        raise ValueError("n must be in [1, 64]")
    rng = np.random.default_rng(seed)
    choices = np.asarray(list(arity_choices), dtype=np.int64)
    arities = rng.choice(choices, size=n).astype(np.int32)
    perm = rng.permutation(n)
    parents: list = [[] for _ in range(n)]
    for p in range(n):
        v = int(perm[p])
        d = min(int(rng.integers(0, dmax + 1)), p)
        if d > 0:
            chosen = rng.choice(perm[:p], size=d, replace=False)
            parents[v] = sorted(int(c) for c in chosen)
    cpts: list = [None] * n
    for p in range(n):
        v = int(perm[p])
        q = 1
        for m in parents[v]:
            q *= int(arities[m])
        cpts[v] = rng.dirichlet(np.ones(int(arities[v])), size=q)
    data = np.zeros((N, n), dtype=np.int8)
    if N > 0:
        u = rng.random((N, n))
        for p in range(n):
            v = int(perm[p])
            k = np.zeros(N, dtype=np.int64)
            for m in parents[v]:
                k = k * int(arities[m]) + data[:, m].astype(np.int64)
            cdf = np.cumsum(cpts[v], axis=1)[k]          # [N, r_v]
            x = (u[:, v:v + 1] > cdf).sum(axis=1)
            data[:, v] = np.minimum(x, int(arities[v]) - 1).astype(np.int8)
    return Network(n=n, arities=arities, perm=perm, parents=parents, data=data, cpts=cpts)


def random_prior(n: int, seed: int, fraction: float = 0.1) -> np.ndarray:
    """Pairwise confidence weights w in [-1, 1] (row = child, column = parent).

    ``round(fraction * n * (n - 1))`` ordered pairs (i != m) are chosen without
    replacement and given w ~ U[-1, 1]; every other entry is 0 (no bias).
    """
    rng = np.random.default_rng(seed)
    w = np.zeros((n, n), dtype=np.float32)
    pairs = [(i, m) for i in range(n) for m in range(n) if i != m]
    k = int(round(fraction * len(pairs)))
    if k:
        idx = rng.choice(len(pairs), size=k, replace=False)
        vals = rng.uniform(-1.0, 1.0, size=k)
        for t, j in enumerate(idx):
            i, m = pairs[int(j)]
            w[i, m] = np.float32(vals[t])
    return w


def random_orders(n: int, B: int, seed: int) -> np.ndarray:
    """``B`` independent uniform random node orders, int32 [B][n] (position -> node id)."""
    rng = np.random.default_rng(seed)
    out = np.empty((B, n), dtype=np.int32)
    for b in range(B):
        out[b] = rng.permutation(n).astype(np.int32)
    return out


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    N: int
    arity_choices: tuple
    dmax: int
    K: int
    data_seed: int
    prior_seed: Optional[int]
    ess: float = 1.0


# The synthetic workloads: a tiny binary net, a 20-node ternary net with a
# prior, a 40-node mixed-arity net, the uneven 20..60-node family (one member
# per seed), the 60-node mixed-arity net used for the headline scoring rate, and
# a 20-node binary net for the structure-recovery study.
WORKLOADS = {
    "tiny8": Workload("tiny8", 8, 200, (2,), 3, 3, 0, None),
    "prior20": Workload("prior20", 20, 1000, (3,), 4, 4, 1, 11),
    "mixed40": Workload("mixed40", 40, 2000, (2, 3, 4), 4, 4, 2, 12),
    "mixed60": Workload("mixed60", 60, 5000, (2, 3, 4), 4, 4, 4, 14),
    # the accuracy study's graph: 20 binary nodes, 1,000 samples (Sec. VI)
    "roc20": Workload("roc20", 20, 1000, (2,), 3, 4, 20, None),
}


def uneven_workload(d: int) -> Workload:
    """Member ``d`` of the uneven family: n ~ U[20,60], N ~ U[1000,5000], dmax 3."""
    rng = np.random.default_rng(1000 + d)
    n = int(rng.integers(20, 61))
    N = int(rng.integers(1000, 5001))
    return Workload(f"uneven{d}", n, N, (2, 3, 4), 3, 4, 1000 + d, None)


def make(w: Workload):
    """Materialise a workload: returns (network, prior weights or None)."""
    net = random_network(w.n, w.N, w.arity_choices, w.dmax, w.data_seed)
    prior = random_prior(w.n, w.prior_seed) if w.prior_seed is not None else None
    return net, prior


MLP_HIDDEN = 128
MLP_FEATURES = 8


def mlp_params(seed: int, scale: float = 1.0) -> np.ndarray:
    """Random network parameters (He-style normal draws), flat FP64 in the order
    W1 [128][8], b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1]."""
    rng = np.random.default_rng(seed)
    H, F = MLP_HIDDEN, MLP_FEATURES
    W1 = rng.standard_normal((H, F)) * np.sqrt(2.0 / F) * scale
    b1 = rng.standard_normal(H) * 0.1 * scale
    W2 = rng.standard_normal((H, H)) * np.sqrt(2.0 / H) * scale
    b2 = rng.standard_normal(H) * 0.1 * scale
    w3 = rng.standard_normal(H) * np.sqrt(1.0 / H) * scale
    b3 = np.zeros(1)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, b3])
