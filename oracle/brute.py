"""Pure-Python checkers that pin the C oracle without sharing its arithmetic.

TEST INFRASTRUCTURE ONLY.

- ``count_dags_robinson``: Robinson's recurrence for the number of labelled
  DAGs (the "# of graphs" column of the paper's Table 1).
- ``enumerate_dags``: every DAG on n <= 5 nodes with in-degree <= K, as one
  parent mask per node, found by exhaustive search with an acyclicity check.
- ``exact_bd_local``: the Bayesian-Dirichlet marginal likelihood of one node
  computed in exact rational arithmetic as a Polya-urn sequential product,
  prod_t (N_jk(t) + a_jk) / (N_k(t) + a_k), which equals the Gamma-function
  ratio of Eq. (3) without evaluating any Gamma function.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np


def count_dags_robinson(n: int) -> int:
    """a(n) = sum_{k=1..n} (-1)^(k+1) C(n,k) 2^(k(n-k)) a(n-k), a(0) = 1."""
    a = [1]
    for m in range(1, n + 1):
        s = 0
        for k in range(1, m + 1):
            s += (-1) ** (k + 1) * math.comb(m, k) * 2 ** (k * (m - k)) * a[m - k]
        a.append(s)
    return a[n]


def enumerate_dags(n: int, K: int) -> np.ndarray:
    """All DAGs with in-degree <= K: int64 array [G][n] of parent masks."""
    per_node = []
    for i in range(n):
        others = [m for m in range(n) if m != i]
        masks = []
        for j in range(0, min(K, n - 1) + 1):
            for c in itertools.combinations(others, j):
                masks.append(sum(1 << m for m in c))
        per_node.append(np.array(masks, dtype=np.int64))
    grids = np.meshgrid(*per_node, indexing="ij")
    pa = np.stack([g.reshape(-1) for g in grids], axis=1)        # [A][n]
    # Kahn-style peeling: a node can be removed once all its parents are removed.
    removed = np.zeros(pa.shape[0], dtype=np.int64)
    for _ in range(n):
        for i in range(n):
            ok = (pa[:, i] & ~removed) == 0
            removed = np.where(ok, removed | (1 << i), removed)
    full = (1 << n) - 1
    return pa[removed == full]


def consistent_with(pa: np.ndarray, order) -> np.ndarray:
    """Boolean mask over DAGs: every parent of every node precedes it in ``order``."""
    pred = {}
    acc = 0
    for v in order:
        pred[int(v)] = acc
        acc |= 1 << int(v)
    ok = np.ones(pa.shape[0], dtype=bool)
    for i, p in pred.items():
        ok &= (pa[:, i] & ~p) == 0
    return ok


def exact_bd_local(data: np.ndarray, arities, node: int, parents, ess: Fraction) -> Fraction:
    """exp(ls) for gamma = 1 and no prior, as an exact fraction (BDeu alphas)."""
    parents = sorted(int(p) for p in parents)
    r = int(arities[node])
    q = 1
    for m in parents:
        q *= int(arities[m])
    a_jk = Fraction(ess) / (q * r)
    a_k = Fraction(ess) / q
    Njk: dict = {}
    Nk: dict = {}
    prob = Fraction(1)
    for row in np.asarray(data):
        k = 0
        for m in parents:
            k = k * int(arities[m]) + int(row[m])
        j = int(row[node])
        prob *= (Njk.get((k, j), 0) + a_jk) / (Nk.get(k, 0) + a_k)
        Njk[(k, j)] = Njk.get((k, j), 0) + 1
        Nk[k] = Nk.get(k, 0) + 1
    return prob


def log_fraction(x: Fraction) -> float:
    """Natural log of a positive fraction with big-integer numerator/denominator."""
    return math.log(x.numerator) - math.log(x.denominator)
