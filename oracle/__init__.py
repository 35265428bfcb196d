"""CPU oracle for order-space Bayesian-network structure learning.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it to check and time the GPU library.  The product never
imports it.  ``bnos_oracle.c`` holds the FP64 arithmetic; this module compiles
it with gcc and wraps it with ctypes.  ``brute`` holds pure-Python checkers
(DAG enumeration, exact rational scores) that pin the C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bnos_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` with gcc -O2."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u64, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
        L.orc_num_sets.restype = i64
        L.orc_num_sets.argtypes = [i32, i32]
        L.orc_counts.restype = i64
        L.orc_counts.argtypes = [P, i64, i32, P, i32, u64, P]
        L.orc_ppf_nats.restype = f64
        L.orc_ppf_nats.argtypes = [f64, i32]
        L.orc_local_score.restype = f64
        L.orc_local_score.argtypes = [P, i64, i32, P, i32, u64, f64, f64, P, i32]
        L.orc_rank.restype = i64
        L.orc_rank.argtypes = [i32, i32, i32, u64]
        L.orc_unrank.restype = u64
        L.orc_unrank.argtypes = [i32, i32, i32, i64]
        L.orc_build_table.restype = None
        L.orc_build_table.argtypes = [P, i64, i32, P, i32, f64, f64, P, i32, P]
        L.orc_score_order.restype = None
        L.orc_score_order.argtypes = [P, i32, i32, P, i32, P, P, P, P, P, P]
        L.orc_score_node_direct.restype = None
        L.orc_score_node_direct.argtypes = [P, i64, i32, P, i32, f64, f64, P, i32, i32, u64, i32,
                                            P, P, P, P]
        L.orc_build_row.restype = None
        L.orc_build_row.argtypes = [P, i64, i32, P, i32, f64, f64, P, i32, i32, i64, i64, P]
        L.orc_score_node_row.restype = None
        L.orc_score_node_row.argtypes = [P, i32, i32, i32, u64, i32, P, P, P, P]
        L.orc_draw.restype = u64
        L.orc_draw.argtypes = [u64, u64, u64, u64]
        L.orc_initial_order.restype = None
        L.orc_initial_order.argtypes = [u64, u64, i32, P]
        L.orc_swap_pair.restype = None
        L.orc_swap_pair.argtypes = [u64, u64, i32, u64, P, P]
        L.orc_accept_uniform.restype = f64
        L.orc_accept_uniform.argtypes = [u64, u64, u64]
        L.orc_run_chain.restype = None
        L.orc_run_chain.argtypes = [P, i32, i32, u64, u64, i64, i32, i32, P, P, P, P, P, P, i32, P, P, P]
        L.orc_mlp_num_params.restype = i32
        L.orc_mlp_num_params.argtypes = []
        L.orc_table_stats.restype = None
        L.orc_table_stats.argtypes = [P, i32, i32, i32, P]
        L.orc_features.restype = None
        L.orc_features.argtypes = [i32, P, P, P, P, P, P]
        L.orc_mlp_forward.restype = None
        L.orc_mlp_forward.argtypes = [P, i32, P, P, P, P]
        L.orc_pair_logq.restype = f64
        L.orc_pair_logq.argtypes = [P, i32, i32, i32, f64]
        L.orc_mlp_loss_grad.restype = f64
        L.orc_mlp_loss_grad.argtypes = [P, i32, P, i32, i32, f64, P]
        L.orc_learned_pair.restype = None
        L.orc_learned_pair.argtypes = [u64, u64, i32, u64, P, P, f64, P, P]
        L.orc_run_chain_learned.restype = None
        L.orc_run_chain_learned.argtypes = [P, i32, i32, u64, u64, i64, i32, i32, P, P, P, P, P, f64,
                                            P, P, P, P, P, P, i32, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _prep(data, arities, prior):
    data = np.ascontiguousarray(data, dtype=np.int8)
    ar = np.ascontiguousarray(arities, dtype=np.int32)
    pr = None if prior is None else np.ascontiguousarray(prior, dtype=np.float32)
    return data, ar, pr


def num_sets(m: int, K: int) -> int:
    return int(lib().orc_num_sets(m, K))


def counts(data, arities, node: int, pmask: int) -> np.ndarray:
    data, ar, _ = _prep(data, arities, None)
    q = 1
    for m in range(data.shape[1]):
        if (pmask >> m) & 1:
            q *= int(ar[m])
    out = np.zeros(q * int(ar[node]), dtype=np.uint32)
    lib().orc_counts(_p(data), data.shape[0], data.shape[1], _p(ar), node, pmask, _p(out))
    return out


def ppf_nats(v: float, mode: int = 0) -> float:
    return float(lib().orc_ppf_nats(v, mode))


def local_score(data, arities, node: int, pmask: int, ess: float = 1.0, log_gamma: float = 0.0,
                prior=None, prior_mode: int = 0) -> float:
    data, ar, pr = _prep(data, arities, prior)
    return float(lib().orc_local_score(_p(data), data.shape[0], data.shape[1], _p(ar), node, pmask,
                                       ess, log_gamma, None if pr is None else _p(pr), prior_mode))


def rank(n: int, K: int, node: int, pmask: int) -> int:
    return int(lib().orc_rank(n, K, node, pmask))


def unrank(n: int, K: int, node: int, idx: int) -> int:
    return int(lib().orc_unrank(n, K, node, idx))


def build_table(data, arities, K: int, ess: float = 1.0, log_gamma: float = 0.0, prior=None,
                prior_mode: int = 0) -> np.ndarray:
    """FP64 table [n][S], indexed by the oracle's own combinatorial rank."""
    data, ar, pr = _prep(data, arities, prior)
    n = data.shape[1]
    S = num_sets(n - 1, K)
    out = np.zeros((n, S), dtype=np.float64)
    lib().orc_build_table(_p(data), data.shape[0], n, _p(ar), K, ess, log_gamma,
                          None if pr is None else _p(pr), prior_mode, _p(out))
    return out


def build_row(data, arities, K: int, node: int, ess: float = 1.0, log_gamma: float = 0.0, prior=None,
              prior_mode: int = 0, threads: int = 1, ranks=None) -> np.ndarray:
    """FP64 row of one node, indexed by the oracle's combinatorial rank.

    ``threads`` > 1 splits the rank range over that many threads (the C call
    releases the GIL); every entry is still computed by the same plain code.
    ``ranks`` = (r0, r1) computes only the entries r0 <= rank < r1 (the rest
    of the returned row stays 0).
    """
    data, ar, pr = _prep(data, arities, prior)
    n = data.shape[1]
    S = num_sets(n - 1, K)
    out = np.zeros(S, dtype=np.float64)
    L = lib()
    lo, hi = (0, S) if ranks is None else (max(0, int(ranks[0])), min(S, int(ranks[1])))

    def part(r0, r1):
        L.orc_build_row(_p(data), data.shape[0], n, _p(ar), K, ess, log_gamma,
                        None if pr is None else _p(pr), prior_mode, node, r0, r1, _p(out))

    if threads <= 1:
        part(lo, hi)
    else:
        from concurrent.futures import ThreadPoolExecutor
        cuts = [lo + (hi - lo) * k // (4 * threads) for k in range(4 * threads + 1)]
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda k: part(cuts[k], cuts[k + 1]), range(4 * threads)))
    return out


def score_node_row(row: np.ndarray, n: int, K: int, node: int, pred: int, round_f32: bool = True):
    """Returns (lse_i, best_i, best_mask_i, second_i) from one node's table row."""
    row = np.ascontiguousarray(row, dtype=np.float64)
    lse, best, bm, sec = ctypes.c_double(), ctypes.c_double(), ctypes.c_uint64(), ctypes.c_double()
    lib().orc_score_node_row(_p(row), n, K, node, pred, int(round_f32), ctypes.byref(lse),
                             ctypes.byref(best), ctypes.byref(bm), ctypes.byref(sec))
    return lse.value, best.value, bm.value, sec.value


def score_order(table: np.ndarray, K: int, order, round_f32: bool = True):
    """Returns (lse, max, best_masks[n] by node id, node_lse[n], node_best[n], node_second[n])."""
    table = np.ascontiguousarray(table, dtype=np.float64)
    n = table.shape[0]
    order = np.ascontiguousarray(order, dtype=np.int32)
    lse = ctypes.c_double()
    mx = ctypes.c_double()
    best = np.zeros(n, dtype=np.uint64)
    nl = np.zeros(n)
    nb = np.zeros(n)
    ns = np.zeros(n)
    lib().orc_score_order(_p(table), n, K, _p(order), int(round_f32), ctypes.byref(lse),
                          ctypes.byref(mx), _p(best), _p(nl), _p(nb), _p(ns))
    return lse.value, mx.value, best, nl, nb, ns


def score_node_direct(data, arities, K: int, node: int, pred: int, ess: float = 1.0,
                      log_gamma: float = 0.0, prior=None, prior_mode: int = 0,
                      round_f32: bool = True):
    """Returns (lse_i, best_i, best_mask_i, second_i) computed from the data directly."""
    data, ar, pr = _prep(data, arities, prior)
    lse = ctypes.c_double()
    best = ctypes.c_double()
    bm = ctypes.c_uint64()
    sec = ctypes.c_double()
    lib().orc_score_node_direct(_p(data), data.shape[0], data.shape[1], _p(ar), K, ess, log_gamma,
                                None if pr is None else _p(pr), prior_mode, node, pred,
                                int(round_f32), ctypes.byref(lse), ctypes.byref(best),
                                ctypes.byref(bm), ctypes.byref(sec))
    return lse.value, best.value, bm.value, sec.value


def draw(seed: int, chain: int, purpose: int, step: int) -> int:
    return int(lib().orc_draw(seed, chain, purpose, step))


def initial_order(seed: int, chain: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.int32)
    lib().orc_initial_order(seed, chain, n, _p(out))
    return out


def swap_pair(seed: int, chain: int, n: int, step: int):
    a = ctypes.c_int()
    b = ctypes.c_int()
    lib().orc_swap_pair(seed, chain, n, step, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def accept_uniform(seed: int, chain: int, step: int) -> float:
    return float(lib().orc_accept_uniform(seed, chain, step))


def _topk_buffers(n: int, topk: int):
    return (np.zeros((max(topk, 1), n), dtype=np.uint64), np.zeros(max(topk, 1)), ctypes.c_int32())


def run_chain(table: np.ndarray, K: int, seed: int, chain: int, iters: int, target: int = 0,
              round_f32: bool = True, topk: int = 0):
    """Returns dict(order, trace[iters+1], acc[iters], best_graph[n], best_score, accepted,
    top_graphs[count][n], top_scores[count]) (the last two empty unless topk > 0)."""
    table = np.ascontiguousarray(table, dtype=np.float64)
    n = table.shape[0]
    order = np.zeros(n, dtype=np.int32)
    trace = np.zeros(iters + 1)
    acc = np.zeros(max(iters, 1), dtype=np.uint8)
    bg = np.zeros(n, dtype=np.uint64)
    bs = ctypes.c_double()
    na = ctypes.c_int64()
    tg, ts, tc = _topk_buffers(n, topk)
    lib().orc_run_chain(_p(table), n, K, seed, chain, iters, target, int(round_f32), _p(order),
                        _p(trace), _p(acc), _p(bg), ctypes.byref(bs), ctypes.byref(na),
                        topk, _p(tg), _p(ts), ctypes.byref(tc))
    return dict(order=order, trace=trace, acc=acc[:iters], best_graph=bg, best_score=bs.value,
                accepted=na.value, top_graphs=tg[:tc.value], top_scores=ts[:tc.value])


# ---------------------------------------------------------------- learned proposal

HIDDEN = 128
FEATURES = 8


def mlp_num_params() -> int:
    return int(lib().orc_mlp_num_params())


def table_stats(table: np.ndarray, K: int, round_f32: bool = True) -> np.ndarray:
    table = np.ascontiguousarray(table, dtype=np.float64)
    n = table.shape[0]
    out = np.zeros((n, 3))
    lib().orc_table_stats(_p(table), n, K, int(round_f32), _p(out))
    return out


def prior_nats(prior, n: int, prior_mode: int = 0) -> np.ndarray:
    """Per-edge prior terms in nats, [child][parent], 0 on the diagonal."""
    out = np.zeros((n, n))
    if prior is not None:
        for i in range(n):
            for m in range(n):
                if i != m:
                    out[i, m] = ppf_nats(float(np.float32(prior[i, m])), prior_mode)
    return out


def features(order, node_best, node_second, prior_nats_m, stats) -> np.ndarray:
    order = np.ascontiguousarray(order, dtype=np.int32)
    n = order.size
    nb = np.ascontiguousarray(node_best, dtype=np.float64)
    ns = np.ascontiguousarray(node_second, dtype=np.float64)
    pn = None if prior_nats_m is None else np.ascontiguousarray(prior_nats_m, dtype=np.float64)
    st = np.ascontiguousarray(stats, dtype=np.float64)
    out = np.zeros((n, FEATURES))
    lib().orc_features(n, _p(order), _p(nb), _p(ns), None if pn is None else _p(pn), _p(st), _p(out))
    return out


def mlp_forward(prm: np.ndarray, z: np.ndarray) -> np.ndarray:
    prm = np.ascontiguousarray(prm, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    n = z.shape[0]
    out = np.zeros(n)
    lib().orc_mlp_forward(_p(prm), n, _p(z), _p(out), None, None)
    return out


def pair_logq(logits, a: int, b: int, eps: float) -> float:
    lg = np.ascontiguousarray(logits, dtype=np.float64)
    return float(lib().orc_pair_logq(_p(lg), lg.size, a, b, eps))


def mlp_loss_grad(prm: np.ndarray, z: np.ndarray, a: int, b: int, eps: float):
    """(loss, gradient) of -ln q({a,b}) for one sample."""
    prm = np.ascontiguousarray(prm, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    g = np.zeros_like(prm)
    loss = lib().orc_mlp_loss_grad(_p(prm), z.shape[0], _p(z), a, b, eps, _p(g))
    return float(loss), g


def learned_pair(seed: int, chain: int, step: int, logits, order, eps: float):
    lg = np.ascontiguousarray(logits, dtype=np.float64)
    order = np.ascontiguousarray(order, dtype=np.int32)
    a, b = ctypes.c_int(), ctypes.c_int()
    lib().orc_learned_pair(seed, chain, order.size, step, _p(lg), _p(order), eps, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def run_chain_learned(table, K, seed, chain, iters, prm, mu, sd, prior_nats_m, stats, eps=0.1, target=0,
                      round_f32=True, topk: int = 0):
    table = np.ascontiguousarray(table, dtype=np.float64)
    n = table.shape[0]
    prm = np.ascontiguousarray(prm, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    sd = np.ascontiguousarray(sd, dtype=np.float64)
    st = np.ascontiguousarray(stats, dtype=np.float64)
    pn = None if prior_nats_m is None else np.ascontiguousarray(prior_nats_m, dtype=np.float64)
    order = np.zeros(n, dtype=np.int32)
    trace = np.zeros(iters + 1)
    acc = np.zeros(max(iters, 1), dtype=np.uint8)
    bg = np.zeros(n, dtype=np.uint64)
    bs = ctypes.c_double()
    na = ctypes.c_int64()
    tg, ts, tc = _topk_buffers(n, topk)
    lib().orc_run_chain_learned(_p(table), n, K, seed, chain, iters, target, int(round_f32), _p(prm), _p(mu), _p(sd),
                                None if pn is None else _p(pn), _p(st), eps, _p(order), _p(trace), _p(acc), _p(bg),
                                ctypes.byref(bs), ctypes.byref(na), topk, _p(tg), _p(ts), ctypes.byref(tc))
    return dict(order=order, trace=trace, acc=acc[:iters], best_graph=bg, best_score=bs.value, accepted=na.value,
                top_graphs=tg[:tc.value], top_scores=ts[:tc.value])

