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
        L.orc_run_chain.argtypes = [P, i32, i32, u64, u64, i64, i32, i32, P, P, P, P, P, P]
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
              prior_mode: int = 0, threads: int = 1) -> np.ndarray:
    """FP64 row of one node, indexed by the oracle's combinatorial rank.

    ``threads`` > 1 splits the rank range over that many threads (the C call
    releases the GIL); every entry is still computed by the same plain code.
    """
    data, ar, pr = _prep(data, arities, prior)
    n = data.shape[1]
    S = num_sets(n - 1, K)
    out = np.zeros(S, dtype=np.float64)
    L = lib()

    def part(r0, r1):
        L.orc_build_row(_p(data), data.shape[0], n, _p(ar), K, ess, log_gamma,
                        None if pr is None else _p(pr), prior_mode, node, r0, r1, _p(out))

    if threads <= 1:
        part(0, S)
    else:
        from concurrent.futures import ThreadPoolExecutor
        cuts = [S * k // (4 * threads) for k in range(4 * threads + 1)]
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


def run_chain(table: np.ndarray, K: int, seed: int, chain: int, iters: int, target: int = 0,
              round_f32: bool = True):
    """Returns dict(order, trace[iters+1], acc[iters], best_graph[n], best_score, accepted)."""
    table = np.ascontiguousarray(table, dtype=np.float64)
    n = table.shape[0]
    order = np.zeros(n, dtype=np.int32)
    trace = np.zeros(iters + 1)
    acc = np.zeros(max(iters, 1), dtype=np.uint8)
    bg = np.zeros(n, dtype=np.uint64)
    bs = ctypes.c_double()
    na = ctypes.c_int64()
    lib().orc_run_chain(_p(table), n, K, seed, chain, iters, target, int(round_f32), _p(order),
                        _p(trace), _p(acc), _p(bg), ctypes.byref(bs), ctypes.byref(na))
    return dict(order=order, trace=trace, acc=acc[:iters], best_graph=bg, best_score=bs.value,
                accepted=na.value)
