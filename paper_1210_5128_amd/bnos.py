"""Thin ctypes binding of ``libbnos.so`` (C ABI in ``include/bnos.h``).

Argument marshalling only: every step of table build and order scoring runs
in the library's HIP kernels.  Device buffers and streams come from PyTorch
(``tensor.data_ptr()``, ``torch.cuda.current_stream().cuda_stream``).
Importing this module loads the library and raises if it is missing.

PyTorch is imported before the library is opened.  A PyTorch ROCm wheel
carries its own HIP and HSA runtimes under the same sonames as the system's;
with PyTorch's copy already mapped, ``libbnos.so`` binds to it, so device
pointers and streams from PyTorch are valid in the library's calls.  Opened
first, the library would map the system runtimes beside PyTorch's, and the
second runtime to start in the process sees no device.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch  # noqa: F401  (maps the HIP runtime the library must share)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbnos.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -c 'import __graft_entry__ as g; g.build()')")

_lib = ctypes.CDLL(LIB_PATH)

OK, E_INVALID, E_RANGE, E_NOMEM, E_DEVICE, E_STATE = 0, -1, -2, -3, -4, -5

P = ctypes.c_void_p
i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class BuildOpts(ctypes.Structure):
    _fields_ = [("log_gamma", ctypes.c_double), ("prior_mode", ctypes.c_int32), ("chunk_steps", ctypes.c_int32),
                ("count_mode", ctypes.c_int32), ("data_on_device", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


class ChainCfg(ctypes.Structure):
    _fields_ = [("chains", ctypes.c_int32), ("target", ctypes.c_int32), ("iterations", ctypes.c_int64),
                ("first_iteration", ctypes.c_int64), ("seed", ctypes.c_uint64), ("chain_offset", ctypes.c_int64),
                ("trace_every", ctypes.c_int32), ("sweep_len", ctypes.c_int32), ("proposal", ctypes.c_int32),
                ("eps", ctypes.c_float), ("mlp", P), ("topk", ctypes.c_int32), ("trace_edges", ctypes.c_int32),
                ("edges", P), ("reserved", ctypes.c_int32 * 2)]


class ChainState(ctypes.Structure):
    _fields_ = [("orders", P), ("scores", P), ("best_graphs", P), ("best_scores", P), ("accepted", P),
                ("trace", P), ("accept_flags", P), ("harvest_feats", P), ("harvest_pairs", P),
                ("harvest_count", P), ("harvest_cap", ctypes.c_int64), ("top_graphs", P), ("top_scores", P),
                ("top_count", P), ("edge_trace", P)]


_SIGS = {
    "bnos_last_error": (ctypes.c_char_p, []),
    "bnos_version": (i32, []),
    "bnos_build_score_table": (i32, [P, i64, i32, P, i32, f64, P, P, P, P]),
    "bnos_table_free": (None, [P]),
    "bnos_table_info": (i32, [P, P, P, P, P]),
    "bnos_table_export": (i32, [P, i32, P, P, i64]),
    "bnos_table_node_features": (i32, [P, P]),
    "bnos_counts": (i32, [P, i32, P, P, P, i64]),
    "bnos_score_orders": (i32, [P, P, i32, P, P, P, P, P, P]),
    "bnos_score_order": (i32, [P, P, P, P, P]),
    "bnos_score_orders_noalloc": (i32, [P, P, i32, P, P, P, P, P, P]),
    "bnos_run_chains": (i32, [P, P, P, P]),
    "bnos_run_chains_multi": (i32, [P, i32, P, P, P]),
    "bnos_mlp_create": (i32, [P]),
    "bnos_mlp_free": (None, [P]),
    "bnos_mlp_set_params": (i32, [P, P, P, P]),
    "bnos_mlp_get_params": (i32, [P, P, P, P]),
    "bnos_mlp_fit_norm": (i32, [P, P, i64, P]),
    "bnos_mlp_forward": (i32, [P, P, i32, i32, P, P]),
    "bnos_mlp_grad": (i32, [P, P, P, i32, i32, ctypes.c_float, P, P, P]),
    "bnos_mlp_train": (i32, [P, P, P, i64, i32, ctypes.c_float, i32, i32, ctypes.c_float, ctypes.c_uint64, P, P]),
    "bnos_table_timing": (i32, [P, i32]),
    "bnos_table_tile_skip": (i32, [P, i32]),
    "bnos_table_score_bound": (i32, [P, i32]),
    "bnos_table_computed_masks": (i32, [P, i32]),
    "bnos_table_count_tiles": (i32, [P, P, i32, P, P]),
    "bnos_table_autotune": (i32, [P, P, i32, i32, P, P, P, P, P]),
    "bnos_table_set_launch": (i32, [P, i32, i32, i32, i32]),
    "bnos_chains_autotune": (i32, [P, P, P, i32, P, P, P, P]),
    "bnos_chains_set_launch": (i32, [P, i32, i32, i32]),
    "bnos_table_timing_read": (i32, [P, P, P, P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class BnosError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bnos status {status}: {msg}")
        self.status = status


def _check(status: int):
    if status != OK:
        raise BnosError(status, _lib.bnos_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(P)


def _dptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Table:
    """A device-resident local-score table of one dataset."""

    def __init__(self, handle: int, n: int, K: int):
        self._h = ctypes.c_void_p(handle)
        self.n = n
        self.K = K

    # -- lifetime
    def free(self):
        if self._h:
            _lib.bnos_table_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- info / export
    def info(self):
        n, K, S, b = i32(), i32(), i64(), i64()
        _check(_lib.bnos_table_info(self._h, ctypes.byref(n), ctypes.byref(K), ctypes.byref(S),
                                    ctypes.byref(b)))
        return dict(n=n.value, K=K.value, entries_per_node=S.value, device_bytes=b.value)

    def export(self, node: int):
        S = self.info()["entries_per_node"]
        masks = np.zeros(S, dtype=np.uint64)
        scores = np.zeros(S, dtype=np.float32)
        _check(_lib.bnos_table_export(self._h, node, _ptr(masks), _ptr(scores), S))
        return masks, scores

    def counts(self, nodes, masks, arities):
        nodes = np.ascontiguousarray(nodes, dtype=np.int32)
        masks = np.ascontiguousarray(masks, dtype=np.uint64)
        sizes = []
        for v, m in zip(nodes, masks):
            c = int(arities[int(v)])
            for b in range(self.n):
                if (int(m) >> b) & 1:
                    c *= int(arities[b])
            sizes.append(c)
        out = np.zeros(max(sum(sizes), 1), dtype=np.uint32)
        _check(_lib.bnos_counts(self._h, len(nodes), _ptr(nodes), _ptr(masks), _ptr(out), out.size))
        res = []
        off = 0
        for c in sizes:
            res.append(out[off:off + c].copy())
            off += c
        return res

    # -- scoring
    def score_orders(self, orders, lse, maxs, best, node_lse=None, node_second=None, stream=None):
        """Asynchronous batched scoring on device tensors (see bnos_score_orders)."""
        B = int(orders.shape[0])
        _check(_lib.bnos_score_orders(self._h, _dptr(orders), B, _dptr(lse), _dptr(maxs), _dptr(best),
                                      _dptr(node_lse), _dptr(node_second), _stream(stream)))

    def score_orders_noalloc(self, orders, lse, maxs, best, node_lse=None, node_second=None, stream=None):
        """score_orders with the partials in the library's fixed per-GPU array (bnos_score_orders_noalloc)."""
        B = int(orders.shape[0])
        _check(_lib.bnos_score_orders_noalloc(self._h, _dptr(orders), B, _dptr(lse), _dptr(maxs), _dptr(best),
                                              _dptr(node_lse), _dptr(node_second), _stream(stream)))

    def score_order(self, order):
        """Synchronous host-side scoring of one order -> (lse, max, best_parents[n])."""
        order = np.ascontiguousarray(order, dtype=np.int32)
        lse, mx = f64(), f64()
        best = np.zeros(self.n, dtype=np.uint64)
        _check(_lib.bnos_score_order(self._h, _ptr(order), ctypes.byref(lse), ctypes.byref(mx), _ptr(best)))
        return lse.value, mx.value, best

    # -- chains
    def node_features(self):
        """Static per-node features [n][5]: prior row sum, column sum, max, mean, sd of the scores."""
        out = np.zeros((self.n, 5))
        _check(_lib.bnos_table_node_features(self._h, _ptr(out)))
        return out

    def new_chain_state(self, chains: int, iterations: int, trace_every: int = 1, flags: bool = False,
                        device=None, harvest_cap: int = 0, topk: int = 0, edges=None):
        """Device tensors holding the state of `chains` chains (see bnos_chain_state).
        edges: optional (child, parent) pairs (at most 32) whose presence in each
        chain's current greedy graph is traced into state["edge_trace"]."""
        import torch
        dev = device or torch.device("cuda")
        n = self.n
        st = dict(
            orders=torch.zeros((chains, n), dtype=torch.int32, device=dev),
            scores=torch.zeros(chains, dtype=torch.float64, device=dev),
            best_graphs=torch.zeros((chains, n), dtype=torch.int64, device=dev),
            best_scores=torch.zeros(chains, dtype=torch.float64, device=dev),
            accepted=torch.zeros(chains, dtype=torch.int64, device=dev),
            trace=(torch.zeros((chains, iterations // trace_every + 1), dtype=torch.float64, device=dev)
                   if trace_every > 0 else None),
            accept_flags=torch.zeros((chains, max(iterations, 1)), dtype=torch.uint8, device=dev) if flags else None,
        )
        if harvest_cap > 0:
            st["harvest_feats"] = torch.zeros((chains, harvest_cap, n, 8), dtype=torch.float32, device=dev)
            st["harvest_pairs"] = torch.zeros((chains, harvest_cap, 2), dtype=torch.int32, device=dev)
            st["harvest_count"] = torch.zeros(chains, dtype=torch.int64, device=dev)
        if edges is not None and len(edges):
            st["edges"] = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
            st["edge_trace"] = torch.zeros((chains, iterations // max(1, trace_every) + 1), dtype=torch.int32,
                                           device=dev)
        if topk > 0:
            st["top_graphs"] = torch.zeros((chains, topk, n), dtype=torch.int64, device=dev)
            st["top_scores"] = torch.zeros((chains, topk), dtype=torch.float64, device=dev)
            st["top_count"] = torch.zeros(chains, dtype=torch.int32, device=dev)
        return st

    def run_chains(self, state: dict, iterations: int, seed: int, target: int = 0, first_iteration: int = 0,
                   trace_every: int = 1, chain_offset: int = 0, sweep_len: int = 0, mlp=None, eps=0.5, stream=None):
        """Run MH chains in place on `state` (from new_chain_state); returns when done.
        With `mlp` the swap pair comes from the learned proposal (exact MH correction)."""
        chains = int(state["orders"].shape[0])
        cfg = _chain_cfg(chains, iterations, seed, target, first_iteration, trace_every, chain_offset, sweep_len,
                         mlp, eps)
        cfg.topk = _state_topk([state])
        edges = _state_edges(cfg, [state])
        st = _chain_state(state, iterations, trace_every)
        _check(_lib.bnos_run_chains(self._h, ctypes.byref(cfg), ctypes.byref(st), _stream(stream)))

    def chains_autotune(self, chains: int, iterations: int, seed: int, state: Optional[dict] = None,
                        first_iteration: int = 0, target: int = 0, reps: int = 1, mlp=None, eps=0.5, stream=None):
        """Pick the chain-sweep launch for `chains` chains by timing `iterations` real
        iterations per shape (bnos_chains_autotune); with first_iteration > 0 each run
        resumes from a copy of `state` -> (chunk steps, chains per block, ms per iteration)."""
        cfg = _chain_cfg(chains, iterations, seed, target, first_iteration, 1, 0, 0, mlp, eps)
        st = None
        if state is not None:           # the tuner copies only the chains' positions, never the traces
            st = _chain_state({k: state.get(k) for k in ("orders", "scores", "best_graphs", "best_scores",
                                                         "accepted")}, iterations, 1)
        cs, bt, ms = i32(), i32(), f64()
        _check(_lib.bnos_chains_autotune(self._h, ctypes.byref(cfg), ctypes.byref(st) if st is not None else None,
                                         reps, _stream(stream), ctypes.byref(cs), ctypes.byref(bt),
                                         ctypes.byref(ms)))
        return cs.value, bt.value, ms.value

    def chains_set_launch(self, chains: int, chunk_steps: int = 0, orders_per_block: int = 0):
        """Fix the chain-sweep launch for `chains` chains (bnos_chains_set_launch); 0, 0 = default."""
        _check(_lib.bnos_chains_set_launch(self._h, int(chains), int(chunk_steps), int(orders_per_block)))

    def autotune(self, orders, reps: int = 5, stream=None):
        """Pick the launch for this batch size (bnos_table_autotune):
        -> (chunk steps, orders per block, gather pass chosen, ms per launch)."""
        cs, bt, g, ms = i32(), i32(), i32(), f64()
        _check(_lib.bnos_table_autotune(self._h, _dptr(orders), int(orders.shape[0]), reps, _stream(stream),
                                        ctypes.byref(cs), ctypes.byref(bt), ctypes.byref(g), ctypes.byref(ms)))
        return cs.value, bt.value, g.value, ms.value

    def set_launch(self, B: int, gather: bool = False, chunk_steps: int = 0, orders_per_block: int = 0):
        """Fix the scoring launch for batches of B orders (bnos_table_set_launch)."""
        _check(_lib.bnos_table_set_launch(self._h, int(B), int(bool(gather)), int(chunk_steps),
                                          int(orders_per_block)))

    def tile_skip(self, enable: bool):
        _check(_lib.bnos_table_tile_skip(self._h, int(enable)))

    def score_bound(self, enable: bool):
        _check(_lib.bnos_table_score_bound(self._h, int(enable)))

    def computed_masks(self, enable: bool):
        """One-order launches compute the masks from per-4-entry anchors (bnos_table_computed_masks)."""
        _check(_lib.bnos_table_computed_masks(self._h, int(enable)))

    def count_tiles(self, orders):
        """-> (tiles a scoring launch of these device orders reads with skipping, tiles per full pass)."""
        a, b = i64(), i64()
        _check(_lib.bnos_table_count_tiles(self._h, _dptr(orders), int(orders.shape[0]), ctypes.byref(a),
                                           ctypes.byref(b)))
        return a.value, b.value

    # -- timing
    def timing(self, enable, every: int = 1):
        """Kernel timing (bnos_table_timing): off, or events on every `every`-th scoring launch."""
        _check(_lib.bnos_table_timing(self._h, int(every) if enable else 0))

    def timing_read(self):
        """-> (total kernel ms, launches, table passes) since timing was enabled."""
        ms, cnt, passes = f64(), i64(), i64()
        _check(_lib.bnos_table_timing_read(self._h, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(passes)))
        return ms.value, cnt.value, passes.value


NPARAM = 17793


class Mlp:
    """The learned swap proposal's network (see bnos_mlp_* in bnos.h)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(_lib.bnos_mlp_create(ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h:
            _lib.bnos_mlp_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def set_params(self, params=None, mu=None, sd=None):
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        if p is not None and p.size != NPARAM:
            raise ValueError("expected 17793 parameters")
        m = None if mu is None else np.ascontiguousarray(mu, dtype=np.float32)
        d = None if sd is None else np.ascontiguousarray(sd, dtype=np.float32)
        _check(_lib.bnos_mlp_set_params(self._h, None if p is None else _ptr(p), None if m is None else _ptr(m),
                                        None if d is None else _ptr(d)))

    def get_params(self):
        p = np.zeros(NPARAM, dtype=np.float32)
        mu = np.zeros(8, dtype=np.float32)
        sd = np.zeros(8, dtype=np.float32)
        _check(_lib.bnos_mlp_get_params(self._h, _ptr(p), _ptr(mu), _ptr(sd)))
        return p, mu, sd

    def fit_norm(self, feats, stream=None):
        rows = int(feats.numel() // 8)
        _check(_lib.bnos_mlp_fit_norm(self._h, _dptr(feats), rows, _stream(stream)))

    def forward(self, feats, logits, stream=None):
        R, n = int(feats.shape[0]), int(feats.shape[1])
        _check(_lib.bnos_mlp_forward(self._h, _dptr(feats), R, n, _dptr(logits), _stream(stream)))

    def grad(self, feats, pairs, grad, loss=None, eps=0.1, stream=None):
        R, n = int(feats.shape[0]), int(feats.shape[1])
        _check(_lib.bnos_mlp_grad(self._h, _dptr(feats), _dptr(pairs), R, n, eps, _dptr(grad), _dptr(loss),
                                  _stream(stream)))

    def train(self, feats, pairs, epochs, batch, lr, seed, eps=0.1, loss_trace=None, count=None, stream=None):
        n = int(feats.shape[1])
        cnt = int(feats.shape[0]) if count is None else int(count)
        _check(_lib.bnos_mlp_train(self._h, _dptr(feats), _dptr(pairs), cnt, n, eps, epochs, batch, lr, seed,
                                   _dptr(loss_trace), _stream(stream)))


def _chain_cfg(chains, iterations, seed, target, first_iteration, trace_every, chain_offset, sweep_len,
               mlp=None, eps=0.5):
    cfg = ChainCfg()
    if mlp is not None:
        cfg.proposal = 1
        cfg.mlp = mlp.handle
        cfg.eps = eps
    cfg.chains = chains
    cfg.target = target
    cfg.iterations = iterations
    cfg.first_iteration = first_iteration
    cfg.seed = seed
    cfg.chain_offset = chain_offset
    cfg.trace_every = max(1, trace_every)
    cfg.sweep_len = sweep_len
    return cfg


def _state_topk(states) -> int:
    """Records per chain of the best-graph record the states carry (0 = none)."""
    ks = {int(s["top_graphs"].shape[1]) if s.get("top_graphs") is not None else 0 for s in states}
    if len(ks) != 1:
        raise ValueError("every state needs the same best-graph record size")
    return ks.pop()


def _state_edges(cfg, states):
    """Set cfg's traced edges from the states (all must trace the same edges);
    returns the host array, which must stay alive during the call."""
    lists = [s.get("edges") for s in states]
    if all(e is None for e in lists):
        return None
    if any(e is None or not np.array_equal(e, lists[0]) for e in lists):
        raise ValueError("every state needs the same traced edges")
    e = lists[0]
    cfg.trace_edges = int(e.shape[0])
    cfg.edges = e.ctypes.data
    return e


def _chain_state(state: dict, iterations: int, trace_every: int) -> ChainState:
    st = ChainState()
    for k in ("orders", "scores", "best_graphs", "best_scores", "accepted", "trace", "accept_flags",
              "harvest_feats", "harvest_pairs", "harvest_count", "top_graphs", "top_scores", "top_count",
              "edge_trace"):
        v = state.get(k)
        setattr(st, k, None if v is None else v.data_ptr())
    if state.get("harvest_feats") is not None:
        st.harvest_cap = int(state["harvest_feats"].shape[1])
    if state.get("trace") is not None and state["trace"].shape[1] < iterations // max(1, trace_every) + 1:
        raise ValueError("trace tensor too small")
    if state.get("accept_flags") is not None and state["accept_flags"].shape[1] < iterations:
        raise ValueError("accept_flags tensor too small")
    if state.get("edge_trace") is not None and state["edge_trace"].shape[1] < iterations // max(1, trace_every) + 1:
        raise ValueError("edge_trace tensor too small")
    return st


def run_chains_multi(tables, states, iterations: int, seed: int, target: int = 0, first_iteration: int = 0,
                     trace_every: int = 1, chain_offset: int = 0, sweep_len: int = 0, mlp=None, eps=0.5, stream=None):
    """Advance the chains of several tables in one set of launches (bnos_run_chains_multi)."""
    T = len(tables)
    chains = int(states[0]["orders"].shape[0])
    if any(int(s["orders"].shape[0]) != chains for s in states):
        raise ValueError("every table needs the same number of chains")
    cfg = _chain_cfg(chains, iterations, seed, target, first_iteration, trace_every, chain_offset, sweep_len,
                     mlp, eps)
    cfg.topk = _state_topk(states)
    edges = _state_edges(cfg, states)
    hs = (P * T)(*[t.handle.value for t in tables])
    sts = (ChainState * T)(*[_chain_state(s, iterations, trace_every) for s in states])
    _check(_lib.bnos_run_chains_multi(hs, T, ctypes.byref(cfg), sts, _stream(stream)))


def build_score_table(data, arities, K: int, ess: float = 1.0, prior=None, prior_mode: int = 0,
                      log_gamma: float = 0.0, chunk_steps: int = 0, count_mode: int = 0, stream=None) -> Table:
    """Build the local-score table (see bnos_build_score_table).  `data` is a host
    array, or a DEVICE int8 torch tensor [N][n] (row-major), passed as a device
    pointer; the other inputs are host arrays."""
    on_dev = hasattr(data, "is_cuda") and data.is_cuda
    if on_dev:
        import torch
        if data.dtype != torch.int8 or data.dim() != 2 or not data.is_contiguous():
            raise ValueError("device data must be a contiguous int8 tensor [N][n]")
    else:
        data = np.ascontiguousarray(data, dtype=np.int8)
        if data.ndim != 2:
            raise ValueError("data must be [N][n]")
    N, n = data.shape
    ar = np.ascontiguousarray(arities, dtype=np.int32)
    pr = None if prior is None else np.ascontiguousarray(prior, dtype=np.float32)
    opts = BuildOpts()
    opts.log_gamma = log_gamma
    opts.prior_mode = prior_mode
    opts.chunk_steps = chunk_steps
    opts.count_mode = count_mode
    opts.data_on_device = 1 if on_dev else 0
    h = ctypes.c_void_p()
    st = ctypes.c_void_p(0) if stream is None else _stream(stream)
    dptr = (_dptr(data) if on_dev else _ptr(data)) if N else None
    _check(_lib.bnos_build_score_table(dptr, N, n, _ptr(ar), K, ess,
                                       None if pr is None else _ptr(pr), ctypes.byref(opts), st,
                                       ctypes.byref(h)))
    return Table(h.value, n, K)


def version() -> int:
    return int(_lib.bnos_version())


def exported_symbols():
    return list(_SIGS)
