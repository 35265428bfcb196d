"""The allocation-free scoring entry point (bnos_score_orders_noalloc), called
through the C-ABI, against bnos_score_orders on the same inputs: bit-for-bit
equal outputs on two calls in a row, the second with a smaller input, and the
size limit of its fixed scratch array."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1210_5128_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bnos():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_5128_amd import bnos as b
    return b


def outputs(B, n):
    dev = torch.device("cuda")
    return dict(lse=torch.empty(B, dtype=torch.float64, device=dev),
                max=torch.empty(B, dtype=torch.float64, device=dev),
                best=torch.empty((B, n), dtype=torch.int64, device=dev),
                node_lse=torch.empty((B, n), dtype=torch.float64, device=dev),
                node_second=torch.empty((B, n), dtype=torch.float32, device=dev))


def call(bnos, fn, table, orders):
    """One C-ABI scoring call (fn = the exported function) on device tensors."""
    B, n = orders.shape
    o = torch.from_numpy(np.ascontiguousarray(orders, dtype=np.int32)).cuda()
    out = outputs(B, n)
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    st = fn(table.handle, p(o), B, p(out["lse"]), p(out["max"]), p(out["best"]), p(out["node_lse"]),
            p(out["node_second"]), ctypes.c_void_p(0))
    torch.cuda.synchronize()
    return st, {k: v.cpu().numpy() for k, v in out.items()}


def same_bits(a, b):
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k


def test_noalloc_scoring_matches_the_workspace_call(bnos):
    lib = bnos._lib
    big = datagen.WORKLOADS["mixed40"]
    net, prior = datagen.make(big)
    t1 = bnos.build_score_table(net.data, net.arities, big.K, prior=prior)
    small = datagen.random_network(12, 300, (2, 3), 3, seed=5)
    t2 = bnos.build_score_table(small.data, small.arities, 3)
    try:
        # first call: 64 orders of the 40-node table (stored masks, several orders per block)
        o1 = datagen.random_orders(big.n, 64, seed=301)
        s_ref, ref = call(bnos, lib.bnos_score_orders, t1, o1)
        s_new, new = call(bnos, lib.bnos_score_orders_noalloc, t1, o1)
        assert s_ref == 0 and s_new == 0, bnos._lib.bnos_last_error()
        same_bits(ref, new)
        # second call, smaller: one order of the same table (computed masks), then 3 of a 12-node table
        s_new, new = call(bnos, lib.bnos_score_orders_noalloc, t1, o1[5:6])
        assert s_new == 0
        s_ref, ref = call(bnos, lib.bnos_score_orders, t1, o1[5:6])
        same_bits(ref, new)
        o2 = datagen.random_orders(12, 3, seed=302)
        o2[1, 0] = o2[1, 3]                       # not a permutation: NaN, best 0, the others unaffected
        s_new, new = call(bnos, lib.bnos_score_orders_noalloc, t2, o2)
        s_ref, ref = call(bnos, lib.bnos_score_orders, t2, o2)
        assert s_new == 0 and s_ref == 0
        same_bits(ref, new)
        assert np.isnan(new["lse"][1]) and np.all(new["best"][1] == 0)
        # above the fixed array: rejected before any device work, nothing written
        Bmax = 20000
        o3 = np.tile(datagen.random_orders(big.n, 1, seed=303), (Bmax, 1))
        s_big, out = call(bnos, lib.bnos_score_orders_noalloc, t1, o3)
        assert s_big == bnos.E_RANGE
        assert b"scratch" in lib.bnos_last_error()
    finally:
        t1.free()
        t2.free()
