"""Edge counting and the random inputs of the structure-recovery study (CPU)."""
import numpy as np
import pytest

from paper_1210_5128_amd import accuracy as A


def masks(n, edges):
    m = [0] * n
    for p, c in edges:
        m[c] |= 1 << p
    return np.array(m, dtype=np.uint64)


def test_edge_rates_by_hand():
    n = 3
    true = masks(n, [(0, 1), (1, 2)])
    learned = masks(n, [(0, 1), (2, 1)])          # second edge reversed
    r = A.edge_rates(learned, true, n)
    assert (r.tp, r.fn, r.fp, r.tn) == (1, 1, 1, 3)
    assert r.tpr == 0.5 and r.fpr == 0.25
    r = A.edge_rates(true, true, n)
    assert (r.tpr, r.fpr) == (1.0, 0.0)
    r = A.edge_rates(masks(n, []), true, n)
    assert (r.tp, r.fp, r.fn, r.tn) == (0, 0, 2, 4)


def test_adjacency_uses_bit_63():
    n = 64
    m = np.zeros(n, dtype=np.uint64)
    m[0] = np.uint64(1 << 63)
    a = A.masks_to_adjacency(m, n)
    assert a[63, 0] and a.sum() == 1


def test_injected_prior_protocol():
    n = 5
    true = masks(n, [(0, 1), (1, 2), (2, 3), (3, 4)])
    learned = masks(n, [(0, 1), (2, 1), (3, 4), (0, 4)])
    missed = [(2, 1), (3, 2)]          # (child, parent): 1->2 and 2->3 not found
    added = [(1, 2), (4, 0)]           # 2->1 and 0->4 not true
    R = A.injected_prior(true, learned, n, 0.8, 0.1, 1.0, seed=1)
    for i in range(n):
        for m in range(n):
            want = 0.8 if (i, m) in missed else (0.1 if (i, m) in added else 0.5)
            assert R[i, m] == np.float32(want), (i, m)
    assert np.all(A.injected_prior(true, learned, n, 0.8, 0.1, 0.0, seed=1) == 0.5)
    # probability: about half of many wrong edges get a prior
    n = 40
    true = masks(n, [(i, i + 1) for i in range(n - 1)])
    R = A.injected_prior(true, masks(n, []), n, 0.7, 0.2, 0.5, seed=3)
    frac = (R == np.float32(0.7)).sum() / (n - 1)
    assert 0.3 < frac < 0.7


def test_flip_states():
    rng = np.random.default_rng(0)
    d = rng.integers(0, 2, size=(400, 50)).astype(np.int8)
    assert np.array_equal(A.flip_states(d, 0.0, 1), d)
    assert np.array_equal(A.flip_states(d, 1.0, 1), 1 - d)
    rate = (A.flip_states(d, 0.1, 2) != d).mean()
    assert abs(rate - 0.1) < 0.01
    with pytest.raises(ValueError):
        A.flip_states(d + 1, 0.1, 1)
