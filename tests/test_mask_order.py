"""The order of a table row and the successor rule the scoring pass uses to
compute masks instead of reading them (no GPU needed).

A row lists every parent set of at most K members over the node's n - 1 other
nodes (as a mask over slots) in ascending numeric order.  The mask after m is
m + 1 when that has at most K members, else m plus its lowest member.  Checked
here against the enumeration of all such masks for small n and K."""
import itertools

import pytest


def next_mask(m, K, bits=64):
    t = m + 1
    r = t if bin(t).count("1") <= K else m + (m & -m)
    return (1 << bits) - 1 if r <= m or r >= (1 << bits) else r


@pytest.mark.parametrize("slots,K", [(1, 0), (1, 1), (5, 0), (5, 2), (7, 3), (8, 8), (10, 4), (12, 1)])
def test_successor_walks_the_row_in_order(slots, K):
    row = sorted(sum(1 << b for b in c) for k in range(K + 1) for c in itertools.combinations(range(slots), k))
    for a, b in zip(row, row[1:]):
        assert next_mask(a, K) == b
    # past the last mask: a slot beyond the row (>= slots) or saturation, never a mask of the row
    last = row[-1]
    m = last
    for _ in range(3):
        m = next_mask(m, K)
        assert m not in row[:-1] and (m >> slots) != 0


def test_saturation_at_64_bits():
    top = 1 << 63
    assert next_mask(top, 1) == (1 << 64) - 1          # top + lowest member overflows
    assert next_mask((1 << 64) - 1, 4) == (1 << 64) - 1
    assert next_mask(0, 0) == (1 << 64) - 1            # K = 0: the empty set is the whole row
