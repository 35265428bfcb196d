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


def next_mask_nosat(m, K):
    t = m + 1
    return t if bin(t).count("1") <= K else m + (m & -m)


@pytest.mark.parametrize("K", [1, 2, 3, 4, 6])
def test_steps_without_saturation_stay_in_range(K):
    """Where the scoring pass drops the saturation test (K >= 2 with n <= 63, K = 1 with
    n <= 61), three steps from the padding anchor 2^(n-1) or from any of the row's last
    masks stay below 2^64 and keep a slot >= n - 1 once past the row."""
    for n in range(2, 64):
        if not ((K >= 2 and n <= 63) or (K == 1 and n <= 61)):
            continue
        slots = n - 1
        top = sorted(sum(1 << b for b in c) for k in range(1, min(K, slots) + 1)
                     for c in itertools.combinations(range(max(0, slots - K - 1), slots), k))[-4:]
        for start in [1 << slots] + top:
            m = start
            for _ in range(3):
                m = next_mask_nosat(m, K)
                assert m < (1 << 64)
                if m >= (1 << slots):
                    assert m >> slots != 0
    # and the excluded case does overflow: K = 1, n = 62 from the padding anchor
    m = 1 << 61
    for _ in range(3):
        m = next_mask_nosat(m, 1)
    assert m >= (1 << 64)
