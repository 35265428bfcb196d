"""Integer arithmetic the counting kernels rely on (no GPU needed).

The joint-histogram build splits a cell index of a contingency table into the
states of its variables by dividing by each arity.  It divides with a
multiply-high: for an arity r in [2, 255] and m = floor(2^32 / r) + 1, the
quotient of x by r is the high 32 bits of x * m for every x from 0 to 2^14 (a
table holds at most 2^14 cells).  Cell byte offsets and the remainders are
formed with 24-bit multiplies, so every factor must stay below 2^24.  Both
facts are checked here over the whole domain."""
import numpy as np

MAX_CELLS = 1 << 14


def test_multiply_high_quotient_is_exact_for_every_cell_index():
    x = np.arange(MAX_CELLS + 1, dtype=np.uint64)
    for r in range(2, 256):
        m = np.uint64((1 << 32) // r + 1)
        q = (x * m) >> np.uint64(32)
        assert np.array_equal(q, x // np.uint64(r)), r
        assert np.all(x - q * np.uint64(r) < np.uint64(r)), r


def test_cell_offsets_fit_24_bit_multiplies():
    # A 24-bit multiply takes operands below 2^24 and returns the low 32 bits of
    # their product.  Operands: a state (< 256) or a quotient (<= 2^14), and a
    # stride in bytes (4 x a stride <= 2^14) or an arity (< 256).  Products: a
    # state times its stride stays inside the table (< 4 x 2^14 bytes), and a
    # quotient times the arity is at most the cell index.
    assert max(255, MAX_CELLS) < (1 << 24) and 4 * MAX_CELLS < (1 << 24)
    for r in range(2, 256):
        stride = MAX_CELLS // r              # the largest stride of a digit of radix r
        assert (r - 1) * 4 * stride < 4 * MAX_CELLS < (1 << 32)
