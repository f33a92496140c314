"""Host check of the integer identity behind the persistent FMA kernel's
index decode: the quotient of 0 <= n < 2^16 by a launch-fixed divisor
1 <= d <= 256 (N, N^2 or the mode count) is taken as a multiply-high by the
rounded-up reciprocal, q = (n * m) >> 32 with m = floor((2^32 - 1) / d) + 1
(d = 1 passes n through).  The error term n (m d - 2^32) / 2^32 stays below
1 when n d < 2^32; here every case is enumerated."""

import numpy as np


def test_multiply_high_quotient_is_exact():
    n = np.arange(1 << 16, dtype=np.uint64)
    for d in range(2, 257):
        m = np.uint64((0xFFFFFFFF // d) + 1)
        q = (n * m) >> np.uint64(32)
        assert np.array_equal(q, n // np.uint64(d)), d

