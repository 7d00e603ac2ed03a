"""The vote's integer average (Σ + floor(k/2)) / k is computed on the GPU as
trunc((n + 1/2) * rk) in float32 with rk the hardware reciprocal of k (within
one ulp of 1/k).  This checks that identity exhaustively for every numerator
the vote can produce (n < 2^16: at most 225 votes of 255 plus 112) and every
vote count k = 1..225, for each of the three float32 values nearest 1/k,
and for the fused form fma(n, rk, rk / 2) the kernel uses: it rounds the
same exact product (n + 1/2) * rk once, so it must give the same floats."""
import numpy as np


def test_float_reciprocal_division_is_exact():
    n = np.arange(0, 1 << 16, dtype=np.int64)
    nf = n.astype(np.float32) + np.float32(0.5)
    for k in range(1, 226):
        r = np.float32(1.0) / np.float32(k)
        for rk in (r, np.nextafter(r, np.float32(0)), np.nextafter(r, np.float32(1))):
            prod = (nf * rk).astype(np.float32)
            q = np.floor(prod).astype(np.int64)
            assert np.array_equal(q, n // k), (k, rk)
            # fma: the exact n * rk + rk / 2 fits a double (42 bits), then one rounding
            r64 = np.float64(rk)
            fused = (n.astype(np.float64) * r64 + r64 * 0.5).astype(np.float32)
            assert np.array_equal(fused, prod), (k, rk)
