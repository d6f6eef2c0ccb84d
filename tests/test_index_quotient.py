"""The ring FFT kernels take index quotients floor(x / d), d workgroup-uniform,
as trunc(fma(x, r, r / 2)) with r the hardware reciprocal of d (correct to
1 ulp), claimed exact for 0 <= x < 2^20.  Emulated here in float32 with r
moved one ulp either way: exhaustive for x < 2^17 and d <= 2048 (every
divisor of the kernels' index arithmetic at the sizes the tests run), and a
random sample up to x < 2^20, d < 2^16."""
import numpy as np


def quotient(x, r):
    # x * r + r/2 formed exactly in float64 (float32 operands), then one
    # rounding to float32: a fused multiply-add
    xf = x.astype(np.float32).astype(np.float64)
    rr = np.float64(np.float32(r)) if np.isscalar(r) else r.astype(np.float64)
    h = (np.float32(0.5) * np.float32(r)) if np.isscalar(r) else (np.float32(0.5) * r).astype(np.float64)
    return (xf * rr + h).astype(np.float32).astype(np.int64)


def reciprocals(d):
    r0 = np.float32(1.0) / np.float32(d)
    return (np.nextafter(r0, np.float32(0)), r0, np.nextafter(r0, np.float32(2)))


def test_exhaustive_small():
    x = np.arange(1 << 17, dtype=np.int64)
    for d in range(1, 2049):
        want = x // d
        for r in reciprocals(d):
            assert np.array_equal(quotient(x, r), want), d


def test_sampled_to_2_20():
    rng = np.random.default_rng(7)
    x = rng.integers(0, 1 << 20, 1 << 21)
    d = rng.integers(1, 1 << 16, 1 << 21)
    r0 = np.float32(1.0) / d.astype(np.float32)
    for r in (np.nextafter(r0, np.float32(0)), r0, np.nextafter(r0, np.float32(2))):
        q = quotient(x, r.astype(np.float32))
        assert np.array_equal(q, x // d)


def test_plain_reciprocal_product_is_not_exact():
    """Without the half-step offset the truncated product undershoots exact
    multiples (x = q d), which is why the offset is there."""
    x = np.arange(1, 1 << 16, dtype=np.int64)
    bad = 0
    for d in (3, 5, 7, 11, 13, 49, 97, 1021):
        r = np.float32(1.0) / np.float32(d)
        q = (x.astype(np.float32) * r).astype(np.int64)
        bad += int(np.count_nonzero(q != x // d))
    assert bad > 0
