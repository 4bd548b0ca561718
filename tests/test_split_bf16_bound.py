"""The error bound behind the split-BF16 tolerances, checked in plain numpy (no GPU, no
library code): an FP32 value v = hi + lo with hi = bf16(v) and lo = bf16(v - hi), both
rounded to nearest even, leaves |v - hi - lo| <= 2^-17 |v| (the first rounding leaves at
most 2^-8 |v|, strictly less but for ties, so the remainder's own rounding error is at
most 2^-17 |v|); a product a x formed as hi_a hi_x + hi_a lo_x + lo_a hi_x (lo_a lo_x,
at most 2^-16 |a x|, dropped) is within 2^-15 |a| |x| of the exact one to first order,
the per-product bound the GPU parity tests build on."""
import numpy as np


def _bf16_rne(v):
    """float32 -> the nearest bfloat16 value (ties to even), returned as float32."""
    u = np.asarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32)


def _split(v):
    hi = _bf16_rne(v)
    lo = _bf16_rne(v.astype(np.float32) - hi)  # v - hi is exact in FP32
    return hi, lo


def _samples(rng, n):
    # mantissas over the whole range of bit patterns, exponents over +-30 binades
    m = rng.uniform(1.0, 2.0, n) * rng.choice([-1.0, 1.0], n)
    return (m * 2.0 ** rng.integers(-30, 31, n)).astype(np.float32)


def test_rounding_helper_matches_known_values():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1) wins; 1 + 3 2^-8 rounds up
    v = np.array([1.0, 1.0 + 2.0**-8, 1.0 + 3 * 2.0**-8, -2.5, 1.0 + 2.0**-9], np.float32)
    assert np.array_equal(_bf16_rne(v), np.array([1.0, 1.0, 1.0 + 2.0**-6, -2.5, 1.0], np.float32))


def test_two_term_split_is_within_2_pow_minus_17():
    rng = np.random.default_rng(7)
    v = _samples(rng, 200000)
    hi, lo = _split(v)
    err = np.abs(v.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    assert np.all(err <= 2.0**-17 * np.abs(v.astype(np.float64)))
    # and it is nearly attained (within a factor of two)
    assert np.max(err / np.abs(v.astype(np.float64))) > 2.0**-18


def test_three_product_form_is_within_2_pow_minus_15():
    rng = np.random.default_rng(8)
    a = _samples(rng, 200000)
    x = _samples(rng, 200000)
    ha, la = _split(a)
    hx, lx = _split(x)
    f = lambda t: t.astype(np.float64)  # noqa: E731
    approx = f(ha) * f(hx) + f(ha) * f(lx) + f(la) * f(hx)
    exact = f(a) * f(x)
    rel = np.abs(approx - exact) / np.abs(exact)
    assert np.all(rel <= 2.0**-15 * (1 + 2.0**-7))
    assert np.max(rel) > 2.0**-16  # the worst cases come within a factor of two
    # dropping a cross term instead breaks it: hi_a hi_x + hi_a lo_x alone is ~2^-9 off
    two = f(ha) * f(hx) + f(ha) * f(lx)
    assert np.max(np.abs(two - exact) / np.abs(exact)) > 2.0**-12
