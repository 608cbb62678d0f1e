"""Error bounds of the split-BF16 product forms, emulated on the host.

The BF16X6 form (and the adjoint's 64- and 128-label FP32 tiles) write every
FP32 operand as three bfloat16 parts a = a0 + a1 + a2, each part the
round-to-nearest-even bfloat16 of what the previous ones left, and keep the six
products a_i b_j with i + j <= 2; the BF16X3 form keeps two parts and the three
products with i + j <= 1.  With u = 2^-8 the bfloat16 unit roundoff,
|a1| <= u |a|, and the remainder after two parts is at most 2^-17 |a|; after
three parts it is zero (an FP32 significand has 24 bits, each part takes 8).
So the six products drop a1 b2 + a2 b1 + a2 b2 <= (2^-25 + 2^-25 + 2^-34) |a b|,
about 2^-24 (FP32-level), and the three drop a1 b1 plus the two remainders'
products, <= (2^-16 + 2^-17 + 2^-17) |a b| = 2^-15 |a b|.  These tests check
the statements on random normal FP32 values over a wide exponent range, with
bfloat16 rounding emulated on the FP32 bit patterns and the products summed
exactly in FP64 (a product of two bfloat16 values is exact in FP32 and FP64).
"""
import numpy as np


def _bf16(x):
    """Round-to-nearest-even FP32 -> bfloat16, returned as FP32."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def _split(a, parts):
    out, rest = [], a.astype(np.float32)
    for _ in range(parts):
        p = _bf16(rest)
        out.append(p)
        rest = (rest - p).astype(np.float32)   # exact in FP32
    return out


def _operands(n, seed):
    rng = np.random.default_rng(seed)
    mant = rng.uniform(1.0, 2.0, size=(2, n))
    sign = rng.choice([-1.0, 1.0], size=(2, n))
    expo = rng.integers(-60, 60, size=(2, n))
    v = (sign * mant * np.ldexp(1.0, expo)).astype(np.float32)
    return v[0], v[1]


def _split_product(a, b, parts, pairs):
    pa, pb = _split(a, parts), _split(b, parts)
    return sum(pa[i].astype(np.float64) * pb[j].astype(np.float64) for i, j in pairs)


def test_remainders_and_parts():
    a, _ = _operands(200_000, 1)
    p = _split(a, 3)
    a64 = a.astype(np.float64)
    # three parts represent a exactly; two leave at most 2^-17 |a|
    assert np.all(a64 - (p[0].astype(np.float64) + p[1] + p[2]) == 0.0)
    two = np.abs(a64 - (p[0].astype(np.float64) + p[1])) / np.abs(a64)
    assert two.max() <= np.ldexp(1.0, -17)
    assert two.max() > np.ldexp(1.0, -18)   # the bound is reached, not 2^-18
    assert np.all(np.abs(p[1]) <= np.ldexp(1.0, -8) * np.abs(a64))


def test_six_products_within_fp32_level():
    a, b = _operands(200_000, 2)
    exact = a.astype(np.float64) * b.astype(np.float64)
    six = _split_product(a, b, 3, [(0, 2), (2, 0), (1, 1), (0, 1), (1, 0), (0, 0)])
    rel = np.abs(six - exact) / np.abs(exact)
    assert rel.max() <= np.ldexp(1.0, -24) * (1 + 2.0 ** -9), rel.max()


def test_three_products_within_stated_bound():
    a, b = _operands(200_000, 3)
    exact = a.astype(np.float64) * b.astype(np.float64)
    three = _split_product(a, b, 2, [(0, 1), (1, 0), (0, 0)])
    rel = np.abs(three - exact) / np.abs(exact)
    assert rel.max() <= np.ldexp(1.0, -15), rel.max()
    # the bound is nearly reached (about 6.8 * 2^-18 here), far above FP32 level
    assert rel.max() > 4 * np.ldexp(1.0, -18)


def test_bf16_rounding_is_nearest_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even 1.0;
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties go to 1 + 2^-6
    x = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20], dtype=np.float32)
    assert list(_bf16(x)) == [1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7]
