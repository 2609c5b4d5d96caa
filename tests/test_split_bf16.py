"""The arithmetic behind the split-bfloat16 range-compression GEMM, on the CPU.

A float32 x splits into three bfloat16 parts x1 = rne(x), x2 = rne(x - x1),
x3 = rne(x - x1 - x2) (rne: round to nearest even at 8 significant bits).  Pinned
here against float64, independently of the library: each remainder is exact in
float32, the three parts reproduce x to 2^-27 of |x|, every partial product
ai * bj is exact in float32, and the six products with i + j <= 4 sum to a b
within 2^-23 of |a b| (the three left out are below 2^-26 of it; float32 rounding
of the partial sums adds at most a few units of 2^-24), for operands whose
products and parts stay in float32's normal range (echo samples and DFT weights
are many orders of magnitude inside it)."""
import numpy as np


def _rne_bf16(x):
    """bfloat16 rounding (nearest even) of float32 values, returned as float32."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _split3(x):
    x = np.asarray(x, np.float32)
    x1 = _rne_bf16(x)
    r1 = (x - x1).astype(np.float32)
    x2 = _rne_bf16(r1)
    r2 = (r1 - x2).astype(np.float32)
    return x1, x2, _rne_bf16(r2), r1, r2


def _sample(n, seed):
    rng = np.random.default_rng(seed)
    mant = rng.uniform(-1.0, 1.0, n)
    expo = rng.integers(-30, 30, n)  # products and their parts stay in float32's normal range
    return (mant * np.exp2(expo)).astype(np.float32)


def test_parts_have_eight_bits_and_remainders_are_exact():
    x = _sample(200000, 1)
    x1, x2, x3, r1, r2 = _split3(x)
    for p in (x1, x2, x3):
        assert np.all((p.view(np.uint32) & 0xFFFF) == 0)  # a bfloat16 value
    xd = x.astype(np.float64)
    assert np.array_equal(r1.astype(np.float64), xd - x1.astype(np.float64))
    assert np.array_equal(r2.astype(np.float64), r1.astype(np.float64) - x2.astype(np.float64))
    err = np.abs(xd - x1.astype(np.float64) - x2.astype(np.float64) - x3.astype(np.float64))
    assert np.all(err <= np.exp2(-27) * np.abs(xd))


def test_six_partial_products_give_float32_accuracy():
    a, b = _sample(200000, 2), _sample(200000, 3)
    pa, pb = _split3(a)[:3], _split3(b)[:3]
    terms = [(i, j) for i in range(3) for j in range(3) if i + j <= 2]
    assert len(terms) == 6
    exact = a.astype(np.float64) * b.astype(np.float64)
    acc = np.zeros_like(a)
    # smallest products first, accumulated in float32 as the MFMA does
    for i, j in sorted(terms, key=lambda t: -(t[0] + t[1])):
        p = pa[i].astype(np.float64) * pb[j].astype(np.float64)
        assert np.array_equal(p, (pa[i] * pb[j]).astype(np.float64))  # exact in float32
        acc = (acc + (pa[i] * pb[j])).astype(np.float32)
    rel = np.abs(acc.astype(np.float64) - exact) / np.abs(exact)
    assert rel.max() <= np.exp2(-23)
    # a single float32 product rounds to 2^-24 of itself: the same order
    f32 = np.abs((a * b).astype(np.float64) - exact) / np.abs(exact)
    assert rel.max() <= 4 * f32.max()


def test_dropping_a_needed_term_is_caught():
    """With five products (x2 y2 left out) the error reaches ~2^-18: the bound
    above would fail, so the test discriminates the six-product rule."""
    a, b = _sample(20000, 4), _sample(20000, 5)
    pa, pb = _split3(a)[:3], _split3(b)[:3]
    acc = np.zeros_like(a)
    for i, j in ((2, 0), (0, 2), (1, 0), (0, 1), (0, 0)):
        acc = (acc + pa[i] * pb[j]).astype(np.float32)
    exact = a.astype(np.float64) * b.astype(np.float64)
    assert (np.abs(acc.astype(np.float64) - exact) / np.abs(exact)).max() > np.exp2(-23)
