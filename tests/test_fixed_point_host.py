"""Host-side checks of the arithmetic the spreading kernel relies on.

The adjoint's spreading accumulates each contribution c = round(w * y) as a
packed 64-bit integer c_re + 2^32 c_im (mod 2^64), where the rounding is one
fused multiply-add: fma(w, y, 1.5 * 2^23) in float32 leaves 0x4B400000 + c in
the bits of the result when |w * y| < 2^22, and the two words' offsets are
removed by subtracting 0x4B4000004B400000. These tests emulate that in numpy
(a float32 fma is the exact product rounded once, which float64 holds exactly
for float32 operands) and check it against the plain definitions: round half
to even, exact integer sums, and the decode of the packed sum.
"""
import numpy as np

MAGIC = np.float32(12582912.0)        # 1.5 * 2^23
BIAS = 0x4B4000004B400000


def fma32(a, b, c):
    """float32 fma, emulated: the product of two float32 values is exact in
    float64; adding the offset there rounds only bits 29 places below the
    integer position, so rounding the float64 sum to float32 gives the fma's
    single rounding (the two could differ only on a float64 tie, which these
    inputs do not produce)."""
    return (a.astype(np.float64) * b.astype(np.float64) + np.float64(c)).astype(np.float32)


def packed_word(w, yr, yi):
    tr = fma32(w, yr, MAGIC).view(np.uint32).astype(np.uint64)
    ti = fma32(w, yi, MAGIC).view(np.uint32).astype(np.uint64)
    return ((ti << np.uint64(32)) | tr) - np.uint64(BIAS)      # wraps mod 2^64 like the GPU


def decode(word):
    """S_re = low word as int32, S_im = (word - S_re) >> 32 as int32."""
    sre = (word & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.int32).astype(np.int64)
    sim = ((word - sre.astype(np.uint64)) >> np.uint64(32)).astype(np.uint32).view(np.int32).astype(np.int64)
    return sre, sim


def test_fma_rounding_is_round_half_even():
    rng = np.random.default_rng(0)
    w = rng.uniform(0, 1, 200_000).astype(np.float32)
    y = (rng.uniform(-1, 1, 200_000) * 2.0 ** 21).astype(np.float32)      # |w y| < 2^21
    bits = fma32(w, y, MAGIC).view(np.uint32).astype(np.int64)
    c = bits - 0x4B400000
    exact = w.astype(np.float64) * y.astype(np.float64)
    assert np.array_equal(c, np.rint(exact).astype(np.int64))             # rint: half to even


def test_fma_rounding_ties_and_edges():
    # exact ties round to even; the extremes of the range stay exact
    w = np.ones(8, np.float32)
    y = np.array([0.5, 1.5, 2.5, -0.5, -1.5, 2.0 ** 21, -(2.0 ** 21), 0.0], np.float32)
    c = fma32(w, y, MAGIC).view(np.uint32).astype(np.int64) - 0x4B400000
    assert c.tolist() == [0, 2, 2, 0, -2, 2 ** 21, -(2 ** 21), 0]


def test_packed_sums_decode_exactly():
    # up to 512 contributions with |c| <= 2^21 per component, added in any order
    rng = np.random.default_rng(1)
    for count in (1, 7, 512):
        w = rng.uniform(0, 1, count).astype(np.float32)
        yr = (rng.uniform(-1, 1, count) * 2.0 ** 21).astype(np.float32)
        yi = (rng.uniform(-1, 1, count) * 2.0 ** 21).astype(np.float32)
        words = packed_word(w, yr, yi)
        with np.errstate(over="ignore"):
            total = np.uint64(0)
            for wd in words[rng.permutation(count)]:
                total = total + wd                               # mod 2^64
        sre, sim = decode(np.array([total], np.uint64))
        cre = np.rint(w.astype(np.float64) * yr).astype(np.int64)
        cim = np.rint(w.astype(np.float64) * yi).astype(np.int64)
        assert sre[0] == cre.sum() and sim[0] == cim.sum()
        assert abs(cre.sum()) < 2 ** 31 and abs(cim.sum()) < 2 ** 31


def test_scale_bound_keeps_sums_in_range():
    # the kernel picks s with m * 2^s < 2^21 (m = largest |Y wy| of the item);
    # with |wx| <= 1 every |c| <= 2^21, so 512 of them stay below 2^30
    rng = np.random.default_rng(2)
    m = np.float32(rng.uniform(1e-3, 1e3))
    _, e = np.frexp(m)                                             # m < 2^e
    s = 21 - int(e)
    assert m * 2.0 ** s < 2.0 ** 21
    assert 512 * 2 ** 21 <= 2 ** 30
