"""CPU: the three-term BF16 split that the BF16-storage contraction feeds to
the BF16 matrix-core instruction.

The kernel cuts each FP32 value w of WH by truncation: hi = w with its low
16 bits cleared, mid = (w - hi) likewise, lo = w - hi - mid, every
subtraction in FP32.  Its products with the stored BF16 fibre values are
exact in FP32 only if every term is a BF16 number, and the contraction
equals the FP32 one (up to the order of the FP32 sums) only if
hi + mid + lo == w exactly.  These pins check both on FP32 values over the
whole normal exponent range, with both signs, and on the shapes WH takes
(products of factor entries and a weight)."""

import numpy as np


def split3(w):
    w = np.asarray(w, dtype=np.float32)
    hi = (w.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)
    r1 = (w - hi).astype(np.float32)
    mid = (r1.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)
    lo = (r1 - mid).astype(np.float32)
    return hi, mid, lo


def is_bf16(x):
    return np.all((np.asarray(x, dtype=np.float32).view(np.uint32) & np.uint32(0xFFFF)) == 0)


def test_split_is_exact_over_the_exponent_range():
    rng = np.random.default_rng(7)
    mant = rng.uniform(1.0, 2.0, 200_000)
    expo = rng.integers(-100, 100, mant.size)
    sign = rng.choice([-1.0, 1.0], mant.size)
    w = (sign * mant * np.exp2(expo)).astype(np.float32)
    hi, mid, lo = split3(w)
    assert is_bf16(hi) and is_bf16(mid) and is_bf16(lo)
    total = hi.astype(np.float64) + mid.astype(np.float64) + lo.astype(np.float64)
    assert np.array_equal(total, w.astype(np.float64))


def test_split_of_weighted_krp_rows():
    # WH(f, r) = w_f * prod_k A^(k)(i_k, r): FP32 products of O(1) entries
    # and a weight 1 / (B p_f)
    rng = np.random.default_rng(11)
    a = rng.standard_normal((3, 4096, 32)).astype(np.float32)
    wf = (1.0 / (128 * rng.uniform(1e-7, 1e-3, 4096))).astype(np.float32)
    wh = (wf[:, None] * a[0] * a[1] * a[2]).astype(np.float32)
    hi, mid, lo = split3(wh)
    assert is_bf16(hi) and is_bf16(mid) and is_bf16(lo)
    assert np.array_equal(hi.astype(np.float64) + mid + lo, wh.astype(np.float64))
    # each product with a BF16 value is exact in FP32 (8 x 8 significant bits)
    x = (rng.standard_normal(4096).astype(np.float32).view(np.uint32)
         & np.uint32(0xFFFF0000)).view(np.float32)
    for part in (hi, mid, lo):
        p32 = (part[:, 0] * x).astype(np.float32)
        assert np.array_equal(p32.astype(np.float64), part[:, 0].astype(np.float64) * x)


def test_two_terms_are_not_enough():
    # why the kernel takes three terms: hi + mid alone leaves up to 8 bits
    # (here 1 + 2^-8 + 2^-23 spans 24 significant bits)
    w = np.float32(1.0 + 2.0 ** -8 + 2.0 ** -23)
    hi, mid, lo = split3(np.array([w]))
    assert lo[0] != 0.0
    assert hi[0] + mid[0] != w
