"""The running minimum of the grouped sweep keeps, per row, one FP64 word:
the FP32 candidate's bits with the sign cleared in the high half and
(visit position + 1) << 16 | u in the low half, updated with v_min_f64.
These CPU checks pin the ordering argument the kernel relies on, on the same
word construction done with numpy: for non-negative values the FP64 order of
the words is the value order, then the visit order (the first minimum a
strict < keeps); NaN of either sign ends above +inf; J_inf with position 0
beats a later J_inf candidate and loses to anything below it."""
import numpy as np

J_INF = np.float32(1.0e4)


def word(value, pos, u):
    hi = np.asarray(value, dtype=np.float32).view(np.uint32) & np.uint32(0x7FFFFFFF)
    lo = np.uint32((pos << 16) | u) if pos >= 0 else np.uint32(0)
    return ((np.uint64(hi) << np.uint64(32)) | np.uint64(lo)).view(np.float64)


def first_min(values):
    """Strict < from J_inf: (value, index) of the first minimum, or (J_inf, -1)."""
    best, arg = J_INF, -1
    for q, v in enumerate(values):
        if v < best:
            best, arg = v, q
    return best, arg


def word_min(values, us):
    best = word(J_INF, -1, 0)
    for q, v in enumerate(values):
        w = word(v, q + 1, us[q])
        # IEEE minimum of two non-NaN doubles (the words are never NaN: the
        # cleared sign keeps the exponent field of a float NaN below 0x7FF
        # unless its top mantissa bits are set, checked below)
        best = w if w < best else best
    hi = int(np.asarray(best).view(np.uint64)) >> 32
    lo = int(np.asarray(best).view(np.uint64)) & 0xFFFFFFFF
    return np.uint32(hi).view(np.float32), (lo & 0xFFFF) if lo else -1


def test_word_order_is_value_then_visit_order():
    rng = np.random.default_rng(5)
    for trial in range(400):
        n = int(rng.integers(1, 40))
        vals = rng.choice(np.float32([0.0, 1.5, 2.0, 7.25, 100.0, 9999.0, J_INF, np.inf, 2.5e4]), n)
        vals = vals + rng.choice(np.float32([0.0, 0.0, 1e-3]), n).astype(np.float32)
        vals = vals.astype(np.float32)
        if trial % 3 == 0:
            vals[rng.integers(0, n)] = np.float32(np.nan)
        us = rng.permutation(32767)[:n]
        bv, bq = first_min(vals)
        wv, wu = word_min(vals, us)
        assert wv == bv or (np.isnan(wv) and np.isnan(bv))
        assert wu == (us[bq] if bq >= 0 else -1)


def test_nan_of_either_sign_sorts_above_inf():
    """The kernel's NaN candidates carry the quiet-NaN pattern of its weights
    (0x7fc00000) or the hardware's default NaN (sign either way, top mantissa
    bits 100): with the sign cleared their words are finite FP64 values above
    the word of +inf, so they never win.  (A float NaN whose top three
    mantissa bits are 111 would give an FP64 NaN word; none is produced.)"""
    for bits in (0x7FC00000, 0xFFC00000, 0x7F800001, 0xFFA00000, 0x7FCAFE00):
        nan = np.uint32(bits).view(np.float32)
        w = word(nan, 1, 0)
        assert np.isfinite(w) and w > word(np.float32(np.inf), 7, 0x7FFF)


def test_jinf_ties_keep_no_control():
    assert first_min([J_INF, J_INF]) == (J_INF, -1)
    assert word_min([J_INF, J_INF], [3, 4]) == (J_INF, -1)
    v, u = word_min([J_INF, np.float32(9999.0)], [3, 4])
    assert v == np.float32(9999.0) and u == 4
