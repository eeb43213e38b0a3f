"""The decode search's float form of the round decision (Sec. III-A search).

The bracketed decode search's candidate rounds carry the boundary as the
binary32 value b = lo_sym + mid - 1/2 and decide with the float test
y < s1 - b, s1 = slot + 1 + lo_sym - 1/2. For y = RN(F (M - N)) >= 0 that
test is the contract's decision slot >= c_mid = mid + floor(y) (pinned
here); the candidate rounds feed it an approximate y, and the exact
confirmation that follows makes the decoded symbol independent of it.
This replays the arithmetic in numpy binary32 over the ranges the library
accepts
(|lo_sym| <= 2^22, N <= 2^15, slot < M <= 2^16):
- every boundary, s1 and s1 - b is exact;
- the float test and the integer decision agree, y at, just below and just
  above integers included.
"""
import numpy as np

f32 = np.float32


def test_boundaries_and_differences_are_exact():
    rng = np.random.default_rng(7)
    n = 1 << 20
    lo_sym = rng.integers(-(1 << 22), (1 << 22) + 1, size=n)
    lo_sym[:4] = [-(1 << 22), 1 << 22, 0, -1]
    mid = rng.integers(0, 1 << 15, size=n)
    slot = rng.integers(0, 1 << 16, size=n)
    lo_mh = (lo_sym.astype(f32) - f32(0.5)).astype(f32)
    assert np.all(lo_mh.astype(np.float64) == lo_sym - 0.5)
    b = (mid.astype(f32) + lo_mh).astype(f32)
    s1 = ((slot + 1).astype(f32) + lo_mh).astype(f32)
    assert np.all(b.astype(np.float64) == lo_sym + mid - 0.5)
    assert np.all(s1.astype(np.float64) == lo_sym + slot + 0.5)
    k1 = (s1 - b).astype(f32)
    assert np.all(k1.astype(np.int64) == slot + 1 - mid)
    # the next boundary from the current one: b + 2^r, exact
    for r in range(0, 15):
        nb = (b + f32(1 << r)).astype(f32)
        assert np.all(nb.astype(np.float64) == lo_sym + mid + (1 << r) - 0.5)


def test_float_test_matches_integer_decision():
    rng = np.random.default_rng(11)
    span = (1 << 16) - 511
    ints = rng.integers(0, span, size=1 << 18).astype(f32)
    y = np.concatenate([
        ints,
        np.nextafter(ints, f32(-1)),          # just below an integer
        np.nextafter(ints, f32(np.inf)),      # just above
        (rng.random(1 << 18) * span).astype(f32),
        np.array([0.0, span], dtype=f32),
    ]).astype(f32)
    y = np.maximum(y, f32(0))
    fl = np.floor(y.astype(np.float64)).astype(np.int64)
    for shift in (-2, -1, 0, 1, 2):
        k = fl + shift  # slot - mid near the decision point
        k1 = (k + 1).astype(f32)  # exact: |k + 1| < 2^17
        float_test = y < k1
        int_decision = k >= fl
        assert np.array_equal(float_test, int_decision), shift
    # slot - mid far below and above
    for k in (-1100, -1, span, 1 << 16):
        assert np.array_equal(y < f32(k + 1), k >= fl)
