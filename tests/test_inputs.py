"""The seeded input generator, host side (no GPU).

The vectorised numpy form is checked against a scalar big-integer form of the
published SplitMix64 definition, and the value map against its stated range.
"""
import numpy as np

import inputs


def scalar_value(seed, stream, idx):
    key = inputs.mix64_int(seed) ^ (stream << 60)
    w = inputs.mix64_int(key + (idx + 1) * inputs.GOLDEN)
    return (w >> 11) * 2.0 ** -53 - 0.5


def test_vector_matches_scalar_definition():
    for seed in (0, 1, 2202, 2 ** 63 + 5):
        idx = np.array([0, 1, 2, 1023, 1 << 33, (1 << 62) + 7], dtype=np.uint64)
        v = inputs.uniform(seed, 0, idx)
        for t, i in enumerate(idx):
            assert v[t] == scalar_value(seed, 0, int(i))
        v1 = inputs.uniform(seed, 1, idx)
        assert not np.array_equal(v, v1)


def test_splitmix_finaliser_known_structure():
    # mix64 is a bijection fixing 0; the first output of SplitMix64 seeded with 0
    # is mix64(golden gamma)
    assert inputs.mix64_int(0) == 0
    w = inputs.words(0, 0, np.array([0], dtype=np.uint64))
    key = inputs.stream_key(0, 0)
    assert int(w[0]) == inputs.mix64_int(key + inputs.GOLDEN)


def test_range_and_moments():
    a = inputs.matrix(2202, 512)
    assert a.min() >= -0.5 and a.max() < 0.5
    assert abs(a.mean()) < 5e-3
    assert abs(a.var() - 1.0 / 12.0) < 2e-3


def test_rows_and_shift_consistent():
    n = 100
    a = inputs.matrix(7, n, shift=float(n))
    rows = inputs.matrix_rows(7, n, [0, 13, 99], shift=float(n))
    assert np.array_equal(rows, a[[0, 13, 99]])
    plain = inputs.matrix(7, n)
    d = np.arange(n)
    assert np.array_equal(a[d, d], plain[d, d] + n)
    off = ~np.eye(n, dtype=bool)
    assert np.array_equal(a[off], plain[off])


def test_rhs_layout():
    b = inputs.rhs(3, 10, 4)
    assert b.shape == (10, 4)
    assert b[2, 3] == scalar_value(3, 1, 2 * 4 + 3)


def test_splitmix64_published_test_vector():
    # SplitMix64 (Steele, Lea & Flood 2014) started from state 1234567: the
    # first five outputs of the published reference generator.  word(idx) is
    # mix64(state + (idx + 1) * golden gamma), so this pins the gamma, both
    # multipliers and all three shifts.
    known = [6457827717110365317, 3203168211198807973, 9817491932198370423,
             4593380528125082431, 16408922859458223821]
    m = (1 << 64) - 1
    got = [inputs.mix64_int((1234567 + (i + 1) * inputs.GOLDEN) & m) for i in range(5)]
    assert got == known


def test_frozen_known_answers():
    # Frozen after the first run (seed 2202, the benchmark seed): the stream
    # key, the counter layout and the value map must never change, or every
    # stored expected value goes stale.
    w0 = [int(v) for v in inputs.words(2202, 0, np.arange(4, dtype=np.uint64))]
    assert w0 == [11679603653836149609, 2546826671173654124, 8944916027041204696,
                  8505917649281692741]
    w1 = [int(v) for v in inputs.words(2202, 1, np.arange(2, dtype=np.uint64))]
    assert w1 == [3395646559196411040, 4722259662302294198]
    a = inputs.matrix(2202, 4)
    assert a[0, 0] == (11679603653836149609 >> 11) * 2.0 ** -53 - 0.5
    assert a[0, 3] == (8505917649281692741 >> 11) * 2.0 ** -53 - 0.5
