"""Pins of the oracle's counter-based generator against numpy's independent
Philox4x64-10 implementation and against the statistics its derived draws must
have."""
import numpy as np
import pytest
from scipy import stats

from helpers import numpy_block


def test_philox_known_answer_zero(orc):
    # all-zero key and counter
    out = orc.philox4x64_10(0, 0, [0, 0, 0, 0])
    assert np.array_equal(out, numpy_block(0, 0, [0, 0, 0, 0]))


def test_philox_matches_numpy_random_keys_and_counters(orc):
    rng = np.random.default_rng(1234)
    for _ in range(300):
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.int64)]
        key[0] |= int(rng.integers(0, 2)) << 63
        ctr = [int(x) for x in rng.integers(0, 2**63, 4, dtype=np.int64)]
        ctr[0] = max(ctr[0], 1)
        assert np.array_equal(orc.philox4x64_10(key[0], key[1], ctr), numpy_block(key[0], key[1], ctr))


def test_u32_is_top_half_of_word0(orc):
    seed, tag, proj = 99, orc.TAG_DR_TGT, 3
    for c in [(0, 0, 0, 0), (7, 11, 13, 2), (123456, 1023, 42, 63)]:
        blk = numpy_block(seed, tag | (proj << 8), list(c))
        assert orc.u32(seed, tag, proj, *c) == int(blk[0]) >> 32


def test_threshold_edges(orc):
    assert orc.threshold(0.0) == 0
    assert orc.threshold(-1.0) == 0
    assert orc.threshold(1.0) == 1 << 32
    assert orc.threshold(1.225) == 1 << 32
    assert orc.threshold(0.5) == 1 << 31
    assert orc.threshold(0.25) == 1 << 30


def test_below_is_uniform(orc):
    n = 7
    counts = np.zeros(n)
    for a in range(14000):
        counts[orc.below(orc.u32(5, orc.TAG_DR_ROW, 0, 1, a, 0), n)] += 1
    chi2, p = stats.chisquare(counts)
    assert p > 1e-4
    assert orc.below(0, 1000) == 0
    assert orc.below(0xFFFFFFFF, 1000) == 999


def test_bernoulli_rate(orc):
    p = 0.1
    T = orc.threshold(p)
    hits = sum(orc.u32(3, orc.TAG_CONN, 0, 0, i, j) < T for i in range(100) for j in range(100))
    n = 10000
    assert abs(hits - n * p) < 4 * np.sqrt(n * p * (1 - p))


def test_normal_distribution(orc):
    x = np.array([orc.normal(11, orc.TAG_WINIT, 1, 0, i, j) for i in range(60) for j in range(60)])
    assert stats.kstest(x, "norm").pvalue > 1e-4
    assert abs(x.mean()) < 4 / np.sqrt(x.size)
