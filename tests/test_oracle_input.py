"""Pins of the oracle's Poisson input source: each spike decision against
numpy's independent Philox4x64-10, the thresholds of a Poisson step in closed
form, and the statistics a Bernoulli(rate*dt) train must have."""
import numpy as np
from scipy import stats

from helpers import numpy_block


def test_rate_thresholds_closed_form(orc):
    thr = orc.rate_thresholds([0.0, 50.0, 250.0, 500.0, 1000.0, 2500.0, -3.0], dt_ms=1.0)
    # floor(p 2^32) with p = rate * dt: 0.05 * 2^32 = 214748364.8
    assert list(thr) == [0, 214748364, 1 << 30, 1 << 31, 1 << 32, 1 << 32, 0]
    # dt enters linearly: 10 Hz at 0.1 ms is p = 1e-3
    assert orc.rate_thresholds([10.0], dt_ms=0.1)[0] == int(np.floor(1e-3 * 2.0**32))


def test_decisions_match_independent_philox(orc):
    seed, B, n_in = 77, 3, 40
    rates = np.linspace(0.0, 900.0, n_in)
    thr = orc.rate_thresholds(rates)
    key1 = orc.TAG_INPUT
    for step in [0, 1, 17, 123456]:
        idx, off = orc.poisson_input(seed, step, B, thr)
        for b in range(B):
            want = [i for i in range(n_in)
                    if (int(numpy_block(seed, key1, [step, b, i, 0])[0]) >> 32) < int(thr[i])]
            assert list(idx[off[b]:off[b + 1]]) == want


def test_edge_rates_and_lists(orc):
    B, n_in = 4, 33
    thr = orc.rate_thresholds(np.r_[np.zeros(11), np.full(11, 1000.0), np.full(11, 20.0)])
    for step in range(5):
        idx, off = orc.poisson_input(5, step, B, thr)
        assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == idx.size
        for b in range(B):
            lst = idx[off[b]:off[b + 1]]
            assert np.all(np.diff(lst) > 0)           # ascending, no repeats
            assert not np.any(lst < 11)               # rate 0 never fires
            assert np.all(np.isin(np.arange(11, 22), lst))  # p = 1 fires every step


def test_per_instance_table(orc):
    n_in = 20
    thr = orc.rate_thresholds(np.array([np.zeros(n_in), np.full(n_in, 1000.0)]))
    idx, off = orc.poisson_input(3, 9, 2, thr)
    assert off[1] == 0 and list(idx[off[1]:off[2]]) == list(range(n_in))


def test_rates_are_bernoulli(orc):
    # 60 channels x 2 instances x 2000 steps: per-channel counts are
    # Binomial(T, p); the summed chi-square over channels is chi2(n_ch) distributed
    n_in, B, T = 60, 2, 2000
    rates = np.linspace(5.0, 120.0, n_in)
    thr = orc.rate_thresholds(rates)
    counts = np.zeros((B, n_in))
    trains = np.zeros((B, T, n_in), bool)
    for t in range(T):
        idx, off = orc.poisson_input(11, t, B, thr)
        for b in range(B):
            trains[b, t, idx[off[b]:off[b + 1]]] = True
    counts = trains.sum(axis=1)
    p = rates * 1e-3
    chi2 = (((counts - T * p) ** 2) / (T * p * (1 - p))).sum()
    assert stats.chi2.sf(chi2, B * n_in) > 1e-4
    # instances and consecutive steps are uncorrelated: the mean product of
    # standardised residuals is N(0, 1/n) for independent trains
    r = (trains - p) / np.sqrt(p * (1 - p))
    for x, y in [(r[0], r[1]), (r[0, 1:], r[0, :-1]), (r[1, 1:], r[1, :-1])]:
        assert abs((x * y).mean()) < 5 / np.sqrt(x.size)
