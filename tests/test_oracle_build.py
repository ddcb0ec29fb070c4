"""Pins of the oracle's network construction: fixed-probability rows, Gaussian
pairwise-Bernoulli rows on a torus, readout init and DEEP R bitfields."""
import numpy as np
import pytest
from scipy import stats

from helpers import bits_to_sets, rows_of
from test_oracle_rng import numpy_block


def build_fixed(orc, seed, n_pre, n_post, p, rec, proj_id=0, sigma=0.5):
    lens, mx = orc.fixed_prob_count(seed, n_pre, n_post, p, rec, proj_id)
    P = orc.Proj(n_pre, n_post, max(2 * mx, 1), rec, proj_id, bitfields=True)
    mx2 = orc.fixed_prob_rows(seed, P, p, sigma)
    assert mx2 == mx and np.array_equal(P.len, lens)
    return P


def test_fixed_prob_decisions_match_library_generator(orc):
    seed, p = 17, 0.1
    P = build_fixed(orc, seed, 20, 50, p, rec=True, proj_id=1)
    T = int(np.floor(p * 2**32))
    for i in range(20):
        expect = [j for j in range(50) if j != i and
                  (int(numpy_block(seed, orc.TAG_CONN | (1 << 8), [0, i, j, 0])[0]) >> 32) < T]
        assert rows_of(P)[i] == expect


def test_fixed_prob_statistics(orc):
    n_pre, n_post, p = 300, 400, 0.1
    P = build_fixed(orc, 3, n_pre, n_post, p, rec=False, sigma=0.25)
    lens = P.len.astype(float)
    # row lengths ~ Binomial(n_post, p)
    assert abs(lens.mean() - n_post * p) < 4 * np.sqrt(n_post * p * (1 - p) / n_pre)
    assert abs(lens.var() / (n_post * p * (1 - p)) - 1.0) < 0.25
    w = np.concatenate([P.w[i * P.cap:i * P.cap + int(P.len[i])] for i in range(n_pre)])
    assert stats.kstest(w / 0.25, "norm").pvalue > 1e-4
    # weights are stored at float32 precision
    assert np.array_equal(w, w.astype(np.float32).astype(np.float64))


def test_recurrent_rows_sorted_unique_no_autapse(orc):
    P = build_fixed(orc, 5, 64, 64, 0.3, rec=True)
    for i, r in enumerate(rows_of(P)):
        assert r == sorted(set(r))
        assert i not in r


def brute_d2(L, i, j):
    xi, yi, xj, yj = i % L, i // L, j % L, j // L
    return min((xi - xj + sx * L) ** 2 + (yi - yj + sy * L) ** 2
               for sx in (-1, 0, 1) for sy in (-1, 0, 1))


def test_torus_distance_brute_force(orc):
    for L in (3, 4, 7, 8):
        for i in range(L * L):
            for j in range(L * L):
                assert orc.torus_d2(L, i, j) == brute_d2(L, i, j)


def test_gauss_rows_expected_degree(orc):
    # topographic map at scale s=4: the expected in/out degree is the sum of
    # connection probabilities over the torus, about 2 pi p sigma^2.
    L, p_form, sigma = 64, 0.16, 2.5
    lens, mx = orc.gauss_count(21, L, p_form, sigma, proj_id=0)
    expect = sum(p_form * np.exp(-brute_d2(L, 0, j) / (2 * sigma ** 2)) for j in range(L * L))
    assert abs(expect - 2 * np.pi * p_form * sigma ** 2) < 0.01
    assert abs(lens.mean() - expect) < 4 * np.sqrt(expect / lens.size)
    P = orc.Proj(L * L, L * L, 32, False, 0)
    orc.gauss_rows(21, P, L, p_form, sigma, 0.2)
    assert np.array_equal(P.len, np.minimum(lens, 32))
    r = rows_of(P)
    assert all(rr == sorted(set(rr)) for rr in r)
    assert all(P.w[i * 32 + k] == np.float32(0.2) for i in range(L * L) for k in range(int(P.len[i])))


def test_gauss_rows_distance_profile(orc):
    # connection frequency by distance follows p_form exp(-d^2 / 2 sigma^2)
    L, p_form, sigma = 32, 1.0, 1.0
    P = orc.Proj(L * L, L * L, 64, False, 2)
    orc.gauss_rows(8, P, L, p_form, sigma, 0.1)
    hit = {}
    tot = {}
    conn = [set(r) for r in rows_of(P)]
    for i in range(0, L * L, 7):
        for j in range(L * L):
            d2 = brute_d2(L, i, j)
            if d2 > 4:
                continue
            tot[d2] = tot.get(d2, 0) + 1
            hit[d2] = hit.get(d2, 0) + (j in conn[i])
    for d2, n in tot.items():
        p = p_form * np.exp(-d2 / (2 * sigma ** 2))
        assert abs(hit[d2] - n * p) <= 4 * np.sqrt(n * p * (1 - p)) + 1e-9


def test_dense_init(orc):
    W = orc.dense_init(4, 2, 20, 300, 0.1)
    assert W.shape == (20, 300)
    assert stats.kstest(W.ravel() / 0.1, "norm").pvalue > 1e-4


def test_deepr_init_bits(orc):
    P = build_fixed(orc, 9, 40, 70, 0.2, rec=True, sigma=1.0)
    orc.deepr_init_bits(9, P)
    conn = bits_to_sets(P.conn, 40, 70)
    sign = bits_to_sets(P.sign, 40, 70)
    rows = rows_of(P)
    n_free_neg = n_free = 0
    for i in range(40):
        assert conn[i] == set(rows[i])
        for k, j in enumerate(rows[i]):
            assert (j in sign[i]) == (P.w[i * P.cap + k] < 0)
        for j in range(70):
            if j not in conn[i]:
                n_free += 1
                n_free_neg += j in sign[i]
    # signs of potential (absent) connections are fair coin flips
    assert abs(n_free_neg - n_free / 2) < 4 * np.sqrt(n_free / 4)
