"""Pins of the oracle's DEEP R rewiring (paper Sec. 2.1.2, Fig. 2): the
removal rule of ragged rows, the closed-form elimination set, the invariants
of formation and the uniformity of its random choices."""
import itertools

import numpy as np
import pytest
from scipy import stats

from helpers import bits_to_sets, canonical_compaction, rows_of, sequential_remove, set_rows


def test_canonical_compaction_equals_sequential_exhaustive():
    # the closed-form pairing of holes and tail survivors used by the parallel
    # kernels equals sequential swap-with-last removal with re-check
    for n in range(0, 13):
        for mask in itertools.product((0, 1), repeat=n):
            assert canonical_compaction(n, list(mask)) == sequential_remove(n, list(mask))


def one_row(orc, n, mask, B=3):
    P = orc.Proj(1, 16, 16, False, 0, batch=B, trained=True, traces="alif", bitfields=True)
    tg = list(range(n))
    set_rows(P, [tg], [[0.1 * (s + 1) for s in range(n)]])
    orc.deepr_init_bits(0, P)  # all sign bits positive now (weights > 0)
    for s in range(n):
        if mask[s]:
            P.w[s] = -0.05  # weight crossed zero: mismatched with its sign bit
        P.m[s], P.v[s], P.G[s] = 10 + s, 20 + s, 30 + s
        P.eps[s * B:(s + 1) * B] = 40 + s
        P.ebar[s * B:(s + 1) * B] = 50 + s
    return P


def test_elimination_order_and_records_exhaustive(orc):
    B = 3
    for n in range(1, 10):
        for mask in itertools.product((0, 1), repeat=n):
            P = one_row(orc, n, list(mask), B)
            dormant, st = orc.deepr_rewire(7, P, step=1000 + n)
            R = sum(mask)
            assert dormant[0] == R and st[0] == R and st[1] == R
            assert P.len[0] == n
            order = canonical_compaction(n, list(mask))
            for s, o in enumerate(order):  # survivors, with their whole record
                assert P.ind[s] == o
                assert P.m[s] == 10 + o and P.v[s] == 20 + o and P.G[s] == 30 + o
                assert np.all(P.eps[s * B:(s + 1) * B] == 40 + o)
                assert np.all(P.ebar[s * B:(s + 1) * B] == 50 + o)
            for s in range(n - R, n):  # new synapses start from zero
                assert P.w[s] == 0 and P.m[s] == 0 and P.v[s] == 0 and P.G[s] == 0
                assert np.all(P.eps[s * B:(s + 1) * B] == 0) and np.all(P.ebar[s * B:(s + 1) * B] == 0)
                assert P.ind[s] >= n or mask[P.ind[s]]  # a free target


def random_proj(orc, seed, n_pre=50, n_post=60, p=0.2, rec=True, B=2, flip=0.15):
    rng = np.random.default_rng(seed)
    lens, mx = orc.fixed_prob_count(seed, n_pre, n_post, p, rec, 1)
    P = orc.Proj(n_pre, n_post, 2 * mx, rec, 1, batch=B, trained=True, traces="alif", bitfields=True)
    orc.fixed_prob_rows(seed, P, p, 0.3)
    orc.deepr_init_bits(seed, P)
    for i in range(n_pre):
        for k in range(int(P.len[i])):
            s = i * P.cap + k
            if rng.random() < flip:
                P.w[s] = -P.w[s]
            P.m[s], P.v[s], P.G[s] = rng.random(3)
            P.eps[s * B:(s + 1) * B] = rng.random(B)
            P.ebar[s * B:(s + 1) * B] = rng.random(B)
    return P


def mismatched(P, i, s):
    j = int(P.ind[s])
    neg = (int(P.sign[i * P.words + (j >> 5)]) >> (j & 31)) & 1
    w = np.float32(P.w[s])
    return (w > 0 and neg) or (w < 0 and not neg)


@pytest.mark.parametrize("rec", [True, False])
def test_deepr_invariants(orc, rec):
    P = random_proj(orc, 11 + rec, rec=rec)
    B = P.batch
    before = rows_of(P)
    rec_of = {}
    elim_expect = []
    for i in range(P.n_pre):
        for k in range(int(P.len[i])):
            s = i * P.cap + k
            rec_of[(i, int(P.ind[s]))] = (P.w[s], P.m[s], P.v[s], P.G[s], P.eps[s * B:(s + 1) * B].copy(),
                                          P.ebar[s * B:(s + 1) * B].copy())
            if mismatched(P, i, s):
                elim_expect.append((i, int(P.ind[s])))
    sign0 = P.sign.copy()
    total = int(P.len.sum())
    dormant, st = orc.deepr_rewire(5, P, step=300)
    after = rows_of(P)
    assert st[0] == len(elim_expect) > 0 and st[1] == st[0]
    assert int(P.len.sum()) == total
    assert np.array_equal(P.sign, sign0)
    conn = bits_to_sets(P.conn, P.n_pre, P.n_post)
    gone = set(elim_expect)
    for i in range(P.n_pre):
        assert len(after[i]) == len(set(after[i])) and P.len[i] <= P.cap
        assert conn[i] == set(after[i])
        if rec:
            assert i not in after[i]
        assert dormant[i] == sum(1 for (r, _) in elim_expect if r == i)
        for k, j in enumerate(after[i]):
            s = i * P.cap + k
            if (i, j) in rec_of and (i, j) not in gone:
                w, m, v, G, e, eb = rec_of[(i, j)]
                assert (P.w[s], P.m[s], P.v[s], P.G[s]) == (w, m, v, G)
                assert np.array_equal(P.eps[s * B:(s + 1) * B], e) and np.array_equal(P.ebar[s * B:(s + 1) * B], eb)
            else:
                assert (P.w[s], P.m[s], P.v[s], P.G[s]) == (0, 0, 0, 0)
                assert not np.any(P.eps[s * B:(s + 1) * B]) and not np.any(P.ebar[s * B:(s + 1) * B])
        kept = [j for j in before[i] if (i, j) not in gone]
        assert set(kept) <= set(after[i])


def test_formation_row_choice_uniform(orc):
    # every row loses exactly one synapse per rewire, so D = n_pre activations
    # are spread over rows: totals over many rewires are uniform
    n_pre, n_post, B = 40, 200, 1
    totals = np.zeros(n_pre)
    for step in range(150):
        P = orc.Proj(n_pre, n_post, 40, False, 3, batch=B, trained=True, traces="lif", bitfields=True)
        set_rows(P, [[i] for i in range(n_pre)], [[0.5]] * n_pre)
        orc.deepr_init_bits(1, P)
        P.w[np.arange(n_pre) * P.cap] = -0.5
        orc.deepr_rewire(1, P, step=step)
        totals += P.len
    assert totals.sum() == 150 * n_pre
    assert stats.chisquare(totals).pvalue > 1e-4


def test_formation_targets_uniform_over_free_non_self(orc):
    n, B = 30, 1
    hist = np.zeros(n)
    for step in range(300):
        P = orc.Proj(n, n, 10, True, 4, batch=B, trained=True, traces="lif", bitfields=True)
        rows = [[(i + 1) % n] for i in range(n)]
        set_rows(P, rows, [[-0.2]] * n)
        orc.deepr_init_bits(2, P)
        for i in range(n):  # flip sign bits so every synapse is eliminated
            j = rows[i][0]
            P.sign[i * P.words + (j >> 5)] ^= np.uint32(1 << (j & 31))
        orc.deepr_rewire(2, P, step=step)
        r0 = rows_of(P)[0]
        for j in r0:
            hist[j] += 1
    assert hist[0] == 0  # never an autapse
    assert stats.chisquare(hist[1:]).pvalue > 1e-4


def test_capacity_respected_when_rows_are_full(orc):
    n_pre, n_post, cap, B = 8, 20, 4, 1
    P = orc.Proj(n_pre, n_post, cap, False, 5, batch=B, trained=True, traces="lif", bitfields=True)
    rows = [[0, 1, 2, 3] for _ in range(n_pre - 1)] + [[0]]
    set_rows(P, rows, [[0.3] * len(r) for r in rows])
    orc.deepr_init_bits(3, P)
    for i in range(n_pre - 1):
        P.w[i * cap + 3] = -0.3  # one mismatch in each full row
    for step in range(20):
        P2 = orc.Proj(n_pre, n_post, cap, False, 5, batch=B, trained=True, traces="lif", bitfields=True)
        for name in ("len", "ind", "w", "m", "v", "G", "ebar", "conn", "sign"):
            getattr(P2, name)[:] = getattr(P, name)
        orc.deepr_rewire(3, P2, step=step)
        assert int(P2.len.sum()) == int(P.len.sum())
        assert np.all(P2.len <= cap)
