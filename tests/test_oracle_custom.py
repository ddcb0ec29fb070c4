"""Pins of the oracle's custom connectivity-update examples (the paper's
add_diagonal and remove_random): brute force over small random projections,
the random targets against numpy's independent Philox, and their uniformity."""
import numpy as np
import pytest

from helpers import numpy_block, rows_of, sequential_remove, set_rows


def proj(orc, rng, n_pre, n_post, cap, B=2, bits=False):
    P = orc.Proj(n_pre, n_post, cap, False, 3, batch=B, trained=True, traces="alif", bitfields=bits)
    rows = []
    for i in range(n_pre):
        k = int(rng.integers(0, cap + 1))
        rows.append(rng.choice(n_post, k, replace=False).tolist())
    set_rows(P, rows, [rng.normal(0, 1, len(r)) for r in rows])
    for a in (P.m, P.v, P.G, P.eps, P.ebar):
        a[:] = rng.normal(0, 1, a.size)
    if bits:
        for i, r in enumerate(rows):
            for j in r:
                P.conn[i * P.words + (j >> 5)] |= np.uint32(1 << (j & 31))
    return P, rows


@pytest.mark.parametrize("bits", [False, True])
def test_add_diagonal_brute_force(orc, bits):
    rng = np.random.default_rng(1)
    P, rows = proj(orc, rng, 30, 20, 6, bits=bits)
    before = [list(r) for r in rows]
    m0, eb0 = P.m.copy(), P.ebar.copy()
    added = orc.add_diagonal(P)
    after = rows_of(P)
    n = 0
    for i in range(30):
        if i < 20 and len(before[i]) < 6 and not (bits and i in before[i]):
            assert after[i] == before[i] + [i]
            s = i * 6 + len(before[i])
            assert P.w[s] == 1.0 and P.m[s] == 0 and P.G[s] == 0 and not P.ebar[s * 2:s * 2 + 2].any()
            n += 1
        else:
            assert after[i] == before[i]
    assert added == n > 0
    for i in range(30):  # existing records untouched
        for k in range(len(before[i])):
            s = i * 6 + k
            assert P.m[s] == m0[s] and (P.ebar[s * 2:s * 2 + 2] == eb0[s * 2:s * 2 + 2]).all()


def test_remove_random_targets_follow_the_generator(orc):
    P, _ = proj(orc, np.random.default_rng(2), 50, 37, 5)
    seed, step = 99, 1234
    t = orc.remove_random_targets(seed, P, step)
    for i in range(50):
        w0 = numpy_block(seed, orc.TAG_CUSTOM | (3 << 8), [step, i, 0, 0])[0]
        assert t[i] == (((int(w0) >> 32) * 37) >> 32)


def test_remove_random_targets_are_uniform(orc):
    from scipy.stats import chisquare
    P = orc.Proj(20000, 16, 1, False, 1)
    t = orc.remove_random_targets(5, P, 7)
    assert chisquare(np.bincount(t, minlength=16)).pvalue > 1e-4


def test_remove_targets_brute_force(orc):
    rng = np.random.default_rng(3)
    P, rows = proj(orc, rng, 40, 15, 8, bits=True)
    post = rng.integers(0, 15, 40).astype(np.uint32)
    for i in range(0, 40, 3):  # some rows certainly hold their target
        if rows[i]:
            post[i] = rows[i][int(rng.integers(0, len(rows[i])))]
    recs = {(i, k): (P.w[i * 8 + k], P.m[i * 8 + k], P.ebar[(i * 8 + k) * 2]) for i in range(40)
            for k in range(len(rows[i]))}
    removed = orc.remove_targets(P, post)
    n = 0
    for i in range(40):
        r = rows[i]
        if post[i] in r:
            k = r.index(post[i])
            order = sequential_remove(len(r), [q == k for q in range(len(r))])
            n += 1
        else:
            order = list(range(len(r)))
        assert rows_of(P)[i] == [r[q] for q in order]
        for slot, q in enumerate(order):  # whole records moved
            assert (P.w[i * 8 + slot], P.m[i * 8 + slot], P.ebar[(i * 8 + slot) * 2]) == recs[(i, q)]
        word = P.conn[i * P.words]
        assert {j for j in range(15) if (int(word) >> j) & 1} == set(rows_of(P)[i])
    assert removed == n > 0
