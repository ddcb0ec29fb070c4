"""Pins of the oracle's topographic-map rewiring (paper Sec. 2.1.3, Fig. 3,
Tab. B and G): the narrated worked example, invariants, and the expected
numbers of formations and eliminations."""
import json
import os

import numpy as np
import pytest

from helpers import bits_to_sets, rows_of, set_rows
from test_oracle_build import brute_d2

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig3_topomap.json")


def u32_of(R):
    return int(np.floor(R * 2**32))


def test_fig3_worked_example(orc):
    g = json.load(open(GOLD))
    P = orc.Proj(g["n_pre"], g["n_post"], g["cap"], False, 0)
    set_rows(P, g["rows_before"], g["weights_before"])
    pr = g["params"]
    tp = orc.TopoParams(L=g["L"], n_attempts=len(g["attempt_rows"]), **pr)
    cand = {int(k): v for k, v in g["candidate_targets"].items()}
    elim = {tuple(int(x) for x in k.split(",")): u32_of(v) for k, v in g["elim_R"].items()}
    form = {tuple(int(x) for x in k.split(",")): u32_of(v) for k, v in g["form_R"].items()}
    seen_elim, seen_form = set(), set()

    def elim_u32(r, s):
        seen_elim.add((r, s))
        return elim[(r, s)]

    def form_u32(r, j):
        seen_form.add((r, j))
        return form[(r, j)]

    stats, bits = orc.topo_rewire_scripted(
        P, tp, attempt_row=lambda a: g["attempt_rows"][a], target=lambda r, q, t: cand[r][q],
        elim_u32=elim_u32, form_u32=form_u32)
    assert rows_of(P) == g["rows_after"]
    for i, ws in enumerate(g["weights_after"]):
        assert list(P.w[i * P.cap:i * P.cap + len(ws)]) == pytest.approx([float(np.float32(w)) for w in ws])
    s = g["stats_after"]
    assert list(stats) == [s["eliminated"], s["formed"], s["blocked"], s["attempts"]]
    assert not bits.any()
    # exactly the narrated elimination and formation candidates were tried
    assert seen_elim == set(elim) and seen_form == set(form)


def fresh(orc, L, cap, rows, w, proj_id=0):
    P = orc.Proj(L * L, L * L, cap, False, proj_id)
    set_rows(P, rows, w)
    return P


def test_topomap_invariants_random(orc):
    L, cap = 8, 6
    rng = np.random.default_rng(4)
    N = L * L
    rows = [sorted(rng.choice(N, rng.integers(0, cap + 1), replace=False).tolist()) for _ in range(N)]
    for r in rows:
        rng.shuffle(r)
    w = [rng.uniform(0, 0.2, len(r)) for r in rows]
    P = fresh(orc, L, cap, rows, w)
    tp = orc.TopoParams(L=L, n_attempts=200, p_form=0.8, sigma_form=1.5, g_theta=0.1,
                        p_elim_dep=0.6, p_elim_pot=0.2, g_new=0.2)
    for step in range(0, 200, 10):
        before = [set(r) for r in rows_of(P)]
        total = int(P.len.sum())
        stats, bits = orc.topo_rewire(42, P, tp, step)
        after = rows_of(P)
        assert not bits.any()
        assert int(P.len.sum()) == total - stats[0] + stats[1]
        for i in range(N):
            assert len(after[i]) == len(set(after[i])) <= cap
            new = set(after[i]) - before[i]
            for j in new:
                k = after[i].index(j)
                assert P.w[i * cap + k] == np.float32(0.2)


def test_topomap_formation_rate_empty_rows(orc):
    # all rows empty: every candidate is a formation attempt with probability
    # p_form exp(-d^2 / 2 sigma^2), d to a uniformly chosen target
    L, n_att, reps = 12, 40, 300
    p_form, sigma = 0.7, 1.5
    tp = orc.TopoParams(L=L, n_attempts=n_att, p_form=p_form, sigma_form=sigma, g_theta=0.1,
                        p_elim_dep=0.5, p_elim_pot=0.1, g_new=0.2)
    pj = np.array([p_form * np.exp(-brute_d2(L, 0, j) / (2 * sigma ** 2)) for j in range(L * L)])
    formed = 0
    for rep in range(reps):
        P = fresh(orc, L, 8, [[]] * (L * L), None)
        stats, _ = orc.topo_rewire(9, P, tp, 10 * rep)
        formed += stats[1]
    n = n_att * reps
    mean = pj.mean()
    assert abs(formed - n * mean) < 4 * np.sqrt(n * mean * (1 - mean))


def test_topomap_elimination_rate_full_rows(orc):
    # every row connected to every target: each candidate hits a synapse, weak
    # (w < g_theta) for even targets and strong for odd ones
    L, reps = 4, 300
    N = L * L
    tp = orc.TopoParams(L=L, n_attempts=12, p_form=0.5, sigma_form=1.0, g_theta=0.1,
                        p_elim_dep=0.6, p_elim_pot=0.1, g_new=0.2)
    elim = 0
    cands = 0
    for rep in range(reps):
        rows = [list(range(N)) for _ in range(N)]
        w = [[0.05 if j % 2 == 0 else 0.15 for j in range(N)] for _ in range(N)]
        P = fresh(orc, L, N, rows, w)
        stats, _ = orc.topo_rewire(13, P, tp, rep)
        elim += stats[0]
        assert stats[1] == 0
        cands += 12
    mean = 0.5 * (0.6 + 0.1)
    var = 0.5 * (0.6 * 0.4 + 0.1 * 0.9) + 0.25 * 0.25  # mixture variance
    assert abs(elim - cands * mean) < 4 * np.sqrt(cands * var)


def test_topomap_full_row_blocks_formation(orc):
    L = 4
    tp = orc.TopoParams(L=L, n_attempts=50, p_form=1.0, sigma_form=100.0, g_theta=0.0,
                        p_elim_dep=0.0, p_elim_pot=0.0, g_new=0.2)
    rows = [[(i + 1) % 16] for i in range(16)]
    P = fresh(orc, L, 1, rows, [[0.2]] * 16)
    stats, bits = orc.topo_rewire(1, P, tp, 0)
    assert stats[0] == 0 and stats[1] == 0 and stats[2] > 0
    assert rows_of(P) == rows and not bits.any()
