"""Pins of the oracle's lateral projection and of the scaled (replicated)
stimulus of the topographic-map model (Tab. A-G; scaling paragraph of the
topographic-map section).

The lateral projection is pinned against the feed-forward path, which the
neuron-equation and STDP-pair pins already tie to the paper: with no lateral
synapses the run is the feed-forward run bit for bit; one lateral spike is
the feed-forward impulse of the same weight one step later; lateral pairs
follow the additive all-to-all pair closed forms of Tab. B / F; an autapse is
depressed by its own spike.  The initial in-degree of the pairwise-Bernoulli
rule is the lattice Gaussian sum, 2 pi p sigma^2 = 2 pi for both projections
(the paper's statement that both start from the same expected count).  The
replicated stimulus is checked against a brute-force nearest-centre search
over the s^2 copies.
"""
import math

import numpy as np
import pytest

import oracle as O

SEED = 11


def silent_model(L=4, **kw):
    base = dict(L=L, f_base=0.0, f_peak=0.0, stdp=0, rewire_steps=0)
    base.update(kw)
    return O.TopoModel(**base)


def rows(L, cap, syn, proj_id=0):
    N = L * L
    P = O.Proj(N, N, cap, False, proj_id)
    for i, j, w in syn:
        k = i * cap + P.len[i]
        P.ind[k] = j
        P.w[k] = w
        P.len[i] += 1
    return P


def step(M, P, PL, S, t, force_spike=()):
    """One step; neurons in force_spike start it far above threshold."""
    for a in force_spike:
        S.V[a] = 0.0
    O.topo_sim_step(SEED, M, P, S, t, PL)


def test_empty_lateral_rows_equal_the_feed_forward_run():
    """A lateral projection without synapses changes nothing: the full model
    (Poisson input, STDP, both rewires off) gives the feed-forward run's state
    bit for bit."""
    L, cap = 8, 16
    M = O.TopoModel(L=L, rewire_steps=0, f_base=40.0)
    P1 = O.Proj(L * L, L * L, cap, False, 0)
    O.gauss_rows(SEED, P1, L, 0.16, 2.5, M.g_max)
    P2 = O.Proj(L * L, L * L, cap, False, 0)
    O.gauss_rows(SEED, P2, L, 0.16, 2.5, M.g_max)
    PL = O.Proj(L * L, L * L, 4, False, 1)
    S1, S2 = O.TopoState(M), O.TopoState(M)
    for t in range(400):
        O.topo_sim_step(SEED, M, P1, S1, t)
        O.topo_sim_step(SEED, M, P2, S2, t, PL)
    assert S1.count.sum() > 0
    for f in ("V", "g", "y", "x", "ref", "count", "zout", "zin"):
        np.testing.assert_array_equal(getattr(S1, f), getattr(S2, f), err_msg=f)
    np.testing.assert_array_equal(P1.w, P2.w)
    # targets that spiked before the last step carry a lateral trace anyway
    assert (S2.xl > 0).sum() >= (S2.count > 0).sum() - S2.zout.sum()


def test_lateral_spike_is_a_feed_forward_impulse_one_step_later():
    """Neuron 5 spikes at step 10; its lateral synapse (weight 0.5) onto
    neuron 3 then acts exactly like a source spike of the same weight
    delivered at step 11 (whose response the neuron-equation pins fix)."""
    M = silent_model()
    w = 0.5
    PL = rows(M.L, 4, [(5, 3, w)], proj_id=1)
    empty = rows(M.L, 4, [])
    S = O.TopoState(M)
    Vl, gl = [], []
    for t in range(300):
        step(M, empty, PL, S, t, force_spike=(5,) if t == 10 else ())
        Vl.append(S.V[3])
        gl.append(S.g[3])
    assert S.count[5] == 1 and S.count[3] == 0
    Pf = rows(M.L, 4, [(0, 3, w)])
    S2 = O.TopoState(M)
    Vf, gf = [], []
    for t in range(300):
        S2.zin[:] = 0
        if t == 11:
            S2.zin[0] = 1
        O.topo_sim_step(SEED, M, Pf, S2, t)
        Vf.append(S2.V[3])
        gf.append(S2.g[3])
    np.testing.assert_array_equal(np.array(Vl), np.array(Vf))
    np.testing.assert_array_equal(np.array(gl), np.array(gf))
    assert gl[10] == 0.0 and gl[11] == w * math.exp(-M.h / M.tau_s)
    assert PL.w[5 * 4] == w  # no STDP in this model
    # the lateral pre trace took the delivery at step 11 and decayed since
    assert abs(S.xl[5] - math.exp(-(299 - 11) * M.h / M.tau_plus)) < 1e-12


@pytest.mark.parametrize("k", [0, 1, 7, 45])
def test_lateral_pair_pre_before_post(k):
    """Neuron 5 spikes at step 10 (delivered at 11), neuron 3 at 11 + k: the
    lateral weight 5 -> 3 gains A_+ exp(-k h / tau_+)."""
    M = silent_model(stdp=1)
    PL = rows(M.L, 4, [(5, 3, 0.1)], proj_id=1)
    empty = rows(M.L, 4, [])
    S = O.TopoState(M)
    t_pre, t_post = 10, 11 + k
    for t in range(t_post + 3):
        force = ((5,) if t == t_pre else ()) + ((3,) if t == t_post else ())
        step(M, empty, PL, S, t, force)
    assert S.count[5] == 1 and S.count[3] == 1
    expect = 0.1 + M.A_plus * math.exp(-k * M.h / M.tau_plus)
    assert abs(PL.w[5 * 4] - expect) < 1e-14


@pytest.mark.parametrize("k", [1, 3, 40])
def test_lateral_pair_post_before_pre(k):
    """Neuron 3 spikes at step 20; neuron 5's spike is delivered k steps later:
    the lateral weight 5 -> 3 loses A_- exp(-k h / tau_-)."""
    M = silent_model(stdp=1)
    PL = rows(M.L, 4, [(5, 3, 0.1)], proj_id=1)
    empty = rows(M.L, 4, [])
    S = O.TopoState(M)
    t_post = 20
    t_pre = t_post + k - 1  # spike at t_pre, delivered at t_post + k
    for t in range(t_post + k + 2):
        force = ((3,) if t == t_post else ()) + ((5,) if t == t_pre else ())
        step(M, empty, PL, S, t, force)
    assert S.count[3] == 1 and S.count[5] == 1
    expect = 0.1 - M.A_minus * math.exp(-k * M.h / M.tau_minus)
    assert abs(PL.w[5 * 4] - expect) < 1e-14


def test_autapse_is_depressed_by_its_own_spike():
    """An autapse 6 -> 6: the neuron's spike at step 4 reaches it at step 5,
    when the neuron's own post trace has decayed once: w loses A_- exp(-h /
    tau_-); the spike step itself potentiates nothing (no earlier pre spike)."""
    M = silent_model(stdp=1)
    PL = rows(M.L, 4, [(6, 6, 0.1)], proj_id=1)
    empty = rows(M.L, 4, [])
    S = O.TopoState(M)
    for t in range(8):
        step(M, empty, PL, S, t, (6,) if t == 4 else ())
        if t == 4:
            assert PL.w[6 * 4] == 0.1
    assert S.count[6] == 1
    assert abs(PL.w[6 * 4] - (0.1 - M.A_minus * math.exp(-M.h / M.tau_minus))) < 1e-15
    # the lateral pre trace took the delivery and decays with tau_+
    assert abs(S.xl[6] - math.exp(-2 * M.h / M.tau_plus)) < 1e-15


@pytest.mark.parametrize("kind", [O.STIM_BLOB, O.STIM_BAR])
@pytest.mark.parametrize("s", [1, 2, 3])
def test_replicated_stimulus_is_the_nearest_copy(kind, s):
    """Scaled map L = 16 s with the input replicated in every 16 x 16 square:
    each channel's squared stimulus distance is its distance on the L torus to
    the nearest of the s^2 copies of the drawn location (brute force)."""
    L0 = 16
    L = L0 * s
    M = O.TopoModel(L=L, stim_kind=kind, stim_tile=L0)
    for e in range(12):
        cx, cy, o = O.topo_stimulus(SEED, M, e * M.stim_steps)
        assert 0 <= cx < L0 and 0 <= cy < L0
        for i in range(0, L * L, 7):
            x, y = i % L, i // L
            best = None
            for a in range(s):
                for b in range(s):
                    ddx = abs(x - (cx + a * L0))
                    ddx = min(ddx, L - ddx)
                    ddy = abs(y - (cy + b * L0))
                    ddy = min(ddy, L - ddy)
                    d2 = (ddy * ddy if o else ddx * ddx) if kind == O.STIM_BAR else ddx * ddx + ddy * ddy
                    best = d2 if best is None else min(best, d2)
            assert O.topo_stim_d2(M, i, cx, cy, o) == best
    if s == 1:  # one square: the unscaled map
        M0 = O.TopoModel(L=L, stim_kind=kind)
        for e in range(12):
            assert O.topo_stimulus(SEED, M, e * M.stim_steps) == O.topo_stimulus(SEED, M0, e * M.stim_steps)


@pytest.mark.parametrize("p,sigma", [(1.0, 1.0), (0.16, 2.5)])
def test_initial_in_degree_is_the_lattice_gaussian_sum(p, sigma):
    """Pairwise-Bernoulli init: the expected row length is the sum of p exp(-d^2
    / 2 sigma^2) over the torus, which for p sigma^2 = 1 is 2 pi up to the
    lattice correction (both projections of the paper start from it); the
    lateral rule with p = 1 always contains the autapse."""
    L = 64
    N = L * L
    P = O.Proj(N, N, 64, False, 1)
    O.gauss_rows(SEED, P, L, p, sigma, 0.2)
    k = np.arange(-L // 2, L // 2)
    lattice = p * np.exp(-k ** 2 / (2 * sigma * sigma)).sum() ** 2
    assert abs(lattice - 2 * math.pi) < 1e-3
    mean = P.len.mean()
    sd = math.sqrt(lattice / N)
    assert abs(mean - lattice) < 5 * sd, (mean, lattice)
    if p == 1.0:
        for i in range(0, N, 97):
            assert i in P.ind[i * 64:i * 64 + P.len[i]]


def test_lateral_rewire_may_form_an_autapse():
    """Lateral formation at distance zero has probability p_form-lat = 1: a
    candidate equal to the row's own neuron is formed whatever its draw."""
    L = 8
    N = L * L
    PL = O.Proj(N, N, 8, False, 1)
    tp = O.TopoParams(L, 1, 1.0, 1.0, 0.1, 0.5, 0.01, 0.2)
    stats, bits = O.topo_rewire_scripted(PL, tp, attempt_row=lambda a: 9, target=lambda r, q, t: 9,
                                         elim_u32=lambda r, s: 0, form_u32=lambda r, j: 0xFFFFFFFF)
    assert list(stats) == [0, 1, 0, 1]
    assert PL.len[9] == 1 and PL.ind[9 * 8] == 9 and PL.w[9 * 8] == np.float32(0.2)
    assert not bits.any()


def test_full_model_with_lateral_invariants():
    """Both projections with STDP and rewiring over 3000 steps of a 16 x 16
    map: weights in [0, g_max], rows duplicate-free within capacity, both
    attempt bitfields clear, both rewires active, the lateral trace bounded by
    the spike count's geometric sum."""
    L, cap = 16, 32
    N = L * L
    M = O.TopoModel(L=L)
    P = O.Proj(N, N, cap, False, 0)
    O.gauss_rows(SEED, P, L, 0.16, 2.5, M.g_max)
    PL = O.Proj(N, N, cap, False, 1)
    O.gauss_rows(SEED, PL, L, 1.0, 1.0, M.g_max)
    tp = O.TopoParams(L, 10, 0.16, 2.5, M.g_max / 2, 2.45e-2 * 50, 1.36e-4 * 50, M.g_max)
    tpl = O.TopoParams(L, 10, 1.0, 1.0, M.g_max / 2, 2.45e-2 * 50, 1.36e-4 * 50, M.g_max)
    S = O.TopoState(M)
    bits = np.zeros(N * P.words, np.uint32)
    bits_l = np.zeros(N * PL.words, np.uint32)
    st, stl = O.topo_run(SEED, M, P, tp, S, 0, 3000, bits, PL, tpl, bits_l)
    # formation is active on both; with weights mostly potentiated, eliminations
    # (p_elim-pot 0.68% per hit) are rare at this length
    assert st[1] > 0 and stl[1] > 0 and st[3] == stl[3] == 3000
    assert S.count.sum() > 0
    for Q in (P, PL):
        for i in range(N):
            r = Q.ind[i * cap:i * cap + Q.len[i]]
            assert Q.len[i] <= cap and len(set(r.tolist())) == len(r)
            wr = Q.w[i * cap:i * cap + Q.len[i]]
            assert np.all(wr >= 0) and np.all(wr <= np.float32(M.g_max))  # new synapses: float g_max
    assert not bits.any() and not bits_l.any()
    assert np.all(S.xl >= 0) and np.all(S.xl <= 1.0 / (1.0 - math.exp(-M.h / M.tau_plus)))
