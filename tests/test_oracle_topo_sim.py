"""Pins of the oracle's topographic-map simulation (conductance LIF, STDP, input).

Each test checks the oracle against something other than its own formulas:
the continuous-time solution of the neuron equation of Tab. B, the algebraic
fixed point of that equation under constant conductance, the closed form of an
all-to-all additive STDP pair (Tab. B, F), the refractory definition of Tab. B,
a dense-matrix sum, and the Poisson rate profile of Tab. E measured from the
spikes the oracle draws.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle as O

SEED = 5


def silent_model(L=4, **kw):
    """Model with no Poisson input, no STDP and no rewiring unless asked."""
    base = dict(L=L, f_base=0.0, f_peak=0.0, stdp=0, rewire_steps=0)
    base.update(kw)
    return O.TopoModel(**base)


def rows(L, cap, syn):
    """Projection on an L x L sheet with the listed (pre, post, weight) synapses."""
    N = L * L
    P = O.Proj(N, N, cap, False, 0)
    for i, j, w in syn:
        k = i * cap + P.len[i]
        P.ind[k] = j
        P.w[k] = w
        P.len[i] += 1
    return P


def run(M, P, S, t0, n, force_in=None):
    """Step one at a time; force_in(t) lists source neurons delivered at step t."""
    out = []
    for t in range(t0, t0 + n):
        if force_in is not None:
            S.zin[:] = 0
            for i in force_in(t):
                S.zin[i] = 1
        O.topo_sim_step(SEED, M, P, S, t)
        out.append((S.V.copy(), S.g.copy(), S.zout.copy(), P.w.copy()))
    return out


def test_single_spike_follows_continuous_neuron_equation():
    """A conductance impulse of w delivered at t = 0 into a resting neuron: the
    discrete trajectory tracks the ODE of Tab. B with g(t) = w exp(-t/tau_s)."""
    M = silent_model()
    w = 0.5
    P = rows(M.L, 4, [(0, 3, w)])
    S = O.TopoState(M)
    tr = run(M, P, S, 0, 600, force_in=lambda t: [0] if t == 0 else [])
    V = np.array([x[0][3] for x in tr])
    g_leak = M.C_m / M.tau_m

    def f(t, v):
        g = w * math.exp(-t / M.tau_s)
        return [(M.V_rest - v[0] + g / g_leak * (M.E_exc - v[0])) / M.tau_m]

    times = (np.arange(600) + 1) * M.h
    sol = solve_ivp(f, (0, times[-1]), [M.V_rest], t_eval=times, rtol=1e-10, atol=1e-12)
    dev = V - M.V_rest
    ref = sol.y[0] - M.V_rest
    assert dev.max() > 1.0  # a visible PSP, well below threshold
    assert np.abs(dev - ref).max() < 0.03 * ref.max()
    # the conductance itself decays exactly as w exp(-(k+1) h / tau_s)
    g = np.array([x[1][3] for x in tr])
    k = np.arange(600)
    np.testing.assert_allclose(g, w * np.exp(-(k + 1) * M.h / M.tau_s), rtol=1e-12)
    # other neurons stay at rest
    assert np.all(tr[-1][0][np.arange(M.L * M.L) != 3] == M.V_rest)


def test_constant_conductance_reaches_ode_fixed_point():
    """One spike every step: the held conductance is w / (1 - exp(-h/tau_s)),
    and V settles where the right-hand side of the Tab. B equation vanishes."""
    M = silent_model()
    w = 0.003
    P = rows(M.L, 4, [(2, 5, w)])
    S = O.TopoState(M)
    tr = run(M, P, S, 0, 20000, force_in=lambda t: [2])
    g_hold = w / (1.0 - math.exp(-M.h / M.tau_s))
    g_leak = M.C_m / M.tau_m
    V_star = (M.V_rest + g_hold / g_leak * M.E_exc) / (1.0 + g_hold / g_leak)
    assert V_star < M.V_th
    assert abs(tr[-1][0][5] - V_star) < 1e-9 * abs(V_star)
    assert not any(x[2].any() for x in tr)


def test_threshold_reset_and_refractory_period():
    """Strong drive: spikes are exactly tau_ref/h + 1 steps apart, V is V_reset
    through each refractory period, and nothing fires during it."""
    M = silent_model()
    P = rows(M.L, 4, [(1, 7, 200.0)])
    S = O.TopoState(M)
    tr = run(M, P, S, 0, 400, force_in=lambda t: [1])
    z = np.array([x[2][7] for x in tr])
    V = np.array([x[0][7] for x in tr])
    spikes = np.flatnonzero(z)
    assert spikes[0] == 0
    assert np.all(np.diff(spikes) == M.ref_steps + 1)
    for s in spikes[:-1]:
        assert np.all(V[s:s + M.ref_steps + 1] == M.V_reset)
    assert S.count[7] == len(spikes)
    assert S.count.sum() == len(spikes)


def test_delivery_equals_dense_matrix_sum():
    """Conductance increments of one step equal W^T z for a random ragged
    projection and random source spikes (brute force, dense float64)."""
    rng = np.random.default_rng(3)
    L, cap = 6, 8
    N = L * L
    syn = []
    for i in range(N):
        for j in rng.choice(N, size=rng.integers(0, cap + 1), replace=False):
            syn.append((i, int(j), float(rng.uniform(0, 0.2))))
    P = rows(L, cap, syn)
    Wd = np.zeros((N, N))
    for i, j, w in syn:
        Wd[i, j] += w
    M = silent_model(L=L, ref_steps=10 ** 6)
    S = O.TopoState(M)
    S.ref[:] = 10 ** 6  # keep V fixed; only g matters here
    z = (rng.random(N) < 0.3).astype(np.uint8)
    S.zin[:] = z
    O.topo_sim_step(SEED, M, P, S, 0)
    np.testing.assert_allclose(S.g, (Wd.T @ z) * math.exp(-M.h / M.tau_s), rtol=1e-13, atol=1e-15)


def pair_model(L=4):
    return silent_model(L=L, stdp=1)


@pytest.mark.parametrize("k", [0, 1, 5, 30, 200])
def test_stdp_pre_before_post(k):
    """Source 0 (weight 0.1 onto neuron 3) is delivered k steps before a strong
    source 1 makes neuron 3 fire: the weight gains A_+ exp(-k h / tau_+)."""
    M = pair_model()
    P = rows(M.L, 4, [(0, 3, 0.1), (1, 3, 500.0)])
    S = O.TopoState(M)
    t_pre, t_post = 10, 10 + k
    run(M, P, S, 0, t_post + 3,
        force_in=lambda t: ([0] if t == t_pre else []) + ([1] if t == t_post else []))
    assert S.count[3] == 1
    expect = 0.1 + M.A_plus * math.exp(-k * M.h / M.tau_plus)
    assert abs(P.w[0] - expect) < 1e-14


@pytest.mark.parametrize("k", [1, 4, 40, 300])
def test_stdp_post_before_pre(k):
    """Neuron 3 fires at t0; source 0 is delivered k steps later: the weight
    loses A_- exp(-k h / tau_-) per earlier postsynaptic spike (the strong
    impulse keeps the neuron firing after each refractory period, so long lags
    pair with several spikes)."""
    M = pair_model()
    P = rows(M.L, 4, [(0, 3, 0.1), (1, 3, 500.0)])
    S = O.TopoState(M)
    t_post, t_pre = 10, 10 + k
    tr = run(M, P, S, 0, t_pre + 1,
             force_in=lambda t: ([1] if t == t_post else []) + ([0] if t == t_pre else []))
    posts = [t for t, x in enumerate(tr) if x[2][3]]
    assert posts[0] == t_post and t_pre not in posts
    if k <= M.ref_steps:
        assert posts == [t_post]
    expect = 0.1 - M.A_minus * sum(math.exp(-(t_pre - p) * M.h / M.tau_minus) for p in posts)
    assert abs(P.w[0] - expect) < 1e-14


def test_stdp_all_to_all_sum_and_clipping():
    """All-to-all pairing sums the pair terms of every earlier spike; weights
    are clipped to [0, g_max]."""
    M = pair_model()
    pre0 = [5, 9]
    post = 20
    # neuron 5 fires first, driven by source 3
    P2 = rows(M.L, 4, [(0, 3, 0.1), (1, 3, 500.0), (2, 3, 0.195), (0, 5, 0.001), (3, 5, 500.0)])
    S = O.TopoState(M)
    run(M, P2, S, 0, 30,
        force_in=lambda t: ([0] if t in pre0 else []) + ([1] if t == post else [])
        + ([2] if t == 2 else []) + ([3] if t == 0 else []))
    x0 = sum(math.exp(-(post - t) * M.h / M.tau_plus) for t in pre0)
    assert abs(P2.w[0] - (0.1 + M.A_plus * x0)) < 1e-14
    # 0.195 + A_+ e^{...} > g_max: clipped
    assert P2.w[2 * 4] == M.g_max
    # neuron 5 fired at step 0; both deliveries of source 0 depress 0.001 below zero
    assert P2.w[1] == 0.0


def test_input_rate_profile_and_stimulus_epochs():
    """Spikes drawn by the source sheet: the per-step probability at squared
    stimulus distance d2 is (f_base + f_peak exp(-d2 / 2 sigma^2)) h (Tab. E),
    the stimulus keeps its position through an epoch of t_stim and moves at
    epoch boundaries."""
    L = 16
    M = O.TopoModel(L=L, stdp=0, rewire_steps=0, stim_steps=200)
    P = rows(L, 1, [])
    S = O.TopoState(M)
    N = L * L
    n_steps = 20000
    hits = {}
    tries = {}
    moves = 0
    prev = None
    for t in range(n_steps):
        O.topo_sim_step(SEED, M, P, S, t)
        c = O.topo_stimulus(SEED, M, t)
        if t % 200:
            assert c == prev
        elif prev is not None and c != prev:
            moves += 1
        prev = c
        cx, cy, _ = c
        xs, ys = np.arange(N) % L, np.arange(N) // L
        dx = np.minimum(np.abs(xs - cx), L - np.abs(xs - cx))
        dy = np.minimum(np.abs(ys - cy), L - np.abs(ys - cy))
        d2 = dx * dx + dy * dy
        for v in (0, 1, 2, 4, 5, 8):
            sel = d2 == v
            hits[v] = hits.get(v, 0) + int(S.zin[sel].sum())
            tries[v] = tries.get(v, 0) + int(sel.sum())
    assert moves >= 90
    for v in hits:
        p = (5.0 + 152.8 * math.exp(-v / 8.0)) * 0.1e-3
        n = tries[v]
        assert abs(hits[v] - n * p) < 5 * math.sqrt(n * p * (1 - p)) + 1, (v, hits[v], n * p)


def test_bar_stimulus_uses_distance_along_one_axis():
    """Bar input: the rate depends on the distance to a line of cells only."""
    L = 16
    M = O.TopoModel(L=L, stim_kind=O.STIM_BAR)
    seen = set()
    for e in range(40):
        cx, cy, o = O.topo_stimulus(SEED, M, e * M.stim_steps)
        seen.add(o)
        for i in range(L * L):
            x, y = i % L, i // L
            d = min(abs(y - cy), L - abs(y - cy)) if o else min(abs(x - cx), L - abs(x - cx))
            assert O.topo_stim_d2(M, i, cx, cy, o) == d * d
    assert seen == {0, 1}


def test_full_model_invariants():
    """Conductance-LIF + STDP + rewiring over 3000 steps on a 16 x 16 map:
    weights stay in [0, g_max], rows stay duplicate-free within capacity, the
    attempt bitfield ends clear, refractory counters stay in range."""
    L, cap = 16, 32
    M = O.TopoModel(L=L)
    P = O.Proj(L * L, L * L, cap, False, 0)
    O.gauss_rows(SEED, P, L, 0.16, 2.5, M.g_max)
    tp = O.TopoParams(L, 10, 0.16, 2.5, M.g_max / 2, 2.45e-2 * 50, 1.36e-4 * 50, M.g_max)
    S = O.TopoState(M)
    bits = np.zeros(P.n_pre * P.words, np.uint32)
    stats = O.topo_run(SEED, M, P, tp, S, 0, 3000, bits)
    assert stats[3] == 300 * 10
    assert stats[0] + stats[1] > 0
    assert not bits.any()
    for i in range(P.n_pre):
        n = P.len[i]
        assert 0 <= n <= cap
        r = P.ind[i * cap:i * cap + n]
        assert len(set(r.tolist())) == n
        w = P.w[i * cap:i * cap + n]
        # new and initial synapses carry g_max rounded to float32, the stored precision
        assert np.all(w >= 0) and np.all(w <= float(np.float32(M.g_max)))
    assert S.count.sum() > 0
    assert np.all((S.ref >= 0) & (S.ref <= M.ref_steps))


def test_input_draws_share_generator_calls_as_stated():
    """Eight channels per generator call: channel i's draw is word (i % 8) / 2
    of the Philox block at counter (t, i // 8), upper half for even i, lower
    half for odd i (the block itself is pinned to numpy's Philox elsewhere)."""
    key1 = 12  # topomap source tag, projection 0
    for t, i in [(0, 0), (0, 1), (7, 5), (123, 4095), (99999, 8), (5, 2046)]:
        words = O.philox4x64_10(SEED, key1, [t, i // 8, 0, 0])
        w = int(words[(i % 8) // 2])
        expect = (w & 0xFFFFFFFF) if i % 2 else (w >> 32)
        assert O.topo_input_u32(SEED, t, i) == expect


def test_input_channels_sharing_a_word_are_independent():
    """Channels 2k and 2k+1 take the two halves of one 64-bit word: at p = 1/2
    their joint firing frequency is 1/4 within 5 sigma."""
    L = 16
    M = O.TopoModel(L=L, f_base=5000.0, f_peak=0.0, stdp=0, rewire_steps=0)
    P = rows(L, 1, [])
    S = O.TopoState(M)
    both = n = 0
    for t in range(400):
        O.topo_sim_step(SEED, M, P, S, t)
        z = S.zin.astype(np.int64)
        both += int((z[0::2] & z[1::2]).sum())
        n += L * L // 2
    assert abs(both - n / 4) < 5 * math.sqrt(n * 3 / 16)
