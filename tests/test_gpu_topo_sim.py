"""GPU parity of the topographic-map simulation (conductance LIF, STDP, Poisson
stimulus, rewiring every interval) against the oracle.

Lockstep protocol: before every rewiring interval the oracle takes the GPU's
rows and state, both run the interval (its steps and the rewire at its end),
and the results are compared: spikes, refractory counts, input draws and row
structure exactly; voltages, conductances, traces and weights within 1e-5 of
max(|oracle|, scale of the variable).
"""
import numpy as np
import pytest

import oracle
from paper_2510_19764_amd import binding as rb

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def f32(x):
    return float(np.float32(x))


def omodel(m: rb.TopoModel, L: int) -> oracle.TopoModel:
    """The oracle model with the float32 constants the library receives."""
    kw = {}
    for k in ("h", "C_m", "tau_m", "V_rest", "E_exc", "V_th", "V_reset", "tau_s", "f_base", "f_peak",
              "sigma_stim", "g_max", "A_plus", "A_minus", "tau_plus", "tau_minus"):
        kw[k] = f32(getattr(m, k))
    for k in ("ref_steps", "stim_steps", "stim_kind", "stdp", "rewire_steps"):
        kw[k] = int(getattr(m, k))
    return oracle.TopoModel(L=L, **kw)


def tparams(cfg: rb.TopoConfig):
    return oracle.TopoParams(L=cfg.L, n_attempts=cfg.n_attempts, p_form=f32(cfg.p_form),
                             sigma_form=f32(cfg.sigma_form), g_theta=f32(cfg.g_theta),
                             p_elim_dep=f32(cfg.p_elim_dep), p_elim_pot=f32(cfg.p_elim_pot), g_new=f32(cfg.g_new))


def unpack(bits, n):
    return np.unpackbits(bits.view(np.uint8), bitorder="little")[:n]


def snapshot(t: rb.TopoNet, cfg: rb.TopoConfig, M: oracle.TopoModel):
    n = cfg.L * cfg.L
    ln, ind, w = t.get_rows()
    P = oracle.Proj(n, n, cfg.cap, False, cfg.proj_id)
    P.len[:] = ln
    P.ind[:] = ind.ravel()
    P.w[:] = w.ravel()
    S = oracle.TopoState(M)
    S.V[:] = t.sim_get(rb.TV_V)
    S.g[:] = t.sim_get(rb.TV_G)
    S.y[:] = t.sim_get(rb.TV_Y)
    S.x[:] = t.sim_get(rb.TV_X)
    S.ref[:] = t.sim_get(rb.TV_REF)
    S.count[:] = t.sim_get(rb.TV_COUNT).astype(np.int32)
    S.zin[:] = unpack(t.sim_get(rb.TV_ZIN), n)
    S.zout[:] = unpack(t.sim_get(rb.TV_ZOUT), n)
    return P, S, int(t.sim_get(rb.TV_STEP)[0])


def close(name, gpu, orc, scale):
    tol = 1e-5 * np.maximum(np.abs(orc), scale)
    bad = np.abs(gpu.astype(np.float64) - orc) > tol
    assert not bad.any(), f"{name}: {bad.sum()} of {bad.size} outside tolerance, e.g. " \
                          f"{gpu[bad][:3]} vs {orc[bad][:3]}"


def compare(t, cfg, M, P, S):
    n = cfg.L * cfg.L
    ln, ind, w = t.get_rows()
    assert np.array_equal(ln, P.len)
    m = np.arange(cfg.cap)[None, :] < ln[:, None]
    assert np.array_equal(ind[m], P.ind.reshape(n, cfg.cap)[m])
    close("w", w[m], P.w.reshape(n, cfg.cap)[m], M.g_max)
    assert np.array_equal(unpack(t.sim_get(rb.TV_ZOUT), n), S.zout)
    assert np.array_equal(unpack(t.sim_get(rb.TV_ZIN), n), S.zin)
    assert np.array_equal(t.sim_get(rb.TV_COUNT).astype(np.int64), S.count)
    assert np.array_equal(t.sim_get(rb.TV_REF), S.ref)
    close("V", t.sim_get(rb.TV_V), S.V, abs(M.V_rest))
    close("g", t.sim_get(rb.TV_G), S.g, M.g_max)
    close("x", t.sim_get(rb.TV_X), S.x, 1.0)
    close("y", t.sim_get(rb.TV_Y), S.y, 1.0)


# a driven map (strong input and weights) so that STDP and refractoriness occur
HOT = rb.TopoModel(f_peak=600.0, g_max=0.5, A_plus=0.05, A_minus=0.05 * 1.2 * 20.0 / 64.0)
CASES = {
    "hot-L16-blob": (rb.TopoConfig(L=16, cap=32, n_attempts=10, proj_id=0, g_theta=0.25, g_new=0.5,
                                   g_init=0.5, seed=3), HOT),
    # capacities above 32 and not a multiple of 4
    "hot-L20-bar": (rb.TopoConfig(L=20, cap=40, n_attempts=40, proj_id=2, g_theta=0.25, g_new=0.5,
                                  g_init=0.5, seed=4),
                    rb.TopoModel(f_peak=600.0, g_max=0.5, A_plus=0.05, A_minus=0.01875, stim_kind=rb.STIM_BAR,
                                 stim_steps=50)),
    "nostdp-L12": (rb.TopoConfig(L=12, cap=18, n_attempts=10, proj_id=1, g_theta=0.25, g_new=0.5,
                                 g_init=0.5, seed=5),
                   rb.TopoModel(f_peak=600.0, g_max=0.5, stdp=0, rewire_steps=7)),
    # the benchmark's map: the paper's parameters with the moving bar
    "paper-L64": (rb.TopoConfig(L=64, cap=32, n_attempts=160, proj_id=0, seed=9),
                  rb.TopoModel(stim_kind=rb.STIM_BAR)),
    # the largest map, driven, bar stimulus moving every 5 ms
    "hot-L64-bar": (rb.TopoConfig(L=64, cap=32, n_attempts=160, proj_id=0, g_theta=0.25, g_new=0.5, g_init=0.5,
                                  seed=10),
                    rb.TopoModel(f_peak=600.0, g_max=0.5, A_plus=0.05, A_minus=0.01875, stim_kind=rb.STIM_BAR,
                                 stim_steps=50)),
    # 36 neurons: the last generator call covers 4 channels beyond the sheet, bit words end mid-word
    "ragged-L6": (rb.TopoConfig(L=6, cap=8, n_attempts=5, proj_id=3, p_form=0.6, sigma_form=1.5, g_theta=0.25,
                                g_new=0.5, g_init=0.5, seed=12),
                  rb.TopoModel(f_base=200.0, f_peak=600.0, g_max=0.5, A_plus=0.05, A_minus=0.02, stim_steps=30,
                               ref_steps=7, rewire_steps=3)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_topo_sim_lockstep_matches_oracle(name):
    cfg, model = CASES[name]
    t = rb.TopoNet(cfg)
    t.sim_init(model)
    M = omodel(model, cfg.L)
    tp = tparams(cfg)
    R = model.rewire_steps
    n_chunks = 12 if cfg.L >= 64 else 40
    spikes = 0
    changed = 0
    for _ in range(n_chunks):
        P, S, t0 = snapshot(t, cfg, M)
        stats = oracle.topo_run(cfg.seed, M, P, tp, S, t0, R)
        t.run(R)
        st = t.run_stats()
        assert (st.eliminated, st.formed, st.blocked) == tuple(stats[:3])
        changed += st.eliminated + st.formed
        compare(t, cfg, M, P, S)
        spikes = int(S.count.sum())
    assert spikes > 0
    assert changed > 0


def test_topo_sim_split_runs_are_identical():
    """Launch boundaries inside and across rewiring intervals change nothing:
    one 200-step run equals runs of 3, 64, 1 and 132 steps, bit for bit."""
    cfg, model = CASES["hot-L16-blob"]
    a, b = rb.TopoNet(cfg), rb.TopoNet(cfg)
    a.sim_init(model)
    b.sim_init(model)
    a.run(200)
    for n in (3, 64, 1, 132):
        b.run(n)
    for var in (rb.TV_V, rb.TV_G, rb.TV_Y, rb.TV_X, rb.TV_REF, rb.TV_COUNT, rb.TV_ZIN, rb.TV_ZOUT, rb.TV_STEP):
        assert np.array_equal(a.sim_get(var), b.sim_get(var)), var
    for x, y in zip(a.get_rows(), b.get_rows()):
        assert np.array_equal(x, y)
    assert a.sim_get(rb.TV_COUNT).sum() > 0


def _same_state(a, b):
    for var in (rb.TV_V, rb.TV_G, rb.TV_Y, rb.TV_X, rb.TV_REF, rb.TV_COUNT, rb.TV_ZIN, rb.TV_ZOUT, rb.TV_STEP):
        assert np.array_equal(a.sim_get(var), b.sim_get(var)), var
    for x, y in zip(a.get_rows(), b.get_rows()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("name", ["hot-L16-blob", "paper-L64"])
def test_topo_sim_graph_replays_match_direct_launches(name):
    """Whole rewiring intervals run as replays of a recorded graph of 64
    intervals.  Replays mixed with direct launches and host reads give the same
    state and rows, bit for bit, as the same steps in 10-step calls."""
    cfg, model = CASES[name]
    a, b = rb.TopoNet(cfg), rb.TopoNet(cfg)
    a.sim_init(model)
    b.sim_init(model)
    a.run(5)                 # direct, within an interval
    a.run(5 + 640 * 2)       # direct to the boundary, then two replays
    a.sim_get(rb.TV_V)       # host read between replays
    a.run(640 * 3 + 7)       # three replays, then a direct partial interval
    total = 5 + 5 + 1280 + 1920 + 7
    b.run(5)
    done = 5
    while done < total:
        n = min(10 - done % 10, total - done)
        b.run(n)
        done += n
    _same_state(a, b)
    assert a.sim_get(rb.TV_COUNT).sum() > 0


def test_topo_sim_graph_follows_new_model():
    """After rs_topo_sim_init with another rewiring interval the recorded
    launches are replaced: replays equal direct 5-step calls under the new model."""
    cfg, model = CASES["hot-L16-blob"]
    m2 = rb.TopoModel(f_peak=600.0, g_max=0.5, A_plus=0.05, A_minus=0.02, rewire_steps=5)
    a = rb.TopoNet(cfg)
    a.sim_init(model)
    a.run(640)
    a.sim_init(m2)
    ln, ind, w = a.get_rows()
    b = rb.TopoNet(cfg)
    b.set_rows(ln, ind, w)
    b.sim_init(m2)
    a.run(320 * 4)
    for _ in range(256):
        b.run(5)
    _same_state(a, b)


def test_topo_sim_phase_timers():
    """The per-phase timers change no result, stay within the run's device
    time, and restart from zero when switched."""
    cfg, model = CASES["hot-L16-blob"]
    a, b = rb.TopoNet(cfg), rb.TopoNet(cfg)
    a.sim_init(model)
    b.sim_init(model)
    a.sim_timing(True)
    a.run(1280 + 35)  # graph replays and direct launches
    b.run(1280 + 35)
    _same_state(a, b)
    ph = a.sim_phase_ms()
    assert all(v > 0 for v in ph.values()), ph
    assert sum(ph.values()) <= a.last_ms() * 1.01
    a.sim_timing(False)
    assert all(v == 0 for v in a.sim_phase_ms().values())
    a.run(20)
    assert all(v == 0 for v in a.sim_phase_ms().values())


def test_topo_sim_uses_rows_set_by_caller():
    """Rows replaced through set_rows (a new column layout) drive both delivery
    and potentiation of the next run."""
    cfg, model = CASES["hot-L16-blob"]
    t = rb.TopoNet(cfg)
    t.sim_init(model)
    t.run(100)
    n = cfg.L * cfg.L
    rng = np.random.default_rng(1)
    ln = rng.integers(0, cfg.cap + 1, n).astype(np.int32)
    ind = np.zeros((n, cfg.cap), np.int32)
    for i in range(n):
        ind[i, :ln[i]] = rng.choice(n, ln[i], replace=False)
    w = rng.uniform(0, 0.5, (n, cfg.cap)).astype(np.float32)
    t.set_rows(ln, ind, w)
    M = omodel(model, cfg.L)
    tp = tparams(cfg)
    for _ in range(5):
        P, S, t0 = snapshot(t, cfg, M)
        oracle.topo_run(cfg.seed, M, P, tp, S, t0, model.rewire_steps)
        t.run(model.rewire_steps)
        compare(t, cfg, M, P, S)


@pytest.mark.parametrize("name", ["hot-L16-blob", "paper-L64"])
def test_topo_sim_long_run_spike_counts(name):
    """Independent runs of 20000 steps (2 s of model time) from the same start:
    total spike counts agree within 1% (the input draws are shared, the
    floating-point state is not resynchronised).  paper-L64 is the benchmark's
    map: 64 x 64, the paper's parameters, the moving bar."""
    cfg, model = CASES[name]
    t = rb.TopoNet(cfg)
    t.sim_init(model)
    M = omodel(model, cfg.L)
    P, S, t0 = snapshot(t, cfg, M)
    oracle.topo_run(cfg.seed, M, P, tparams(cfg), S, t0, 20000)
    t.run(20000)
    g = int(t.sim_get(rb.TV_COUNT).sum())
    o = int(S.count.sum())
    assert o > 1000
    assert abs(g - o) <= 0.01 * o, (g, o)


def test_topo_sim_errors():
    # maps above 64 x 64 run on the tiled kernel only
    big = rb.TopoNet(rb.TopoConfig(L=72, cap=8, n_attempts=10, seed=1))
    big.sim_kernel(rb.TOPO_KERNEL_ONE_WG)
    with pytest.raises(RuntimeError, match="4096"):
        big.sim_init(rb.TopoModel())
    big.sim_kernel(rb.TOPO_KERNEL_AUTO)
    big.sim_init(rb.TopoModel())
    big.run(20)
    assert int(big.sim_get(rb.TV_STEP)[0]) == 20
    t = rb.TopoNet(rb.TopoConfig(L=8, cap=8, n_attempts=10, seed=1))
    with pytest.raises(RuntimeError, match="sim_init"):
        t.run(10)
    with pytest.raises(RuntimeError):
        t.sim_init(rb.TopoModel(tau_s=0.0))
    with pytest.raises(RuntimeError):
        t.sim_init(rb.TopoModel(stim_steps=0))
    t.sim_init(rb.TopoModel())
    with pytest.raises(RuntimeError, match="read-only"):
        t.sim_set(rb.TV_ZOUT, np.zeros(2, np.uint32))
    with pytest.raises(RuntimeError, match="negative"):
        t.sim_set(rb.TV_REF, np.full(64, -1, np.int32))
    t.run(25)
    assert int(t.sim_get(rb.TV_STEP)[0]) == 25
    ln, ind, w = t.get_rows()
    i = int(np.argmax(ln))
    ind[i, 1] = ind[i, 0]  # a target twice in one row
    with pytest.raises(RuntimeError, match="twice"):
        t.set_rows(ln, ind, w)
