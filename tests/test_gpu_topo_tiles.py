"""GPU parity of the tiled topographic-map simulation (one workgroup per 256
targets, a device-wide barrier per step) against the oracle, with and without
the lateral projection, on maps of one tile, several tiles with a ragged last
one, the 64 x 64 benchmark map and the paper's largest scaled map (s = 7,
112 x 112, input replicated in every 16 x 16 square).

Lockstep protocol as for the one-workgroup kernel: before every rewiring
interval the oracle takes the GPU's rows and state, both run the interval
(its steps, then the feed-forward and lateral rewires), and the results are
compared: spikes, refractory counts, input draws, rewire counts and row
structure exactly; voltages, conductances, traces and weights within 1e-5 of
max(|oracle|, scale of the variable).
"""
import numpy as np
import pytest

import oracle
from paper_2510_19764_amd import binding as rb
from test_gpu_topo_sim import close, f32, tparams, unpack

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def omodel(m: rb.TopoModel, L: int) -> oracle.TopoModel:
    kw = {}
    for k in ("h", "C_m", "tau_m", "V_rest", "E_exc", "V_th", "V_reset", "tau_s", "f_base", "f_peak",
              "sigma_stim", "g_max", "A_plus", "A_minus", "tau_plus", "tau_minus"):
        kw[k] = f32(getattr(m, k))
    for k in ("ref_steps", "stim_steps", "stim_kind", "stdp", "rewire_steps", "stim_tile"):
        kw[k] = int(getattr(m, k))
    return oracle.TopoModel(L=L, **kw)


def oproj(t, cfg, lateral):
    n = cfg.L * cfg.L
    c = t.lat_cfg if lateral else cfg
    ln, ind, w = t.get_rows(lateral=lateral)
    P = oracle.Proj(n, n, c.cap, False, c.proj_id)
    P.len[:] = ln
    P.ind[:] = ind.ravel()
    P.w[:] = w.ravel()
    return P


def snapshot(t, cfg, M, lateral):
    n = cfg.L * cfg.L
    P = oproj(t, cfg, False)
    PL = oproj(t, cfg, True) if lateral else None
    S = oracle.TopoState(M)
    S.V[:] = t.sim_get(rb.TV_V)
    S.g[:] = t.sim_get(rb.TV_G)
    S.y[:] = t.sim_get(rb.TV_Y)
    S.x[:] = t.sim_get(rb.TV_X)
    if lateral:
        S.xl[:] = t.sim_get(rb.TV_XLAT)
    S.ref[:] = t.sim_get(rb.TV_REF)
    S.count[:] = t.sim_get(rb.TV_COUNT).astype(np.int32)
    S.zin[:] = unpack(t.sim_get(rb.TV_ZIN), n)
    S.zout[:] = unpack(t.sim_get(rb.TV_ZOUT), n)
    return P, PL, S, int(t.sim_get(rb.TV_STEP)[0])


def compare_rows(t, cfg, P, lateral, g_max):
    n = cfg.L * cfg.L
    cap = (t.lat_cfg if lateral else cfg).cap
    ln, ind, w = t.get_rows(lateral=lateral)
    assert np.array_equal(ln, P.len), "lateral len" if lateral else "len"
    m = np.arange(cap)[None, :] < ln[:, None]
    assert np.array_equal(ind[m], P.ind.reshape(n, cap)[m])
    close("w_lat" if lateral else "w", w[m], P.w.reshape(n, cap)[m], g_max)


def compare(t, cfg, M, P, PL, S):
    n = cfg.L * cfg.L
    compare_rows(t, cfg, P, False, M.g_max)
    if PL is not None:
        compare_rows(t, cfg, PL, True, M.g_max)
        close("xl", t.sim_get(rb.TV_XLAT), S.xl, 1.0)
    assert np.array_equal(unpack(t.sim_get(rb.TV_ZOUT), n), S.zout)
    assert np.array_equal(unpack(t.sim_get(rb.TV_ZIN), n), S.zin)
    assert np.array_equal(t.sim_get(rb.TV_COUNT).astype(np.int64), S.count)
    assert np.array_equal(t.sim_get(rb.TV_REF), S.ref)
    close("V", t.sim_get(rb.TV_V), S.V, abs(M.V_rest))
    close("g", t.sim_get(rb.TV_G), S.g, M.g_max)
    close("x", t.sim_get(rb.TV_X), S.x, 1.0)
    close("y", t.sim_get(rb.TV_Y), S.y, 1.0)


HOT = dict(f_peak=600.0, g_max=0.5, A_plus=0.05, A_minus=0.05 * 1.2 * 20.0 / 64.0)


def ff(L, cap=32, attempts=10, seed=3, **kw):
    base = dict(L=L, cap=cap, n_attempts=attempts, proj_id=0, g_theta=0.25, g_new=0.5, g_init=0.5, seed=seed)
    base.update(kw)
    return rb.TopoConfig(**base)


def lat(L, cap=16, attempts=10, **kw):
    """The lateral rule of Tab. G: p_form-lat 1, sigma_form-lat 1."""
    base = dict(L=L, cap=cap, n_attempts=attempts, proj_id=1, p_form=1.0, sigma_form=1.0, g_theta=0.25,
                g_new=0.5, g_init=0.5)
    base.update(kw)
    return rb.TopoConfig(**base)


# name: (feed-forward config, lateral config or None, model, intervals)
CASES = {
    # one tile, the one-workgroup kernel's test map
    "ff-L16": (ff(16), None, rb.TopoModel(**HOT), 30),
    # two tiles, the second ragged (400 = 256 + 144), bar stimulus, capacity 40
    "ff-L20-bar": (ff(20, cap=40, attempts=40, seed=4, proj_id=2), None,
                   rb.TopoModel(stim_kind=rb.STIM_BAR, stim_steps=50, **HOT), 30),
    # 36 neurons in one partial tile; bit words end mid-word
    "ff-L6": (ff(6, cap=8, attempts=5, seed=12, p_form=0.6, sigma_form=1.5), None,
              rb.TopoModel(f_base=200.0, f_peak=600.0, g_max=0.5, A_plus=0.05, A_minus=0.02, stim_steps=30,
                           ref_steps=7, rewire_steps=3), 40),
    # the benchmark's map on 16 tiles
    "ff-L64-bar": (ff(64, attempts=160, seed=10), None, rb.TopoModel(stim_kind=rb.STIM_BAR, stim_steps=50, **HOT),
                   10),
    # lateral projection, one tile
    "lat-L16": (ff(16, seed=5), lat(16), rb.TopoModel(**HOT), 30),
    # lateral, two tiles, ragged
    "lat-L20-bar": (ff(20, cap=40, attempts=40, seed=6), lat(20, cap=20, attempts=20, proj_id=3),
                    rb.TopoModel(stim_kind=rb.STIM_BAR, stim_steps=50, **HOT), 25),
    # s = 3 scaled map: input replicated in 16 x 16 squares, 9 tiles
    "lat-L48-tiled-input": (ff(48, attempts=90, seed=7), lat(48, attempts=90),
                            rb.TopoModel(stim_tile=16, **HOT), 12),
    # the paper's model at s = 7 (112 x 112, 49 tiles): its parameters, 490 attempts per projection
    "paper-L112": (rb.TopoConfig(L=112, cap=32, n_attempts=490, proj_id=0, seed=9),
                   rb.TopoConfig(L=112, cap=32, n_attempts=490, proj_id=1, p_form=1.0, sigma_form=1.0),
                   rb.TopoModel(stim_tile=16), 20),
}


def run_lockstep(cfg, lcfg, model, n_chunks, kernel=rb.TOPO_KERNEL_TILED):
    t = rb.TopoNet(cfg)
    if lcfg is not None:
        t.add_lateral(lcfg)
    t.sim_kernel(kernel)
    t.sim_init(model)
    M = omodel(model, cfg.L)
    tp = tparams(cfg)
    tpl = tparams(lcfg) if lcfg is not None else None
    R = model.rewire_steps
    spikes = changed = changed_l = 0
    for _ in range(n_chunks):
        P, PL, S, t0 = snapshot(t, cfg, M, lcfg is not None)
        if lcfg is None:
            stats = oracle.topo_run(cfg.seed, M, P, tp, S, t0, R)
        else:
            stats, stats_l = oracle.topo_run(cfg.seed, M, P, tp, S, t0, R, PL=PL, tpl=tpl)
        t.run(R)
        st = t.run_stats()
        assert (st.eliminated, st.formed, st.blocked) == tuple(stats[:3])
        changed += st.eliminated + st.formed
        if lcfg is not None:
            sl = t.run_stats(lateral=True)
            assert (sl.eliminated, sl.formed, sl.blocked) == tuple(stats_l[:3])
            changed_l += sl.eliminated + sl.formed
        compare(t, cfg, M, P, PL, S)
        spikes = int(S.count.sum())
    return t, spikes, changed, changed_l


@pytest.mark.parametrize("name", list(CASES))
def test_tiled_lockstep_matches_oracle(name):
    cfg, lcfg, model, n_chunks = CASES[name]
    print(f"[tiles] {name}", flush=True)
    t, spikes, changed, changed_l = run_lockstep(cfg, lcfg, model, n_chunks)
    assert spikes > 0
    assert changed > 0
    if lcfg is not None:
        assert changed_l > 0
    t.close()


def test_graph_replay_equals_direct_launches():
    """64 whole rewiring intervals replayed from the recorded graph (tiled
    kernel, lateral projection) give the state of interval-by-interval calls
    bit for bit."""
    cfg, lcfg, model, _ = CASES["lat-L48-tiled-input"]
    nets = []
    for _ in range(2):
        t = rb.TopoNet(cfg)
        t.add_lateral(lcfg)
        t.sim_init(model)  # AUTO: the lateral projection selects the tiled kernel
        nets.append(t)
    R = model.rewire_steps
    nets[0].run(R * 64)
    for _ in range(64):
        nets[1].run(R)
    for var in (rb.TV_V, rb.TV_G, rb.TV_Y, rb.TV_X, rb.TV_XLAT, rb.TV_REF, rb.TV_COUNT, rb.TV_ZIN, rb.TV_ZOUT,
                rb.TV_STEP):
        assert np.array_equal(nets[0].sim_get(var), nets[1].sim_get(var)), var
    for lateral in (False, True):
        a, b = nets[0].get_rows(lateral=lateral), nets[1].get_rows(lateral=lateral)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    assert int(nets[0].sim_get(rb.TV_COUNT).sum()) > 0


def test_kernel_choice_and_limits():
    """AUTO keeps the one-workgroup kernel for small maps without a lateral
    projection; the one-workgroup kernel refuses a lateral projection; the
    lateral projection must come before the simulation and needs its own id."""
    t = rb.TopoNet(ff(16))
    with pytest.raises(rb.RagsnnError):
        t.add_lateral(lat(16, proj_id=0))
    t.add_lateral(lat(16))
    with pytest.raises(rb.RagsnnError):
        t.add_lateral(lat(16))
    with pytest.raises(rb.RagsnnError):
        t.sim_kernel(rb.TOPO_KERNEL_ONE_WG)
        t.sim_init(rb.TopoModel())
    t.close()
    t = rb.TopoNet(ff(16))
    t.sim_init(rb.TopoModel())
    with pytest.raises(rb.RagsnnError):
        t.add_lateral(lat(16))
    with pytest.raises(rb.RagsnnError):
        t.sim_init(rb.TopoModel(stim_tile=5))
    t.close()
