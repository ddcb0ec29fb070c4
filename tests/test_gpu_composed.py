"""Composed networks (rs_create / rs_add_pop / rs_add_proj / rs_build): the
e-prop classifier and the topographic map declared population by population
and projection by projection, their device memory taken from torch's caching
allocator, run bit-identical to the same models built by rs_eprop_create and
rs_topo_create; compositions no model implements are refused."""
import numpy as np
import pytest

from gpu_harness import gpu_input, snapshot
from paper_2510_19764_amd import binding as rb
from paper_2510_19764_amd import workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def f32(x):
    return float(np.float32(x))


def classifier_cfg():
    return rb.EpropConfig(n_in=60, n_rec=96, n_out=5, batch=64, alif=True, p_in=0.2, p_rec=0.2,
                          sigma_in=f32(wl.sigma_init(0.2, 60)), sigma_rec=f32(wl.sigma_init(0.2, 96)),
                          sigma_out=f32(1 / np.sqrt(96)), deepr_mask=2, l1=0.005, lr=0.02, update_interval=25,
                          sample_steps=100, seed=21)


def composed_classifier(cfg):
    net = rb.ComposedNet(seed=cfg.seed, allocator=True)
    src = net.add_pop(rb.POP_SPIKE_SOURCE, cfg.n_in)
    rec = net.add_pop(rb.POP_ALIF, cfg.n_rec, dt_ms=cfg.dt_ms, tau_mem_ms=cfg.tau_mem_ms,
                      tau_adapt_ms=cfg.tau_adapt_ms, v_thr=cfg.v_thr, beta=cfg.beta)
    out = net.add_pop(rb.POP_READOUT, cfg.n_out)
    opt = dict(learn=rb.LEARN_EPROP, lr=cfg.lr, update_interval=cfg.update_interval)
    net.add_proj(src, rec, init=rb.INIT_FIXED_PROB, p=cfg.p_in, sigma_w=cfg.sigma_in, **opt)
    net.add_proj(rec, rec, init=rb.INIT_FIXED_PROB, p=cfg.p_rec, sigma_w=cfg.sigma_rec, rewire=rb.REWIRE_DEEPR,
                 l1=cfg.l1, **opt)
    net.add_proj(rec, out, init=rb.INIT_DENSE, sigma_w=cfg.sigma_out, **opt)
    return net


def test_classifier_composed_equals_preset():
    cfg = classifier_cfg()
    rates = wl.poisson_rates(cfg.seed, cfg.n_in, 120.0)
    raster = wl.poisson_raster(cfg.seed, rates, cfg.sample_steps, cfg.batch)
    labels = np.random.default_rng(0).integers(0, cfg.n_out, cfg.batch).astype(np.int32)
    dev = gpu_input(raster, labels)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    net = composed_classifier(cfg)
    net.build(batch=cfg.batch, sample_steps=cfg.sample_steps)
    held = torch.cuda.memory_allocated() - before
    a = net.eprop(cfg)
    assert held >= a.info().device_bytes > 0  # every buffer from torch's allocator
    a.set_input(*dev)
    b = rb.EpropNet(cfg)
    b.set_input(*dev)
    flags = rb.RS_LEARN | rb.RS_AUTO_UPDATE | rb.RS_AUTO_RESET
    net.step(130, flags)
    b.step(130, flags)
    assert net.step_counter() == 130 and a.info().eliminated > 0
    sa, sb = snapshot(a), snapshot(b)
    for k in sa:
        if isinstance(sa[k], dict):
            for f in sa[k]:
                assert np.array_equal(sa[k][f], sb[k][f]), (k, f)
        else:
            assert np.array_equal(sa[k], sb[k]), k
    st = net.rewire(1)
    assert st.eliminated == st.attempts
    net.close()
    b.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before == 0  # returned at destroy


def test_topomap_composed_equals_preset():
    cfg = rb.TopoConfig(L=16, cap=24, n_attempts=20, proj_id=0, g_theta=0.25, g_new=0.5, g_init=0.5, seed=3)
    model = rb.TopoModel(f_peak=600.0, g_max=0.5, A_plus=0.05, A_minus=0.02, stim_kind=rb.STIM_BAR, stim_steps=50)
    net = rb.ComposedNet(seed=cfg.seed, allocator=True)
    src = net.add_pop(rb.POP_POISSON_SHEET, cfg.L * cfg.L, L=cfg.L, model=model)
    tgt = net.add_pop(rb.POP_COND_LIF_SHEET, cfg.L * cfg.L, L=cfg.L, model=model)
    net.add_proj(src, tgt, init=rb.INIT_GAUSS_TORUS, p_form=cfg.p_form, sigma_form=cfg.sigma_form,
                 g_init=cfg.g_init, cap=cfg.cap, learn=rb.LEARN_STDP, rewire=rb.REWIRE_TOPO,
                 n_attempts=cfg.n_attempts, g_theta=cfg.g_theta, p_elim_dep=cfg.p_elim_dep,
                 p_elim_pot=cfg.p_elim_pot, g_new=cfg.g_new, update_interval=model.rewire_steps)
    net.build()
    a = net.topo(cfg)
    b = rb.TopoNet(cfg)
    b.sim_init(model)
    net.step(700)
    b.run(700)
    for var in (rb.TV_V, rb.TV_G, rb.TV_Y, rb.TV_X, rb.TV_REF, rb.TV_COUNT, rb.TV_ZIN, rb.TV_ZOUT, rb.TV_STEP):
        assert np.array_equal(a.sim_get(var), b.sim_get(var)), var
    for x, y in zip(a.get_rows(), b.get_rows()):
        assert np.array_equal(x, y)
    assert a.sim_get(rb.TV_COUNT).sum() > 0
    net.close()
    b.close()


def test_topomap_with_lateral_composed_equals_preset():
    """A map with a lateral projection (target sheet onto itself, Tab. G lateral
    formation rule) built from descriptors equals rs_topo_add_lateral's, bit for
    bit, on the tiled kernel with the input replicated in 16 x 16 squares."""
    cfg = rb.TopoConfig(L=32, cap=24, n_attempts=40, proj_id=0, g_theta=0.25, g_new=0.5, g_init=0.5, seed=4)
    lcfg = rb.TopoConfig(L=32, cap=16, n_attempts=40, proj_id=1, p_form=1.0, sigma_form=1.0, g_theta=0.25,
                         g_new=0.5, g_init=0.5, seed=4)
    model = rb.TopoModel(f_peak=600.0, g_max=0.5, A_plus=0.05, A_minus=0.02, stim_tile=16)
    net = rb.ComposedNet(seed=cfg.seed, allocator=True)
    src = net.add_pop(rb.POP_POISSON_SHEET, cfg.L * cfg.L, L=cfg.L, model=model)
    tgt = net.add_pop(rb.POP_COND_LIF_SHEET, cfg.L * cfg.L, L=cfg.L, model=model)
    common = dict(init=rb.INIT_GAUSS_TORUS, learn=rb.LEARN_STDP, rewire=rb.REWIRE_TOPO,
                  update_interval=model.rewire_steps)
    net.add_proj(src, tgt, p_form=cfg.p_form, sigma_form=cfg.sigma_form, g_init=cfg.g_init, cap=cfg.cap,
                 n_attempts=cfg.n_attempts, g_theta=cfg.g_theta, p_elim_dep=cfg.p_elim_dep,
                 p_elim_pot=cfg.p_elim_pot, g_new=cfg.g_new, **common)
    net.add_proj(tgt, tgt, p_form=lcfg.p_form, sigma_form=lcfg.sigma_form, g_init=lcfg.g_init, cap=lcfg.cap,
                 n_attempts=lcfg.n_attempts, g_theta=lcfg.g_theta, p_elim_dep=lcfg.p_elim_dep,
                 p_elim_pot=lcfg.p_elim_pot, g_new=lcfg.g_new, **common)
    net.build()
    a = net.topo(cfg, lcfg)
    b = rb.TopoNet(cfg)
    b.add_lateral(lcfg)
    b.sim_init(model)
    net.step(700)
    b.run(700)
    for var in (rb.TV_V, rb.TV_G, rb.TV_Y, rb.TV_X, rb.TV_XLAT, rb.TV_REF, rb.TV_COUNT, rb.TV_ZIN, rb.TV_ZOUT,
                rb.TV_STEP):
        assert np.array_equal(a.sim_get(var), b.sim_get(var)), var
    for lateral in (False, True):
        for x, y in zip(a.get_rows(lateral=lateral), b.get_rows(lateral=lateral)):
            assert np.array_equal(x, y)
    assert a.sim_get(rb.TV_COUNT).sum() > 0
    st = net.rewire(1)  # the lateral projection through the generic call
    assert st.attempts == lcfg.n_attempts
    net.close()
    b.close()


def test_unsupported_compositions_are_refused():
    cfg = classifier_cfg()
    net = rb.ComposedNet(seed=1, allocator=False)
    s = net.add_pop(rb.POP_SPIKE_SOURCE, 10)
    r = net.add_pop(rb.POP_LIF, 20)
    net.add_proj(s, r, init=rb.INIT_FIXED_PROB, p=0.1, sigma_w=0.3, learn=rb.LEARN_EPROP, update_interval=25)
    with pytest.raises(rb.RagsnnError) as e:
        net.build()  # no readout
    assert e.value.code == rb.RS_EINVAL and "readout" in str(e.value)
    net.close()
    net = composed_classifier(cfg)
    net.add_pop(rb.POP_LIF, 5)
    with pytest.raises(rb.RagsnnError) as e:
        net.build(batch=4)
    assert e.value.code == rb.RS_EINVAL
    net.close()
