"""Batched networks (rs_multi_*): a set of e-prop classifiers of different
sizes and densities trained together, through the C-ABI.  Every network of the
set ends bit-identical to the same network trained alone (rs_eprop_*), for
every e-prop schedule the tuner tries and for graph replay as for direct
launches; a reduced set matches the oracle (spike counts and rows exact,
weights within their bounds)."""
import numpy as np
import pytest

import oracle
from gpu_harness import (_adam_bounds, _carry, close, compare_rows_exact, gpu_input, oracle_net, real_slots,
                         snapshot)
from paper_2510_19764_amd import binding as rb
from paper_2510_19764_amd import workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def f32(x):
    return float(np.float32(x))


def member_cfg(n_rec, p, seed, n_in=60, n_out=4, B=1, T=50, U=25, alif=True, lr=1e-3):
    return rb.EpropConfig(n_in=n_in, n_rec=n_rec, n_out=n_out, batch=B, alif=alif, p_in=p, p_rec=p,
                          sigma_in=f32(wl.sigma_init(p, n_in)), sigma_rec=f32(wl.sigma_init(p, n_rec)),
                          sigma_out=f32(1.0 / np.sqrt(n_rec)), deepr_mask=3, update_interval=U, sample_steps=T,
                          seed=seed, lr=lr)


def member_input(cfg, rate=120.0):
    rates = wl.poisson_rates(cfg.seed, cfg.n_in, rate)
    raster = wl.poisson_raster(cfg.seed, rates, cfg.sample_steps, cfg.batch)
    labels = np.random.default_rng(cfg.seed).integers(0, cfg.n_out, cfg.batch).astype(np.int32)
    return raster, labels


SET = [(40, 0.3, 1), (300, 0.1, 2), (97, 0.2, 3), (1200, 0.05, 4), (25, 0.5, 5)]


def snap_member(getter, cfg, info):
    class View:
        pass
    v = View()
    v.cfg = cfg
    v.get = getter
    v.info = lambda: info
    return snapshot(v)


def same(a, b, where):
    for k in a:
        if isinstance(a[k], dict):
            for f in a[k]:
                assert np.array_equal(a[k][f], b[k][f]), (where, k, f)
        else:
            assert np.array_equal(a[k], b[k]), (where, k)


@pytest.mark.parametrize("B,alif", [(1, True), (3, False)])
def test_set_matches_networks_trained_alone(B, alif):
    """Seven samples: five tuning samples (each e-prop schedule once, direct
    launches) and two graph replays; every member equals the same network
    trained alone for the same samples, bit for bit."""
    cfgs = [member_cfg(n, p, s, B=B, alif=alif, lr=0.01) for n, p, s in SET]
    inputs = [member_input(c) for c in cfgs]
    m = rb.MultiNet(cfgs)
    dev = []
    for i, (raster, labels) in enumerate(inputs):
        d = gpu_input(raster, labels)
        dev.append(d)
        m.set_input(i, *d)
    n_samples = 7
    print("set of", len(cfgs), "networks:", n_samples, "samples", flush=True)
    m.train(n_samples)
    sch = m.schedule()
    assert sch["tuned"] and sch["samples"] == n_samples and all(t > 0 for t in sch["sample_ms"]), sch
    flags = rb.RS_LEARN | rb.RS_AUTO_UPDATE | rb.RS_AUTO_RESET
    for i, c in enumerate(cfgs):
        alone = rb.EpropNet(c)
        alone.set_input(*dev[i])
        alone.step(n_samples * c.sample_steps, flags)
        inf_a, inf_m = alone.info(), m.info(i)
        assert (inf_a.step, inf_a.adam_step, inf_a.spikes, inf_a.eliminated, inf_a.formed) == \
               (inf_m.step, inf_m.adam_step, inf_m.spikes, inf_m.eliminated, inf_m.formed), i
        assert inf_m.eliminated > 0 and inf_m.spikes > 0
        a = snapshot(alone)
        b = snap_member(lambda var, i=i: m.get(i, var), c, inf_m)
        same(a, b, f"network {i}")
        alone.close()
    m.close()


def test_graph_replay_equals_direct_launches():
    cfgs = [member_cfg(n, p, s, lr=0.01) for n, p, s in SET[:3]]
    snaps = []
    for graph in (True, False):
        m = rb.MultiNet(cfgs)
        refs = []
        for i, c in enumerate(cfgs):
            refs.append(gpu_input(*member_input(c)))
            m.set_input(i, *refs[-1])
        m.set_schedule(3, use_graph=graph)
        m.train(3)
        assert m.schedule()["graph"] == graph
        snaps.append([snap_member(lambda var, i=i: m.get(i, var), c, m.info(i)) for i, c in enumerate(cfgs)])
        m.close()
    for i in range(len(cfgs)):
        same(snaps[0][i], snaps[1][i], f"network {i}")


def test_reduced_set_matches_oracle():
    """One training sample of one update interval (T = U = 25: the update and
    both DEEP R rewires, then the reset) of three networks in one set, against
    the oracle running each network's steps, update, rewires and reset: spike
    counts exact, rows and bitfields bit for bit, weights and readout within
    the bounds the gradient's rounding allows through Adam."""
    cfgs = [member_cfg(n, p, s, T=25, U=25, lr=0.05) for n, p, s in SET[:3]]
    inputs = [member_input(c) for c in cfgs]
    m = rb.MultiNet(cfgs)
    m.set_schedule(1, use_graph=True)
    refs = []
    for i, (raster, labels) in enumerate(inputs):
        refs.append(gpu_input(raster, labels))
        m.set_input(i, *refs[-1])
    pre = [snap_member(lambda var, i=i: m.get(i, var), c, m.info(i)) for i, c in enumerate(cfgs)]
    m.train(1)
    for i, c in enumerate(cfgs):
        raster, labels = inputs[i]
        post = snap_member(lambda var, i=i: m.get(i, var), c, m.info(i))
        N = oracle_net(pre[i], c)
        counts = np.zeros((c.batch, c.n_rec), np.int64)
        for t in range(c.sample_steps):
            idx, off = raster.step_lists(t)
            N.step(idx, off, labels)
            counts += N.z
        assert np.array_equal(m.get(i, rb.ZCOUNT).astype(np.int64), counts), f"network {i}: spike counts"
        G = {tag: (P.G.reshape(-1, P.cap).copy(), P.Gabs.reshape(-1, P.cap).copy(), P.m.reshape(-1, P.cap).copy())
             for tag, P in (("in", N.inp), ("rec", N.rec))}
        ro = (N.Gout.copy(), N.Goutabs.copy(), N.Mout.copy())
        N.adam_update(1, lr=c.lr, b1=c.adam_b1, b2=c.adam_b2, eps=c.adam_eps, l1=c.l1, deepr_mask=c.deepr_mask)
        bounds = {}
        for tag, P, sig in (("in", N.inp, c.sigma_in), ("rec", N.rec, c.sigma_rec)):
            Gp, Ga, m_old = G[tag]
            ind = P.ind.reshape(-1, P.cap)
            words = P.sign.reshape(P.n_pre, -1)
            neg = (words[np.arange(P.n_pre)[:, None], ind >> 5] >> (ind & 31)) & 1
            g = Gp / c.batch + np.where(neg == 1, -c.l1, c.l1)
            bm, bv, bw = _adam_bounds(P, Gp, Ga, m_old, g, P.m.reshape(-1, P.cap), P.v.reshape(-1, P.cap),
                                      P.w.reshape(-1, P.cap), c, 1, sig)
            bounds[tag] = (P.len.copy(), ind.copy(), bw)
        _, _, bwo = _adam_bounds(None, ro[0], ro[1], ro[2], ro[0] / c.batch, N.Mout, N.Vout, N.Wout, c, 1,
                                 c.sigma_out)
        for tag, P in (("in", N.inp), ("rec", N.rec)):
            oracle.deepr_rewire(c.seed, P, c.sample_steps)
        N.reset()
        for tag, P in (("in", N.inp), ("rec", N.rec)):
            g = post[tag]
            compare_rows_exact(f"{i}.{tag}", g, P)
            assert np.array_equal(g["conn"].ravel(), P.conn) and np.array_equal(g["sign"].ravel(), P.sign)
            ln, ind, bw = bounds[tag]
            carried = _carry(bw, ln, ind, P.len, P.ind.reshape(-1, P.cap), P.n_post)
            close(f"{i}.{tag}.w", g["w"][real_slots(g)], P.w.reshape(-1, P.cap)[real_slots(g)], 0.0, bound=carried)
        close(f"{i}.Wout", post["Wout"], N.Wout, 0.0, bound=bwo)
        assert not post["v"].any() and not post["rec"]["ebar"].any()  # the reset
        assert m.info(i).eliminated > 0
    m.close()


def test_set_errors():
    a = member_cfg(40, 0.3, 1)
    with pytest.raises(rb.RagsnnError) as e:
        rb.MultiNet([a, rb.EpropConfig(**{**a.__dict__, "n_in": 61})])
    assert e.value.code == rb.RS_EINVAL
    with pytest.raises(rb.RagsnnError) as e:
        rb.MultiNet([rb.EpropConfig(**{**a.__dict__, "batch": 4})])
    assert e.value.code == rb.RS_EINVAL
    with pytest.raises(rb.RagsnnError) as e:
        rb.MultiNet([rb.EpropConfig(**{**a.__dict__, "sample_steps": 30})])
    assert e.value.code == rb.RS_EINVAL
    m = rb.MultiNet([a])
    with pytest.raises(rb.RagsnnError) as e:
        m.train(1)
    assert e.value.code == rb.RS_ESTATE
    import ctypes
    buf = np.zeros(a.n_rec, np.float64)
    assert rb.lib().rs_multi_get(m._h, 1, rb.V, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes) == rb.RS_EINVAL
    m.close()
