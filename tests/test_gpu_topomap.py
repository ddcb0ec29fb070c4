"""GPU parity of topographic-map rewiring against the oracle: pairwise-Bernoulli
build and repeated connectivity updates, compared bit for bit from the same
pre-update rows."""
import numpy as np
import pytest

import oracle
from paper_2510_19764_amd import binding as rb
from paper_2510_19764_amd import workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def f32(x):
    return float(np.float32(x))


def oracle_proj(ln, ind, w, n, cap, pid):
    P = oracle.Proj(n, n, cap, False, pid)
    P.len[:] = ln
    P.ind[:] = ind.ravel()
    P.w[:] = w.ravel()
    return P


def tparams(cfg: rb.TopoConfig):
    return oracle.TopoParams(L=cfg.L, n_attempts=cfg.n_attempts, p_form=f32(cfg.p_form),
                             sigma_form=f32(cfg.sigma_form), g_theta=f32(cfg.g_theta),
                             p_elim_dep=f32(cfg.p_elim_dep), p_elim_pot=f32(cfg.p_elim_pot), g_new=f32(cfg.g_new))


CASES = {
    "small-L16": rb.TopoConfig(L=16, cap=12, n_attempts=120, proj_id=3, p_form=0.6, sigma_form=2.0, g_theta=0.1,
                               p_elim_dep=0.5, p_elim_pot=0.1, g_new=0.2, g_init=0.2, seed=7),
    "paper-ff-L64": rb.TopoConfig(L=64, cap=32, n_attempts=160, proj_id=0, p_form=0.16, sigma_form=2.5,
                                  g_theta=0.1, p_elim_dep=2.45e-2 * 50, p_elim_pot=1.36e-4 * 50, g_new=0.2,
                                  g_init=0.2, seed=9),
    "paper-lat-L64": rb.TopoConfig(L=64, cap=32, n_attempts=160, proj_id=1, p_form=1.0, sigma_form=1.0,
                                   g_theta=0.1, p_elim_dep=2.45e-2 * 50, p_elim_pot=1.36e-4 * 50, g_new=0.2,
                                   g_init=0.2, seed=9),
    "full-rows-L8": rb.TopoConfig(L=8, cap=4, n_attempts=300, proj_id=2, p_form=1.0, sigma_form=50.0,
                                  g_theta=0.1, p_elim_dep=0.0, p_elim_pot=0.0, g_new=0.2, g_init=0.2, seed=5),
    # more attempts than the one-launch form takes: the separate distribution launch
    "many-attempts-L32": rb.TopoConfig(L=32, cap=16, n_attempts=3000, proj_id=4, p_form=0.5, sigma_form=2.0,
                                       g_theta=0.1, p_elim_dep=0.3, p_elim_pot=0.05, g_new=0.2, g_init=0.2,
                                       seed=11),
}


@pytest.mark.parametrize("name", list(CASES))
def test_topo_build_matches_oracle(name):
    cfg = CASES[name]
    t = rb.TopoNet(cfg)
    ln, ind, w = t.get_rows()
    n = cfg.L * cfg.L
    P = oracle.Proj(n, n, cfg.cap, False, cfg.proj_id)
    oracle.gauss_rows(cfg.seed, P, cfg.L, f32(cfg.p_form), f32(cfg.sigma_form), f32(cfg.g_init))
    assert np.array_equal(ln, P.len)
    m = np.arange(cfg.cap)[None, :] < ln[:, None]
    assert np.array_equal(ind[m], P.ind.reshape(n, cfg.cap)[m])
    assert np.all(w[m] == np.float32(cfg.g_init))
    assert not t.get_bits().any()


@pytest.mark.parametrize("name", list(CASES))
def test_topo_rewire_bit_exact(name):
    cfg = CASES[name]
    t = rb.TopoNet(cfg)
    n = cfg.L * cfg.L
    rng = np.random.default_rng(cfg.seed)
    ln, ind, w = t.get_rows()
    # weights spread over [0, g_max] so both elimination probabilities occur
    w = rng.uniform(0.0, 0.2, w.shape).astype(np.float32)
    t.set_rows(ln, ind, w)
    tp = tparams(cfg)
    totals = np.zeros(3, np.int64)
    for step in range(0, 400, 10):
        ln0, ind0, w0 = t.get_rows()
        st = t.rewire(step)
        ln1, ind1, w1 = t.get_rows()
        P = oracle_proj(ln0, ind0, w0, n, cfg.cap, cfg.proj_id)
        ost, bits = oracle.topo_rewire(cfg.seed, P, tp, step)
        assert (st.eliminated, st.formed, st.blocked) == tuple(int(x) for x in ost[:3]), step
        assert np.array_equal(ln1, P.len), step
        m = np.arange(cfg.cap)[None, :] < ln1[:, None]
        assert np.array_equal(ind1[m], P.ind.reshape(n, cfg.cap)[m]), step
        assert np.array_equal(w1[m], P.w.reshape(n, cfg.cap)[m].astype(np.float32)), step
        assert not t.get_bits().any()
        totals += [st.eliminated, st.formed, st.blocked]
    assert totals.sum() > 0
    if name == "full-rows-L8":
        assert totals[2] > 0
