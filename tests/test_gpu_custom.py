"""Custom connectivity updates through the C-ABI (rs_eprop_custom_update,
rs_topo_custom_update): the paper's add_diagonal and remove_random examples
against the oracle, DEEP R and the topographic rule re-expressed on the
row-update interface bit-identical to the dedicated entry points, and a host
function changing a rule's per-row variable."""
import numpy as np
import pytest

import oracle
from gpu_harness import compare_rows_exact, gpu_input, oracle_net, real_slots, snapshot
from paper_2510_19764_amd import binding as rb
from paper_2510_19764_amd import workload as wl
from test_gpu_eprop import CASES, flip_some_signs, setup_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def records_equal(g, P, B, alif):
    cap = g["ind"].shape[1]
    m = real_slots(g)
    compare_rows_exact("rows", g, P)
    for name, arr in (("w", P.w), ("m", P.m), ("vv", P.v), ("G", P.G)):
        assert np.array_equal(g[name][m], arr.reshape(-1, cap)[m].astype(np.float32)), name
    assert np.array_equal(g["ebar"][m], P.ebar.reshape(-1, cap, B)[m].astype(np.float32))
    if alif:
        assert np.array_equal(g["eps"][m], P.eps.reshape(-1, cap, B)[m].astype(np.float32))


@pytest.mark.parametrize("name", ["alif-b64-col", "alif-b3-narrow"])
def test_add_diagonal_matches_oracle(name):
    base, _ = CASES[name]
    cfg = rb.EpropConfig(**{**base.__dict__, "deepr_mask": 2})  # the input projection has no bitfield
    net = rb.EpropNet(cfg)
    rates = wl.poisson_rates(cfg.seed, cfg.n_in, 150.0)
    raster = wl.poisson_raster(cfg.seed, rates, cfg.sample_steps, cfg.batch)
    labels = np.zeros(cfg.batch, np.int32)
    net.set_input(*gpu_input(raster, labels))
    net.step(10, rb.RS_LEARN)
    pre = snapshot(net)
    st = net.custom_update(0, rb.RULE_ADD_DIAGONAL, 0)
    post = snapshot(net)
    N = oracle_net(pre, cfg)
    added = oracle.add_diagonal(N.inp)
    assert st.formed == added > 0 and st.eliminated == 0
    records_equal(post["in"], N.inp, cfg.batch, cfg.alif)
    # the next steps use the new synapses (the column view followed them)
    net.step(5, rb.RS_LEARN)


@pytest.mark.parametrize("name", ["alif-b64-col", "lif-b256-col", "alif-b3-narrow"])
def test_remove_random_matches_oracle(name):
    cfg, net, raster, labels = setup_case(name)
    net.step(10, rb.RS_LEARN)
    pre = snapshot(net)
    step = 777
    st = net.custom_update(1, rb.RULE_REMOVE_RANDOM, step)
    post = snapshot(net)
    N = oracle_net(pre, cfg)
    post_ind = oracle.remove_random_targets(cfg.seed, N.rec, step)
    removed = oracle.remove_targets(N.rec, post_ind)
    assert st.eliminated == removed > 0 and st.formed == 0
    records_equal(post["rec"], N.rec, cfg.batch, cfg.alif)
    assert np.array_equal(post["rec"]["conn"].ravel(), N.rec.conn)


def test_host_function_chooses_the_targets():
    """remove_random with a host function that picks each row's first target
    instead: every row that has synapses loses the one in slot 0."""
    cfg, net, raster, labels = setup_case("alif-b64-col")
    net.step(10, rb.RS_LEARN)
    pre = snapshot(net)
    first = pre["rec"]["ind"][:, 0].astype(np.uint32)
    seen = {}

    def host(ln, post_ind, info):
        seen.update(info)
        assert np.array_equal(ln, pre["rec"]["len"])
        post_ind[:] = np.where(ln > 0, first, cfg.n_rec)  # n_rec: no target
    st = net.custom_update(1, rb.RULE_REMOVE_RANDOM, 5, host_fn=host)
    assert seen["rule"] == rb.RULE_REMOVE_RANDOM and seen["n_pre"] == cfg.n_rec and seen["step"] == 5
    N = oracle_net(pre, cfg)
    removed = oracle.remove_targets(N.rec, np.where(pre["rec"]["len"] > 0, first, cfg.n_rec))
    assert st.eliminated == removed == int((pre["rec"]["len"] > 0).sum())
    records_equal(snapshot(net)["rec"], N.rec, cfg.batch, cfg.alif)


@pytest.mark.parametrize("name", ["alif-b64-col", "alif-b3-narrow", "tiny-lif-b1", "alif-b64-dense"])
def test_deepr_on_the_interface_equals_rs_eprop_rewire(name):
    nets = []
    for _ in range(2):
        cfg, net, raster, labels = setup_case(name)
        net.step(20, rb.RS_LEARN)
        net.update()
        flip_some_signs(net, cfg, 0.15, cfg.seed)
        nets.append(net)
    a, b = nets
    step = a.info().step
    for p in (0, 1):
        sa = a.rewire(p)
        sb = b.custom_update(p, rb.RULE_DEEPR, step)
        assert (sa.eliminated, sa.formed, sa.attempts, sa.blocked) == \
               (sb.eliminated, sb.formed, sb.attempts, sb.blocked)
        assert sa.eliminated > 0 or (cfg.p_in if p == 0 else cfg.p_rec) == 0
    x, y = snapshot(a), snapshot(b)
    for tag in ("in", "rec"):
        for f in x[tag]:
            assert np.array_equal(x[tag][f], y[tag][f]), (tag, f)
    # and training continues alike
    a.step(10, rb.RS_LEARN)
    b.step(10, rb.RS_LEARN)
    assert np.array_equal(a.get(rb.V), b.get(rb.V))


@pytest.mark.parametrize("L,cap,att", [(16, 12, 40), (32, 32, 160), (20, 4, 300)])
def test_topo_rule_on_the_interface_equals_rs_topo_rewire(L, cap, att):
    cfg = rb.TopoConfig(L=L, cap=cap, n_attempts=att, proj_id=2, p_form=0.6, sigma_form=2.0, g_theta=0.1,
                        p_elim_dep=0.5, p_elim_pot=0.1, g_new=0.2, g_init=0.2, seed=L)
    a, b = rb.TopoNet(cfg), rb.TopoNet(cfg)
    rng = np.random.default_rng(L)
    ln, ind, w = a.get_rows()
    w = rng.uniform(0, 0.2, w.shape).astype(np.float32)
    a.set_rows(ln, ind, w)
    b.set_rows(ln, ind, w)
    tot = 0
    for s in range(0, 200, 10):
        sa = a.rewire(s)
        sb = b.custom_update(rb.RULE_TOPO, s)
        assert (sa.eliminated, sa.formed, sa.blocked, sa.attempts) == \
               (sb.eliminated, sb.formed, sb.blocked, sb.attempts), s
        tot += sa.eliminated + sa.formed
        for x, y in zip(a.get_rows(), b.get_rows()):
            assert np.array_equal(x, y), s
    assert tot > 0
    assert not b.get_bits().any()


def test_topo_rule_keeps_an_attached_simulation_consistent():
    """A custom rewire between simulation runs: the simulation's column view
    is rebuilt, so the run matches a map rewired by rs_topo_rewire."""
    cfg = rb.TopoConfig(L=16, cap=24, n_attempts=30, proj_id=0, g_theta=0.25, g_new=0.5, g_init=0.5, seed=8)
    model = rb.TopoModel(f_peak=600.0, g_max=0.5, A_plus=0.05, A_minus=0.02, rewire_steps=0)
    a, b = rb.TopoNet(cfg), rb.TopoNet(cfg)
    a.sim_init(model)
    b.sim_init(model)
    a.run(50)
    b.run(50)
    a.rewire(50)
    b.custom_update(rb.RULE_TOPO, 50)
    a.run(100)
    b.run(100)
    for var in (rb.TV_V, rb.TV_G, rb.TV_COUNT, rb.TV_X, rb.TV_Y):
        assert np.array_equal(a.sim_get(var), b.sim_get(var)), var
