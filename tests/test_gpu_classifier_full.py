"""Parity at the full sparse-classifier size (700 inputs, 1024 ALIF, 20
readouts, 10% connectivity, batch 256): 120 steps in the schedule the
benchmark times (blocks of 10, 30, 30 and 30 steps per update interval
through the two-stream hand-off ring, the
automatic Adam update and both DEEP R rewires inside the call, the column view
rebuilt beside the next forward block) compared element by element with the
oracle; single full-size steps; DEEP R bit-exact on the full rows; invariants
after a complete training interval; and a whole training batch run twice."""
import numpy as np
import pytest

import oracle
from gpu_harness import (MARGINS, compare_state, gpu_input, interval_vs_oracle, oracle_net, oracle_step_resync,
                         real_slots, snapshot)
from paper_2510_19764_amd import binding as rb
from paper_2510_19764_amd import workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def classifier_cfg():
    c = wl.SHD_CLASSIFIER
    f32 = lambda x: float(np.float32(x))
    return rb.EpropConfig(n_in=c["n_in"], n_rec=c["n_rec"], n_out=c["n_out"], batch=c["batch"], alif=True,
                          p_in=c["p_in"], p_rec=c["p_rec"], sigma_in=f32(wl.sigma_init(c["p_in"], c["n_in"])),
                          sigma_rec=f32(wl.sigma_init(c["p_rec"], c["n_rec"])),
                          sigma_out=f32(1.0 / np.sqrt(c["n_rec"])), deepr_mask=c["deepr_mask"], l1=c["l1"],
                          lr=c["lr"], update_interval=c["update_interval"], sample_steps=c["T"], seed=1)


@pytest.fixture(scope="module")
def setup():
    cfg = classifier_cfg()
    labels, raster = wl.ShdLike().batch(seed=1, batch_index=0, B=cfg.batch)
    net = rb.EpropNet(cfg)
    dev = gpu_input(raster, labels)
    net.set_input(*dev)
    yield cfg, net, raster, labels, dev
    net.close()


def test_full_size_step_matches_oracle(setup):
    cfg, net, raster, labels, _ = setup
    print("classifier full size: warm-up 40 steps", flush=True)
    net.step(40, rb.RS_LEARN)
    for t in (40, 41):
        pre = snapshot(net)
        net.step(1, rb.RS_LEARN)
        post = snapshot(net)
        N = oracle_net(pre, cfg)
        oracle_step_resync(N, raster, t, labels, post["z"])
        compare_state(post, N, cfg)
    assert int(post["z"].sum()) > 0


def test_full_size_update_and_rewire_bit_exact(setup):
    cfg, net, raster, labels, _ = setup
    net.update()
    rng = np.random.default_rng(0)
    w = net.get(rb.PROJ(1, rb.P_W))
    w[rng.random(w.shape) < 0.05] *= -1
    net.set(rb.PROJ(1, rb.P_W), w)
    pre = snapshot(net)
    step = net.info().step
    st = net.rewire(1)
    post = snapshot(net)
    N = oracle_net(pre, cfg)
    dormant, ost = oracle.deepr_rewire(cfg.seed, N.rec, step)
    assert (st.eliminated, st.formed) == (int(ost[0]), int(ost[1])) and st.eliminated > 1000
    g = post["rec"]
    cap = g["ind"].shape[1]
    m = real_slots(g)
    assert np.array_equal(g["len"], N.rec.len)
    assert np.array_equal(g["ind"][m], N.rec.ind.reshape(-1, cap)[m])
    assert np.array_equal(g["w"][m], N.rec.w.reshape(-1, cap)[m].astype(np.float32))
    assert np.array_equal(g["eps"][m], N.rec.eps.reshape(-1, cap, cfg.batch)[m].astype(np.float32))
    assert np.array_equal(g["ebar"][m], N.rec.ebar.reshape(-1, cap, cfg.batch)[m].astype(np.float32))
    assert np.array_equal(g["conn"].ravel(), N.rec.conn)


def test_full_training_interval_invariants(setup):
    cfg, net, raster, labels, _ = setup
    lens0 = [int(net.get(rb.PROJ(p, rb.P_LEN)).sum()) for p in (0, 1)]
    net.reset()
    s0 = net.info().step
    # advance to the next interval boundary, then one full interval with update + rewire
    net.step(int(cfg.update_interval - s0 % cfg.update_interval) + cfg.update_interval,
             rb.RS_LEARN | rb.RS_AUTO_UPDATE | rb.RS_AUTO_RESET)
    for p in (0, 1):
        ln = net.get(rb.PROJ(p, rb.P_LEN))
        ind = net.get(rb.PROJ(p, rb.P_IND))
        assert int(ln.sum()) == lens0[p]
        for i in range(0, ln.size, 37):
            row = ind[i, :ln[i]]
            assert len(np.unique(row)) == row.size
    y = net.get(rb.Y)
    assert np.isfinite(y).all()


def test_full_batch_training_deterministic():
    """One whole training batch (1000 steps, 10 updates, 20 DEEP R rewires and
    the reset) at the full size, in the benchmark's schedule, twice from the
    same seed: bit-identical state, constant synapse counts, finite values."""
    cfg = classifier_cfg()
    labels, raster = wl.ShdLike().batch(seed=1, batch_index=0, B=cfg.batch)
    flags = rb.RS_LEARN | rb.RS_AUTO_UPDATE | rb.RS_AUTO_RESET
    snaps = []
    for rep in range(2):
        net = rb.EpropNet(cfg)
        net.set_input(*gpu_input(raster, labels))
        lens0 = [int(net.get(rb.PROJ(p, rb.P_LEN)).sum()) for p in (0, 1)]
        net.step(cfg.sample_steps, flags)
        inf = net.info()
        assert inf.adam_step == cfg.sample_steps // cfg.update_interval
        assert inf.eliminated == inf.formed
        s = snapshot(net)
        for p, tag in ((0, "in"), (1, "rec")):
            assert int(s[tag]["len"].sum()) == lens0[p]
            m = real_slots(s[tag])
            for k in ("w", "m", "vv", "G"):
                assert np.isfinite(s[tag][k][m]).all(), (tag, k)
        for k in ("Wout", "bout", "Mout", "Vout"):
            assert np.isfinite(s[k]).all(), k
        snaps.append(s)
        net.close()
    a, b = snaps
    for k in a:
        if isinstance(a[k], dict):
            for f in a[k]:
                assert np.array_equal(a[k][f], b[k][f]), (k, f)
        else:
            assert np.array_equal(a[k], b[k]), k


def test_full_size_interval_in_bench_schedule():
    """From the update boundary at step 100, one call of 100 steps with
    RS_LEARN | RS_AUTO_UPDATE and the default block lengths (10, 30, 30 and
    30 steps through the two-stream ring, the update and both rewires at step
    200, the column view rebuilt beside the next block), against the oracle's
    100 steps, Adam update and two rewires from the same snapshot: spike
    counts and the last block's raster exact, rows, bitfields and dormant
    counts bit for bit, state and parameters within their bounds.  Then 20
    more steps past the boundary from the GPU's updated state."""
    cfg = classifier_cfg()
    labels, raster = wl.ShdLike().batch(seed=1, batch_index=0, B=cfg.batch)
    net = rb.EpropNet(cfg)
    net.set_input(*gpu_input(raster, labels))
    net.step(cfg.update_interval, rb.RS_LEARN | rb.RS_AUTO_UPDATE)
    info = net.info()
    assert (info.first_block, info.trace_block) == (10, 30)
    print("classifier full size: 100 + 20 steps against the oracle", flush=True)
    assert interval_vs_oracle(net, cfg, raster, labels, 100, after=20) == 1
    print("worst error / bound:", {k: round(v, 3) for k, v in sorted(MARGINS.items())}, flush=True)
    net.close()
