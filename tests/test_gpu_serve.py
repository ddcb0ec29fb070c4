"""Served inference (rs_serve_*) through the C-ABI: continuous batching of
classification requests on trained networks of different sizes.  Each
request's result (sum over steps of the softmax, its argmax, spike and event
counts) is identical whether it runs alone or among others, matches the
oracle, and admission follows the memory budget."""
import numpy as np
import pytest

import oracle
from gpu_harness import close, oracle_net, snapshot
from paper_2510_19764_amd import binding as rb
from paper_2510_19764_amd import workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def f32(x):
    return float(np.float32(x))


def model_cfg(n_rec, seed, n_in=60, n_out=4, p=0.15):
    return rb.EpropConfig(n_in=n_in, n_rec=n_rec, n_out=n_out, batch=1, alif=True, p_in=p, p_rec=p,
                          sigma_in=f32(2.0 * wl.sigma_init(p, n_in)), sigma_rec=f32(wl.sigma_init(p, n_rec)),
                          sigma_out=f32(1.0 / np.sqrt(n_rec)), update_interval=0, sample_steps=1000, seed=seed)


SIZES = [(96, 1), (250, 2), (700, 3)]


@pytest.fixture(scope="module")
def models():
    ms = [rb.EpropNet(model_cfg(n, s)) for n, s in SIZES]
    yield ms
    for m in ms:
        m.close()


def raster_pool(n, T=160, n_in=60, seed=7):
    pool = []
    for q in range(n):
        rates = wl.poisson_rates(seed + q, n_in, 150.0)
        r = wl.poisson_raster(seed + q, rates, T, 1)
        pool.append((r, torch.tensor(r.off, dtype=torch.int32, device="cuda"),
                     torch.tensor(r.idx if r.idx.size else np.zeros(1, np.int32), dtype=torch.int32, device="cuda")))
    return pool


def requests(n, seed=3):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(0, len(SIZES))), int(rng.integers(0, 8)), int(rng.integers(25, 200)))
            for _ in range(n)]


def run_all(server, pool, reqs, T=160):
    tickets = [server.submit(m, pool[p][1], pool[p][2], T, n) for m, p, n in reqs]
    assert all(t is not None for t in tickets)
    out = {}
    while len(out) < len(reqs):
        server.step()
        for r in server.poll():
            out[r["ticket"]] = r
    return [out[t] for t in tickets]


def test_results_same_alone_and_in_the_mix(models):
    pool = raster_pool(8)
    reqs = requests(40)
    mix = rb.Server(models, slots_per_model=16, block_steps=20, max_running=48)
    res_mix = run_all(mix, pool, reqs)
    st = mix.stats()
    assert st["completed"] == len(reqs) and st["running"] == 0 and st["queued"] == 0
    mix.close()
    alone = rb.Server(models, slots_per_model=1, block_steps=20, max_running=1)
    for q, rq in enumerate(reqs):
        (r,) = run_all(alone, pool, [rq])
        a, b = r, res_mix[q]
        assert (a["decision"], a["spikes"], a["events"], a["steps"]) == \
               (b["decision"], b["spikes"], b["events"], b["steps"]), q
        assert np.array_equal(a["scores"], b["scores"]), q
    alone.close()
    assert sum(r["spikes"] for r in res_mix) > 0


def test_results_match_oracle(models):
    """Each request against the oracle's forward pass of the same model and
    input (state reset, no learning): spike counts exact, the summed softmax
    within 1e-5 of its value per step summed."""
    pool = raster_pool(4)
    reqs = [(0, 0, 60), (1, 1, 120), (2, 2, 90), (2, 3, 33)]
    srv = rb.Server(models, slots_per_model=4, block_steps=16, max_running=8)
    res = run_all(srv, pool, reqs)
    srv.close()
    for (mi, pi, n), r in zip(reqs, res):
        cfg = models[mi].cfg
        N = oracle_net(snapshot(models[mi]), cfg)
        N.reset()
        raster = pool[pi][0]
        score = np.zeros(cfg.n_out)
        spikes = 0
        for t in range(n):
            idx, off = raster.step_lists(t % raster.T)
            N.step(idx, off, np.array([-1], np.int32), learn=False)
            score += N.delta[0]  # no target: delta is the softmax itself
            spikes += int(N.z.sum())
        assert r["spikes"] == spikes
        close("score", r["scores"][:cfg.n_out], score, 0.0, bound=1e-5 * n)
        assert r["decision"] == int(np.argmax(score))


def test_admission_follows_the_budget(models):
    pool = raster_pool(2)
    probe = rb.Server(models, slots_per_model=2, block_steps=20)
    probe.submit(2, pool[0][1], pool[0][2], 160, 100)
    probe.step()  # one block: the request is still running
    fp = probe.stats()["state_bytes_used"]  # one request of the largest model
    assert fp > 0
    probe.close()
    srv = rb.Server(models, slots_per_model=8, block_steps=20, max_running=64, max_queue=4,
                    state_budget_bytes=2 * fp + fp // 2)
    tickets = [srv.submit(2, pool[0][1], pool[0][2], 160, 100) for _ in range(4)]
    assert all(t is not None for t in tickets)
    assert srv.submit(2, pool[0][1], pool[0][2], 160, 100) is None  # queue full: rejected
    srv.step()
    st = srv.stats()
    assert st["rejected"] == 1 and st["running"] == 2 and st["queued"] == 2
    assert st["state_bytes_used"] == 2 * fp
    done = []
    while len(done) < 4:
        srv.step()
        st = srv.stats()
        assert st["running"] <= 2 and st["state_bytes_used"] <= st["state_budget_bytes"]
        done += srv.poll()
    assert sorted(r["ticket"] for r in done) == sorted(tickets)
    srv.close()
    tight = rb.Server(models, slots_per_model=8, state_budget_bytes=1024)
    assert tight.submit(0, pool[0][1], pool[0][2], 160, 10) is None  # never fits
    assert tight.stats()["rejected"] == 1
    tight.close()


def test_replay_of_a_trace(models):
    pool = raster_pool(4)
    rng = np.random.default_rng(11)
    n = 60
    arrivals = np.cumsum(rng.exponential(1 / 2000.0, n))
    ms = rng.integers(0, len(SIZES), n)
    lens = rng.integers(25, 150, n)
    rasters = [(pool[q % 4][1], pool[q % 4][2], 160) for q in range(n)]
    srv = rb.Server(models, slots_per_model=32, block_steps=20, max_running=96)
    lat, dec, spk = srv.replay(arrivals, ms, lens, rasters)
    assert (lat > 0).all() and (dec >= 0).all()
    # the same requests in a mix without timing: identical decisions and spikes
    res = run_all(srv, pool, [(int(ms[q]), q % 4, int(lens[q])) for q in range(n)])
    assert [r["decision"] for r in res] == dec.tolist()
    assert [r["spikes"] for r in res] == spk.tolist()
    srv.close()
