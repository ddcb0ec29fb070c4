"""GPU parity of the Poisson input source against the oracle's, through the
C-ABI: lockstep single steps and whole trace blocks with one shared rate table
and with one table per instance, the edge rates, the equivalence of a device
source with a raster holding the same spikes, and argument errors."""
import numpy as np
import pytest

import oracle
from gpu_harness import compare_state, gpu_input, oracle_net, oracle_step_resync, snapshot
from paper_2510_19764_amd import binding as rb
from paper_2510_19764_amd import workload as wl
from test_gpu_eprop import CASES

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


class PoissonLists:
    """The oracle's input lists of absolute step t, in the raster interface."""

    def __init__(self, seed, thr, B):
        self.seed, self.thr, self.B = seed, thr, B

    def step_lists(self, t):
        return oracle.poisson_input(self.seed, t, self.B, self.thr)


def poisson_case(name, per_instance, max_hz=None):
    cfg, rate = CASES[name]
    net = rb.EpropNet(cfg)
    rng = np.random.default_rng(cfg.seed + 100)
    shape = (cfg.batch, cfg.n_in) if per_instance else (cfg.n_in,)
    rates = rng.uniform(0.0, max_hz or rate, shape)
    labels = rng.integers(0, cfg.n_out, cfg.batch).astype(np.int32)
    lab = torch.tensor(labels, dtype=torch.int32, device="cuda")
    net.set_input_poisson(rates, lab)
    src = PoissonLists(cfg.seed, oracle.rate_thresholds(rates, cfg.dt_ms), cfg.batch)
    return cfg, net, src, labels, lab


@pytest.mark.parametrize("name,per_instance", [("tiny-lif-b1", False), ("alif-b64-col", False),
                                               ("alif-b3-narrow", True), ("lif-b256-col", True)])
def test_poisson_lockstep(name, per_instance):
    cfg, net, src, labels, _ = poisson_case(name, per_instance)
    N = oracle_net(snapshot(net), cfg)
    resync, t, nx = 0, 0, 0
    for _ in range(40):  # one step per launch
        net.step(1, rb.RS_LEARN)
        snap = snapshot(net)
        nx += src.step_lists(t)[0].size
        resync += oracle_step_resync(N, src, t, labels, snap["z"])
        compare_state(snap, N, cfg)
        t += 1
    for blk in range(3):  # whole trace blocks: the block's draws made at its start
        net.step(20, rb.RS_LEARN)
        for _ in range(20):
            idx, off = src.step_lists(t)
            nx += idx.size
            N.step(idx, off, labels)
            t += 1
        snap = snapshot(net)
        assert np.array_equal(snap["z"], N.z), f"spikes differ in block {blk}"
        compare_state(snap, N, cfg)
    assert nx > 0
    assert resync <= 2, f"{resync} threshold ties"


def test_poisson_edge_rates():
    """Rate 0 never fires and rate * dt >= 1 fires every step: the input traces
    are 0 and the geometric sum of the trace decay."""
    cfg, _ = CASES["alif-b3-narrow"]
    net = rb.EpropNet(cfg)
    rates = np.zeros((cfg.batch, cfg.n_in))
    rates[1] = 1000.0 / cfg.dt_ms
    rates[2] = 5000.0
    net.set_input_poisson(rates, torch.zeros(cfg.batch, dtype=torch.int32, device="cuda"))
    net.step(25, 0)
    xbar = net.get(rb.XBAR).T  # [n_in][B]
    a = np.float32(np.exp(-cfg.dt_ms / cfg.tau_mem_ms))
    f = np.float32(0.0)
    for _ in range(25):
        f = np.float32(a * f + np.float32(1.0))
    assert np.all(xbar[:, 0] == 0.0)
    np.testing.assert_allclose(xbar[:, 1:], f, rtol=1e-6)
    # every synapse of the firing instances carried an event in every step
    assert net.info().synaptic_events >= 2 * 25 * int(net.get(rb.PROJ(0, rb.P_LEN)).sum())


@pytest.mark.parametrize("name", ["alif-b64-col", "alif-b3-narrow"])
def test_poisson_source_equals_raster_of_its_spikes(name):
    """A raster holding the oracle's Poisson spikes (ascending lists) and the
    device source (lists in arrival order) give the same state bit for bit:
    the input sums are exact whatever the order."""
    cfg, rate = CASES[name]
    T = 45
    cfg = rb.EpropConfig(**{**cfg.__dict__, "sample_steps": T})
    rng = np.random.default_rng(7)
    rates = rng.uniform(0.0, rate, cfg.n_in)
    labels = rng.integers(0, cfg.n_out, cfg.batch).astype(np.int32)
    src = PoissonLists(cfg.seed, oracle.rate_thresholds(rates, cfg.dt_ms), cfg.batch)
    spk = np.zeros((T, cfg.batch, cfg.n_in), bool)
    for t in range(T):
        idx, off = src.step_lists(t)
        for b in range(cfg.batch):
            spk[t, b, idx[off[b]:off[b + 1]]] = True
    raster = wl._to_raster(spk)
    a, b = rb.EpropNet(cfg), rb.EpropNet(cfg)
    a.set_input(*gpu_input(raster, labels))
    b.set_input_poisson(rates, torch.tensor(labels, dtype=torch.int32, device="cuda"))
    for n in (7, 20, 18):
        a.step(n, rb.RS_LEARN)
        b.step(n, rb.RS_LEARN)
        sa, sb = snapshot(a), snapshot(b)
        for k in sa:
            if isinstance(sa[k], dict):
                for f in sa[k]:
                    assert np.array_equal(sa[k][f], sb[k][f]), (k, f)
            else:
                assert np.array_equal(sa[k], sb[k]), k
    assert a.info().synaptic_events == b.info().synaptic_events


def test_poisson_argument_errors():
    cfg, _ = CASES["alif-b3-narrow"]
    net = rb.EpropNet(cfg)
    lab = torch.zeros(cfg.batch, dtype=torch.int32, device="cuda")
    with pytest.raises(rb.RagsnnError):
        net.set_input_poisson(np.ones(cfg.n_in + 1), lab)
    bad = np.ones(cfg.n_in)
    bad[3] = np.nan
    with pytest.raises(rb.RagsnnError):
        net.set_input_poisson(bad, lab)
    with pytest.raises(rb.RagsnnError):  # still no input attached
        net.step(1, 0)
    net.set_input_poisson(np.full(cfg.n_in, 20.0), lab)
    net.step(3, 0)
