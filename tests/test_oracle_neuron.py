"""Closed-form pins of the oracle's neuron, readout and propagation arithmetic
(paper, recurrent classifier equations)."""
import numpy as np
import pytest
import torch

from helpers import dense, set_rows


def tiny_net(orc, n_in, n_rec, n_out, B, alif, in_rows, in_w, rec_rows, rec_w, cap=None, traces=True):
    cap_in = cap or max(1, max(len(r) for r in in_rows))
    cap_rec = cap or max(1, max([len(r) for r in rec_rows] + [1]))
    tr = ("alif" if alif else "lif") if traces else "none"
    inp = orc.Proj(n_in, n_rec, cap_in, False, 0, batch=B, trained=True, traces=tr, bitfields=True)
    rec = orc.Proj(n_rec, n_rec, cap_rec, True, 1, batch=B, trained=True, traces=tr, bitfields=True)
    set_rows(inp, in_rows, in_w)
    set_rows(rec, rec_rows, rec_w)
    prm = orc.EpropParams(n_in=n_in, n_rec=n_rec, n_out=n_out, batch=B, alif=alif)
    return orc.Net(prm, inp, rec)


def no_input(B):
    return np.zeros(0, np.int32), np.zeros(B + 1, np.int32)


def one_input(B, i):
    return np.array([i] * B, np.int32), np.arange(B + 1, dtype=np.int32)


def test_lif_single_spike_impulse_response(orc):
    w = 0.3
    N = tiny_net(orc, 1, 1, 1, 1, False, [[0]], [[w]], [[]], [[]])
    alpha = N.prm.alpha
    N.step(*one_input(1, 0), labels=[0])
    for k in range(40):
        assert N.v[0, 0] == pytest.approx(w * alpha ** k, rel=1e-14, abs=0)
        N.step(*no_input(1), labels=[0])


def test_subtractive_reset(orc):
    N = tiny_net(orc, 1, 1, 1, 1, False, [[0]], [[0.25]], [[]], [[]])
    alpha, vt = N.prm.alpha, N.prm.v_thr
    N.v[0, 0] = 0.7  # above threshold: spikes this step
    N.step(*one_input(1, 0), labels=[0])
    assert N.z[0, 0] == 1
    assert N.v[0, 0] == pytest.approx(alpha * (0.7 - vt) + 0.25, rel=1e-14)
    N.v[0, 0] = 0.59
    N.step(*no_input(1), labels=[0])
    assert N.z[0, 0] == 0
    assert N.v[0, 0] == pytest.approx(alpha * 0.59, rel=1e-14)


def test_heaviside_at_threshold(orc):
    N = tiny_net(orc, 1, 1, 1, 1, False, [[0]], [[0.0]], [[]], [[]])
    N.v[0, 0] = N.prm.v_thr
    z, margin = N.spikes()
    assert z[0, 0] == 1 and margin[0, 0] == 0.0


def test_alif_adaptation_decay(orc):
    N = tiny_net(orc, 1, 1, 1, 1, True, [[0]], [[0.0]], [[]], [[]])
    rho = N.prm.rho
    assert rho == pytest.approx(np.exp(-1 / 2000.0))
    N.v[0, 0] = 1.0
    N.step(*no_input(1), labels=[0])
    assert N.z[0, 0] == 1
    for k in range(30):
        assert N.a[0, 0] == pytest.approx(rho ** k, rel=1e-14)
        N.step(*no_input(1), labels=[0])
        assert N.z[0, 0] == 0


def test_alif_threshold_rises_with_adaptation(orc):
    N = tiny_net(orc, 1, 1, 1, 1, True, [[0]], [[0.0]], [[]], [[]])
    N.a[0, 0] = 10.0
    N.v[0, 0] = 0.6 + 0.0174 * 10.0 - 1e-9
    z, _ = N.spikes()
    assert z[0, 0] == 0
    N.v[0, 0] += 2e-9
    z, _ = N.spikes()
    assert z[0, 0] == 1


def test_surrogate_shape(orc):
    N = tiny_net(orc, 1, 3, 1, 1, True, [[0]], [[0.0]], [[], [], []], [[], [], []])
    vt, beta = 0.6, 0.0174
    N.a[0, :] = [0.0, 2.0, 0.0]
    N.v[0, :] = [0.6, 0.6 + beta * 2.0 - 0.3, -0.1]
    N.step(*no_input(1), labels=[0])
    assert N.psi[0, 0] == pytest.approx(0.3 / vt, rel=1e-14)
    assert N.psi[0, 1] == pytest.approx((0.3 / vt) * 0.5, rel=1e-12)
    assert N.psi[0, 2] == 0.0


def test_readout_impulse_and_bias_step(orc):
    N = tiny_net(orc, 1, 2, 3, 1, False, [[0]], [[0.0]], [[], []], [[], []])
    alpha = N.prm.alpha
    N.Wout[:] = np.array([[0.5, -0.2], [0.1, 0.3], [-0.4, 0.7]])
    N.bout[:] = [0.0, 0.0, 0.0]
    N.v[0, 1] = 1.0  # neuron 1 spikes at the first step only
    N.step(*no_input(1), labels=[0])
    for m in range(25):
        assert N.y[0] == pytest.approx(alpha ** m * N.Wout[:, 1], rel=1e-13)
        N.step(*no_input(1), labels=[0])
    # bias step response with no spikes: sum_{m<k} alpha^m b
    N.reset()
    N.bout[:] = [0.1, -0.3, 0.05]
    for k in range(1, 20):
        N.step(*no_input(1), labels=[0])
        assert N.y[0] == pytest.approx(N.bout * (1 - alpha ** k) / (1 - alpha), rel=1e-12)


def test_output_error_is_cross_entropy_gradient(orc):
    N = tiny_net(orc, 1, 2, 5, 3, False, [[0]], [[0.0]], [[], []], [[], []])
    rng = np.random.default_rng(0)
    N.y[:] = rng.normal(0, 3, (3, 5))
    N.bout[:] = 0
    labels = np.array([4, 0, 2], np.int32)
    yy = torch.tensor(N.prm.alpha * N.y, dtype=torch.float64, requires_grad=True)
    N.step(*no_input(3), labels=labels)
    torch.nn.functional.cross_entropy(yy, torch.tensor(labels, dtype=torch.long), reduction="sum").backward()
    assert np.allclose(N.delta, yy.grad.numpy(), rtol=0, atol=1e-14)


def test_propagation_dense_equivalence(orc):
    # ragged accumulation == dense W @ s on random tiny networks
    rng = np.random.default_rng(7)
    for trial in range(20):
        n_in, n_rec, B = int(rng.integers(1, 20)), int(rng.integers(1, 32)), int(rng.integers(1, 4))
        in_rows = [sorted(rng.choice(n_rec, int(rng.integers(0, n_rec + 1)), replace=False).tolist())
                   for _ in range(n_in)]
        rec_rows = [[j for j in rng.choice(n_rec, int(rng.integers(0, n_rec + 1)), replace=False) if j != i]
                    for i in range(n_rec)]
        rng.shuffle(in_rows)  # unsorted rows are fine
        in_w = [rng.normal(0, 0.3, len(r)) for r in in_rows]
        rec_w = [rng.normal(0, 0.3, len(r)) for r in rec_rows]
        N = tiny_net(orc, n_in, n_rec, 2, B, bool(trial % 2), in_rows, in_w, rec_rows, rec_w,
                     cap=max(n_rec, 1))
        N.v[:] = rng.normal(0.3, 0.4, (B, n_rec))
        N.a[:] = rng.uniform(0, 3, (B, n_rec))
        x = rng.random((B, n_in)) < 0.3
        idx = np.concatenate([np.nonzero(x[b])[0] for b in range(B)]).astype(np.int32)
        off = np.concatenate([[0], np.cumsum(x.sum(1))]).astype(np.int32)
        zf = (rng.random((B, n_rec)) < 0.4).astype(np.uint8)
        v0, a0 = N.v.copy(), N.a.copy()
        Win, Wrec = dense(N.inp), dense(N.rec)
        N.step(idx, off, labels=np.zeros(B, np.int32), z_force=zf)
        p = N.prm
        expect = p.alpha * (v0 - zf * p.v_thr) + x.astype(float) @ Win.T + zf.astype(float) @ Wrec.T
        assert np.allclose(N.v, expect, rtol=1e-13, atol=1e-13)
        assert np.allclose(N.a, p.rho * a0 + zf, rtol=1e-14, atol=0)


@pytest.mark.parametrize("alpha_trace", [None, 0.95122945])
def test_trace_impulse_response(orc, alpha_trace):
    """An input spike at step 0 leaves xbar = a^k after k further steps, with a
    the trace decay: tau_mem's alpha itself, or alpha as a float
    implementation stores it; the membrane keeps alpha."""
    N = tiny_net(orc, 1, 1, 1, 1, False, [[0]], [[0.1]], [[]], [[]])
    N.prm.alpha_trace_value = alpha_trace
    a = N.prm.alpha if alpha_trace is None else alpha_trace
    N.step(*one_input(1, 0), labels=[0])
    for k in range(30):
        assert N.xbar[0, 0] == pytest.approx(a ** k, rel=1e-14, abs=0)
        assert N.v[0, 0] == pytest.approx(0.1 * N.prm.alpha ** k, rel=1e-14, abs=0)
        N.step(*no_input(1), labels=[0])
