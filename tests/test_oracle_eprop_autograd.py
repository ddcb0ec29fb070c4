"""Pin of the oracle's e-prop eligibility traces and gradients against torch
autograd in float64.

e-prop (Bellec et al. 2020, as used in the paper's classifier section) is the
exact gradient of the summed per-step cross-entropy loss once two paths are cut:
the reset term and the recurrent spikes entering other neurons.  Spikes use the
paper's surrogate derivative psi w.r.t. v (and -beta psi w.r.t. a).  The
forward pass is driven by the oracle's own spike raster so threshold ties cannot
split the two.  The bias gradient follows the paper's delta rule (sum of output
errors), which ignores the readout leak; it is pinned by that closed form."""
import numpy as np
import pytest
import torch

from helpers import set_rows


class Spike(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, z_given, v_thr):
        ctx.save_for_backward(u)
        ctx.v_thr = v_thr
        return z_given.clone()

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        psi = (0.3 / ctx.v_thr) * torch.clamp(1.0 - u.abs() / ctx.v_thr, min=0.0)
        return g * psi, None, None


def build(orc, rng, n_in, n_rec, n_out, B, alif, p_in=0.6, p_rec=0.5):
    in_rows = [sorted(rng.choice(n_rec, rng.binomial(n_rec, p_in), replace=False).tolist()) for _ in range(n_in)]
    rec_rows = []
    for i in range(n_rec):
        c = [j for j in range(n_rec) if j != i and rng.random() < p_rec]
        rng.shuffle(c)
        rec_rows.append(c)
    tr = "alif" if alif else "lif"
    inp = orc.Proj(n_in, n_rec, n_rec, False, 0, batch=B, trained=True, traces=tr, bitfields=True)
    rec = orc.Proj(n_rec, n_rec, n_rec, True, 1, batch=B, trained=True, traces=tr, bitfields=True)
    set_rows(inp, in_rows, [rng.normal(0.25, 0.3, len(r)) for r in in_rows])
    set_rows(rec, rec_rows, [rng.normal(0.0, 0.3, len(r)) for r in rec_rows])
    N = orc.Net(orc.EpropParams(n_in=n_in, n_rec=n_rec, n_out=n_out, batch=B, alif=alif), inp, rec)
    N.Wout[:] = rng.normal(0, 0.5, (n_out, n_rec))
    N.bout[:] = rng.normal(0, 0.2, n_out)
    return N


def dense_param(P):
    W = np.zeros((P.n_post, P.n_pre))
    for i in range(P.n_pre):
        for k in range(int(P.len[i])):
            W[P.ind[i * P.cap + k], i] = P.w[i * P.cap + k]
    return W


def slot_grad(P, Gdense):
    out = np.zeros_like(P.G)
    for i in range(P.n_pre):
        for k in range(int(P.len[i])):
            out[i * P.cap + k] = Gdense[P.ind[i * P.cap + k], i]
    return out


@pytest.mark.parametrize("alif", [False, True])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_eprop_equals_truncated_autograd(orc, alif, seed):
    rng = np.random.default_rng(100 + seed)
    n_in, n_rec, n_out, B, T = 6, 10, 3, 2, 45
    N = build(orc, rng, n_in, n_rec, n_out, B, alif)
    labels = rng.integers(0, n_out, B).astype(np.int32)
    xs = rng.random((T, B, n_in)) < 0.3
    Win0, Wrec0, Wout0, b0 = dense_param(N.inp), dense_param(N.rec), N.Wout.copy(), N.bout.copy()

    zs, vs = [], []
    for t in range(T):
        x = xs[t]
        idx = np.concatenate([np.nonzero(x[b])[0] for b in range(B)]).astype(np.int32)
        off = np.concatenate([[0], np.cumsum(x.sum(1))]).astype(np.int32)
        vs.append(N.v.copy())
        N.step(idx, off, labels)
        zs.append(N.z.copy())
    zs = np.array(zs, dtype=np.float64)
    assert 0.05 < zs.mean() < 0.6, "test network should spike moderately"

    p = N.prm
    dt = torch.float64
    Win = torch.tensor(Win0, dtype=dt, requires_grad=True)
    Wrec = torch.tensor(Wrec0, dtype=dt, requires_grad=True)
    Wout = torch.tensor(Wout0, dtype=dt, requires_grad=True)
    bout = torch.tensor(b0, dtype=dt, requires_grad=True)
    v = torch.zeros(B, n_rec, dtype=dt)
    a = torch.zeros(B, n_rec, dtype=dt)
    y = torch.zeros(B, n_out, dtype=dt)
    lab = torch.tensor(labels, dtype=torch.long)
    loss = torch.zeros((), dtype=dt)
    delta_sum = torch.zeros(n_out, dtype=dt)
    for t in range(T):
        assert np.allclose(v.detach().numpy(), vs[t], rtol=1e-12, atol=1e-12)
        A = p.v_thr + p.beta_eff * a
        z = Spike.apply(v - A, torch.tensor(zs[t], dtype=dt), p.v_thr)
        x = torch.tensor(xs[t], dtype=dt)
        I = x @ Win.T + z.detach() @ Wrec.T
        v = p.alpha * (v - z.detach() * p.v_thr) + I
        a = p.rho * a + z
        y = p.alpha * y + z @ Wout.T + bout
        loss = loss + torch.nn.functional.cross_entropy(y, lab, reduction="sum")
        delta_sum += (torch.softmax(y, dim=1) - torch.nn.functional.one_hot(lab, n_out)).sum(0).detach()
    loss.backward()

    gin = slot_grad(N.inp, Win.grad.numpy())
    grec = slot_grad(N.rec, Wrec.grad.numpy())
    scale_in = max(1e-3, np.abs(gin).max())
    scale_rec = max(1e-3, np.abs(grec).max())
    assert np.abs(N.inp.G - gin).max() <= 1e-10 * scale_in
    assert np.abs(N.rec.G - grec).max() <= 1e-10 * scale_rec
    assert np.abs(grec).max() > 1e-4 and np.abs(gin).max() > 1e-4
    assert np.allclose(N.Gout, Wout.grad.numpy(), rtol=1e-10, atol=1e-12)
    assert np.allclose(N.Gb, delta_sum.numpy(), rtol=1e-10, atol=1e-12)
