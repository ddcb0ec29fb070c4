"""Pin of the oracle's parameter update (batch mean, DEEP R L1 term, Adam)
against torch.optim.Adam with its default hyper-parameters."""
import numpy as np
import torch

from helpers import set_rows


def test_adam_with_l1_matches_torch(orc):
    rng = np.random.default_rng(3)
    n_in, n_rec, n_out, B = 4, 6, 3, 5
    inp = orc.Proj(n_in, n_rec, 6, False, 0, batch=B, trained=True, traces="lif", bitfields=True)
    rec = orc.Proj(n_rec, n_rec, 6, True, 1, batch=B, trained=True, traces="lif", bitfields=True)
    set_rows(inp, [[0, 2, 5], [1], [], [3, 4, 0, 2]], [rng.normal(0, 0.3, n) for n in (3, 1, 0, 4)])
    rows = [[j for j in range(n_rec) if j != i and rng.random() < 0.5] for i in range(n_rec)]
    set_rows(rec, rows, [rng.normal(0, 0.3, len(r)) for r in rows])
    for P in (inp, rec):
        orc.deepr_init_bits(1, P)
    N = orc.Net(orc.EpropParams(n_in=n_in, n_rec=n_rec, n_out=n_out, batch=B, alif=False), inp, rec)
    N.Wout[:] = rng.normal(0, 0.3, (n_out, n_rec))
    N.bout[:] = rng.normal(0, 0.1, n_out)

    l1, deepr_mask = 0.005, 2  # L1 only on the recurrent projection
    slots = {id(P): [(i, k) for i in range(P.n_pre) for k in range(int(P.len[i]))] for P in (inp, rec)}

    def sgn(P, i, k):
        j = int(P.ind[i * P.cap + k])
        neg = (int(P.sign[i * P.words + (j >> 5)]) >> (j & 31)) & 1
        return -1.0 if neg else 1.0

    params = {}
    for P in (inp, rec):
        params[id(P)] = torch.tensor([P.w[i * P.cap + k] for i, k in slots[id(P)]], dtype=torch.float64,
                                     requires_grad=True)
    tw = torch.tensor(N.Wout, requires_grad=True)
    tb = torch.tensor(N.bout, requires_grad=True)
    opt = torch.optim.Adam([params[id(inp)], params[id(rec)], tw, tb])
    for k in range(1, 8):
        for P in (inp, rec):
            P.G[:] = 0
            for (i, kk) in slots[id(P)]:
                P.G[i * P.cap + kk] = rng.normal(0, 1e-2) * B
        N.Gout[:] = rng.normal(0, 1e-2, N.Gout.shape) * B
        N.Gb[:] = rng.normal(0, 1e-2, N.Gb.shape) * B
        opt.zero_grad()
        for P, use_l1 in ((inp, False), (rec, True)):
            g = [P.G[i * P.cap + kk] / B + (l1 * sgn(P, i, kk) if use_l1 else 0.0) for (i, kk) in slots[id(P)]]
            params[id(P)].grad = torch.tensor(g, dtype=torch.float64)
        tw.grad = torch.tensor(N.Gout / B)
        tb.grad = torch.tensor(N.Gb / B)
        opt.step()
        N.adam_update(k, l1=l1, deepr_mask=deepr_mask)
        for P in (inp, rec):
            got = np.array([P.w[i * P.cap + kk] for i, kk in slots[id(P)]])
            assert np.allclose(got, params[id(P)].detach().numpy(), rtol=1e-12, atol=1e-14)
            assert np.all(P.G == 0)
        assert np.allclose(N.Wout, tw.detach().numpy(), rtol=1e-12, atol=1e-14)
        assert np.allclose(N.bout, tb.detach().numpy(), rtol=1e-12, atol=1e-14)
        assert np.all(N.Gout == 0) and np.all(N.Gb == 0)


def test_l1_pushes_towards_zero(orc):
    # with zero gradient, the L1 term alone moves positive weights down and
    # negative weights up by lr on the first Adam step
    B = 1
    P = orc.Proj(1, 4, 4, False, 0, batch=B, trained=True, traces="lif", bitfields=True)
    set_rows(P, [[0, 1, 2, 3]], [[0.3, -0.2, 0.05, -0.01]])
    orc.deepr_init_bits(0, P)
    R = orc.Proj(4, 4, 4, True, 1, batch=B, trained=True, traces="lif", bitfields=True)
    N = orc.Net(orc.EpropParams(n_in=1, n_rec=4, n_out=1, batch=B, alif=False), P, R)
    w0 = P.w[:4].copy()
    N.adam_update(1, lr=1e-3, l1=0.005, deepr_mask=1)
    # Adam step = lr * lambda / (lambda + eps): within lr * eps / lambda = 2e-9 of lr
    assert np.allclose(P.w[:4], w0 - 1e-3 * np.sign(w0), rtol=0, atol=1e-8)
