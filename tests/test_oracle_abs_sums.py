"""The oracle's error-bound bookkeeping: beside each sum with cancellation
(learning signal L, gradients G, Gout, Gb) it keeps the first-order error
scale of its terms (for L the magnitude of its terms; for the gradients the
magnitude of each term's factors times the error scales of the others), which
the GPU parity tests use as the per-element scale of their tolerance.
Checked against the terms recomputed from the oracle's per-step values, and
for the invariants |sum| <= scale, its closed form when every term has one
sign, and clearing with the update."""
import numpy as np

from helpers import set_rows


def net(orc, rng, B=3, n_in=6, n_rec=7, n_out=3):
    inp = orc.Proj(n_in, n_rec, n_rec, False, 0, batch=B, trained=True, traces="alif", bitfields=True,
                   abs_sums=True)
    rec = orc.Proj(n_rec, n_rec, n_rec, True, 1, batch=B, trained=True, traces="alif", bitfields=True,
                   abs_sums=True)
    in_rows = [sorted(rng.choice(n_rec, 4, replace=False).tolist()) for _ in range(n_in)]
    rec_rows = [[j for j in range(n_rec) if j != i and rng.random() < 0.5] for i in range(n_rec)]
    set_rows(inp, in_rows, [rng.normal(0.3, 0.3, len(r)) for r in in_rows])
    set_rows(rec, rec_rows, [rng.normal(0.0, 0.3, len(r)) for r in rec_rows])
    N = orc.Net(orc.EpropParams(n_in=n_in, n_rec=n_rec, n_out=n_out, batch=B, alif=True), inp, rec,
                abs_sums=True)
    N.Wout[:] = rng.normal(0, 0.5, (n_out, n_rec))
    return N


def test_magnitude_sums_follow_their_terms(orc):
    rng = np.random.default_rng(4)
    B = 3
    N = net(orc, rng, B=B)
    labels = np.array([0, 2, 1], np.int32)
    expect = {id(P): np.zeros_like(P.G) for P in (N.inp, N.rec)}
    gout = np.zeros_like(N.Gout)
    gb = np.zeros_like(N.Gb)
    for t in range(25):
        x = rng.random((B, N.prm.n_in)) < 0.4
        idx = np.nonzero(x)[1].astype(np.int32)
        off = np.concatenate([[0], np.cumsum(x.sum(1))]).astype(np.int32)
        N.step(idx, off, labels)
        # L and its error scale over the readout units, this step
        pi = N.delta + (np.arange(N.prm.n_out)[None, :] == labels[:, None])
        terms = N.Wout[None, :, :] * N.delta[:, :, None]          # [B][k][j]
        assert np.allclose(N.L, terms.sum(1), rtol=1e-13, atol=1e-15)
        scale = (np.abs(N.Wout)[None, :, :] * (np.abs(N.delta) + pi)[:, :, None]).sum(1)
        assert np.allclose(N.Labs, scale, rtol=1e-13, atol=1e-15)
        assert (np.abs(N.L) <= N.Labs).all()
        gout += (np.abs(N.zbar[:, None, :]) * (2 * np.abs(N.delta) + pi)[:, :, None]).sum(0)
        gb += (np.abs(N.delta) + pi).sum(0)
        for P in (N.inp, N.rec):
            eb = P.ebar.reshape(P.n_pre, P.cap, B)
            for i in range(P.n_pre):
                for k in range(int(P.len[i])):
                    j = P.ind[i * P.cap + k]
                    expect[id(P)][i * P.cap + k] += (np.abs(eb[i, k]) * (2 * np.abs(N.L[:, j]) + N.Labs[:, j])).sum()
    for P in (N.inp, N.rec):
        assert np.allclose(P.Gabs, expect[id(P)], rtol=1e-12, atol=0)
        assert (np.abs(P.G) <= P.Gabs * (1 + 1e-12) + 1e-300).all()
        assert P.Gabs.max() > 0
    assert np.allclose(N.Goutabs, gout, rtol=1e-12, atol=0)
    assert np.allclose(N.Gbabs, gb, rtol=1e-12, atol=0)
    assert (np.abs(N.Gb) <= N.Gbabs).all() and (np.abs(N.Gout) <= N.Goutabs).all()
    N.adam_update(1, l1=0.005, deepr_mask=3)
    for P in (N.inp, N.rec):
        assert not P.Gabs.any() and not P.G.any()
    assert not N.Goutabs.any() and not N.Gbabs.any()


def test_single_sign_terms_closed_form(orc):
    """One instance, two readout units, label 1: delta of unit 0 is pi_0 > 0
    at every step, so its scale sum_t (|delta| + pi) is exactly 2 Gb[0]."""
    rng = np.random.default_rng(5)
    N = net(orc, rng, B=1, n_out=2)
    for t in range(10):
        N.step(np.zeros(1, np.int32), np.zeros(2, np.int32), np.array([1], np.int32))
    assert N.Gb[0] > 0 and np.isclose(2 * N.Gb[0], N.Gbabs[0], rtol=1e-14)
