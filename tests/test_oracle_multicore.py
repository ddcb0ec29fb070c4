"""The oracle's multi-core timing build (OpenMP over independent batch
instances, rows and readout units) computes exactly what the single-threaded
parity build computes: same state, traces and gradients bit for bit after
learning steps, an update and DEEP R."""
import os

import numpy as np

from helpers import set_rows


def run(orc, steps=12):
    rng = np.random.default_rng(9)
    B, NI, NR, K = 16, 30, 40, 3
    inp = orc.Proj(NI, NR, NR, False, 0, batch=B, trained=True, traces="alif", bitfields=True)
    rec = orc.Proj(NR, NR, NR, True, 1, batch=B, trained=True, traces="alif", bitfields=True)
    set_rows(inp, [sorted(rng.choice(NR, 12, replace=False)) for _ in range(NI)],
             [rng.normal(0.3, 0.3, 12) for _ in range(NI)])
    rr = [[j for j in rng.choice(NR, 10, replace=False) if j != i] for i in range(NR)]
    set_rows(rec, rr, [rng.normal(0, 0.3, len(r)) for r in rr])
    orc.deepr_init_bits(3, inp)
    orc.deepr_init_bits(3, rec)
    N = orc.Net(orc.EpropParams(n_in=NI, n_rec=NR, n_out=K, batch=B, alif=True), inp, rec)
    N.Wout[:] = rng.normal(0, 0.4, (K, NR))
    labels = rng.integers(0, K, B).astype(np.int32)
    for t in range(steps):
        x = rng.random((B, NI)) < 0.3
        idx = np.nonzero(x)[1].astype(np.int32)
        off = np.concatenate([[0], np.cumsum(x.sum(1))]).astype(np.int32)
        N.step(idx, off, labels)
    N.adam_update(1, lr=0.05, l1=0.005, deepr_mask=3)
    orc.deepr_rewire(3, N.rec, steps)
    return N


def test_multicore_build_is_bit_identical(orc):
    os.environ.setdefault("OMP_NUM_THREADS", "4")
    a = run(orc)
    threads = orc.use_multicore(True)
    try:
        b = run(orc)
    finally:
        orc.use_multicore(False)
    assert threads >= 1
    for k in ("v", "a", "y", "xbar", "zbar", "Wout", "bout", "Mout", "Vout", "psi", "L", "z", "delta"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    for P, Q in ((a.inp, b.inp), (a.rec, b.rec)):
        for k in ("len", "ind", "w", "m", "v", "G", "eps", "ebar", "conn"):
            assert np.array_equal(getattr(P, k), getattr(Q, k)), k
