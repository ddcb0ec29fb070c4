"""Shared machinery of the GPU parity tests: GPU snapshots in the oracle's
layout, oracle networks built from a snapshot, and the comparison rules.

Tolerance (single precision against the fp64 oracle): |gpu - orc| <=
RTOL * max(|orc|, scale) with RTOL = 1e-5, scale = v_thr for voltages and the
readout, 1 for spike traces and eligibility traces, the initial weight spread
for weights, and the largest magnitude in the array for accumulated sums
(gradients, learning signals), whose cancellation makes a per-element relative
bound meaningless."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2510_19764_amd import binding as rb

RTOL = 1e-5


def snapshot(net: rb.EpropNet, with_traces=True):
    s = {}
    for name, var in [("v", rb.V), ("a", rb.A), ("y", rb.Y), ("xbar", rb.XBAR), ("zbar", rb.ZBAR),
                      ("psiT", rb.PSI), ("LT", rb.LSIG), ("deltaT", rb.DELTA), ("z", rb.Z),
                      ("Wout", rb.WOUT), ("bout", rb.BOUT), ("Gout", rb.GOUT), ("Gb", rb.GB),
                      ("Mout", rb.MOUT), ("Vout", rb.VOUT), ("Mb", rb.MB), ("Vb", rb.VB)]:
        s[name] = net.get(var)
    for p, tag in ((0, "in"), (1, "rec")):
        d = {}
        fl = [("len", rb.P_LEN), ("ind", rb.P_IND), ("w", rb.P_W), ("m", rb.P_M), ("vv", rb.P_V),
              ("G", rb.P_G), ("dormant", rb.P_DORMANT)]
        if with_traces:
            fl.append(("ebar", rb.P_EBAR))
            if net.cfg.alif:
                fl.append(("eps", rb.P_EPS))
        if (net.cfg.deepr_mask >> p) & 1:
            fl += [("conn", rb.P_CONN), ("sign", rb.P_SIGN)]
        for name, f in fl:
            d[name] = net.get(rb.PROJ(p, f))
        s[tag] = d
    return s


def f32(x):
    return float(np.float32(x))


def effective_params(cfg: rb.EpropConfig):
    """The parameter values the library actually runs with: parameters cross the
    C-ABI as float32, and the decay factors are exp(-dt/tau) evaluated in double
    from the float32 dt and tau.  The oracle receives these same values so that
    the comparison measures arithmetic, not parameter rounding."""
    dt, tm, ta = np.float64(np.float32(cfg.dt_ms)), np.float64(np.float32(cfg.tau_mem_ms)), \
        np.float64(np.float32(cfg.tau_adapt_ms))
    alpha = float(np.exp(-dt / tm))
    # the presynaptic traces decay by the float-rounded alpha
    return dict(v_thr=f32(cfg.v_thr), beta=f32(cfg.beta), alpha_value=alpha,
                rho_value=float(np.exp(-dt / ta)), alpha_trace_value=f32(alpha))


def oracle_net(snap, cfg: rb.EpropConfig, with_traces=True):
    """fp64 oracle network initialised from a GPU snapshot."""
    B = cfg.batch
    projs = []
    for tag, n_pre, rec, pid in (("in", cfg.n_in, False, 0), ("rec", cfg.n_rec, True, 1)):
        d = snap[tag]
        cap = d["ind"].shape[1]
        P = oracle.Proj(n_pre, cfg.n_rec, cap, rec, pid, batch=B, trained=True,
                        traces=("alif" if cfg.alif else "lif") if with_traces else "none",
                        bitfields="conn" in d)
        P.len[:] = d["len"]
        P.ind[:] = d["ind"].ravel()
        P.w[:] = d["w"].ravel()
        P.m[:] = d["m"].ravel()
        P.v[:] = d["vv"].ravel()
        P.G[:] = d["G"].ravel()
        if with_traces:
            P.ebar[:] = d["ebar"].ravel()
            if cfg.alif:
                P.eps[:] = d["eps"].ravel()
        if "conn" in d:
            P.conn[:] = d["conn"].ravel()
            P.sign[:] = d["sign"].ravel()
        projs.append(P)
    prm = oracle.EpropParams(n_in=cfg.n_in, n_rec=cfg.n_rec, n_out=cfg.n_out, batch=B, alif=cfg.alif,
                             dt_ms=cfg.dt_ms, tau_mem_ms=cfg.tau_mem_ms, tau_adapt_ms=cfg.tau_adapt_ms,
                             **effective_params(cfg))
    N = oracle.Net(prm, projs[0], projs[1])
    N.v[:] = snap["v"]
    N.a[:] = snap["a"]
    N.y[:] = snap["y"]
    N.xbar[:] = snap["xbar"]
    N.zbar[:] = snap["zbar"]
    for k in ("Wout", "bout", "Gout", "Gb", "Mout", "Vout", "Mb", "Vb"):
        getattr(N, k)[:] = snap[k]
    return N


def close(name, gpu, orc, scale, rtol=RTOL):
    gpu = np.asarray(gpu, np.float64)
    orc = np.asarray(orc, np.float64)
    assert gpu.shape == orc.shape, (name, gpu.shape, orc.shape)
    bound = rtol * np.maximum(np.abs(orc), scale)
    err = np.abs(gpu - orc)
    bad = err > bound
    if bad.any():
        q = np.argwhere(bad)[0]
        raise AssertionError(f"{name}: {int(bad.sum())} elements off, first at {tuple(q)}: "
                             f"gpu={gpu[tuple(q)]!r} oracle={orc[tuple(q)]!r} bound={bound[tuple(q)]!r}")


def real_slots(d):
    """Boolean mask [n_pre, cap] of slots holding synapses."""
    cap = d["ind"].shape[1]
    return np.arange(cap)[None, :] < d["len"][:, None]


def compare_rows_exact(tag, g, o: oracle.Proj):
    cap = g["ind"].shape[1]
    assert np.array_equal(g["len"], o.len), f"{tag}: row lengths differ"
    m = real_slots(g)
    assert np.array_equal(g["ind"][m], o.ind.reshape(-1, cap)[m]), f"{tag}: indices differ"


def compare_state(snap, N: oracle.Net, cfg: rb.EpropConfig, sigma_w=(1.0, 1.0), learn=True, rtol=RTOL):
    close("v", snap["v"], N.v, cfg.v_thr, rtol)
    close("a", snap["a"], N.a, 1.0, rtol)
    close("y", snap["y"], N.y, cfg.v_thr, rtol)
    close("xbar", snap["xbar"], N.xbar, 1.0, rtol)
    close("zbar", snap["zbar"], N.zbar, 1.0, rtol)
    close("psi", snap["psiT"].T, N.psi, 0.3 / cfg.v_thr, rtol)
    close("delta", snap["deltaT"].T, N.delta, 1.0, rtol)
    close("L", snap["LT"].T, N.L, max(1e-12, np.abs(N.L).max()), rtol)
    if not learn:
        return
    close("Gout", snap["Gout"], N.Gout, max(1e-12, np.abs(N.Gout).max()), rtol)
    close("Gb", snap["Gb"], N.Gb, max(1e-12, np.abs(N.Gb).max()), rtol)
    B = cfg.batch
    for tag, P in (("in", N.inp), ("rec", N.rec)):
        g = snap[tag]
        cap = g["ind"].shape[1]
        m = real_slots(g)
        compare_rows_exact(tag, g, P)
        close(tag + ".G", g["G"][m], P.G.reshape(-1, cap)[m], max(1e-12, np.abs(P.G).max()), rtol)
        eb = P.ebar.reshape(-1, cap, B)
        close(tag + ".ebar", g["ebar"][m], eb[m], 1.0, rtol)
        if cfg.alif:
            close(tag + ".eps", g["eps"][m], P.eps.reshape(-1, cap, B)[m], 1.0, rtol)


def gpu_input(raster, labels):
    import torch
    off = torch.tensor(raster.off, dtype=torch.int32, device="cuda")
    idx = torch.tensor(raster.idx if raster.idx.size else np.zeros(1, np.int32), dtype=torch.int32, device="cuda")
    lab = torch.tensor(np.asarray(labels, np.int32), dtype=torch.int32, device="cuda")
    return off, idx, lab


def oracle_step_resync(N: oracle.Net, raster, t_local: int, labels, z_gpu, learn=True, tie_tol=1e-5):
    """Step the oracle; where its spikes differ from the GPU's, require a
    near-threshold tie and adopt the GPU's spikes.  Returns the resync count."""
    idx, off = raster.step_lists(t_local)
    z_orc, margin = N.spikes()
    diff = z_orc != z_gpu
    n_resync = int(diff.sum())
    if n_resync:
        worst = np.abs(margin[diff]).max()
        assert worst <= tie_tol * N.prm.v_thr, \
            f"spike mismatch away from threshold: |v - thr| = {worst} at {np.argwhere(diff)[0]}"
        N.step(idx, off, labels, z_force=z_gpu, learn=learn)
    else:
        N.step(idx, off, labels, learn=learn)
    return n_resync
