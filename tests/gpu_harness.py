"""Shared machinery of the GPU parity tests: GPU snapshots in the oracle's
layout, oracle networks built from a snapshot, and the comparison rules.

Tolerance (single precision against the fp64 oracle): |gpu - orc| <=
RTOL * max(|orc|, scale) with RTOL = 1e-5, scale = v_thr for voltages and the
readout, 1 for spike traces and eligibility traces, the initial weight spread
for weights.  A sum with cancellation (learning signal, gradients) is bounded
per element by RTOL * (|orc| + sum of its terms' magnitudes): each term may
carry the relative error of its factors, and the sum its own rounding.  The
oracle accumulates those magnitude sums beside the sums themselves."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2510_19764_amd import binding as rb

RTOL = 1e-5
# largest error / bound seen per compared quantity (reported by tests)
MARGINS: dict = {}


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


def effective_params(cfg: rb.EpropConfig, paper_alpha=False):
    """The parameter values the library is given: parameters cross the C-ABI as
    float32, and the decay factors are exp(-dt/tau) evaluated in double from the
    float32 dt and tau.  The library keeps the presynaptic traces in float, with
    their decay alpha rounded to float; the oracle receives that rounded factor
    for them (alpha_trace) unless paper_alpha asks for tau_mem's alpha itself,
    which the paper's filters share."""
    dt, tm, ta = np.float64(np.float32(cfg.dt_ms)), np.float64(np.float32(cfg.tau_mem_ms)), \
        np.float64(np.float32(cfg.tau_adapt_ms))
    alpha = float(np.exp(-dt / tm))
    return dict(v_thr=f32(cfg.v_thr), beta=f32(cfg.beta), alpha_value=alpha,
                rho_value=float(np.exp(-dt / ta)), alpha_trace_value=None if paper_alpha else f32(alpha))


def oracle_net(snap, cfg: rb.EpropConfig, with_traces=True, paper_alpha=False):
    """fp64 oracle network initialised from a GPU snapshot."""
    B = cfg.batch
    projs = []
    for tag, n_pre, rec, pid in (("in", cfg.n_in, False, 0), ("rec", cfg.n_rec, True, 1)):
        d = snap[tag]
        cap = d["ind"].shape[1]
        P = oracle.Proj(n_pre, cfg.n_rec, cap, rec, pid, batch=B, trained=True,
                        traces=("alif" if cfg.alif else "lif") if with_traces else "none",
                        bitfields="conn" in d, abs_sums=True)
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
                             **effective_params(cfg, paper_alpha))
    N = oracle.Net(prm, projs[0], projs[1], abs_sums=True)
    N.v[:] = snap["v"]
    N.a[:] = snap["a"]
    N.y[:] = snap["y"]
    N.xbar[:] = snap["xbar"]
    N.zbar[:] = snap["zbar"]
    for k in ("Wout", "bout", "Gout", "Gb", "Mout", "Vout", "Mb", "Vb"):
        getattr(N, k)[:] = snap[k]
    return N


def close(name, gpu, orc, scale, rtol=RTOL, bound=None):
    """|gpu - orc| <= rtol * max(|orc|, scale) per element, or <= bound."""
    gpu = np.asarray(gpu, np.float64)
    orc = np.asarray(orc, np.float64)
    assert gpu.shape == orc.shape, (name, gpu.shape, orc.shape)
    if bound is None:
        bound = rtol * np.maximum(np.abs(orc), scale)
    err = np.abs(gpu - orc)
    bound = np.broadcast_to(np.asarray(bound, np.float64), err.shape)
    if err.size:
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = np.where(err > 0, err / bound, 0.0)
        MARGINS[name] = max(MARGINS.get(name, 0.0), float(np.nanmax(ratio)))
    bad = err > bound
    if bad.any():
        q = np.argwhere(bad)[0]
        raise AssertionError(f"{name}: {int(bad.sum())} of {err.size} elements off (worst error/bound "
                             f"{MARGINS[name]:.3g}), first at {tuple(q)}: "
                             f"gpu={gpu[tuple(q)]!r} oracle={orc[tuple(q)]!r} bound={bound[tuple(q)]!r}")


# Float traces decay to zero below float's range (about 1e-38 and under, as
# flushed denormals) where the fp64 oracle's keep tiny values: sums of at most
# ~1e6 such terms stay below this absolute floor.
SUM_FLOOR = 1e-30


def close_sum(name, gpu, orc, abs_sum, rtol=RTOL):
    """A sum with cancellation: rtol * (|orc| + the terms' error scale), and
    at least SUM_FLOOR."""
    orc = np.asarray(orc, np.float64)
    close(name, gpu, orc, 0.0, bound=rtol * (np.abs(orc) + np.asarray(abs_sum, np.float64)) + SUM_FLOOR)


def real_slots(d):
    """Boolean mask [n_pre, cap] of slots holding synapses."""
    cap = d["ind"].shape[1]
    return np.arange(cap)[None, :] < d["len"][:, None]


def compare_rows_exact(tag, g, o: oracle.Proj):
    cap = g["ind"].shape[1]
    assert np.array_equal(g["len"], o.len), f"{tag}: row lengths differ"
    m = real_slots(g)
    assert np.array_equal(g["ind"][m], o.ind.reshape(-1, cap)[m]), f"{tag}: indices differ"


def compare_state(snap, N: oracle.Net, cfg: rb.EpropConfig, sigma_w=(1.0, 1.0), learn=True, rtol=RTOL,
                  trace_rtol=None):
    """State after a step against the oracle's; trace_rtol (default rtol) for
    the presynaptic and eligibility traces."""
    trt = rtol if trace_rtol is None else trace_rtol
    close("v", snap["v"], N.v, cfg.v_thr, rtol)
    close("a", snap["a"], N.a, 1.0, rtol)
    close("y", snap["y"], N.y, cfg.v_thr, rtol)
    close("xbar", snap["xbar"], N.xbar, 1.0, trt)
    close("zbar", snap["zbar"], N.zbar, 1.0, trt)
    close("psi", snap["psiT"].T, N.psi, 0.3 / cfg.v_thr, rtol)
    close("delta", snap["deltaT"].T, N.delta, 1.0, rtol)
    close_sum("L", snap["LT"].T, N.L, N.Labs, rtol)
    if not learn:
        return
    close_sum("Gout", snap["Gout"], N.Gout, N.Goutabs, rtol)
    close_sum("Gb", snap["Gb"], N.Gb, N.Gbabs, rtol)
    B = cfg.batch
    for tag, P in (("in", N.inp), ("rec", N.rec)):
        g = snap[tag]
        cap = g["ind"].shape[1]
        m = real_slots(g)
        compare_rows_exact(tag, g, P)
        close_sum(tag + ".G", g["G"][m], P.G.reshape(-1, cap)[m], P.Gabs.reshape(-1, cap)[m], rtol)
        eb = P.ebar.reshape(-1, cap, B)
        close(tag + ".ebar", g["ebar"][m], eb[m], 1.0, trt)
        if cfg.alif:
            close(tag + ".eps", g["eps"][m], P.eps.reshape(-1, cap, B)[m], 1.0, trt)


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


# ---------------------------------------------------------------------------
# One step call in the benchmark's schedule (blocks of steps, the two-stream
# hand-off ring, automatic update and DEEP R of both projections inside the
# call) against the oracle stepping the same steps one by one.

def _adam_bounds(P_or_none, G_pre, Gabs_pre, m_old, g, m, v, w, cfg, k, wscale):
    """Bounds on m, v and w after one Adam step whose gradient g = G/B (+ L1)
    carries the error rtol * (|G| + sum of |terms|) / B of the accumulated sum:
    first-order propagation through the step, plus each value's own rounding."""
    b1, b2, lr, eps = cfg.adam_b1, cfg.adam_b2, cfg.lr, cfg.adam_eps
    c1, c2 = 1 - b1 ** k, 1 - b2 ** k
    g_err = RTOL * (np.abs(G_pre) + Gabs_pre) / cfg.batch
    bm = RTOL * (np.abs(m) + b1 * np.abs(m_old) + (1 - b1) * np.abs(g)) + (1 - b1) * g_err
    bv = 2 * RTOL * np.abs(v) + (1 - b2) * 2 * (np.abs(g) + g_err) * g_err
    s = np.sqrt(v / c2)
    mh = m / c1
    with np.errstate(divide="ignore", invalid="ignore"):
        dm = (1 - b1) / c1 / (s + eps)
        ds = np.where(s > 0, (1 - b2) * (np.abs(g) + g_err) / (c2 * s), 0.0)
        dratio = dm + np.abs(mh) / (s + eps) ** 2 * ds
    bw = RTOL * np.maximum(np.abs(w), wscale) + 2 * lr * dratio * g_err
    return bm, bv, bw


def _carry(bound_pre, len_pre, ind_pre, len_post, ind_post, n_post):
    """Move per-slot bounds along with their synapses through a rewire: a
    synapse is identified by (row, target).  New synapses get bound 0 (they
    start at exactly zero on both sides)."""
    n_pre, cap = ind_pre.shape
    slot_of = np.full((n_pre, n_post), -1, np.int64)
    rows = np.repeat(np.arange(n_pre), len_pre)
    m_pre = np.arange(cap)[None, :] < len_pre[:, None]
    slot_of[rows, ind_pre[m_pre]] = np.nonzero(m_pre)[1]
    m_post = np.arange(cap)[None, :] < len_post[:, None]
    rows_post = np.repeat(np.arange(n_pre), len_post)
    s = slot_of[rows_post, ind_post[m_post]]
    out = np.zeros(m_post.sum())
    have = s >= 0
    out[have] = bound_pre[rows_post[have], s[have]]
    return out


def interval_vs_oracle(net, cfg, raster, labels, n_steps, after=0):
    """Run net.step(n_steps, LEARN | AUTO_UPDATE) from the current state, which
    must sit at an update boundary and within one sample, the call ending at
    the next update, and the oracle over the same steps with its own update and
    DEEP R rewires.  Compares spike counts and the last block's raster exactly,
    rows, bitfields and dormant counts bit for bit, and every value within its
    bound.  Then, with `after` > 0, the oracle takes the GPU's state after the
    update (its weights carry the gradient's rounding, which Adam may amplify)
    and both run `after` more steps in one call each, compared again.  Returns
    the number of updates inside the first call."""
    U, T = cfg.update_interval, cfg.sample_steps
    t0 = int(net.info().step)
    assert t0 % U == 0 and (t0 + n_steps) % U == 0 and t0 % T + n_steps + after <= T and after < U
    pre = snapshot(net)
    zc0 = net.get(rb.ZCOUNT).astype(np.int64)
    adam0 = int(net.info().adam_step)
    net.step(n_steps, rb.RS_LEARN | rb.RS_AUTO_UPDATE)
    post = snapshot(net)
    zc1 = net.get(rb.ZCOUNT).astype(np.int64)
    zbits = net.get(rb.ZBITS)
    last_blk = int(net.info().last_block)

    N = oracle_net(pre, cfg)
    counts = np.zeros((cfg.batch, cfg.n_rec), np.int64)
    raster_tail = []
    bounds = None
    n_upd = 0
    for t in range(t0, t0 + n_steps):
        idx, off = raster.step_lists(t % T)
        N.step(idx, off, labels)
        counts += N.z
        if t >= t0 + n_steps - last_blk:
            raster_tail.append(N.z.T.copy())
        if (t + 1) % U == 0:
            n_upd += 1
            k = adam0 + n_upd
            snap_pre = {}
            for tag, P in (("in", N.inp), ("rec", N.rec)):
                cap = P.cap
                snap_pre[tag] = dict(G=P.G.reshape(-1, cap).copy(), Gabs=P.Gabs.reshape(-1, cap).copy(),
                                     m=P.m.reshape(-1, cap).copy())
            ro = dict(G=N.Gout.copy(), Gabs=N.Goutabs.copy(), m=N.Mout.copy(),
                      Gb=N.Gb.copy(), Gbabs=N.Gbabs.copy(), mb=N.Mb.copy())
            N.adam_update(k, lr=cfg.lr, b1=cfg.adam_b1, b2=cfg.adam_b2, eps=cfg.adam_eps, l1=cfg.l1,
                          deepr_mask=cfg.deepr_mask)
            bounds = {}
            for tag, P, sig, bit in (("in", N.inp, cfg.sigma_in, 1), ("rec", N.rec, cfg.sigma_rec, 2)):
                cap = P.cap
                d = snap_pre[tag]
                g = d["G"] / cfg.batch
                if cfg.deepr_mask & bit:
                    words = P.sign.reshape(P.n_pre, -1)
                    ind = P.ind.reshape(-1, cap)
                    neg = (words[np.arange(P.n_pre)[:, None], ind >> 5] >> (ind & 31)) & 1
                    g = g + np.where(neg == 1, -cfg.l1, cfg.l1)
                bm, bv, bw = _adam_bounds(P, d["G"], d["Gabs"], d["m"], g, P.m.reshape(-1, cap),
                                          P.v.reshape(-1, cap), P.w.reshape(-1, cap), cfg, k, sig)
                bounds[tag] = dict(len=P.len.copy(), ind=P.ind.reshape(-1, cap).copy(), m=bm, v=bv, w=bw)
            bm, bv, bw = _adam_bounds(None, ro["G"], ro["Gabs"], ro["m"], ro["G"] / cfg.batch, N.Mout, N.Vout,
                                      N.Wout, cfg, k, cfg.sigma_out)
            bounds["out"] = dict(m=bm, v=bv, w=bw)
            bm, bv, bw = _adam_bounds(None, ro["Gb"], ro["Gbabs"], ro["mb"], ro["Gb"] / cfg.batch, N.Mb, N.Vb,
                                      N.bout, cfg, k, 1e-3)
            bounds["b"] = dict(m=bm, v=bv, w=bw)
            step = t + 1
            dormant = {}
            for p, (tag, P) in enumerate((("in", N.inp), ("rec", N.rec))):
                if (cfg.deepr_mask >> p) & 1:
                    dormant[tag], _ = oracle.deepr_rewire(cfg.seed, P, step)
    assert n_upd >= 1, "the call must contain an update"
    assert int(net.info().adam_step) == adam0 + n_upd

    # spikes: per-neuron counts over the call and the last block's raster
    assert np.array_equal(zc1 - zc0, counts), "spike counts differ"
    for q, z in enumerate(raster_tail):
        assert np.array_equal((zbits >> q) & 1, z.astype(np.uint32)), f"raster differs at block step {q}"

    # neuron, readout and trace state
    compare_state(post, N, cfg)
    # rows, bitfields and dormant counts bit for bit; parameters within bounds
    for p, (tag, P) in enumerate((("in", N.inp), ("rec", N.rec))):
        g = post[tag]
        cap = P.cap
        compare_rows_exact(tag, g, P)
        if "conn" in g:
            assert np.array_equal(g["conn"].ravel(), P.conn), tag + ": connectivity bits differ"
            assert np.array_equal(g["sign"].ravel(), P.sign), tag + ": sign bits differ"
            assert np.array_equal(g["dormant"], dormant[tag]), tag + ": dormant counts differ"
        b = bounds[tag]
        m = real_slots(g)
        for f, arr in (("w", P.w), ("m", P.m), ("vv", P.v)):
            bf = b["v" if f == "vv" else f]
            carried = _carry(bf, b["len"], b["ind"], P.len, P.ind.reshape(-1, cap), P.n_post)
            close(f"{tag}.{f}", g[f][m], arr.reshape(-1, cap)[m], 0.0, bound=carried)
    for f, arr, key in (("Wout", N.Wout, "w"), ("Mout", N.Mout, "m"), ("Vout", N.Vout, "v")):
        close(f, post[f], arr, 0.0, bound=bounds["out"][key])
    for f, arr, key in (("bout", N.bout, "w"), ("Mb", N.Mb, "m"), ("Vb", N.Vb, "v")):
        close(f, post[f], arr, 0.0, bound=bounds["b"][key])
    if after:
        t1 = t0 + n_steps
        zc0 = net.get(rb.ZCOUNT).astype(np.int64)
        N = oracle_net(post, cfg)
        net.step(after, rb.RS_LEARN | rb.RS_AUTO_UPDATE)
        post2 = snapshot(net)
        counts = np.zeros((cfg.batch, cfg.n_rec), np.int64)
        for t in range(t1, t1 + after):
            idx, off = raster.step_lists(t % T)
            N.step(idx, off, labels)
            counts += N.z
        assert np.array_equal(net.get(rb.ZCOUNT).astype(np.int64) - zc0, counts), "spike counts differ after the update"
        compare_state(post2, N, cfg)
    return n_upd
