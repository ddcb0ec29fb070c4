"""Benchmark: e-prop training of the sparse classifier (700 synthetic input
channels -> 1024 ALIF -> 20 readouts, 10% ragged connectivity, batch 256,
1000 steps per sample batch, Adam + DEEP R every 100 steps) on one MI355X.

One benchmark step = one training batch: 1000 timesteps of the whole path
(input, spikes, propagation, neurons, readout, learning signal, eligibility
traces and gradients) plus 10 parameter updates and 20 DEEP R rewires, and the
state reset at the end of the batch.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# fp32 vector FMA rate without packed instructions (the library is built with
# them disabled): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
FP32_PEAK_TFLOPS = 78.6
# the chip's fp32 vector figure counts packed FMAs (two per lane and cycle)
FP32_PACKED_PEAK_TFLOPS = 157.3


def classifier_config(seed=1, trace_block=0):
    from paper_2510_19764_amd import binding as rb
    from paper_2510_19764_amd import workload as wl
    c = wl.SHD_CLASSIFIER
    f32 = lambda x: float(np.float32(x))
    return rb.EpropConfig(n_in=c["n_in"], n_rec=c["n_rec"], n_out=c["n_out"], batch=c["batch"], alif=c["alif"],
                          p_in=c["p_in"], p_rec=c["p_rec"], sigma_in=f32(wl.sigma_init(c["p_in"], c["n_in"])),
                          sigma_rec=f32(wl.sigma_init(c["p_rec"], c["n_rec"])),
                          sigma_out=f32(1.0 / np.sqrt(c["n_rec"])), deepr_mask=c["deepr_mask"], l1=c["l1"],
                          lr=c["lr"], update_interval=c["update_interval"], sample_steps=c["T"], seed=seed,
                          trace_block=trace_block)


def eprop_algorithmic_bytes(cfg, n_syn: int, n_launch: int, n_steps: int) -> int:
    """HBM bytes the e-prop launches must move at minimum over n_steps steps in
    n_launch launches.  Per launch and synapse: eps and ebar of every batch
    instance read and written once (16 B per instance; 8 B for LIF), its
    column-view entry (8 B) and gradient read and written (8 B), and the
    readout gradient.
    Per step: each per-neuron, per-instance input read once (presynaptic
    traces before the step, psi, L, the recurrent trace after the step) and
    the output errors."""
    B = cfg.batch
    per_unit = 16 if cfg.alif else 8
    per_launch = n_syn * (per_unit * B + 16) + 8 * cfg.n_out * cfg.n_rec + 8 * cfg.n_out
    per_step = 4 * B * (cfg.n_in + 4 * cfg.n_rec + cfg.n_out)
    return n_launch * per_launch + n_steps * per_step


def eprop_algorithmic_flops(cfg, n_syn: int, n_steps: int) -> int:
    """Float operations of the method over n_steps steps: per synapse, instance
    and step e = psi (p - beta eps) (3), eps' = psi p + (rho - psi beta) eps
    as eps + (e - (1 - rho) eps) (3), ebar' = alpha ebar + e (2) and
    G += L ebar' (2) for ALIF; e = psi p (1), ebar' (2), G (2) for LIF; plus
    the readout gradient, 2 per readout weight, instance and step."""
    per_syn = 10 if cfg.alif else 5
    B = cfg.batch
    return n_steps * B * (n_syn * per_syn + 2 * cfg.n_out * cfg.n_rec + cfg.n_out)


EPROP_KERNEL = "k_eprop_tc<true>"  # the classifier's e-prop kernel (batch 256, ALIF)


def recorded_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes (calibrated against a plain copy), or None when the
    kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "eprop_tc_classifier_traffic.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("kernel") != kernel or hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return int(rec["hbm_bytes_per_dispatch"])


def tiny_config(seed=1):
    from paper_2510_19764_amd import binding as rb
    from paper_2510_19764_amd import workload as wl
    c = wl.TINY_EPROP
    f32 = lambda x: float(np.float32(x))
    return rb.EpropConfig(n_in=c["n_in"], n_rec=c["n_rec"], n_out=c["n_out"], batch=c["batch"], alif=c["alif"],
                          p_in=c["p_in"], p_rec=c["p_rec"], sigma_in=f32(wl.sigma_init(c["p_in"], c["n_in"])),
                          sigma_rec=f32(wl.sigma_init(c["p_rec"], c["n_rec"])),
                          sigma_out=f32(1.0 / np.sqrt(c["n_rec"])), deepr_mask=c["deepr_mask"], l1=c["l1"],
                          lr=c["lr"], update_interval=c["update_interval"], sample_steps=c["T"], seed=seed)


def oracle_from_seed(cfg):
    """The oracle network built from the same seed as the library's."""
    import oracle
    B = cfg.batch
    f32 = lambda x: float(np.float32(x))
    projs = []
    for n_pre, rec, p, sig, pid in ((cfg.n_in, False, cfg.p_in, cfg.sigma_in, 0),
                                    (cfg.n_rec, True, cfg.p_rec, cfg.sigma_rec, 1)):
        _, mx = oracle.fixed_prob_count(cfg.seed, n_pre, cfg.n_rec, p, rec, pid)
        P = oracle.Proj(n_pre, cfg.n_rec, min(2 * mx, cfg.n_rec), rec, pid, batch=B, trained=True,
                        traces="alif" if cfg.alif else "lif", bitfields=True)
        oracle.fixed_prob_rows(cfg.seed, P, p, sig)
        oracle.deepr_init_bits(cfg.seed, P)
        projs.append(P)
    prm = oracle.EpropParams(n_in=cfg.n_in, n_rec=cfg.n_rec, n_out=cfg.n_out, batch=B, alif=cfg.alif,
                             v_thr=f32(cfg.v_thr), beta=f32(cfg.beta))
    N = oracle.Net(prm, projs[0], projs[1])
    N.Wout[:] = oracle.dense_init(cfg.seed, 2, cfg.n_out, cfg.n_rec, cfg.sigma_out)
    return N


def host_cpu_info():
    """The timing host: logical CPUs, those this process may use, the model."""
    import platform
    import subprocess
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
            else None, "omp_num_threads": os.environ.get("OMP_NUM_THREADS"), "machine": platform.machine()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)"):
                info["lscpu " + k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def time_oracle_interval(cfg, raster, labels, n_steps: int):
    """Seconds per timestep and per update + two DEEP R rewires of the oracle
    (whichever build is in use) over n_steps steps of the workload."""
    import oracle
    N = oracle_from_seed(cfg)
    t0 = time.perf_counter()
    for t in range(n_steps):
        idx, off = raster.step_lists(t)
        N.step(idx, off, labels)
    t_step = (time.perf_counter() - t0) / n_steps
    t1 = time.perf_counter()
    N.adam_update(1, lr=cfg.lr, l1=cfg.l1, deepr_mask=cfg.deepr_mask)
    oracle.deepr_rewire(cfg.seed, N.inp, n_steps)
    oracle.deepr_rewire(cfg.seed, N.rec, n_steps)
    return t_step, time.perf_counter() - t1


def run_cpu_baseline(cfg, raster, labels, n_steps: int):
    """The oracle (fp64 C) timed on the host's cores: its multi-core build
    (OpenMP over independent instances, rows and readout units; results equal
    to the parity build's bit for bit) over one whole update interval (the
    interval's steps, the update and both DEEP R rewires), and the
    single-threaded parity build over n_steps steps and one update; each
    extrapolated linearly to the 1000-step, 10-update batch."""
    import oracle
    B, T, U = cfg.batch, cfg.sample_steps, cfg.update_interval
    threads = oracle.use_multicore(True)
    try:
        mc_step, mc_upd = time_oracle_interval(cfg, raster, labels, U)
    finally:
        oracle.use_multicore(False)
    st_step, st_upd = time_oracle_interval(cfg, raster, labels, n_steps)
    mc_batch = T * mc_step + (T // U) * mc_upd
    st_batch = T * st_step + (T // U) * st_upd
    return {"value": B / mc_batch, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"one whole update interval ({U} timesteps, the Adam update and both DEEP R rewires) of one "
                      f"{B}-sample batch on {threads} threads, extrapolated linearly to the {T}-step batch",
            "seconds_per_timestep": mc_step, "seconds_per_update_rewire": mc_upd,
            "single_thread": {"value": B / st_batch, "unit": "samples/s", "cores": 1,
                              "sample": f"{n_steps} of {T} timesteps and one update + DEEP R, extrapolated",
                              "seconds_per_timestep": st_step, "seconds_per_update_rewire": st_upd},
            "host": host_cpu_info()}


def tiny_net_leg(samples=20, oracle_samples=2):
    """The tiny e-prop network (100 Poisson inputs at U[0, 50) Hz -> 128 LIF ->
    4 readouts, p = 0.1, batch 1, 500 steps per sample, Adam + DEEP R every 25
    steps) trained sample after sample with the device Poisson source; the
    oracle runs the same workload (its own Poisson source) beside it."""
    import torch
    import oracle
    from paper_2510_19764_amd import binding as rb
    from paper_2510_19764_amd import workload as wl
    cfg = tiny_config()
    T, U = cfg.sample_steps, cfg.update_interval
    rates = wl.poisson_rates(cfg.seed, cfg.n_in, wl.TINY_EPROP["max_rates_hz"])
    labels = np.zeros(cfg.batch, np.int32)
    net = rb.EpropNet(cfg)
    net.set_input_poisson(rates, torch.tensor(labels, device="cuda"))
    flags = rb.RS_LEARN | rb.RS_AUTO_UPDATE | rb.RS_AUTO_RESET
    net.step(T, flags)
    torch.cuda.synchronize()
    i0 = net.info()
    ev0, el0 = i0.synaptic_events, i0.eliminated
    t0 = time.perf_counter()
    for _ in range(samples):
        net.step(T, flags)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    i1 = net.info()
    n_syn = int(net.get(rb.PROJ(0, rb.P_LEN)).sum() + net.get(rb.PROJ(1, rb.P_LEN)).sum())
    net.close()
    steps = samples * T
    # the oracle: same steps, updates, rewires and resets
    N = oracle_from_seed(cfg)
    thr = oracle.rate_thresholds(rates, cfg.dt_ms)
    k = 0
    t1 = time.perf_counter()
    for t in range(oracle_samples * T):
        idx, off = oracle.poisson_input(cfg.seed, t, cfg.batch, thr)
        N.step(idx, off, labels)
        if (t + 1) % U == 0:
            k += 1
            N.adam_update(k, lr=cfg.lr, l1=cfg.l1, deepr_mask=cfg.deepr_mask)
            oracle.deepr_rewire(cfg.seed, N.inp, t + 1)
            oracle.deepr_rewire(cfg.seed, N.rec, t + 1)
        if (t + 1) % T == 0:
            N.reset()
    orc_s = (time.perf_counter() - t1) / (oracle_samples * T)
    return {"workload": "tiny e-prop net 100 Poisson (U[0,50) Hz) -> 128 LIF -> 4, p=0.1, batch 1, "
                        "500 steps/sample, Adam + DEEP R every 25 steps",
            "samples": samples, "steps_per_s": round(steps / el, 1), "us_per_step": round(1e6 * el / steps, 3),
            "synaptic_events_per_s": round((i1.synaptic_events - ev0) / el, 1),
            "synapses": n_syn,
            "rewired_fraction_per_update": (i1.eliminated - el0) / (samples * (T // U) * n_syn),
            "oracle_us_per_step": round(1e6 * orc_s, 3), "oracle_cores": 1,
            "oracle_sample": f"{oracle_samples} samples of the same workload",
            "gpu_over_oracle": round(orc_s / (el / steps), 2)}


def batched_configs(n=None, seed=1):
    """The batched-instances workload: n classifiers (recurrent sizes
    log-uniform in [256, 4096], connection probabilities uniform in
    [0.05, 0.2]) on the sparse classifier's input, batch 1 each."""
    from paper_2510_19764_amd import binding as rb
    from paper_2510_19764_amd import workload as wl
    c = wl.BATCHED
    n = n or c["n_inst"]
    f32 = lambda x: float(np.float32(x))
    cfgs = []
    for i, (n_rec, p) in enumerate(wl.batched_sizes(seed, n, c["n_rec_lo"], c["n_rec_hi"], c["p_lo"], c["p_hi"])):
        cfgs.append(rb.EpropConfig(n_in=c["n_in"], n_rec=n_rec, n_out=c["n_out"], batch=c["batch"], alif=c["alif"],
                                   p_in=p, p_rec=p, sigma_in=f32(wl.sigma_init(p, c["n_in"])),
                                   sigma_rec=f32(wl.sigma_init(p, n_rec)), sigma_out=f32(1.0 / np.sqrt(n_rec)),
                                   deepr_mask=c["deepr_mask"], l1=c["l1"], lr=c["lr"],
                                   update_interval=c["update_interval"], sample_steps=c["T"], seed=seed + 1 + i))
    return cfgs


def batched_leg(n=None, samples=3, plain_rounds=1):
    """Batched instances: the set trained together (rs_multi: one launch per
    kernel and block for all instances, the sample replayed from a graph,
    the tuned e-prop schedule) against the plain loop that trains the same
    networks one after another (rs_eprop_step per network), on the same GPU.
    Both compute the same results bit for bit (tests/test_gpu_multi.py); one
    round of the plain loop and one sample of the set both train every
    instance on one sample."""
    import torch
    from paper_2510_19764_amd import binding as rb
    from paper_2510_19764_amd import workload as wl
    cfgs = batched_configs(n)
    T = cfgs[0].sample_steps
    gen = wl.ShdLike(T=T)
    dev = []
    for i in range(len(cfgs)):
        labels, raster = gen.batch(seed=1, batch_index=i, B=1)
        dev.append((torch.tensor(raster.off, dtype=torch.int32, device="cuda"),
                    torch.tensor(raster.idx, dtype=torch.int32, device="cuda"),
                    torch.tensor(labels, dtype=torch.int32, device="cuda")))
    m = rb.MultiNet(cfgs)
    for i, d in enumerate(dev):
        m.set_input(i, *d)
    n_syn = sum(int(m.get(i, rb.PROJ(0, rb.P_LEN)).sum() + m.get(i, rb.PROJ(1, rb.P_LEN)).sum())
                for i in range(len(cfgs)))
    m.train(5)  # tuning: one sample per e-prop schedule
    m.train(1)  # the graph is recorded
    torch.cuda.synchronize()
    ev0 = sum(m.info(i).synaptic_events for i in range(len(cfgs)))
    t0 = time.perf_counter()
    m.train(samples)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ev1 = sum(m.info(i).synaptic_events for i in range(len(cfgs)))
    sch = m.schedule()
    m.close()
    nets = [rb.EpropNet(c) for c in cfgs]
    flags = rb.RS_LEARN | rb.RS_AUTO_UPDATE | rb.RS_AUTO_RESET
    for net, d in zip(nets, dev):
        net.set_input(*d)
        net.step(T, flags)  # warm-up round
    torch.cuda.synchronize()
    pev0 = sum(net.info().synaptic_events for net in nets)
    t1 = time.perf_counter()
    for _ in range(plain_rounds):
        for net in nets:
            net.step(T, flags)
    torch.cuda.synchronize()
    pel = time.perf_counter() - t1
    pev1 = sum(net.info().synaptic_events for net in nets)
    for net in nets:
        net.close()
    ni = len(cfgs)
    batched = ni * samples / el
    plain = ni * plain_rounds / pel
    return {"workload": f"{ni} e-prop classifiers 700 -> N_i ALIF -> 20, N_i log-uniform in [256, 4096], "
                        f"p_i uniform in [0.05, 0.2], batch 1 each, {T} steps/sample, Adam + DEEP R every "
                        f"{cfgs[0].update_interval} steps, synthetic SHD-shaped input",
            "instances": ni, "synapses": n_syn,
            "batched": {"samples_per_s": round(batched, 2), "ms_per_sample_of_the_set": round(1e3 * el / samples, 3),
                        "synaptic_events_per_s": round((ev1 - ev0) / el, 1), "samples_timed": samples,
                        "schedule": sch},
            "plain_loop": {"samples_per_s": round(plain, 2), "ms_per_round": round(1e3 * pel / plain_rounds, 3),
                           "synaptic_events_per_s": round((pev1 - pev0) / pel, 1), "rounds_timed": plain_rounds},
            "batched_over_plain": round(batched / plain, 2),
            "results": "identical bit for bit (tests/test_gpu_multi.py)"}


def served_leg(duration_s=2.0, rate_hz=2000.0, baseline_requests=150, seed=1):
    """Served inference: a Poisson request stream (mean rate_hz) of
    classification runs on networks of 512, 1024, 2048 and 4096 ALIF neurons
    (p = 0.1, 700 inputs, 20 readouts, weights from a fixed seed), presentation
    lengths uniform in [200, 1500] steps, inputs from a pool of synthetic
    SHD-shaped samples resident on the device.  Replayed against the wall
    clock with continuous batching (rs_serve: requests join the running block
    launches as slots free), and the first requests of the same trace with one
    request per launch."""
    import torch
    from paper_2510_19764_amd import binding as rb
    from paper_2510_19764_amd import workload as wl
    f32 = lambda x: float(np.float32(x))
    sizes = (512, 1024, 2048, 4096)
    models = [rb.EpropNet(rb.EpropConfig(n_in=700, n_rec=n, n_out=20, batch=1, alif=True, p_in=0.1, p_rec=0.1,
                                         sigma_in=f32(wl.sigma_init(0.1, 700)), sigma_rec=f32(wl.sigma_init(0.1, n)),
                                         sigma_out=f32(1.0 / np.sqrt(n)), update_interval=0, sample_steps=1500,
                                         seed=seed + q))
              for q, n in enumerate(sizes)]
    T = 1500
    gen = wl.ShdLike(T=T)
    pool = []
    for q in range(16):
        labels, raster = gen.batch(seed=seed, batch_index=100 + q, B=1)
        pool.append((torch.tensor(raster.off, dtype=torch.int32, device="cuda"),
                     torch.tensor(raster.idx, dtype=torch.int32, device="cuda"), T))
    rng = np.random.Generator(np.random.Philox(seed + 31337))
    n = int(rate_hz * duration_s)
    arrivals = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    ms = rng.integers(0, len(sizes), n)
    lens = rng.integers(200, 1501, n)
    rasters = [pool[q % len(pool)] for q in range(n)]
    out = {"workload": f"Poisson requests at {rate_hz:g}/s for {duration_s:g} s on 700 -> N ALIF -> 20 classifiers, "
                       f"N in {list(sizes)}, p = 0.1, presentation lengths uniform in [200, 1500] steps, "
                       f"synthetic SHD-shaped inputs", "requests": n}
    srv = rb.Server(models, slots_per_model=1024, block_steps=20, max_running=4096, state_budget_bytes=2 << 30)
    # warm-up: a few requests through every model
    srv.replay(np.zeros(8), np.arange(8) % 4, np.full(8, 40), rasters[:8])
    t0 = time.perf_counter()
    lat, dec, spk = srv.replay(arrivals, ms, lens, rasters)
    el = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    ok = lat >= 0
    out["continuous_batching"] = {
        "p50_ms": round(float(np.percentile(lat[ok], 50)), 3), "p99_ms": round(float(np.percentile(lat[ok], 99)), 3),
        "mean_ms": round(float(lat[ok].mean()), 3), "completed": int(ok.sum()), "rejected": int((~ok).sum()),
        "samples_per_s": round(float(ok.sum()) / el, 1), "wall_s": round(el, 3),
        "request_steps_per_s": round(float(lens[ok].sum()) / el, 1), "blocks": st["blocks"]}
    nb = min(baseline_requests, n)
    one = rb.Server(models, slots_per_model=1, block_steps=20, max_running=1, state_budget_bytes=2 << 30)
    t0 = time.perf_counter()
    lat1, dec1, spk1 = one.replay(arrivals[:nb], ms[:nb], lens[:nb], rasters[:nb])
    el1 = time.perf_counter() - t0
    one.close()
    out["one_request_per_launch"] = {
        "requests": nb, "p50_ms": round(float(np.percentile(lat1, 50)), 3),
        "p99_ms": round(float(np.percentile(lat1, 99)), 3), "samples_per_s": round(nb / el1, 1),
        "wall_s": round(el1, 3)}
    out["same_results_as_continuous"] = bool(np.array_equal(dec1, dec[:nb]) and np.array_equal(spk1, spk[:nb]))
    for m in models:
        m.close()
    return out


def forward_only_leg(steps=1000):
    """The classifier's forward pass alone (no eligibility work): wall time and
    the forward launches' device time over `steps` steps, after as many
    warm-up steps."""
    import torch
    from paper_2510_19764_amd import binding as rb
    from paper_2510_19764_amd import workload as wl
    cfg = classifier_config()
    labels, raster = wl.ShdLike(T=cfg.sample_steps).batch(seed=1, batch_index=0, B=cfg.batch)
    dev = (torch.tensor(raster.off, dtype=torch.int32, device="cuda"),
           torch.tensor(raster.idx, dtype=torch.int32, device="cuda"),
           torch.tensor(labels, dtype=torch.int32, device="cuda"))
    net = rb.EpropNet(cfg)
    net.set_input(*dev)
    net.step(steps, 0)
    torch.cuda.synchronize()
    net.timing(0b00001)  # the forward launches
    net.phase_times()
    t0 = time.perf_counter()
    net.step(steps, 0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, n = net.phase_times()["forward"]
    net.close()
    return {"steps": steps, "trace_block": cfg.trace_block, "wall_ms": round(1e3 * el, 3),
            "forward_ms": round(ms, 3), "forward_launches": n}


def topo_rewire_latency(n_rewires=200):
    """Topographic-map rewiring (64 x 64 sheets, cap 32, 160 attempts)."""
    from paper_2510_19764_amd import binding as rb
    from paper_2510_19764_amd import workload as wl
    import torch
    c = wl.TOPO_S4
    out = {}
    for name, ff in (("ff", c["ff"]), ("lat", c["lat"])):
        t = rb.TopoNet(rb.TopoConfig(L=c["L"], cap=c["cap"], n_attempts=c["n_attempts"], proj_id=0 if name == "ff" else 1,
                                     p_form=ff["p_form"], sigma_form=ff["sigma"], g_theta=c["g_max"] / 2,
                                     p_elim_dep=c["p_elim_dep"], p_elim_pot=c["p_elim_pot"], g_new=c["g_max"],
                                     g_init=c["g_max"], seed=1))
        for s in range(10):
            t.rewire(s * 10, stats=False)
        torch.cuda.synchronize()
        ms = []
        for s in range(n_rewires):
            t.rewire(1000 + 10 * s, stats=False)
            ms.append(t.last_ms())
        t0 = time.perf_counter()
        for s in range(n_rewires):
            t.rewire(10**6 + 10 * s, stats=False)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / n_rewires
        out[name] = {"device_us": 1e3 * float(np.mean(ms)), "wall_us": 1e6 * wall}
        t.close()
    return out


def topo_sim_leg(steps=1_000_000, oracle_steps=5000, stim="bar"):
    """The topographic map end to end (64 x 64 Poisson sheet -> 64 x 64
    conductance-LIF sheet, cap 32, STDP, 160 rewiring attempts every 10 steps,
    h = 0.1 ms), from a fresh build: realtime factor, steps/s, and the split
    between simulation and rewiring from a second run with rewiring off.  The
    oracle runs the first `oracle_steps` steps of the same workload."""
    import torch
    import oracle
    from paper_2510_19764_amd import binding as rb
    from paper_2510_19764_amd import workload as wl
    c = wl.TOPO_S4
    kind = rb.STIM_BAR if stim == "bar" else rb.STIM_BLOB
    cfg = rb.TopoConfig(L=c["L"], cap=c["cap"], n_attempts=c["n_attempts"], proj_id=0,
                        p_form=c["ff"]["p_form"], sigma_form=c["ff"]["sigma"], g_theta=c["g_max"] / 2,
                        p_elim_dep=c["p_elim_dep"], p_elim_pot=c["p_elim_pot"], g_new=c["g_max"],
                        g_init=c["g_max"], seed=1)
    out = {"workload": f"topographic map 64x64 -> 64x64 conductance LIF, cap 32, STDP, {stim} stimulus, "
                       f"160 rewiring attempts every 10 steps, h = 0.1 ms",
           "steps": steps, "model_seconds": steps * 1e-4}
    for name, R in (("with_rewiring", c["rewire_every"]), ("simulation_only", 0)):
        model = rb.TopoModel(stim_kind=kind, rewire_steps=R)
        t = rb.TopoNet(cfg)
        t.sim_init(model)
        t.run(1000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t.run(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        dev_ms = t.last_ms()
        st = t.run_stats()
        n_syn = int(t.get_rows()[0].sum())
        spikes = int(t.sim_get(rb.TV_COUNT).sum())
        if R:
            # the Fig. 10 style split, from the kernel's phase timers over 100000 further steps
            n_ph = 100_000
            t.sim_timing(True)
            t.run(n_ph)
            torch.cuda.synchronize()
            ph = t.sim_phase_ms()
            tot = t.last_ms()
            t.sim_timing(False)
            split = {k: round(1e3 * v / n_ph, 3) for k, v in ph.items()}
            split["rewire_kernels_and_launch_gaps"] = round(1e3 * (tot - sum(ph.values())) / n_ph, 3)
            out["phase_us_per_step"] = split
        t.close()
        out[name] = {"wall_s": round(el, 4), "device_ms": round(dev_ms, 3),
                     "steps_per_s": round(steps / el, 1), "us_per_step": round(1e6 * el / steps, 3),
                     "realtime_factor": round(steps * 1e-4 / el, 2), "target_spikes": spikes,
                     "synapses_at_end": n_syn}
        if R:
            out[name].update(eliminated=st.eliminated, formed=st.formed, blocked=st.blocked)
    w, s_ = out["with_rewiring"]["wall_s"], out["simulation_only"]["wall_s"]
    out["phase_split"] = {"simulation_s": s_, "rewiring_and_remap_s": round(w - s_, 4),
                          "rewiring_fraction": round((w - s_) / w, 4)}
    # the oracle on the same workload
    M = oracle.TopoModel(L=c["L"], stim_kind=kind, h=float(np.float32(0.1)))
    P = oracle.Proj(c["L"] ** 2, c["L"] ** 2, c["cap"], False, 0)
    f = lambda x: float(np.float32(x))
    oracle.gauss_rows(cfg.seed, P, c["L"], f(cfg.p_form), f(cfg.sigma_form), f(cfg.g_init))
    tp = oracle.TopoParams(L=c["L"], n_attempts=c["n_attempts"], p_form=f(cfg.p_form), sigma_form=f(cfg.sigma_form),
                           g_theta=f(cfg.g_theta), p_elim_dep=f(cfg.p_elim_dep), p_elim_pot=f(cfg.p_elim_pot),
                           g_new=f(cfg.g_new))
    S = oracle.TopoState(M)
    t0 = time.perf_counter()
    oracle.topo_run(cfg.seed, M, P, tp, S, 0, oracle_steps)
    orc = (time.perf_counter() - t0) / oracle_steps
    out["oracle"] = {"us_per_step": round(1e6 * orc, 3), "cores": 1,
                     "sample": f"the first {oracle_steps} steps of the same workload"}
    out["gpu_over_oracle"] = round(orc / (out["with_rewiring"]["wall_s"] / steps), 2)
    return out


def topo_scaling_leg(steps=20000, scales=(1, 2, 3, 4, 5, 6, 7)):
    """The paper's scaling experiment (Fig. 10): the full topographic-map model
    -- feed-forward and lateral projections with STDP and rewiring, blob input
    replicated in every 16 x 16 square -- at L = 16 s for s = 1..7, 10 s^2
    rewiring attempts per projection every 1 ms, h = 0.1 ms, on the tiled
    kernel: wall time per step, realtime factor and the kernel's phase split.
    Also the 64 x 64 feed-forward map of the end-to-end leg on both kernels."""
    import torch
    from paper_2510_19764_amd import binding as rb
    from paper_2510_19764_amd import workload as wl
    c = wl.TOPO_S4
    gm = c["g_max"]
    out = {"workload": "topographic map L = 16 s, s = 1..7: Poisson sheet -> conductance-LIF sheet (p_form 0.16, "
                       "sigma 2.5) plus lateral target -> target rows (p_form 1, sigma 1), cap 64, STDP on both, "
                       "10 s^2 rewiring attempts per projection every 10 steps, blob stimulus replicated per "
                       "16 x 16 square, h = 0.1 ms",
           "steps": steps, "model_seconds": steps * 1e-4, "by_scale": {}}
    for sc in scales:
        L = 16 * sc
        ffc = rb.TopoConfig(L=L, cap=64, n_attempts=10 * sc * sc, proj_id=0, p_form=0.16, sigma_form=2.5,
                            g_theta=gm / 2, p_elim_dep=c["p_elim_dep"], p_elim_pot=c["p_elim_pot"], g_new=gm,
                            g_init=gm, seed=sc)
        latc = rb.TopoConfig(L=L, cap=64, n_attempts=10 * sc * sc, proj_id=1, p_form=1.0, sigma_form=1.0,
                             g_theta=gm / 2, p_elim_dep=c["p_elim_dep"], p_elim_pot=c["p_elim_pot"], g_new=gm,
                             g_init=gm, seed=sc)
        t = rb.TopoNet(ffc)
        t.add_lateral(latc)
        t.sim_init(rb.TopoModel(stim_tile=16, rewire_steps=10))
        t.run(1000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t.run(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st, sl = t.run_stats(), t.run_stats(lateral=True)
        n_ph = min(steps, 10000)
        t.sim_timing(True)
        t.run(n_ph)
        torch.cuda.synchronize()
        ph = t.sim_phase_ms()
        tot = t.last_ms()
        t.sim_timing(False)
        split = {k: round(1e3 * v / n_ph, 3) for k, v in ph.items()}
        split["rewire_kernels_and_launch_gaps"] = round(1e3 * (tot - sum(ph.values())) / n_ph, 3)
        out["by_scale"][str(sc)] = {
            "L": L, "neurons_per_sheet": L * L, "us_per_step": round(1e6 * el / steps, 3),
            "realtime_factor": round(steps * 1e-4 / el, 2), "target_spikes": int(t.sim_get(rb.TV_COUNT).sum()),
            "ff_synapses": int(t.get_rows()[0].sum()), "lateral_synapses": int(t.get_rows(lateral=True)[0].sum()),
            "ff_rewires": {"eliminated": st.eliminated, "formed": st.formed, "blocked": st.blocked},
            "lateral_rewires": {"eliminated": sl.eliminated, "formed": sl.formed, "blocked": sl.blocked},
            "phase_us_per_step": split}
        t.close()
        print(f"[bench] topomap scale {sc}: {out['by_scale'][str(sc)]['us_per_step']} us/step", file=sys.stderr,
              flush=True)
    us = [out["by_scale"][str(sc)]["us_per_step"] for sc in scales]
    out["time_ratio_largest_to_smallest"] = round(us[-1] / us[0], 2)
    # the end-to-end leg's 64 x 64 feed-forward map on both kernels
    cfg = rb.TopoConfig(L=c["L"], cap=c["cap"], n_attempts=c["n_attempts"], proj_id=0, p_form=c["ff"]["p_form"],
                        sigma_form=c["ff"]["sigma"], g_theta=gm / 2, p_elim_dep=c["p_elim_dep"],
                        p_elim_pot=c["p_elim_pot"], g_new=gm, g_init=gm, seed=1)
    kern = {}
    for name, kind in (("one_workgroup", rb.TOPO_KERNEL_ONE_WG), ("tiled", rb.TOPO_KERNEL_TILED)):
        t = rb.TopoNet(cfg)
        t.sim_kernel(kind)
        t.sim_init(rb.TopoModel(stim_kind=rb.STIM_BAR, rewire_steps=c["rewire_every"]))
        t.run(1000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t.run(steps)
        torch.cuda.synchronize()
        kern[name] = round(1e6 * (time.perf_counter() - t0) / steps, 3)
        t.close()
    out["map64_feed_forward_us_per_step"] = kern
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--no-topo", action="store_true")
    ap.add_argument("--no-tiny", action="store_true")
    ap.add_argument("--only-tiny", action="store_true",
                    help="run only the tiny-network leg and print its figures (for profiling)")
    ap.add_argument("--only-topo", action="store_true",
                    help="run only the topographic-map end-to-end leg and print its figures (for profiling)")
    ap.add_argument("--only-topo-scaling", action="store_true",
                    help="run only the topographic-map scaling leg (s = 1..7, lateral projection)")
    ap.add_argument("--topo-scaling-steps", type=int, default=20000)
    ap.add_argument("--topo-steps", type=int, default=1_000_000,
                    help="steps of the topographic-map leg (default 10^6 = 100 s of model time)")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched-instances leg and print its figures (for profiling)")
    ap.add_argument("--batched-instances", type=int, default=0, help="instances of the batched leg (default 64)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--only-served", action="store_true",
                    help="run only the served-inference leg and print its figures (for profiling)")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--forward-only", action="store_true",
                    help="time only the classifier's forward pass, without learning (for profiling)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain copy of this many MiB 20 times (byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this engine runs on one GPU; multi-GPU runs are not part of this build "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_19764_amd import binding as rb
    from paper_2510_19764_amd import workload as wl
    torch.cuda.set_device(0)

    if args.calib_copy_mib:
        n = args.calib_copy_mib << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        for _ in range(20):
            rb.calib_copy(b, a, n)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": n, "launches": 20}))
        return

    if args.only_tiny:
        print(json.dumps({"tiny_net": tiny_net_leg()}), flush=True)
        return
    if args.only_topo:
        print(json.dumps({"topomap_sim": topo_sim_leg(steps=args.topo_steps)}), flush=True)
        return
    if args.only_served:
        print(json.dumps({"served": served_leg()}), flush=True)
        return
    if args.only_topo_scaling:
        print(json.dumps({"topomap_scaling": topo_scaling_leg(steps=args.topo_scaling_steps)}), flush=True)
        return
    if args.only_batched:
        print(json.dumps({"batched": batched_leg(args.batched_instances or None)}), flush=True)
        return
    if args.forward_only:
        print(json.dumps({"forward_only": forward_only_leg()}), flush=True)
        return

    cfg = classifier_config()
    print(f"[bench] generating synthetic input ({cfg.batch} samples x {cfg.sample_steps} steps)",
          file=sys.stderr, flush=True)
    gen = wl.ShdLike(T=cfg.sample_steps)
    batches = [gen.batch(seed=1, batch_index=q, B=cfg.batch) for q in range(2)]
    dev = []
    for labels, raster in batches:
        dev.append((torch.tensor(raster.off, dtype=torch.int32, device="cuda"),
                    torch.tensor(raster.idx, dtype=torch.int32, device="cuda"),
                    torch.tensor(labels, dtype=torch.int32, device="cuda")))
    net = rb.EpropNet(cfg)
    inf = net.info()
    n_syn = int(net.get(rb.PROJ(0, rb.P_LEN)).sum() + net.get(rb.PROJ(1, rb.P_LEN)).sum())
    flags = rb.RS_LEARN | rb.RS_AUTO_UPDATE | rb.RS_AUTO_RESET
    T = cfg.sample_steps

    def one_batch(q):
        net.set_input(*dev[q % 2])
        net.step(T, flags)

    print(f"[bench] warmup {args.warmup} batch(es)", file=sys.stderr, flush=True)
    for q in range(args.warmup):
        one_batch(q)
    torch.cuda.synchronize()
    inf0 = net.info()
    ev0 = inf0.synaptic_events
    # the timed region times the e-prop launches only (each timed phase adds
    # two events to the stream; timing every phase costs about 3%)
    net.timing(0b00010)
    net.phase_times()
    print(f"[bench] timing {args.steps} batch(es)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in range(args.steps):
        one_batch(args.warmup + q)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    phases = net.phase_times()
    net.timing(False)
    inf = net.info()
    # per-phase split from one more batch, outside the timed region
    net.timing(0b11110)  # every phase except the per-block forward launch
    net.phase_times()
    one_batch(args.warmup + args.steps)
    torch.cuda.synchronize()
    split = net.phase_times()
    net.timing(False)
    events = inf.synaptic_events - ev0
    n_syn_after = int(net.get(rb.PROJ(0, rb.P_LEN)).sum() + net.get(rb.PROJ(1, rb.P_LEN)).sum())
    assert n_syn_after == n_syn, "DEEP R must keep the synapse count"

    inf_k, inf_k0 = net.info().trace_block, net.info().first_block
    samples = args.steps * cfg.batch
    value = samples / elapsed
    ep_ms, ep_n = phases["eprop"]
    ep_avg_s = ep_ms / 1e3 / max(ep_n, 1)
    alg_bytes = eprop_algorithmic_bytes(cfg, n_syn, ep_n, args.steps * T)
    achieved = alg_bytes / (ep_ms / 1e3) / 1e9
    alg_flops = eprop_algorithmic_flops(cfg, n_syn, args.steps * T)
    achieved_tf = alg_flops / (ep_ms / 1e3) / 1e12
    result = {
        "metric": "train samples/s (e-prop + DEEP R, sparse classifier)",
        "value": round(value, 2),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": "sparse-classifier 700->1024 ALIF->20, p=0.1, batch 256, 1000 steps/sample, "
                               "Adam + DEEP R every 100 steps, synthetic SHD-shaped input",
                   "global_batch": cfg.batch, "seq_len": T, "parallelism": "single GPU",
                   "synapses": n_syn, "row_capacity": [inf.cap_in, inf.cap_rec]},
        "synaptic_events_per_s": round(events / elapsed, 1),
        "timesteps_per_s": round(args.steps * T / elapsed, 1),
        "phase_ms_per_batch": {k: round(v[0], 3) for k, v in split.items() if k != "forward"},
        "phase_split_from": "one batch after the timed region, every phase timed",
        # DEEP R: synapses eliminated (and as many formed) per update, over all synapses
        "rewired_fraction_per_update": (inf.eliminated - inf0.eliminated) / (args.steps * (T // cfg.update_interval)
                                                                             * n_syn),
        "roofline": {"bound": "hbm", "kernel": EPROP_KERNEL, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic(EPROP_KERNEL),
                     "algorithmic_bytes_per_launch": round(alg_bytes / max(ep_n, 1)),
                     "avg_launch_us": round(ep_avg_s * 1e6, 2), "launches": ep_n,
                     "trace_block": inf_k, "first_block": inf_k0,
                     # the method's float operations (the step-by-step recursion) per second of e-prop
                     "alu": {"achieved": round(achieved_tf, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": round(achieved_tf / FP32_PEAK_TFLOPS, 4),
                             "peak_note": "fp32 FMA without packed instructions, which the build disables",
                             "algorithmic_flops_per_launch": round(alg_flops / max(ep_n, 1))}},
    }
    net.close()
    if not args.no_tiny:
        print("[bench] tiny e-prop network", file=sys.stderr, flush=True)
        result["tiny_net"] = tiny_net_leg()
    if not args.no_batched:
        print("[bench] batched instances against the plain loop", file=sys.stderr, flush=True)
        result["batched"] = batched_leg(args.batched_instances or None)
    if not args.no_served:
        print("[bench] served inference", file=sys.stderr, flush=True)
        result["served"] = served_leg()
    if not args.no_topo:
        print("[bench] topographic-map rewiring latency", file=sys.stderr, flush=True)
        result["topomap_rewire"] = topo_rewire_latency()
        print("[bench] topographic map end to end", file=sys.stderr, flush=True)
        result["topomap_sim"] = topo_sim_leg(steps=args.topo_steps)
        print("[bench] topographic map scaling, s = 1..7", file=sys.stderr, flush=True)
        result["topomap_scaling"] = topo_scaling_leg(steps=args.topo_scaling_steps)
    if not args.no_cpu_baseline:
        print(f"[bench] oracle CPU baseline ({args.cpu_steps} timesteps)", file=sys.stderr, flush=True)
        labels, raster = batches[0]
        result["cpu_baseline"] = run_cpu_baseline(cfg, raster, labels, args.cpu_steps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
