"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module holds none of the method's arithmetic: it only produces input spike
rasters, labels and parameter sets that stand in for the paper's datasets
(N-MNIST, DVS gesture, and the SHD-shaped 700-channel classifier input are not
available).  Its randomness comes from numpy's own generators and is *data*,
not one of the method's draws.

Raster format (compressed rows, one list per (timestep, batch instance)):
    off : int32[T*B + 1]
    idx : int32[off[-1]]
    spikes of instance b at step t are idx[off[t*B + b] : off[t*B + b + 1]],
    ascending channel indices.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Raster:
    T: int
    B: int
    n_in: int
    off: np.ndarray
    idx: np.ndarray

    def at(self, t: int, b: int) -> np.ndarray:
        q = t * self.B + b
        return self.idx[self.off[q]:self.off[q + 1]]

    def step_lists(self, t: int):
        """(idx, off[B+1]) of step t, re-based to start at zero."""
        lo, hi = self.off[t * self.B], self.off[(t + 1) * self.B]
        return self.idx[lo:hi].copy(), (self.off[t * self.B:(t + 1) * self.B + 1] - lo).astype(np.int32)

    @property
    def n_spikes(self) -> int:
        return int(self.off[-1])


def _to_raster(spk: np.ndarray) -> Raster:
    """spk: bool[T, B, n_in] -> Raster."""
    T, B, n = spk.shape
    counts = spk.reshape(T * B, n).sum(axis=1)
    off = np.zeros(T * B + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    idx = np.nonzero(spk.reshape(T * B, n))[1].astype(np.int32)
    assert off[-1] < 2**31
    return Raster(T, B, n, off.astype(np.int32), idx)


def poisson_rates(seed: int, n_in: int, max_hz: float = 50.0) -> np.ndarray:
    """Per-neuron rates drawn U[0, max_hz) (tiny e-prop network inputs)."""
    return np.random.Generator(np.random.Philox(seed)).uniform(0.0, max_hz, n_in)


def poisson_raster(seed: int, rates_hz: np.ndarray, T: int, B: int, dt_ms: float = 1.0) -> Raster:
    rng = np.random.Generator(np.random.Philox(seed + 7919))
    p = np.asarray(rates_hz, np.float64) * dt_ms * 1e-3
    spk = rng.random((T, B, p.size)) < p[None, None, :]
    return _to_raster(spk)


@dataclass
class ShdLike:
    """Class-dependent Gaussian rate bumps over (channel, time): a 700-channel,
    20-class stand-in for the Spiking Heidelberg Digits shape."""
    n_ch: int = 700
    n_classes: int = 20
    T: int = 1000
    bumps: int = 4
    base_hz: float = 2.0
    peak_hz: float = 100.0
    sigma_ch: float = 20.0
    sigma_t_ms: float = 50.0
    jitter_ch: float = 10.0
    jitter_t_ms: float = 30.0
    dt_ms: float = 1.0

    def prototypes(self, seed: int):
        rng = np.random.Generator(np.random.Philox(seed))
        ch = rng.integers(0, self.n_ch, (self.n_classes, self.bumps)).astype(np.float64)
        t = rng.uniform(100.0, 900.0, (self.n_classes, self.bumps)) * (self.T / 1000.0)
        return ch, t

    def batch(self, seed: int, batch_index: int, B: int):
        """Labels int32[B] and the raster of one batch of B samples."""
        ch0, t0 = self.prototypes(seed)
        rng = np.random.Generator(np.random.Philox(seed * 1000003 + 17 + batch_index))
        labels = rng.integers(0, self.n_classes, B).astype(np.int32)
        chs = np.arange(self.n_ch, dtype=np.float64)
        ts = np.arange(self.T, dtype=np.float64) * self.dt_ms
        spk = np.zeros((self.T, B, self.n_ch), dtype=bool)
        for b in range(B):
            c = labels[b]
            cc = ch0[c] + rng.normal(0.0, self.jitter_ch, self.bumps)
            tc = t0[c] + rng.normal(0.0, self.jitter_t_ms, self.bumps)
            rate = np.full((self.T, self.n_ch), self.base_hz)
            for m in range(self.bumps):  # separable Gaussian bump in (time, channel)
                gt = np.exp(-(ts - tc[m]) ** 2 / (2 * self.sigma_t_ms ** 2))
                gc = np.exp(-(chs - cc[m]) ** 2 / (2 * self.sigma_ch ** 2))
                rate += self.peak_hz * np.outer(gt, gc)
            spk[:, b, :] = rng.random((self.T, self.n_ch)) < rate * self.dt_ms * 1e-3
        return labels, _to_raster(spk)


# ------------------------------------------------------------------ parameter sets
TINY_EPROP = dict(name="tiny-eprop-100-128-4", n_in=100, n_rec=128, n_out=4, batch=1, alif=False,
                  p_in=0.1, p_rec=0.1, T=500, update_interval=25, deepr_mask=3, l1=0.005,
                  lr=1e-3, max_rates_hz=50.0)

SHD_CLASSIFIER = dict(name="sparse-classifier-700-1024alif-20", n_in=700, n_rec=1024, n_out=20,
                      batch=256, alif=True, p_in=0.1, p_rec=0.1, T=1000, update_interval=100,
                      deepr_mask=3, l1=0.005, lr=1e-3)

# Topographic map at scale s = 4: two 64 x 64 sheets, feed-forward and lateral
# projections with row capacity 32, N_attempts = 10 s^2 per projection every
# 10 steps of 0.1 ms (Tab. C-H).  Conductances in uS.
TOPO_S4 = dict(name="topomap-64x64-cap32", L=64, cap=32, n_attempts=160, g_max=0.2,
               ff=dict(p_form=0.16, sigma=2.5), lat=dict(p_form=1.0, sigma=1.0),
               p_elim_dep=2.45e-2 * 50, p_elim_pot=1.36e-4 * 50, rewire_every=10)


def sigma_init(p: float, n_pre: int) -> float:
    """Initial weight spread 1/sqrt(expected in-degree)."""
    return float(1.0 / np.sqrt(p * n_pre))

# Batched instances: 64 classifiers on the sparse-classifier input, recurrent
# sizes log-uniform in [256, 4096], connection probabilities uniform in
# [0.05, 0.2], one sample per instance and step.
BATCHED = dict(name="batched-64-classifiers", n_inst=64, n_rec_lo=256, n_rec_hi=4096, p_lo=0.05, p_hi=0.2,
               n_in=700, n_out=20, batch=1, alif=True, T=1000, update_interval=100, deepr_mask=3, l1=0.005,
               lr=1e-3)


def batched_sizes(seed: int, n: int, lo: int = 256, hi: int = 4096, p_lo: float = 0.05, p_hi: float = 0.2):
    """Recurrent sizes (log-uniform in [lo, hi]) and connection probabilities
    (uniform in [p_lo, p_hi]) of n network instances."""
    rng = np.random.Generator(np.random.Philox(seed + 104729))
    n_rec = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), n))).astype(int)
    p = rng.uniform(p_lo, p_hi, n)
    return [(int(a), float(b)) for a, b in zip(n_rec, p)]
