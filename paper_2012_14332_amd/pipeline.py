"""Host orchestration of the plain rejection-ABC path (Sec. 3.1 / 3.2).

Only control flow lives here -- which entry point of libabc.so runs next,
on which stream, with which index range. Every step of the computation is a
HIP kernel behind the C ABI.

One pass over a batch of N prior samples of one series is:
  1. simulate + distance in float32, theta drawn in-kernel from the prior,
     early exit at eps (1 + w);
  2. wavefront-ballot compaction of the candidates d <= eps (1 + w);
  3. float64 decision of the candidates inside the band (eps (1 - w), eps (1 + w)];
  4. float64 posterior mean and covariance of the accepted theta.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import torch

from . import abc
from . import workloads as W

DEFAULT_BAND = 0.02


def observed_series(s: W.Series, device="cuda") -> abc.DeviceSeries:
    """Synthesise the observed A, R, D series of `s`: one float64 model run at
    theta_true on the observation stream (domain 0, seed s.obs_seed)."""
    th = torch.tensor(np.asarray(s.theta_true, np.float32)[None], device=device)
    ser0 = abc.DeviceSeries(s.P, s.T, A0=s.A0, R0=s.R0, D0=s.D0, device=device)
    traj = abc.simulate_record(ser0, th, s.obs_seed, domain=W.DOMAIN_OBS, series=s.series_id,
                               flags=abc.ABC_FP64, device=device)
    obs = traj[0, 1:, 2:5].T.contiguous()
    return abc.DeviceSeries(s.P, s.T, obs, A0=s.A0, R0=s.R0, D0=s.D0, device=device)


def pilot_distances(ser: abc.DeviceSeries, seed: int, n: int, series: int = 0,
                    first: int = 0) -> np.ndarray:
    """Float32 distances of a pilot prefix without early exit (host copy)."""
    return abc.simulate_distance(ser, n, seed, first=first, series=series).cpu().numpy()


def pilot_eps(ser: abc.DeviceSeries, seed: int, n: int = 100_000, q: float = 1e-4,
              series: int = 0) -> float:
    """Tolerance that a fraction q of a pilot run falls under: the ceil(q n)-th
    smallest pilot distance."""
    d = np.sort(pilot_distances(ser, seed, n, series))
    k = max(1, int(math.ceil(q * n)))
    return float(d[k - 1])


@dataclasses.dataclass
class PlainResult:
    idx: torch.Tensor      # [cap] int64, first `count` valid
    theta: torch.Tensor    # [cap, 8]
    dist: torch.Tensor     # [cap]
    count: torch.Tensor    # [1] int64 (device)
    mean: torch.Tensor     # [8] float64
    cov: torch.Tensor      # [8, 8] float64
    rechecked: Optional[torch.Tensor] = None

    def n(self) -> int:
        """Accepted rows. An overflowed candidate list (more candidates than
        the pass's capacity) has no float64 band decision and only part of the
        rows, so it raises instead of returning a partial answer."""
        c = int(self.count.item())
        if c > self.idx.shape[0]:
            raise abc.AbcError("%d candidates exceed the capacity %d: run again with a larger "
                               "capacity" % (c, self.idx.shape[0]))
        return c


class PlainABC:
    """Reusable buffers for repeated plain-ABC passes over one series."""

    def __init__(self, ser: abc.DeviceSeries, seed: int, eps: float, n: int, *, series: int = 0,
                 band_w: float = DEFAULT_BAND, capacity: int = 1 << 16, flags: int = 0,
                 device="cuda"):
        self.ser, self.seed, self.eps, self.n = ser, int(seed), float(eps), int(n)
        self.series, self.band_w, self.cap, self.flags = int(series), float(band_w), int(capacity), flags
        self.dist = torch.empty(self.n, dtype=torch.float32, device=device)
        self.device = device

    def run(self, first: int, want_rechecked: bool = False) -> PlainResult:
        eps_hi = self.eps * (1.0 + self.band_w) if self.band_w > 0 else self.eps
        abc.simulate_distance(self.ser, self.n, self.seed, first=first, series=self.series,
                              eps_exit=eps_hi, flags=self.flags, out=self.dist,
                              device=self.device)
        idx, th, d, _, cnt = abc.accept_compact(self.dist, eps_hi, self.cap, first=first,
                                                seed=self.seed, series=self.series,
                                                device=self.device)
        nre = None
        if self.band_w > 0:
            nre = abc.recheck_band(self.ser, self.seed, self.eps, self.band_w, idx, th, d, cnt,
                                   series=self.series, flags=self.flags,
                                   want_rechecked=want_rechecked)
        mean, cov = abc.posterior_moments(th, n_dev=cnt, device=self.device)
        return PlainResult(idx, th, d, cnt, mean, cov, nre)


@dataclasses.dataclass
class NearestResult:
    idx: torch.Tensor      # [k] int64, index order
    theta: torch.Tensor    # [k, 8]
    dist: torch.Tensor     # [k] float64
    mean: torch.Tensor     # [8] float64
    cov: torch.Tensor      # [8, 8] float64
    candidates: int        # rows decided in float64


class NearestABC:
    """Keep the k nearest of n prior samples (the single-country workload):
    float32 simulation of every day, device nearest-k, then the float64
    decision -- every sample within (1 + band_w) of the k-th float32 distance
    is simulated again in float64 and the k nearest of those by (float64
    distance, index) are kept; float64 moments of their theta."""

    def __init__(self, ser: abc.DeviceSeries, seed: int, n: int, k: int, *, series: int = 0,
                 band_w: float = DEFAULT_BAND, capacity: int = 1 << 16, device="cuda"):
        self.ser, self.seed, self.n, self.k = ser, int(seed), int(n), int(k)
        self.series, self.band_w, self.cap = int(series), float(band_w), int(capacity)
        self.dist = torch.empty(self.n, dtype=torch.float32, device=device)
        self.device = device

    def run(self, first: int = 0) -> NearestResult:
        abc.simulate_distance(self.ser, self.n, self.seed, first=first, series=self.series,
                              out=self.dist, device=self.device)
        _, _, _, kth = abc.nearest_k(self.dist, self.k, first=first, seed=self.seed,
                                     series=self.series, device=self.device)
        tau = float(kth.item()) * (1.0 + self.band_w)
        cidx, cth, _, _, cnt = abc.accept_compact(self.dist, tau, self.cap, first=first,
                                                  seed=self.seed, series=self.series,
                                                  device=self.device)
        c = int(cnt.item())
        if c > self.cap:
            raise abc.AbcError("nearest-k band holds %d rows, capacity %d" % (c, self.cap))
        d64 = abc.simulate_rows_f64(self.ser, self.seed, cidx[:c], cth[:c], series=self.series,
                                    device=self.device)
        idx, th, d = abc.nearest_k_rows(d64, cidx[:c], cth[:c], self.k, device=self.device)
        mean, cov = abc.posterior_moments(th, device=self.device)
        return NearestResult(idx, th, d, mean, cov, c)


# ----------------------------------------------------------------------------
# learned proposal (importance-weighted rejection ABC)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class WeightedResult:
    idx: torch.Tensor      # [q] int64 sample indices (first q accepted by index)
    theta: torch.Tensor    # [q, 8]
    weight: torch.Tensor   # [q] prior / proposal
    dist: torch.Tensor     # [q]
    mean: torch.Tensor     # [8] float64, weighted
    cov: torch.Tensor      # [8, 8] float64, weighted
    samples: int           # proposal draws simulated
    ess: float             # (sum w)^2 / sum w^2
    accepted_total: int    # accepted among all `samples` draws (before keeping the first q)

    def n(self) -> int:
        return int(self.idx.shape[0])


def train_proposal(n_pairs: int = 1_000_000, epochs: int = 20, batch: int = 4096,
                   lr: float = 1e-3, seed: int = 6, init_seed: int = 0,
                   T_range=(30, 200), log10P_range=(5.0, 9.0)):
    """Simulate (theta, x) pairs from the prior (domain 2) and train the
    mixture-density network on them. Returns (net, loss log, steps, train ms,
    data ms)."""
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    feats, theta, _ = abc.simulate_features(n_pairs, seed, domain=W.DOMAIN_MDN_DATA,
                                            T_lo=T_range[0], T_hi=T_range[1],
                                            log10P_lo=log10P_range[0], log10P_hi=log10P_range[1])
    net = abc.Mdn(init_seed)
    net.fit_standardizer(feats)
    t1.record()
    torch.cuda.synchronize()
    data_ms = t0.elapsed_time(t1)
    log, steps, ms = net.train(feats, theta, epochs=epochs, batch=batch, lr=lr, shuffle_seed=seed)
    del feats, theta
    return net, log, steps, ms, data_ms


class LearnedABC:
    """Rejection ABC with theta drawn from the trained mixture for one series
    (defensive weight lam on the prior), importance weights prior / proposal,
    the same eps, float32 simulation, compaction with weights, float64 band
    decision and weighted float64 moments."""

    def __init__(self, net, ser: abc.DeviceSeries, eps: float, seed: int, *, series: int = 0,
                 lam: float = 0.05, inflate: float = 1.5, band_w: float = DEFAULT_BAND,
                 chunk0: int = 1 << 14, chunk_max: int = 1 << 20):
        self.net, self.ser, self.eps, self.seed = net, ser, float(eps), int(seed)
        self.series, self.lam, self.band_w = int(series), float(lam), float(band_w)
        self.inflate = float(inflate)
        self.chunk0, self.chunk_max = int(chunk0), int(chunk_max)
        self.mix = net.forward(abc.series_features(ser)[None])[0].contiguous()
        self.dist = torch.empty(self.chunk_max, dtype=torch.float32, device="cuda")

    def run(self, quota: int, max_samples: int = 1 << 34) -> WeightedResult:
        """Consume proposal indices 0, 1, 2, ... in growing contiguous chunks until
        `quota` samples are accepted; keep the first `quota` by index."""
        e_hi = self.eps * (1.0 + self.band_w)
        parts = []
        got = 0
        first = 0
        chunk = self.chunk0
        while got < quota and first < max_samples:
            th, w = self.net.sample(self.mix, chunk, self.seed, lam=self.lam,
                                    inflate=self.inflate, domain=W.DOMAIN_PROPOSAL,
                                    series=self.series, first=first)
            dist = self.dist[:chunk]
            abc.simulate_distance(self.ser, chunk, self.seed, theta=th, first=first,
                                  series=self.series, eps_exit=e_hi, out=dist)
            # capacity = chunk: every draw could be a candidate
            idx, thc, dc, wc, cnt = abc.accept_compact(dist, e_hi, chunk, theta=th, weight=w,
                                                       first=first)
            abc.recheck_band(self.ser, self.seed, self.eps, self.band_w, idx, thc, dc, cnt,
                             weight=wc, series=self.series)
            c = int(cnt.item())
            if c:
                parts.append((idx[:c], thc[:c], wc[:c], dc[:c]))
                got += c
            first += chunk
            chunk = min(chunk * 2, self.chunk_max)
        idx = torch.cat([p[0] for p in parts])[:quota]
        th = torch.cat([p[1] for p in parts])[:quota].contiguous()
        w = torch.cat([p[2] for p in parts])[:quota].contiguous()
        d = torch.cat([p[3] for p in parts])[:quota]
        mean, cov = abc.posterior_moments(th, w)
        wn = w.double().cpu().numpy()
        ess = float(wn.sum() ** 2 / (wn * wn).sum()) if wn.size else 0.0
        return WeightedResult(idx, th, w, d, mean, cov, first, ess, got)


DOMAIN_PROJECTION = 6


def predictive_bands(s: W.Series, theta: torch.Tensor, horizon: int = 120, seed: int = 7,
                     quantiles=(0.05, 0.5, 0.95), flags: int = 0):
    """Posterior-predictive projection (Sec. 5): simulate every accepted theta
    over `horizon` days from the series' initial state on a fresh stream
    (domain 6), return (trajectories [n, horizon+1, 6], bands [nq, horizon+1, 6])."""
    ser = abc.DeviceSeries(s.P, horizon, A0=s.A0, R0=s.R0, D0=s.D0)
    traj = abc.simulate_record(ser, theta.contiguous(), seed, domain=DOMAIN_PROJECTION,
                               series=s.series_id, flags=flags)
    return traj, abc.trajectory_bands(traj, quantiles)


# ----------------------------------------------------------------------------
# posterior agreement of two ABC samplers (measurement, not the hot path)
# ----------------------------------------------------------------------------
def _weighted_summary(theta: np.ndarray, w: np.ndarray):
    """Weighted mean and sd (reliability-weight variance, as the moments kernel
    forms it) of rows theta [n, 8], the Kish effective size, and standard
    errors of the mean and of the sd from the sample's own second and fourth
    central moments: SE(mean) = sd / sqrt(ess), SE(sd) = sd sqrt((k - 1) / (4 ess))
    with k the kurtosis (delta method for the square root of the variance)."""
    w = w / w.sum()
    ess = 1.0 / float((w * w).sum())
    m = (w[:, None] * theta).sum(0)
    c = theta - m
    m2 = (w[:, None] * c * c).sum(0)
    m4 = (w[:, None] * c ** 4).sum(0)
    sd = np.sqrt(m2 / max(1.0 - 1.0 / ess, 1e-12))
    kurt = m4 / np.maximum(m2 * m2, 1e-300)
    se_m = sd / np.sqrt(ess)
    se_sd = sd * np.sqrt(np.maximum(kurt - 1.0, 0.0) / (4.0 * ess))
    return m, sd, ess, se_m, se_sd


class _Pool:
    """Running form of _weighted_summary over runs added one at a time: the
    weight sums and the weighted power sums of theta - c up to the fourth,
    with c the first run's weighted mean (which keeps the central moments
    free of cancellation), so a summary costs O(1) in the pooled runs."""

    def __init__(self):
        self.runs = 0
        self.c = None

    def add(self, theta: np.ndarray, w: np.ndarray):
        w = np.asarray(w, np.float64)
        theta = np.asarray(theta, np.float64)
        if self.c is None:
            self.c = (w[:, None] * theta).sum(0) / w.sum()
            self.W = self.W2 = 0.0
            self.S = np.zeros((4, theta.shape[1]))
        y = theta - self.c
        wy = w[:, None] * y
        self.W += float(w.sum())
        self.W2 += float((w * w).sum())
        for k in range(4):
            self.S[k] += wy.sum(0)
            wy = wy * y
        self.runs += 1

    def summary(self):
        s1, s2, s3, s4 = self.S / self.W
        ess = self.W * self.W / self.W2
        mu = s1
        m2 = s2 - mu * mu
        m4 = s4 - 4.0 * mu * s3 + 6.0 * mu * mu * s2 - 3.0 * mu ** 4
        sd = np.sqrt(np.maximum(m2, 0.0) / max(1.0 - 1.0 / ess, 1e-12))
        kurt = m4 / np.maximum(m2 * m2, 1e-300)
        se_m = sd / np.sqrt(ess)
        se_sd = sd * np.sqrt(np.maximum(kurt - 1.0, 0.0) / (4.0 * ess))
        return self.c + mu, sd, ess, se_m, se_sd


def compare_posteriors(sers, eps, run_a, run_b, *, quota: int = 4096, seeds_a=(2, 3, 4),
                       seeds_b=(2, 3, 4), max_runs: int = 48, resolution: float = 4.0,
                       min_ess: float = 1e4, rel: float = 0.05, time_limit_s: float = None,
                       progress=None):
    """Posterior mean and sd of sampler B against sampler A, series by series
    (the learned-proposal criterion: per parameter |dmean| <= rel max(|mean_A|,
    sd_A) and |dsd| <= rel sd_A). run_a(seed, idxs) and run_b(seed, idxs) return
    (theta [len(idxs), quota, 8], weights [len(idxs), quota]) as host arrays for
    the series idxs. Each side pools runs on further seeds, series by series,
    until B's effective size is at least min_ess and the standard error of every
    difference is at most tolerance / resolution -- the criterion is then
    decided at `resolution` standard errors rather than at Monte Carlo noise --
    or until max_runs runs (or time_limit_s seconds of pooling). progress(text),
    if given, is called after every pooling pass. Returns per-series records."""
    import time

    t_start = time.perf_counter()
    m = len(sers)
    pools = {"a": [_Pool() for _ in range(m)], "b": [_Pool() for _ in range(m)]}
    next_seed = {"a": list(seeds_a), "b": list(seeds_b)}
    # further runs take fresh seeds per side (so no series sees a seed twice)
    extra = {"a": 100, "b": 200}
    runs = {"a": [0] * m, "b": [0] * m}

    def pull(side, idxs):
        if not idxs:
            return
        fn = run_a if side == "a" else run_b
        seq = next_seed[side]
        if seq:
            seed = seq.pop(0)
        else:
            seed = extra[side]
            extra[side] += 1
        th, w = fn(seed, idxs)
        for q, j in enumerate(idxs):
            pools[side][j].add(th[q], w[q])
            runs[side][j] += 1

    for _ in range(max(len(seeds_a), len(seeds_b))):
        pull("a", list(range(m)) if next_seed["a"] else [])
        pull("b", list(range(m)) if next_seed["b"] else [])
    out = [None] * m
    todo = list(range(m))
    while todo:
        need_a, need_b = [], []
        for j in todo:
            sa = pools["a"][j].summary()
            sb = pools["b"][j].summary()
            tol_m = rel * np.maximum(np.abs(sa[0]), sa[1])
            tol_s = rel * sa[1]
            se_dm = np.sqrt(sa[3] ** 2 + sb[3] ** 2)
            se_ds = np.sqrt(sa[4] ** 2 + sb[4] ** 2)
            res = max(float((se_dm / tol_m).max()), float((se_ds / tol_s).max()))
            out[j] = {"mean_ratio": float((np.abs(sb[0] - sa[0]) / tol_m).max()),
                      "sd_ratio": float((np.abs(sb[1] - sa[1]) / tol_s).max()),
                      "se_over_tol": res, "ess_a": sa[2], "ess_b": sb[2],
                      "runs_a": runs["a"][j], "runs_b": runs["b"][j],
                      "mean_ok": [bool(x) for x in np.abs(sb[0] - sa[0]) <= tol_m],
                      "sd_ok": [bool(x) for x in np.abs(sb[1] - sa[1]) <= tol_s]}
            if res * resolution <= 1.0 and sb[2] >= min_ess:
                continue
            # pool on the side whose standard errors dominate (both if close)
            va = max(float((sa[3] / tol_m).max()), float((sa[4] / tol_s).max()))
            vb = max(float((sb[3] / tol_m).max()), float((sb[4] / tol_s).max()))
            if (vb >= 0.5 * va or sb[2] < min_ess) and runs["b"][j] < max_runs:
                need_b.append(j)
            if va >= 0.5 * vb and runs["a"][j] < max_runs:
                need_a.append(j)
        if not need_a and not need_b:
            break
        if time_limit_s is not None and time.perf_counter() - t_start > time_limit_s:
            break
        pull("a", need_a)
        pull("b", need_b)
        todo = sorted(set(need_a) | set(need_b))
        if progress:
            progress("posterior check: %d series pooling, runs so far %d / %d (max), %.0f s"
                     % (len(todo), max(runs["a"]), max(runs["b"]), time.perf_counter() - t_start))
    return out
