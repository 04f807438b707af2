"""Seeded synthetic workloads: shapes, sizes and seeds only.

This module holds none of the method's arithmetic (no model step, no
distance, no Philox); it states *what* to run. The HIP path and the CPU
oracle each turn these descriptions into observed series and results on
their own. Random choices made here (the 64 uneven series) use numpy's PCG64,
not the method's generator.

The paper fits real case/recovery/death counts for Italy, New Zealand and the
USA over 49 days (Sec. 4, Sec. 5). That data is not used: every observed
series is synthesised by one model run at a fixed ground-truth parameter
vector on the observation stream, which keeps the same roles (49..100-day
fits at three population scales). The ground-truth vectors are the
1000-sample posterior means the paper reports per country (Table
"t:trajectories").
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

# Prior of eq. (2): U(0, [1, 100, 2, 1, 1, 1, 1, 2]) over
# theta = [alpha0, alpha, n, beta, gamma, delta, eta, kappa] (eq. 1).
PRIOR_LO = np.zeros(8, dtype=np.float32)
PRIOR_HI = np.array([1, 100, 2, 1, 1, 1, 1, 2], dtype=np.float32)
THETA_NAMES = ("alpha0", "alpha", "n", "beta", "gamma", "delta", "eta", "kappa")

# Table "t:trajectories", 1000 accepted samples, posterior averages.
THETA_ITALY = np.array([0.309, 15.012, 0.406, 0.013, 0.407, 0.009, 0.507, 0.603], np.float32)
THETA_NZ = np.array([0.480, 50.932, 1.238, 0.030, 0.504, 0.001, 0.527, 1.172], np.float32)
THETA_USA = np.array([0.342, 11.051, 0.319, 0.007, 0.468, 0.005, 0.501, 0.706], np.float32)

# stream domains (fourth counter word carries day<<8 | domain<<4 | block)
DOMAIN_OBS = 0     # synthesis of the observed series
DOMAIN_ABC = 1     # prior draws and simulation noise of rejection ABC
DOMAIN_MDN_DATA = 2
DOMAIN_MDN_INIT = 3
DOMAIN_PROPOSAL = 5


@dataclasses.dataclass
class Series:
    """One observed series: population P, horizon T, initial observed
    compartments, the ground-truth theta and the seed of its observation run."""

    name: str
    P: int
    T: int
    theta_true: np.ndarray
    obs_seed: int
    A0: int = 100
    R0: int = 0
    D0: int = 0
    series_id: int = 0


def single_country() -> Series:
    """One synthetic country: P = 1e7, 100 active at day 0, T = 49, Italy's
    parameter averages, observation seed 1 (100k prior samples, 100 nearest
    kept)."""
    return Series("country-1e7-T49", 10_000_000, 49, THETA_ITALY, 1)


def three_countries() -> List[Series]:
    """Three synthetic countries run separately: (6e7, 49 days), (8.3e7, 72),
    (3.3e8, 100), observation seeds 2..4, Italy / New Zealand / USA averages."""
    return [Series("country-6e7-T49", 60_000_000, 49, THETA_ITALY, 2),
            Series("country-8.3e7-T72", 83_000_000, 72, THETA_NZ, 3),
            Series("country-3.3e8-T100", 330_000_000, 100, THETA_USA, 4)]


def uneven_series(n: int = 64, seed: int = 5) -> List[Series]:
    """n series with T uniform in [30, 200], P log-uniform in [1e5, 1e9] and
    ground-truth theta uniform over the prior box; observation seed = seed,
    series id j distinguishes their streams."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n):
        T = int(30 + rng.integers(0, 171))
        P = int(round(10 ** (5 + 4 * rng.random())))
        th = (PRIOR_LO + (PRIOR_HI - PRIOR_LO) * rng.random(8)).astype(np.float32)
        out.append(Series("uneven-%02d" % j, P, T, th, seed, series_id=j))
    return out


def epidemic_curve(T: int, P: int, seed: int) -> np.ndarray:
    """A stand-in observed series [3, T] (A, R, D) with epidemic shape, made
    from a logistic curve plus seeded jitter; used where a test needs a series
    that does not come from the model. Not part of any workload above."""
    rng = np.random.default_rng(seed)
    t = np.arange(1, T + 1, dtype=np.float64)
    peak = min(P * 0.02, 5e5)
    cum = peak / (1 + np.exp(-(t - T * 0.4) / (T * 0.08 + 1)))
    A = cum * np.exp(-t / (T * 1.5))
    R = np.cumsum(cum * 0.02)
    D = np.cumsum(cum * 0.002)
    obs = np.stack([A, R, D]) * np.exp(rng.normal(0, 0.05, size=(3, T)))
    return np.clip(np.round(obs), 0, P // 4).astype(np.int32)
