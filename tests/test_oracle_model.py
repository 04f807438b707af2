"""Pins of the oracle's model (Sec. 2.1, eqs. 3-5), distance (Sec. 2.2) and
accept/moment rules against facts fixed by the paper and by mathematics:

* conservation and sign invariants of the compartment model;
* transitions that a zero rate switches off stay frozen, noise or not;
* single-transition set-ups whose draw count has a known mean and variance
  (mean h - 1/2 after the floor, variance h + 1/12), which pins each hazard
  of eq. (5) and the noise scale separately;
* the noise-free linear limit (alpha = 0, S ~ P) against the exact linear
  recurrence, which pins the coefficient structure of the update;
* the noise-free map in exact rational arithmetic on tiny populations;
* a distance of exactly zero for the series the model itself generated;
* brute-force accept / nearest / quantile rules and numpy's weighted
  covariance.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import pyref

ITALY = np.array([0.309, 15.012, 0.406, 0.013, 0.407, 0.009, 0.507, 0.603], np.float32)
NZ = np.array([0.480, 50.932, 1.238, 0.030, 0.504, 0.001, 0.527, 1.172], np.float32)


def test_c_oracle_matches_python_restatement():
    cases = [(ITALY, 1e7, 49, 1), (NZ, 5e6, 30, 2), (ITALY, 1e5, 20, 3),
             (np.array([0, 0, 0, 0, 0, 0, 0, 0], np.float32), 1e4, 5, 4),
             (np.array([0.99, 99.0, 1.99, 0.99, 0.99, 0.99, 0.99, 1.99], np.float32), 1e9, 40, 5)]
    for th, P, T, seed in cases:
        m = oracle.make_model(P, T)
        obs = oracle.observe(m, NZ, seed + 100)
        tr, d = oracle.trajectory(m, th, seed, 1, 2, 77, obs=obs)
        tr2, d2 = pyref.trajectory(th, P, T, seed=seed, domain=1, series=2, sample=77, obs=obs)
        np.testing.assert_array_equal(tr, tr2)
        assert math.isclose(d, d2, rel_tol=1e-14)
    # literal-variance noise and raw distance modes
    m = oracle.make_model(2e6, 25, noise_mode=1, dist_mode=1)
    obs = oracle.observe(m, ITALY, 8)
    tr, d = oracle.trajectory(m, NZ, 9, obs=obs)
    tr2, d2 = pyref.trajectory(NZ, 2e6, 25, seed=9, noise_mode=1, dist_mode=1, obs=obs)
    np.testing.assert_array_equal(tr, tr2)
    assert math.isclose(d, d2, rel_tol=1e-14)


@pytest.mark.parametrize("P", [1000, 1e5, 1e7, 3.3e8, 1e9])
def test_invariants(P):
    T = 120
    m = oracle.make_model(P, T)
    th = oracle.prior(300, seed=int(P) % 1000 + 1)
    tr = oracle.record(m, th, seed=11)
    assert np.all(tr.sum(axis=2) == int(P))
    assert np.all(tr >= 0)
    S, I, A, R, D, Ru = (tr[..., k] for k in range(6))
    assert np.all(np.diff(S, axis=1) <= 0)
    for X in (R, D, Ru, A + R + D):
        assert np.all(np.diff(X, axis=1) >= 0)
    # day-0 state: Ru = 0, I0 = floor(kappa*A0), S = P - (A0 + R0 + D0 + I0)
    assert np.all(tr[:, 0, 5] == 0)
    np.testing.assert_array_equal(tr[:, 0, 1], np.floor(th[:, 7].astype(np.float64) * 100))
    assert np.all(tr[:, 0, 2] == 100)


def test_future_days_lower_bound_holds():
    """R and D never fall, so after day t each later day s contributes at
    least max(0, log1p X_t - log1p O_s)^2 per cumulative count: the lower
    bound the float32 kernel adds to its running sum before the early-exit
    test. Checked on oracle trajectories against a series of another theta."""
    P, T = 3.3e8, 100
    m = oracle.make_model(P, T)
    obs = oracle.observe(m, NZ, 4)
    th = oracle.prior(400, seed=12)
    tr = oracle.record(m, th, seed=13)
    X = np.log1p(tr[:, 1:, 3:5].astype(np.float64))          # R, D on days 1..T
    O = np.log1p(obs[1:3].T.astype(np.float64))               # [T, 2]
    term = ((X - O[None]) ** 2).sum(-1)                       # [n, T]
    rest = np.cumsum(term[:, ::-1], 1)[:, ::-1]               # sum over s >= t
    hit = 0
    for t in range(T - 1):
        lb = (np.maximum(0.0, X[:, t:t + 1, :] - O[None, t + 1:, :]) ** 2).sum((1, 2))
        assert np.all(lb <= rest[:, t + 1] * (1 + 1e-12) + 1e-12)
        hit += int(np.count_nonzero(lb > 0))
    assert hit > 0


def _with(th, **kw):
    names = ["alpha0", "alpha", "n", "beta", "gamma", "delta", "eta", "kappa"]
    t = np.array(th, np.float32).copy()
    for k, v in kw.items():
        t[..., names.index(k)] = v
    return t


def test_zero_rates_freeze_their_transitions():
    m = oracle.make_model(1e7, 60)
    base = oracle.prior(200, seed=21)
    # gamma = 0: no I -> A, so A + R + D is constant
    tr = oracle.record(m, _with(base, gamma=0), seed=3)
    ard = tr[..., 2] + tr[..., 3] + tr[..., 4]
    assert np.all(ard == ard[:, :1])
    # beta = delta = 0: R, D, Ru frozen
    tr = oracle.record(m, _with(base, beta=0, delta=0), seed=3)
    for k in (3, 4, 5):
        assert np.all(tr[..., k] == tr[:, :1, k])
    # alpha0 = alpha = 0: no infections, S frozen
    tr = oracle.record(m, _with(base, alpha0=0, alpha=0), seed=3)
    assert np.all(tr[..., 0] == tr[:, :1, 0])
    # eta = 0: Ru frozen
    tr = oracle.record(m, _with(base, eta=0), seed=3)
    assert np.all(tr[..., 5] == 0)
    # kappa = 0: I stays 0, S frozen, A only drains
    tr = oracle.record(m, _with(base, kappa=0), seed=3)
    assert np.all(tr[..., 1] == 0) and np.all(tr[..., 0] == tr[:, :1, 0])
    assert np.all(np.diff(tr[..., 2], axis=1) <= 0)
    # delta = 0: D frozen
    tr = oracle.record(m, _with(base, delta=0), seed=3)
    assert np.all(tr[..., 4] == 0)


def _one_day_counts(th, P, n, seed=7, noise_mode=0, A0=100):
    m = oracle.make_model(P, 1, A0=A0, noise_mode=noise_mode)
    tr = oracle.record(m, np.tile(th, (n, 1)), seed=seed)
    return tr[:, 0, :], tr[:, 1, :]


def _floor_moments_check(counts, h, sd):
    """A floored N(h, sd^2) draw has mean h - 1/2 and variance sd^2 + 1/12
    (exact up to terms of order exp(-2 pi^2 sd^2))."""
    n = counts.size
    mean_ref = h - 0.5
    var_ref = sd * sd + 1.0 / 12.0
    assert abs(counts.mean() - mean_ref) < 6 * sd / math.sqrt(n), (counts.mean(), mean_ref)
    assert abs(counts.var() - var_ref) < 6 * math.sqrt(2.0 / n) * var_ref, (counts.var(), var_ref)


@pytest.mark.parametrize("noise_mode", [0, 1])
def test_single_transition_mean_and_variance(noise_mode):
    n = 20000
    sdf = (lambda h: math.sqrt(h)) if noise_mode == 0 else (lambda h: h ** 0.25)
    # A -> R only: kappa = 0 (no I), gamma = delta = 0, alpha0 = alpha = 0
    A0 = 20000
    th = np.array([0, 0, 0, 0.05, 0, 0, 0, 0], np.float32)
    d0, d1 = _one_day_counts(th, 1e7, n, A0=A0, noise_mode=noise_mode)
    h = float(np.float32(0.05)) * A0
    _floor_moments_check(d1[:, 3] - d0[:, 3], h, sdf(h))
    # A -> D only
    th = np.array([0, 0, 0, 0, 0, 0.03, 0, 0], np.float32)
    d0, d1 = _one_day_counts(th, 1e7, n, A0=A0, noise_mode=noise_mode)
    h = float(np.float32(0.03)) * A0
    _floor_moments_check(d1[:, 4] - d0[:, 4], h, sdf(h))
    # I -> A and I -> Ru: kappa = 2 -> I0 = 2*A0; no infections
    th = np.array([0, 0, 0, 0.5, 0.2, 0, 0.1, 2.0], np.float32)
    d0, d1 = _one_day_counts(th, 1e7, n, A0=A0, noise_mode=noise_mode)
    I0 = 2 * A0
    h2 = float(np.float32(0.2)) * I0
    h5 = float(np.float32(0.5)) * float(np.float32(0.1)) * I0
    _floor_moments_check(d1[:, 4 + 1] - d0[:, 5], h5, sdf(h5))  # Ru gain
    # A gains n2 and loses n3 (beta A); R gain isolates n3, so n2 = dA + dR
    n2 = (d1[:, 2] - d0[:, 2]) + (d1[:, 3] - d0[:, 3])
    _floor_moments_check(n2, h2, sdf(h2))
    # S -> I: g = alpha0 + alpha/(1 + M^n) with n = 0 -> g = alpha0 + alpha/2
    th = np.array([0.3, 0.4, 0, 0, 0, 0, 0, 1.5], np.float32)
    P = 1e5
    d0, d1 = _one_day_counts(th, P, n, A0=A0, noise_mode=noise_mode)
    g = float(np.float32(0.3)) + float(np.float32(0.4)) / 2.0
    S0, I0 = float(d0[0, 0]), float(d0[0, 1])
    h1 = g * S0 * I0 / P
    _floor_moments_check(d0[:, 0] - d1[:, 0], h1, sdf(h1))
    # the five draws of a day are independent
    th = np.array([0.3, 0.4, 0, 0.2, 0.3, 0.1, 0.5, 1.5], np.float32)
    d0, d1 = _one_day_counts(th, P, n, A0=A0, noise_mode=noise_mode)
    dS = d0[:, 0] - d1[:, 0]
    dRu = d1[:, 5] - d0[:, 5]
    dR = d1[:, 3] - d0[:, 3]
    dD = d1[:, 4] - d0[:, 4]
    c = np.corrcoef(np.stack([dS, dRu, dR, dD]).astype(np.float64))
    assert np.all(np.abs(c - np.eye(4)) < 6 / math.sqrt(n))


def test_linear_limit_matches_exact_recurrence():
    """alpha = 0 makes g = alpha0; with P >> counts, S/P ~ 1 and the noise-free
    map is the linear recurrence v' = M v on (I, A, R, D, Ru). The floors lose
    less than one individual per transition per day; the test propagates that
    bound through |M| and checks the oracle stays within it."""
    T = 25
    P = 2_000_000_000  # counts stay far below P, so S/P stays close to 1
    for seed, th in enumerate([
            np.array([0.35, 0, 0, 0.05, 0.2, 0.01, 0.3, 1.0], np.float32),
            np.array([0.6, 0, 0, 0.1, 0.5, 0.02, 0.9, 0.5], np.float32),
            np.array([0.1, 0, 0, 0.2, 0.05, 0.1, 0.2, 2.0], np.float32)]):
        a0, _, _, b, gmm, dl, et, ka = (float(x) for x in th)
        m = oracle.make_model(P, T, A0=10000, noise_scale=0.0)
        tr = oracle.record(m, th[None], seed=seed)[0].astype(np.float64)
        Mx = np.array([
            [1 + a0 - gmm - b * et, 0, 0, 0, 0],
            [gmm, 1 - b - dl, 0, 0, 0],
            [0, b, 1, 0, 0],
            [0, dl, 0, 1, 0],
            [b * et, 0, 0, 0, 1]])
        v = tr[0, 1:].copy()
        err = np.zeros(5)
        floors = np.array([3.0, 3.0, 1.0, 1.0, 1.0])  # floors touching I, A, R, D, Ru per day
        for t in range(1, T + 1):
            v = Mx @ v
            # componentwise propagation through |M|; S/P deviates from 1 by
            # (P - S)/P, which scales the infection term a0*I
            s_dev = (P - tr[t - 1, 0]) / P
            err = np.abs(Mx) @ err + floors
            err[0] += a0 * tr[t - 1, 1] * s_dev
            assert np.all(np.abs(tr[t, 1:] - v) <= err + 1e-6), (t, tr[t, 1:], v, err)
        # the trajectory is not trivial: counts moved by much more than the bound
        moved = np.abs(tr[T, 1:] - tr[0, 1:])
        assert np.all(moved[1:] > 10 * err[1:]), (moved, err)


def test_noise_free_map_in_exact_arithmetic():
    """With noise_scale = 0 and n in {0, 1} every rate is rational; the exact
    floor map must equal the oracle's double-precision path (cases whose exact
    pre-floor value sits within 1e-9 of an integer are excluded)."""
    rng = np.random.default_rng(3)
    checked = 0
    for case in range(40):
        th = oracle.prior(1, seed=1000 + case)[0]
        th[2] = np.float32(case % 2)  # n = 0 or 1
        P = int(rng.integers(300, 20000))
        T = 12
        m = oracle.make_model(P, T, A0=int(rng.integers(1, 50)), noise_scale=0.0)
        tr = oracle.record(m, th[None], seed=1)[0]
        a0, al, n, b, gmm, dl, et, ka = (Fraction(float(x)) for x in th)
        A = int(m.A0)
        R = D = Ru = 0
        I = math.floor(ka * A)
        S = P - (A + I)
        ok = True
        for t in range(1, T + 1):
            M = A + R + D
            g = a0 + al / (1 + (Fraction(M) ** int(n)))
            hs = [g * S * I / P, gmm * I, b * A, dl * A, b * et * I]
            for h in hs:
                if abs(h - round(h)) < Fraction(1, 10**9) and h != round(h):
                    ok = False
            avail = [S, I, A, None, None]
            n1 = min(max(math.floor(hs[0]), 0), S)
            n2 = min(max(math.floor(hs[1]), 0), I)
            n3 = min(max(math.floor(hs[2]), 0), A)
            n4 = min(max(math.floor(hs[3]), 0), A - n3)
            n5 = min(max(math.floor(hs[4]), 0), I - n2)
            del avail
            S -= n1
            I += n1 - n2 - n5
            A += n2 - n3 - n4
            R += n3
            D += n4
            Ru += n5
            if not ok:
                break
            assert tuple(int(x) for x in tr[t]) == (S, I, A, R, D, Ru), (case, t)
        checked += ok
    assert checked >= 30


def test_distance_zero_on_own_series_and_alignment():
    m = oracle.make_model(1e7, 49)
    obs = oracle.observe(m, ITALY, seed=1)
    # the same stream (domain 0, sample 0) reproduces the series exactly
    d = oracle.distances(m, obs, seed=1, n=1, theta=ITALY[None], domain=oracle.DOMAIN_OBS)
    assert d[0] == 0.0
    # shifting the series by one day must give a positive distance
    shifted = np.concatenate([obs[:, 1:], obs[:, -1:]], axis=1)
    d = oracle.distances(m, shifted, seed=1, n=1, theta=ITALY[None], domain=oracle.DOMAIN_OBS)
    assert d[0] > 0.1


def test_distance_against_high_precision_restatement():
    import mpmath

    mpmath.mp.dps = 40
    m = oracle.make_model(8.3e7, 72)
    obs = oracle.observe(m, NZ, seed=3)
    th = oracle.prior(20, seed=4)
    d = oracle.distances(m, obs, seed=4, n=20, theta=th)
    tr = oracle.record(m, th, seed=4)
    for i in range(20):
        acc = mpmath.mpf(0)
        for t in range(1, 73):
            for c in range(3):
                X = int(tr[i, t, 2 + c])
                O = int(obs[c, t - 1])
                acc += (mpmath.log(1 + X) - mpmath.log(1 + O)) ** 2
        assert abs(float(mpmath.sqrt(acc)) - d[i]) <= 1e-12 * d[i]
    # raw-count distance is an exact integer sum of squares
    m = oracle.make_model(8.3e7, 72, dist_mode=1)
    d = oracle.distances(m, obs, seed=4, n=20, theta=th)
    for i in range(20):
        s = sum((int(tr[i, t, 2 + c]) - int(obs[c, t - 1])) ** 2
                for t in range(1, 73) for c in range(3))
        assert abs(d[i] - math.sqrt(s)) <= 1e-12 * math.sqrt(s)


def test_prior_drawn_distances_use_the_prior_stream():
    m = oracle.make_model(1e7, 30)
    obs = oracle.observe(m, ITALY, seed=1)
    th = oracle.prior(50, seed=6, first=200)
    a = oracle.distances(m, obs, seed=6, n=50, first=200)
    b = oracle.distances(m, obs, seed=6, n=50, first=200, theta=th)
    np.testing.assert_array_equal(a, b)


def test_accept_nearest_pilot_brute_force():
    rng = np.random.default_rng(0)
    d = rng.exponential(size=5000)
    d[10] = d[20] = d[30] = 0.0  # ties resolved to the lower index
    eps = 0.05
    np.testing.assert_array_equal(oracle.accept(d, eps),
                                  [i for i in range(d.size) if d[i] <= eps])
    near = oracle.nearest(d, 2)
    np.testing.assert_array_equal(near, [10, 20])
    k = oracle.nearest(d, 100)
    assert len(k) == 100 and d[k].max() <= np.sort(d)[99]
    e = oracle.pilot_eps(d, 1e-3)
    assert np.sum(d <= e) >= 5 and np.sum(d < e) < 5
    q = oracle.first_accepted(d, 0.2, 7)
    assert list(q) == [i for i in range(d.size) if d[i] <= 0.2][:7]


def test_moments_match_numpy_weighted_covariance():
    rng = np.random.default_rng(1)
    th = rng.uniform(0, 1, size=(500, 8)) * oracle.PRIOR_HI
    w = rng.exponential(size=500)
    mean, cov = oracle.moments(th, w)
    np.testing.assert_allclose(mean, np.average(th, axis=0, weights=w), rtol=1e-13)
    np.testing.assert_allclose(cov, np.cov(th.T, aweights=w, ddof=1), rtol=1e-11, atol=1e-13)
    mean, cov = oracle.moments(th)
    np.testing.assert_allclose(mean, th.mean(0), rtol=1e-13)
    np.testing.assert_allclose(cov, np.cov(th.T), rtol=1e-11, atol=1e-13)
