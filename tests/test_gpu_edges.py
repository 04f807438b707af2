"""Edge cases of the plain pass at the limits of the method and of the boundary.

* the shortest and longest horizons the boundary accepts (T = 1 and
  T = ABC_T_MAX = 1024), the largest population (1e9) and the smallest ones:
  P = A0 + R0 + D0 + 2 A0 (room for the most an upper-box kappa moves into I)
  and P = A0 (no room at all: I0 is limited to 0 and S = 0);
* a start with recovered and dead counts already present (R0, D0 > 0);
* an infinite tolerance: every sample is accepted, in index order;
* a tolerance of 0: only an exact match is accepted. The observed series is
  the trajectory of one sample on the sampling stream itself, so that sample
  has distance exactly 0 (decided by the float64 path, since a relative band
  has no width at eps = 0);
* a point prior (lo = hi) and, with it, the noise-free model, where every
  sample has the same trajectory and so the same distance: all of them are
  accepted just above that distance and none just below it.

Each case compares the device pass (float32 simulation, compaction at
eps (1 + w), float64 decision of the band) with the oracle's accept rule
dist <= eps, outside the tie band |d - eps| < 1e-5 eps.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2012_14332_amd import workloads as W

pytestmark = pytest.mark.gpu

TIE = 1e-5
BAND = 0.02


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_14332_amd import abc

    abc.lib()
    abc.set_launch_config(0, 0, 0)
    return abc


def _device_pass(A, ser, eps, n, seed, *, first=0, prior=None, flags=0, noise=1.0, cap=1 << 16):
    eps_hi = eps * (1.0 + BAND) if math.isfinite(eps) else math.inf
    d = A.simulate_distance(ser, n, seed, first=first, eps_exit=eps_hi, prior=prior, flags=flags,
                            noise_scale=noise)
    idx, th, dd, _, cnt = A.accept_compact(d, eps_hi, cap, first=first, seed=seed, prior=prior)
    A.recheck_band(ser, seed, eps, BAND, idx, th, dd, cnt, flags=flags, noise_scale=noise)
    c = int(cnt.item())
    assert c <= cap
    return idx[:c].cpu().numpy(), th[:c].cpu().numpy()


def _eps_between(ref, q):
    """A tolerance near the q-quantile that lies halfway between two distinct
    distances, so that no sample sits on it (short horizons give many ties)."""
    u = np.unique(ref)
    k = max(1, int(np.searchsorted(u, np.quantile(ref, q))))
    return float(0.5 * (u[k - 1] + u[k]))


def _agree(got, ref, eps, first=0):
    want = np.nonzero(ref <= eps)[0] + first
    diff = np.setxor1d(got, want)
    tie = diff[np.abs(ref[diff - first] - eps) < TIE * eps] if diff.size else diff
    assert diff.size == tie.size, [(int(i), ref[i - first], eps) for i in np.setdiff1d(diff, tie)][:10]
    return want


@pytest.mark.parametrize("P,T,n", [(1_000_000, 1, 200_000), (1_000_000_000, 1024, 20_000),
                                   (300, 60, 200_000), (100, 40, 100_000)])
def test_horizon_and_population_limits(A, P, T, n):
    th_true = W.THETA_NZ
    m = oracle.make_model(P, T)
    obs = oracle.observe(m, th_true, 21)
    ser = A.DeviceSeries(P, T, torch.from_numpy(obs))
    ref = oracle.distances(m, obs, seed=5, n=n)
    eps = _eps_between(ref, 0.01)
    got, th = _device_pass(A, ser, eps, n, 5)
    want = _agree(got, ref, eps)
    print("P=%d T=%d: %d accepted of %d" % (P, T, got.size, n))
    if np.array_equal(got, want):
        np.testing.assert_array_equal(th, oracle.prior(n, seed=5)[want])
    # the float64 device distance at the horizon limit, sample by sample
    if T == 1024:
        d64 = A.simulate_distance(ser, 300, 5, flags=A.ABC_FP64, want64=True)[1].cpu().numpy()
        np.testing.assert_allclose(d64, ref[:300], rtol=1e-12)


def test_population_below_the_initial_counts_is_rejected(A):
    obs = torch.zeros((3, 10), dtype=torch.int32)
    ser = A.DeviceSeries(99, 10, obs)            # A0 = 100 > P
    with pytest.raises(A.AbcError):
        A.simulate_distance(ser, 10, 1)
    with pytest.raises(A.AbcError):
        A.simulate_distance(A.DeviceSeries(2**31, 10, obs), 10, 1)   # P beyond int32


def test_start_with_recovered_and_dead(A):
    P, T, n = 50_000_000, 40, 200_000
    m = oracle.make_model(P, T, A0=500, R0=20, D0=3)
    obs = oracle.observe(m, W.THETA_ITALY, 22)
    ser = A.DeviceSeries(P, T, torch.from_numpy(obs), A0=500, R0=20, D0=3)
    ref = oracle.distances(m, obs, seed=6, n=n)
    eps = _eps_between(ref, 0.005)
    got, _ = _device_pass(A, ser, eps, n, 6)
    _agree(got, ref, eps)
    assert got.size > 0


def test_infinite_tolerance_accepts_everything(A):
    s = W.three_countries()[0]
    m = oracle.make_model(s.P, s.T)
    obs = oracle.observe(m, s.theta_true, s.obs_seed)
    ser = A.DeviceSeries(s.P, s.T, torch.from_numpy(obs))
    n, first = 70_001, 5_000_000_000
    got, th = _device_pass(A, ser, math.inf, n, 7, first=first, cap=n)
    np.testing.assert_array_equal(got, np.arange(first, first + n))
    ref_th = oracle.prior(n, seed=7, first=first)
    np.testing.assert_array_equal(th, ref_th)
    mean, cov = A.posterior_moments(torch.from_numpy(th).cuda())
    rm, rc = oracle.moments(ref_th)
    np.testing.assert_allclose(mean.cpu().numpy(), rm, rtol=1e-12)
    np.testing.assert_allclose(cov.cpu().numpy(), rc, rtol=1e-9, atol=1e-12)


def test_zero_tolerance_accepts_only_exact_matches(A):
    P, T, n, seed, star = 2_000_000, 30, 50_000, 8, 12_345
    m = oracle.make_model(P, T)
    th_star = oracle.prior(1, seed=seed, first=star)[0]
    traj, _ = oracle.trajectory(m, th_star, seed, sample=star)      # sampling stream, domain 1
    obs = np.ascontiguousarray(traj[1:, 2:5].T.astype(np.int32))
    ser = A.DeviceSeries(P, T, torch.from_numpy(obs))
    ref = oracle.distances(m, obs, seed=seed, n=n)
    assert ref[star] == 0.0
    got, _ = _device_pass(A, ser, 0.0, n, seed, flags=A.ABC_FP64)
    np.testing.assert_array_equal(got, np.nonzero(ref == 0.0)[0])
    assert star in got


@pytest.mark.parametrize("noise", [1.0, 0.0])
def test_point_prior(A, noise):
    P, T, n, seed = 80_000_000, 50, 100_000, 9
    pt = W.THETA_ITALY.astype(np.float32)
    pr = A.make_prior(pt.tolist(), pt.tolist())
    m = oracle.make_model(P, T, noise_scale=noise)
    obs = oracle.observe(oracle.make_model(P, T), W.THETA_NZ, 23)
    ser = A.DeviceSeries(P, T, torch.from_numpy(obs))
    ref = oracle.distances(m, obs, seed=seed, n=n, lo=pt, hi=pt)
    if noise == 0.0:
        # one trajectory for every sample: all distances tie
        assert np.all(ref == ref[0])
        for f, k in ((1.0 + 1e-4, n), (1.0 - 1e-4, 0)):
            got, th = _device_pass(A, ser, float(ref[0] * f), n, seed, prior=pr, noise=0.0,
                                   cap=n)
            assert got.size == k
            if k:
                np.testing.assert_array_equal(got, np.arange(n))
                assert np.all(th == pt)
    else:
        # one theta: the distances crowd together, so most samples fall in the band
        eps = _eps_between(ref, 0.02)
        got, th = _device_pass(A, ser, eps, n, seed, prior=pr, cap=n)
        _agree(got, ref, eps)
        assert got.size > 0 and np.all(th == pt)


def test_band_decision_many_rows_per_wavefront(A):
    """A wide band (w = 0.5) around the median distance puts most of ~5e4
    candidates in the band, so each band-decision wavefront gathers several
    groups of rows. Every kept row, its order and its distance follow the
    float64 distances of the same samples: in-band rows are kept when their
    float64 distance is <= eps and carry it (rounded to float32); the others
    keep the float32 decision."""
    s = W.single_country()
    m = oracle.make_model(s.P, s.T)
    obs = oracle.observe(m, s.theta_true, s.obs_seed)
    ser = A.DeviceSeries(s.P, s.T, torch.from_numpy(obs))
    n, seed, w = 60_000, 12, 0.5
    d32 = A.simulate_distance(ser, n, seed)
    eps = float(np.float32(np.median(d32.cpu().numpy())))
    e_hi = eps * (1.0 + w)
    idx, th, dd, _, cnt = A.accept_compact(d32, e_hi, n, seed=seed)
    c0 = int(cnt.item())
    assert c0 > 2048 * 16
    cand_idx = idx[:c0].cpu().numpy().copy()
    cand_d = dd[:c0].cpu().numpy().copy()
    nre = A.recheck_band(ser, seed, eps, w, idx, th, dd, cnt, want_rechecked=True)
    _, d64 = A.simulate_distance(ser, n, seed, flags=A.ABC_FP64, want64=True)
    d64 = d64.cpu().numpy()
    e32, w64 = np.float64(np.float32(eps)), np.float64(np.float32(w))
    lo, hi = np.float32(e32 * (1.0 - w64)), np.float32(e32 * (1.0 + w64))
    inb = (cand_d > lo) & (cand_d <= hi)
    keep = np.where(inb, d64[cand_idx] <= e32, cand_d <= np.float32(eps))
    want_d = np.where(inb, d64[cand_idx].astype(np.float32), cand_d)[keep]
    c = int(cnt.item())
    assert int(nre.item()) == int(inb.sum())
    np.testing.assert_array_equal(idx[:c].cpu().numpy(), cand_idx[keep])
    np.testing.assert_array_equal(dd[:c].cpu().numpy(), want_d)
