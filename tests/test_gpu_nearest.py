"""Nearest-k selection on the GPU (the single-country workload keeps the 100
nearest of 1e5 prior samples) through the C ABI.

Bars: abc_nearest_k returns exactly the oracle's nearest set (k smallest
distances, ties to the lower index) in index order, with theta copied or
re-drawn bit-exactly, for random, tied, infinite and NaN inputs; the float64
row path ranks by (float64 distance, index) exactly; the single-country
pipeline (float32 simulation, nearest-k, float64 decision of the band)
returns the oracle's 100 nearest of the float64 distances bit-exactly.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2012_14332_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_14332_amd import abc

    abc.lib()
    return abc


def _check(A, d, k, first=0, theta=None):
    dist = torch.from_numpy(d).cuda()
    th = None if theta is None else torch.from_numpy(theta).cuda()
    idx, tho, do, kth = A.nearest_k(dist, k, theta=th, first=first, seed=3, series=2)
    want = oracle.nearest(d, k)
    got = idx.cpu().numpy() - first
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(do.cpu().numpy(), d[want])
    assert kth.item() == np.max(d[want]) or (np.isnan(kth.item()) and np.isnan(d[want]).any())
    if theta is None:
        ref = oracle.prior(1, 3, 1, 2, 0)  # shape check of the re-draw helper
        assert ref.shape == (1, 8)
        for r, i in enumerate(want[:50]):
            np.testing.assert_array_equal(tho[r].cpu().numpy(),
                                          oracle.prior(1, 3, 1, 2, first + int(i))[0])
    else:
        np.testing.assert_array_equal(tho.cpu().numpy(), theta[want])


@pytest.mark.parametrize("n,k", [(1, 1), (100, 100), (4097, 1), (4097, 100), (1_000_003, 100),
                                 (1_000_003, 4096), (1 << 24, 100)])
def test_nearest_random(A, n, k):
    rng = np.random.default_rng(n + k)
    d = rng.gamma(20.0, 1.0, size=n).astype(np.float32)
    _check(A, d, k, first=12345)


def test_nearest_with_theta_and_infinite_and_nan(A):
    rng = np.random.default_rng(1)
    n = 300_000
    d = rng.exponential(size=n).astype(np.float32)
    d[rng.random(n) < 0.9] = np.inf          # early-exited samples
    d[rng.integers(0, n, 50)] = np.nan
    th = rng.random((n, 8)).astype(np.float32)
    _check(A, d, 500, theta=th)


def test_nearest_heavy_ties_use_the_index(A):
    # integer-valued distances: long runs of equal keys
    rng = np.random.default_rng(2)
    n = 2_000_000
    d = rng.integers(0, 3, size=n).astype(np.float32)
    _check(A, d, 4096)
    d[:] = 1.0
    _check(A, d, 100, first=7)
    d = np.zeros(100_000, dtype=np.float32)
    d[::2] = -0.0
    _check(A, d, 33)


def test_nearest_fewer_finite_than_k_is_an_error(A):
    d = np.full(1000, np.inf, dtype=np.float32)
    d[:10] = 1.0
    with pytest.raises(A.AbcError, match="finite"):
        A.nearest_k(torch.from_numpy(d).cuda(), 11)
    with pytest.raises(A.AbcError):
        A.nearest_k(torch.from_numpy(d).cuda(), 5000)


def test_nearest_rows_rank_by_float64_then_index(A):
    rng = np.random.default_rng(4)
    n = 5000
    d = rng.random(n)
    d[100:200] = d[50]  # ties resolved by idx
    idx = np.sort(rng.choice(10**9, size=n, replace=False)).astype(np.int64)
    th = rng.random((n, 8)).astype(np.float32)
    oi, ot, od = A.nearest_k_rows(torch.from_numpy(d).cuda(), torch.from_numpy(idx).cuda(),
                                  torch.from_numpy(th).cuda(), 300)
    order = np.lexsort((idx, d))[:300]
    sel = np.sort(order)
    np.testing.assert_array_equal(oi.cpu().numpy(), idx[sel])
    np.testing.assert_array_equal(ot.cpu().numpy(), th[sel])
    np.testing.assert_array_equal(od.cpu().numpy(), d[sel])


def test_simulate_rows_f64_matches_oracle(A):
    s = W.three_countries()[1]
    m = oracle.make_model(s.P, s.T)
    obs = oracle.observe(m, s.theta_true, s.obs_seed)
    ser = A.DeviceSeries(s.P, s.T, torch.from_numpy(obs))
    idx = np.array([0, 5, 77, 1 << 33, 123456789], dtype=np.int64)
    th = oracle.prior(5, seed=9)
    d = A.simulate_rows_f64(ser, 1, torch.from_numpy(idx).cuda(), torch.from_numpy(th).cuda(),
                            series=1).cpu().numpy()
    for q in range(5):
        ref = oracle.distances(m, obs, 1, 1, first=int(idx[q]), series=1, theta=th[q:q + 1])[0]
        assert abs(d[q] - ref) <= 1e-12 * ref


@pytest.mark.parametrize("country,n", [(0, 1), (0, 63), (0, 3 * 1024 + 17), (0, 9000), (2, 5000)])
def test_simulate_rows_f64_side_by_side_rows(A, country, n):
    """Several rows per wavefront (n above 1024 rows), ragged last blocks: the
    same doubles as the one-lane-per-sample float64 simulation of the same
    samples and parameters."""
    s = W.three_countries()[country]
    m = oracle.make_model(s.P, s.T)
    obs = oracle.observe(m, s.theta_true, s.obs_seed)
    ser = A.DeviceSeries(s.P, s.T, torch.from_numpy(obs))
    first = 1 << 20
    th = A.sample_prior(n, 4, first=first)
    idx = torch.arange(first, first + n, dtype=torch.int64, device="cuda")
    d = A.simulate_rows_f64(ser, 4, idx, th).cpu().numpy()
    _, d64 = A.simulate_distance(ser, n, 4, theta=th, first=first, flags=A.ABC_FP64, want64=True)
    np.testing.assert_array_equal(d, d64.cpu().numpy())


@pytest.mark.parametrize("T,n", [(1, 2000), (13, 5000), (1024, 1500)])
def test_simulate_rows_f64_short_and_long_horizons(A, T, n):
    """Horizons that end inside the first window (T = 1), a ragged last window
    (T = 13) and the longest horizon (T = 1024): the row kernel's doubles equal
    the one-lane float64 simulation's."""
    P = 1_000_000
    m = oracle.make_model(P, T)
    obs = oracle.observe(m, W.THETA_NZ, 21)
    ser = A.DeviceSeries(P, T, torch.from_numpy(obs))
    th = A.sample_prior(n, 5)
    idx = torch.arange(n, dtype=torch.int64, device="cuda")
    d = A.simulate_rows_f64(ser, 5, idx, th).cpu().numpy()
    _, d64 = A.simulate_distance(ser, n, 5, theta=th, flags=A.ABC_FP64, want64=True)
    np.testing.assert_array_equal(d, d64.cpu().numpy())


def test_single_country_nearest_100_of_1e5(A):
    """The single-country workload end to end against the oracle's rule."""
    from paper_2012_14332_amd import pipeline as P

    s = W.single_country()
    m = oracle.make_model(s.P, s.T)
    obs = oracle.observe(m, s.theta_true, s.obs_seed)
    ref = oracle.distances(m, obs, 1, 100_000)
    want = oracle.nearest(ref, 100)
    ser = P.observed_series(s)
    res = P.NearestABC(ser, 1, 100_000, 100).run(0)
    np.testing.assert_array_equal(res.idx.cpu().numpy(), want)
    np.testing.assert_array_equal(res.theta.cpu().numpy(), oracle.prior(100_000, 1)[want])
    d = res.dist.cpu().numpy()
    assert np.max(np.abs(d - ref[want]) / ref[want]) <= 1e-12
    mean, cov = oracle.moments(oracle.prior(100_000, 1)[want])
    np.testing.assert_allclose(res.mean.cpu().numpy(), mean, rtol=1e-12)
    np.testing.assert_allclose(res.cov.cpu().numpy(), cov, rtol=1e-10, atol=1e-14)
    assert 100 <= res.candidates < 2000
