"""Launch-shape independence of the float32 simulate+distance kernel.

Every random number is fixed by (seed, domain, series, sample index, day), so
samples-per-lane, workgroup size, resident grid, call splitting, in-kernel vs
supplied theta and early exit must all give bit-identical distances (early
exit only replaces distances above the bound by +INF).
"""
import math

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
    yield abc
    abc.set_launch_config(0, 0, 0)


@pytest.fixture(scope="module")
def ser(A):
    s = W.three_countries()[2]
    obs = oracle.observe(oracle.make_model(s.P, s.T), s.theta_true, s.obs_seed)
    return A.DeviceSeries(s.P, s.T, torch.from_numpy(obs))


N = 100_003


def _run(A, ser, n=N, **kw):
    return A.simulate_distance(ser, n, 3, **kw).cpu().numpy()


def test_launch_configs_bit_identical(A, ser):
    A.set_launch_config(0, 0, 0)
    ref_inf = _run(A, ser)
    eps = float(np.quantile(ref_inf, 0.01))
    ref_eps = _run(A, ser, eps_exit=eps)
    for spl, block, bpc in [(1, 64, 1), (1, 1024, 2), (2, 128, 8), (2, 512, 4), (4, 256, 3),
                            (8, 128, 8), (8, 64, 16)]:
        A.set_launch_config(spl, block, bpc)
        assert A.get_launch_config() == (spl, block, bpc)
        np.testing.assert_array_equal(_run(A, ser), ref_inf, err_msg=str((spl, block, bpc)))
        np.testing.assert_array_equal(_run(A, ser, eps_exit=eps), ref_eps,
                                      err_msg=str((spl, block, bpc)))
    A.set_launch_config(0, 0, 0)


def test_refill_threshold_bit_identical(A, ser):
    A.set_launch_config(0, 0, 0)
    A.set_refill_min(0)
    assert A.get_refill_min() == 8
    ref_inf = _run(A, ser)
    eps = float(np.quantile(ref_inf, 0.01))
    ref_eps = _run(A, ser, eps_exit=eps)
    for lanes, shape in [(1, (1, 512, 4)), (32, (2, 256, 4)), (64, (1, 64, 1)), (17, (4, 128, 2))]:
        A.set_refill_min(lanes)
        A.set_launch_config(*shape)
        np.testing.assert_array_equal(_run(A, ser), ref_inf, err_msg=str(lanes))
        np.testing.assert_array_equal(_run(A, ser, eps_exit=eps), ref_eps, err_msg=str(lanes))
    with pytest.raises(A.AbcError):
        A.set_refill_min(65)
    A.set_refill_min(0)
    A.set_launch_config(0, 0, 0)


def test_invalid_launch_config(A):
    with pytest.raises(A.AbcError):
        A.set_launch_config(3, 256, 8)
    with pytest.raises(A.AbcError):
        A.set_launch_config(4, 512, 8)
    with pytest.raises(A.AbcError):
        A.set_launch_config(1, 100, 8)
    A.set_launch_config(0, 0, 0)


def test_early_exit_only_masks_rejections(A, ser):
    full = _run(A, ser)
    for q in (1e-4, 1e-2, 0.5):
        eps = float(np.quantile(full, q))
        d = _run(A, ser, eps_exit=eps)
        inf = np.isinf(d)
        np.testing.assert_array_equal(d[~inf], full[~inf])
        assert np.all(full[inf] > eps)
        np.testing.assert_array_equal(np.nonzero(d <= eps)[0], np.nonzero(full <= eps)[0])


def test_split_calls_and_supplied_theta(A, ser):
    whole = _run(A, ser, n=N)
    parts = []
    cuts = [0, 1, 4096, 50_000, 77_777, N]
    for a, b in zip(cuts[:-1], cuts[1:]):
        parts.append(A.simulate_distance(ser, b - a, 3, first=a).cpu().numpy())
    np.testing.assert_array_equal(np.concatenate(parts), whole)
    th = A.sample_prior(N, seed=3)
    np.testing.assert_array_equal(A.simulate_distance(ser, N, 3, theta=th).cpu().numpy(), whole)


def test_kahan_close_to_naive(A, ser):
    a = _run(A, ser)
    b = _run(A, ser, flags=A.ABC_KAHAN)
    rel = np.abs(a - b) / a
    assert rel.max() < 1e-5


@pytest.mark.parametrize("flags,kw", [(0x4, dict(noise_mode=1)), (0x8, dict(dist_mode=1)),
                                      (0x0, dict(noise_scale=0.0)), (0x0, dict(noise_scale=0.3))])
def test_fp32_modes_track_oracle(A, flags, kw):
    s = W.three_countries()[0]
    m = oracle.make_model(s.P, s.T, **kw)
    obs = oracle.observe(oracle.make_model(s.P, s.T), s.theta_true, s.obs_seed)
    ser = A.DeviceSeries(s.P, s.T, torch.from_numpy(obs))
    n = 20000
    d = A.simulate_distance(ser, n, 5, flags=flags, noise_scale=kw.get("noise_scale", 1.0))
    ref = oracle.distances(m, obs, seed=5, n=n)
    rel = np.abs(d.cpu().numpy() - ref) / np.maximum(ref, 1e-30)
    assert np.median(rel) < 1e-4, np.median(rel)
    assert np.quantile(rel, 0.99) < 1e-2, np.quantile(rel, 0.99)


def _days(A, ser, n, **kw):
    days = torch.zeros(1, dtype=torch.int64, device="cuda")
    d = A.simulate_distance(ser, n, 3, days=days, **kw).cpu().numpy()
    return d, int(days.item())


@pytest.mark.parametrize("which", ["country-T72", "country-T100", "T1024"])
def test_future_bound_only_masks_rejections(A, which):
    """The lower bound on the days still to come (R and D never fall) may
    exit a sample earlier than the running sum alone, never later, and only
    where the float32 distance run to day T ends above the exit bound."""
    if which == "T1024":
        P, T, th, seed = 1_000_000_000, 1024, W.THETA_NZ, 7
    else:
        s = W.three_countries()[1 if which == "country-T72" else 2]
        P, T, th, seed = s.P, s.T, s.theta_true, s.obs_seed
    obs = oracle.observe(oracle.make_model(P, T), th, seed)
    ser = A.DeviceSeries(P, T, torch.from_numpy(obs))
    n = 100_003 if T <= 100 else 20_011
    A.set_launch_config(0, 0, 0)
    full = _run(A, ser, n=n)
    for q in (1e-3, 0.05):
        eps = float(np.quantile(full, q))
        d_b, days_b = _days(A, ser, n, eps_exit=eps)
        d_n, days_n = _days(A, ser, n, eps_exit=eps, flags=A.ABC_NO_BOUND)
        inf_b, inf_n = np.isinf(d_b), np.isinf(d_n)
        np.testing.assert_array_equal(d_b[~inf_b], full[~inf_b])
        assert np.all(inf_b[inf_n])                  # never exits later
        assert np.all(full[inf_b] > eps)             # +INF keeps its meaning
        np.testing.assert_array_equal(np.nonzero(d_b <= eps)[0], np.nonzero(full <= eps)[0])
        assert days_b <= days_n
        if which == "country-T72" and q == 1e-3:
            assert days_b <= 0.8 * days_n   # the low-death country: the bound must bite
        print("%s q=%g: sample-days %d -> %d (%.1f%% fewer)"
              % (which, q, days_n, days_b, 100.0 * (1 - days_b / days_n)))
        # compensated sums take the same bound
        if which == "country-T72":
            fullk = _run(A, ser, n=n, flags=A.ABC_KAHAN)
            d_k = _run(A, ser, n=n, eps_exit=eps, flags=A.ABC_KAHAN)
            inf_k = np.isinf(d_k)
            np.testing.assert_array_equal(d_k[~inf_k], fullk[~inf_k])
            assert np.all(fullk[inf_k] > eps)
        # the bound is part of the launch-independent result
        for shape in [(1, 64, 1), (4, 256, 3)]:
            A.set_launch_config(*shape)
            np.testing.assert_array_equal(_run(A, ser, n=n, eps_exit=eps), d_b, err_msg=str(shape))
        A.set_launch_config(0, 0, 0)
