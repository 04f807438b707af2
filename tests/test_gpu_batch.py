"""Batched persistent path (many uneven series, hipGraph rounds, per-series
quota) against the oracle's rule: for series j, the first Q sample indices i
of its stream with dist_i <= eps_j, in index order.

Also: the result does not depend on the round size, the rounds per graph
replay or the launch shape, and equals the plain path on the same prefix.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2012_14332_amd import workloads as W

pytestmark = pytest.mark.gpu
TIE = 1e-5


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_14332_amd import abc, pipeline

    abc.lib()
    yield abc, pipeline
    abc.set_launch_config(0, 0, 0)


def _setup(env, m, q):
    abc, P = env
    ss = W.uneven_series(64, 5)[:m]
    sers = [P.observed_series(s) for s in ss]
    eps = [P.pilot_eps(ser, 9, n=20000, q=q, series=j) for j, ser in enumerate(sers)]
    return ss, sers, eps


def _oracle_first(s, j, eps, used, quota):
    m = oracle.make_model(s.P, s.T)
    obs = oracle.observe(m, s.theta_true, s.obs_seed, series=s.series_id)
    d = oracle.distances(m, obs, seed=9, n=used, series=j)
    return d, oracle.first_accepted(d, eps, quota)


def test_batch_matches_oracle_first_quota(env):
    abc, _ = env
    ss, sers, eps = _setup(env, 16, 5e-3)
    quota = 40
    out = abc.batch_run(sers, eps, 9, quota, round_size=1 << 16)
    cnt = out["count"].cpu().numpy()
    used = out["used"].cpu().numpy()
    idx = out["idx"].cpu().numpy()
    assert np.all(cnt == quota), cnt
    for j, s in enumerate(ss):
        d, want = _oracle_first(s, j, eps[j], int(used[j]), quota)
        got = idx[j]
        if not np.array_equal(got, want):
            diff = set(got.tolist()) ^ set(want.tolist())
            assert all(abs(d[i] - eps[j]) < TIE * eps[j] for i in diff if i < len(d)), (j, diff)
        th = oracle.prior(1, seed=9, series=j, first=int(got[0]))[0]
        np.testing.assert_array_equal(out["theta"][j, 0].cpu().numpy(), th)
    st = out["stats"]
    assert st["rounds"] >= 1 and st["sample_days"] > 0


def test_batch_independent_of_round_size_and_launch(env):
    abc, _ = env
    ss, sers, eps = _setup(env, 12, 1e-2)
    ref = abc.batch_run(sers, eps, 9, 30, round_size=1 << 15, rounds_per_graph=1,
                        cand_capacity=4096)
    ref_idx = ref["idx"].cpu().numpy()
    for rs, rpg, cfg, lanes in [(1 << 17, 4, (1, 512, 4), 1), (1 << 16, 8, (2, 256, 4), 16),
                                (50_000, 2, (4, 128, 2), 64), (1 << 20, 1, (1, 1024, 1), 9),
                                (1 << 18, 2, (8, 128, 4), 8), (1 << 16, 4, (8, 64, 8), 24)]:
        abc.set_launch_config(*cfg)
        abc.set_refill_min(lanes)
        o = abc.batch_run(sers, eps, 9, 30, round_size=rs, rounds_per_graph=rpg,
                          cand_capacity=4096)
        np.testing.assert_array_equal(o["idx"].cpu().numpy(), ref_idx, err_msg=str((rs, rpg, cfg)))
        np.testing.assert_array_equal(o["theta"].cpu().numpy(), ref["theta"].cpu().numpy())
        np.testing.assert_array_equal(o["dist"].cpu().numpy(), ref["dist"].cpu().numpy())
        np.testing.assert_allclose(o["mean"].cpu().numpy(), ref["mean"].cpu().numpy(), rtol=1e-13)
        assert o["stats"]["spl"] == cfg[0] and o["stats"]["block"] == cfg[1]
    abc.set_launch_config(0, 0, 0)
    abc.set_refill_min(0)


def test_batch_equals_plain_path(env):
    abc, P = env
    ss, sers, eps = _setup(env, 6, 1e-2)
    quota = 25
    o = abc.batch_run(sers, eps, 9, quota, round_size=1 << 15)
    for j, ser in enumerate(sers):
        used = int(o["used"][j].item())
        run = P.PlainABC(ser, 9, eps[j], used, series=j, band_w=0.02, capacity=1 << 14)
        r = run.run(0)
        c = r.n()
        assert c >= quota
        np.testing.assert_array_equal(o["idx"][j].cpu().numpy(), r.idx[:quota].cpu().numpy())
        rm, rc = oracle.moments(r.theta[:quota].cpu().numpy())
        np.testing.assert_allclose(o["mean"][j].cpu().numpy(), rm, rtol=1e-12)
        np.testing.assert_allclose(o["cov"][j].cpu().numpy(), rc, rtol=1e-9, atol=1e-12)


def test_batch_continues_a_series_left_short(env):
    """A first target far below the quota (margin -Q/2) makes the first
    finalisation keep about half of each series' rows; the series continue
    their streams and are finalised again. The rows kept are the default
    run's, whatever the schedule."""
    abc, _ = env
    ss, sers, eps = _setup(env, 8, 5e-3)
    quota = 40
    ref = abc.batch_run(sers, eps, 9, quota, round_size=1 << 16)
    for margin in (-quota // 2, -quota + 1):
        try:
            abc.set_batch_margin(margin)
            o = abc.batch_run(sers, eps, 9, quota, round_size=1 << 16)
        finally:
            abc.set_batch_margin(0)
        assert o["stats"]["phases"] >= 2, (margin, o["stats"])
        for k in ("idx", "theta", "dist", "count"):
            np.testing.assert_array_equal(o[k].cpu().numpy(), ref[k].cpu().numpy(), err_msg=k)
        np.testing.assert_allclose(o["mean"].cpu().numpy(), ref["mean"].cpu().numpy(), rtol=1e-13)


def test_batch_limits(env):
    abc, _ = env
    ss, sers, eps = _setup(env, 4, 1e-3)
    o = abc.batch_run(sers, eps, 9, 50, round_size=1 << 12, max_samples=5000, check=False)
    assert o["status"] == -5  # quota not reachable within max_samples
    assert np.all(o["used"].cpu().numpy() <= 5000)
    assert np.all(o["count"].cpu().numpy() < 50)
    with pytest.raises(abc.AbcError):
        abc.batch_run(sers, eps, 9, 0)
    # a capacity below what one round produces is reported, never overrun
    o = abc.batch_run(sers, [e * 3 for e in eps], 9, 20, round_size=1 << 18, cand_capacity=20,
                      check=False)
    assert o["status"] == -5


def _agree_first(d, eps, got, want):
    if not np.array_equal(got, want):
        diff = set(got.tolist()) ^ set(want.tolist())
        assert all(abs(d[i] - eps) < TIE * eps for i in diff if i < len(d)), diff


def test_batch_extremes(env):
    """Series at the limits in one batch: T = 1, T = 200 at P = 1e9, the
    smallest population (P = A0: no room for I0), quota 1, and a tolerance
    above every distance (the first Q indices are the answer)."""
    abc, P = env
    specs = [(1_000_000, 1, W.THETA_NZ), (1_000_000_000, 200, W.THETA_USA), (100, 40, W.THETA_ITALY),
             (50_000_000, 60, W.THETA_ITALY)]
    sers, obs_l = [], []
    for j, (Pp, T, th) in enumerate(specs):
        obs = oracle.observe(oracle.make_model(Pp, T), th, 31, series=j)
        obs_l.append(obs)
        sers.append(abc.DeviceSeries(Pp, T, torch.from_numpy(obs)))
    eps = []
    refs = []
    for j, (Pp, T, _) in enumerate(specs):
        d = oracle.distances(oracle.make_model(Pp, T), obs_l[j], seed=9, n=40_000, series=j)
        refs.append(d)
        u = np.unique(d)
        k = max(1, int(np.searchsorted(u, np.quantile(d, 2e-3))))
        eps.append(float(0.5 * (u[k - 1] + u[k])))
    eps[3] = 1e30                                  # every sample of series 3 is accepted
    for quota in (1, 25):
        out = abc.batch_run(sers, eps, 9, quota, round_size=1 << 14)
        cnt, used, idx = (out[k].cpu().numpy() for k in ("count", "used", "idx"))
        assert np.all(cnt == quota), cnt
        for j, (Pp, T, _) in enumerate(specs):
            d = refs[j]
            if used[j] > d.size:
                d = oracle.distances(oracle.make_model(Pp, T), obs_l[j], seed=9, n=int(used[j]),
                                     series=j)
            _agree_first(d, eps[j], idx[j], oracle.first_accepted(d, eps[j], quota))
        np.testing.assert_array_equal(idx[3], np.arange(quota))


def test_batch_single_series_equals_plain_path(env):
    abc, P = env
    s = W.uneven_series(64, 5)[7]
    ser = P.observed_series(s)
    eps = P.pilot_eps(ser, 9, n=20000, q=5e-3, series=0)
    out = abc.batch_run([ser], [eps], 9, 60, round_size=1 << 15)
    used = int(out["used"][0].item())
    run = P.PlainABC(ser, 9, eps, used, series=0, capacity=1 << 14)
    res = run.run(0)
    plain = res.idx[:res.n()].cpu().numpy()[:60]
    np.testing.assert_array_equal(out["idx"][0].cpu().numpy(), plain)


def test_batch_one_series_large_rounds_stay_within_capacity(env):
    """One series, rounds of 2^22 samples and a candidate capacity of three
    times the quota: the first round is short (nothing is known of the rate
    yet), and the rounds sized from its few candidates must not overrun the
    capacity on seeds where those undercount the rate. Every seed completes,
    and the accepted set does not depend on the round size."""
    abc, P = env
    s = W.uneven_series(64, 5)[13]
    ser = P.observed_series(s)
    eps = P.pilot_eps(ser, 9, n=100_000, q=2e-3, series=0)
    quota = 1024
    failed = []
    for seed in range(100, 300):
        try:
            out = abc.batch_run([ser], [eps], seed, quota, round_size=1 << 22, cand_capacity=3 * quota)
        except abc.AbcError as e:
            failed.append((seed, str(e)))
            continue
        assert int(out["count"][0]) == quota
        if seed < 103:
            small = abc.batch_run([ser], [eps], seed, quota, round_size=1 << 16, cand_capacity=3 * quota)
            assert torch.equal(small["idx"], out["idx"]) and torch.equal(small["count"], out["count"])
    assert not failed, failed[:3]


def test_batch_series_count_limit(env):
    """256 series (the most one batch takes; short ones, since every series'
    observations sit in LDS at once) and 257 rejected."""
    abc, P = env
    obs = oracle.observe(oracle.make_model(1_000_000, 20), W.THETA_ITALY, 32)
    ser = abc.DeviceSeries(1_000_000, 20, torch.from_numpy(obs))
    eps = P.pilot_eps(ser, 9, n=20000, q=2e-2, series=0)
    m = 256
    out = abc.batch_run([ser] * m, [eps] * m, 9, 3, round_size=1 << 16, series_ids=list(range(m)))
    assert np.all(out["count"].cpu().numpy() == 3)
    with pytest.raises(abc.AbcError):
        abc.batch_run([ser] * (m + 1), [eps] * (m + 1), 9, 3, series_ids=list(range(m + 1)))
