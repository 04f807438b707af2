"""One launch for several series (abc_simulate_distance_multi) against one
launch per series (abc_simulate_distance): every distance bit-identical,
including +INF early exits, for the three countries at ragged sizes, the
uneven series, every model option the multi launch takes, several launch
shapes and refill thresholds, empty jobs, one job and the maximum of eight;
the sample-day counter equals the per-series counters' sum. Together with the
per-series kernel's parity against the FP64 oracle (test_gpu_core,
test_gpu_pipeline, test_gpu_fullsize) this carries the oracle's bar over."""
import math

import numpy as np
import pytest
import torch

from paper_2012_14332_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_14332_amd import abc, pipeline as P

    abc.lib()
    abc.set_launch_config(0, 0, 0)
    abc.set_refill_min(0)
    return abc, P


@pytest.fixture(scope="module")
def countries(env):
    abc, P = env
    out = []
    for c, s in enumerate(W.three_countries()):
        ser = P.observed_series(s)
        eps = P.pilot_eps(ser, 1, n=100_000, q=1e-3, series=c)
        out.append((ser, eps))
    return out


def _per_series(abc, jobs, seed, flags=0, days=None):
    return [abc.simulate_distance(j["ser"], j["n"], seed, first=j.get("first", 0),
                                  series=j.get("series", q), eps_exit=j.get("eps_exit", math.inf),
                                  flags=flags, days=days)
            for q, j in enumerate(jobs)]


def _same(a, b):
    return a.shape == b.shape and torch.equal(a, b)


def _jobs(countries, ns, firsts, w=0.02):
    return [{"ser": ser, "n": n, "first": f, "series": c, "eps_exit": eps * (1 + w)}
            for c, ((ser, eps), n, f) in enumerate(zip(countries, ns, firsts))]


@pytest.mark.parametrize("shape", [(1, 1024, 1), (1, 512, 2), (1, 1024, 2)])
def test_three_countries_bit_identical_and_days(env, countries, shape):
    """At one 1024-thread workgroup per CU the three bound tables fit at the
    per-series resolution and the sample-days match exactly; two workgroups
    per CU (the bench's two 1024-thread ones among them) get coarser time
    blocks (a weaker bound: some samples exit a few days later), never a
    different distance."""
    abc, _ = env
    jobs = _jobs(countries, [300_001, 250_037, 199_999], [100_000, 7, (1 << 32) - 1000])
    dm = torch.zeros(1, dtype=torch.int64, device="cuda")
    ds = torch.zeros(1, dtype=torch.int64, device="cuda")
    want = _per_series(abc, jobs, 1, days=ds)
    abc.set_launch_config(*shape)
    try:
        got = abc.simulate_distance_multi(jobs, 1, days=dm)
    finally:
        abc.set_launch_config(0, 0, 0)
    torch.cuda.synchronize()
    for g, w_ in zip(got, want):
        assert _same(g, w_)
        assert torch.isinf(g).any() and torch.isfinite(g).any()
    if shape == (1, 1024, 1):
        assert int(dm.item()) == int(ds.item())
    else:
        assert int(dm.item()) >= int(ds.item())


@pytest.mark.parametrize("flags", ["raw", "kahan", "literal", "no_bound", "inf"])
def test_model_options_bit_identical(env, countries, flags):
    abc, _ = env
    f = {"raw": abc.ABC_DIST_RAW, "kahan": abc.ABC_KAHAN, "literal": abc.ABC_NOISE_LITERAL,
         "no_bound": abc.ABC_NO_BOUND, "inf": 0}[flags]
    jobs = _jobs(countries, [70_001, 64 * 700, 33_333], [5, 1000, 123_456])
    if flags == "raw":
        # raw-count tolerances: the 1e-3 quantile of each series' raw distances
        for j in jobs:
            d = abc.simulate_distance(j["ser"], 20_000, 1, series=j["series"], flags=f).cpu().numpy()
            j["eps_exit"] = float(np.quantile(d, 1e-2))
    if flags == "inf":
        for j in jobs:
            j["eps_exit"] = math.inf
    got = abc.simulate_distance_multi(jobs, 1, flags=f)
    want = _per_series(abc, jobs, 1, flags=f)
    torch.cuda.synchronize()
    for g, w_ in zip(got, want):
        assert _same(g, w_)


@pytest.mark.parametrize("shape,refill", [((1, 1024, 1), 8), ((1, 512, 2), 1), ((1, 256, 4), 64),
                                          ((1, 64, 8), 16)])
def test_launch_shapes_bit_identical(env, countries, shape, refill):
    abc, _ = env
    jobs = _jobs(countries, [100_003, 90_001, 80_009], [0, 0, 0])
    want = _per_series(abc, jobs, 3)
    abc.set_launch_config(*shape)
    abc.set_refill_min(refill)
    try:
        got = abc.simulate_distance_multi(jobs, 3)
    finally:
        abc.set_launch_config(0, 0, 0)
        abc.set_refill_min(0)
    torch.cuda.synchronize()
    for g, w_ in zip(got, want):
        assert _same(g, w_)


def test_uneven_series_eight_jobs_empty_and_single(env):
    abc, P = env
    ss = W.uneven_series(8, 5)
    sers = [P.observed_series(s) for s in ss]
    eps = [P.pilot_eps(ser, 2, n=20_000, q=1e-2, series=j) for j, ser in enumerate(sers)]
    ns = [20_000 + 17 * j for j in range(8)]
    ns[3] = 0  # an empty job among the others
    jobs = [{"ser": ser, "n": n, "series": j, "first": 11 * j, "eps_exit": e * 1.02}
            for j, (ser, n, e) in enumerate(zip(sers, ns, eps))]
    got = abc.simulate_distance_multi(jobs, 2)
    want = _per_series(abc, jobs, 2)
    torch.cuda.synchronize()
    for g, w_ in zip(got, want):
        assert _same(g, w_)
    one = abc.simulate_distance_multi(jobs[:1], 2)[0]
    torch.cuda.synchronize()
    assert _same(one, want[0])


def test_short_and_long_horizons_together(env):
    """T = 1 and T = 1024 (the longest horizon) in one launch: the bound tables
    of long series get coarser time blocks, never different distances."""
    abc, P = env
    import oracle

    jobs = []
    for j, (Pp, T) in enumerate([(10**6, 1), (10**9, 1024), (5 * 10**7, 200)]):
        m = oracle.make_model(Pp, T)
        th = W.single_country().theta_true
        obs = torch.from_numpy(oracle.observe(m, th, 9, series=j)).cuda()
        ser = abc.DeviceSeries(Pp, T, obs)
        d = abc.simulate_distance(ser, 5000, 4, series=j).cpu().numpy()
        jobs.append({"ser": ser, "n": 30_001, "series": j, "eps_exit": float(np.quantile(d, 0.05))})
    got = abc.simulate_distance_multi(jobs, 4)
    want = _per_series(abc, jobs, 4)
    torch.cuda.synchronize()
    for g, w_ in zip(got, want):
        assert _same(g, w_)
