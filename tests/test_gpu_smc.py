"""ABC-SMC on the GPU against the float64 oracle (oracle/smc.py), through the
C ABI.

Bars: per generation, given the same previous population (the oracle's), the
tolerance is the same float32 value, the population's candidate indices,
ancestors and float32 parameters are identical, the float64 distances agree to
1e-12 relative and the normalised weights to 1e-10 relative (exp and the
Mahalanobis form round differently on the two sides); the sample and
in-support counts are identical. A whole run from the same seed reproduces the
oracle's generations the same way.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import smc as osmc
from paper_2012_14332_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_14332_amd import abc, pipeline as P

    abc.lib()
    s = W.single_country()
    m = oracle.make_model(s.P, s.T)
    obs = oracle.observe(m, s.theta_true, s.obs_seed)
    eps0 = oracle.pilot_eps(oracle.distances(m, obs, 1, 20000), 0.02)
    ser = P.observed_series(s)
    return abc, s, m, obs, eps0, ser


def _upload(g):
    return (torch.from_numpy(np.ascontiguousarray(g.theta)).cuda(),
            torch.from_numpy(np.ascontiguousarray(g.W)).cuda(),
            torch.from_numpy(np.ascontiguousarray(g.dist)).cuda())


def _compare(out, g, tag):
    st = out["stats"]
    assert st["eps"] == np.float32(g.eps), (tag, st["eps"], g.eps)
    np.testing.assert_array_equal(out["idx"].cpu().numpy(), g.idx, err_msg=tag)
    np.testing.assert_array_equal(out["theta"].cpu().numpy(), g.theta, err_msg=tag)
    d = out["dist"].cpu().numpy()
    assert np.max(np.abs(d - g.dist) / g.dist) <= 1e-12, tag
    w = out["w"].cpu().numpy()
    assert np.max(np.abs(w - g.W) / g.W) <= 1e-10, (tag, np.max(np.abs(w - g.W) / g.W))
    assert st["samples"] == g.samples, (tag, st["samples"], g.samples)
    assert st["in_support"] == g.in_support, (tag, st["in_support"], g.in_support)
    assert abs(st["ess"] - g.ess()) <= 1e-9 * g.ess()
    if out.get("ancestors") is not None and g.ancestors is not None:
        np.testing.assert_array_equal(out["ancestors"].cpu().numpy(), g.ancestors, err_msg=tag)


def test_support_flag_rejects_out_of_box_rows(env):
    abc, s, m, obs, eps0, ser = env
    n = 3000
    th = abc.sample_prior(n, seed=4).clone()
    bad = torch.arange(0, n, 7, device="cuda")
    th[bad, 3] = -0.01          # negative beta
    th[bad[::2], 3] = 0.5
    th[bad[::2], 1] = 100.5     # alpha above the box
    th[5, 6] = float("nan")
    outside = torch.zeros(n, dtype=torch.bool, device="cuda")
    outside[bad] = True
    outside[5] = True
    for flags in (0, abc.ABC_FP64):
        d_plain = abc.simulate_distance(ser, n, 4, theta=th, flags=flags)
        d_sup = abc.simulate_distance(ser, n, 4, theta=th, flags=flags | abc.ABC_SUPPORT)
        assert torch.all(torch.isinf(d_sup[outside]))
        assert torch.equal(d_sup[~outside], d_plain[~outside])


def test_generation_zero_is_rejection_abc(env):
    abc, s, m, obs, eps0, ser = env
    gens = osmc.smc_abc(m, obs, seed=5, N=300, generations=1, alpha=0.5, eps0=eps0)
    cfg = abc.smc_config(300, eps0, chunk0=1000, chunk_max=1 << 13)
    out = abc.smc_generation(ser, cfg, 5, 0)
    _compare(out, gens[0], "gen0")
    assert out["stats"]["proposed"] >= out["stats"]["samples"]


@pytest.mark.parametrize("N,alpha,chunk0", [(256, 0.5, 777), (100, 0.3, 1 << 14)])
def test_generations_match_oracle_stepwise(env, N, alpha, chunk0):
    """Each GPU generation from the oracle's previous population."""
    abc, s, m, obs, eps0, ser = env
    gens = osmc.smc_abc(m, obs, seed=6, N=N, generations=4, alpha=alpha, eps0=eps0)
    cfg = abc.smc_config(N, eps0, alpha=alpha, chunk0=chunk0, chunk_max=1 << 16)
    for t in range(1, len(gens)):
        out = abc.smc_generation(ser, cfg, 6, t, _upload(gens[t - 1]), want_ancestors=True)
        _compare(out, gens[t], "gen%d" % t)


@pytest.mark.parametrize("N,alpha", [(12, 1.0), (16, 0.1)])
def test_small_populations_and_extreme_quantiles(env, N, alpha):
    """Few particles (the covariance of 8 parameters needs at least 9) and
    the extreme tolerance quantiles: alpha = 1 keeps the previous generation's
    largest distance, alpha = 0.1 its second smallest of 16."""
    abc, s, m, obs, eps0, ser = env
    gens = osmc.smc_abc(m, obs, seed=8, N=N, generations=3, alpha=alpha, eps0=eps0)
    cfg = abc.smc_config(N, eps0, alpha=alpha, chunk0=1 << 12, chunk_max=1 << 16)
    for t in range(1, len(gens)):
        out = abc.smc_generation(ser, cfg, 8, t, _upload(gens[t - 1]), want_ancestors=True)
        _compare(out, gens[t], "gen%d" % t)


@pytest.mark.parametrize("alpha", [0.5, 0.37, 1.0])
def test_tolerance_quantile_with_ties(env, alpha):
    """eps_t is the ceil(alpha N)-th smallest previous distance also when many
    previous distances are equal (rounded to one decimal) and some are zero."""
    abc, s, m, obs, eps0, ser = env
    g = osmc.smc_abc(m, obs, seed=6, N=256, generations=1, alpha=0.5, eps0=eps0)[0]
    d = np.round(g.dist, 1)
    d[[3, 77, 200]] = 0.0
    assert len(np.unique(d)) < d.size // 2
    cfg = abc.smc_config(256, eps0, alpha=alpha, chunk0=1 << 14, chunk_max=1 << 16)
    prev = (torch.from_numpy(np.ascontiguousarray(g.theta)).cuda(),
            torch.from_numpy(np.ascontiguousarray(g.W)).cuda(),
            torch.from_numpy(d).cuda())
    out = abc.smc_generation(ser, cfg, 6, 1, prev)
    assert out["stats"]["eps"] == np.float32(osmc.quantile_eps(d, alpha, 0.0))


def test_full_run_matches_oracle(env):
    abc, s, m, obs, eps0, ser = env
    gens = osmc.smc_abc(m, obs, seed=8, N=200, generations=5, alpha=0.5, eps0=eps0)
    cfg = abc.smc_config(200, eps0, generations=5, chunk0=4096, chunk_max=1 << 15)
    outs = abc.smc_run(ser, cfg, 8)
    assert len(outs) == len(gens)
    for t, (o, g) in enumerate(zip(outs, gens)):
        _compare(o, g, "run gen%d" % t)


def test_eps_floor_stops_the_run(env):
    abc, s, m, obs, eps0, ser = env
    gens = osmc.smc_abc(m, obs, seed=8, N=200, generations=3, alpha=0.5, eps0=eps0)
    floor = float(gens[1].eps) * 0.999
    og = osmc.smc_abc(m, obs, seed=8, N=200, generations=8, alpha=0.5, eps0=eps0, eps_min=floor)
    cfg = abc.smc_config(200, eps0, generations=8, eps_min=floor, chunk0=4096, chunk_max=1 << 15)
    outs = abc.smc_run(ser, cfg, 8)
    assert len(outs) == len(og) < 8
    assert outs[-1]["stats"]["eps"] == np.float32(floor)
    for t, (o, g) in enumerate(zip(outs, og)):
        _compare(o, g, "floor gen%d" % t)


def test_largest_population(env):
    """N = 8192 (the maximum): generation 1 from the oracle's generation 0."""
    abc, s, m, obs, eps0, ser = env
    N = 8192
    gens = osmc.smc_abc(m, obs, seed=9, N=N, generations=2, alpha=0.5, eps0=eps0, chunk=1 << 16)
    cfg = abc.smc_config(N, eps0, chunk0=1 << 16, chunk_max=1 << 18)
    out0 = abc.smc_generation(ser, cfg, 9, 0)
    _compare(out0, gens[0], "N8192 gen0")
    out1 = abc.smc_generation(ser, cfg, 9, 1, _upload(gens[0]), want_ancestors=True)
    _compare(out1, gens[1], "N8192 gen1")


def test_errors(env):
    abc, s, m, obs, eps0, ser = env
    # a collapsed population has a singular kernel covariance
    th = abc.sample_prior(1, seed=1).repeat(50, 1).contiguous()
    w = torch.full((50,), 1.0 / 50, dtype=torch.float64, device="cuda")
    d = torch.ones(50, dtype=torch.float64, device="cuda")
    cfg = abc.smc_config(50, eps0)
    with pytest.raises(abc.AbcError, match="positive definite"):
        abc.smc_generation(ser, cfg, 1, 1, (th, w, d))
    with pytest.raises(abc.AbcError):
        abc.smc_generation(ser, abc.smc_config(8193, eps0), 1, 0)
    with pytest.raises(abc.AbcError):
        abc.smc_generation(ser, cfg, 1, 1)  # no previous population
    # candidate budget exhausted
    tight = abc.smc_config(50, 1e-3, chunk0=1024, chunk_max=1024, max_samples=4096)
    with pytest.raises(abc.AbcError, match="particles after"):
        abc.smc_generation(ser, tight, 1, 0)
