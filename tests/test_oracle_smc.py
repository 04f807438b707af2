"""Pins of the ABC-SMC oracle (oracle/smc.py) against library routines,
closed forms and statistical identities, independent of the oracle's own
formulas."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import smc
from paper_2012_14332_amd import workloads as W


def test_proposal_draws_are_uniform_and_standard_normal():
    u, z = smc.proposal_draws(seed=5, series=2, gen=3, first=1000, n=200_000)
    assert np.all((u >= 0) & (u < 1))
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    for k in range(8):
        assert stats.kstest(z[:, k], "norm").pvalue > 1e-3, k
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(8))) < 0.02
    # disjoint streams: other generation / series / seed give other numbers
    u2, _ = smc.proposal_draws(seed=5, series=2, gen=4, first=1000, n=1000)
    u3, _ = smc.proposal_draws(seed=5, series=3, gen=3, first=1000, n=1000)
    assert not np.any(u2 == u[:1000]) and not np.any(u3 == u[:1000])


def test_ancestor_uses_53_bits():
    # u takes distinct values below 2^-32 spacing: more than 32 bits enter it
    u, _ = smc.proposal_draws(seed=1, series=0, gen=1, first=0, n=1000)
    frac = (u * 2.0 ** 32) % 1.0
    assert np.mean(frac != 0.0) > 0.99


def test_cholesky_matches_lapack_and_rejects_indefinite():
    rng = np.random.default_rng(0)
    for _ in range(5):
        A = rng.standard_normal((8, 8))
        S = A @ A.T + 0.1 * np.eye(8)
        L = smc.cholesky(S)
        np.testing.assert_allclose(L, np.linalg.cholesky(S), rtol=1e-12, atol=1e-14)
        assert np.all(np.triu(L, 1) == 0)
    S = np.eye(8)
    S[3, 3] = -1.0
    with pytest.raises(ValueError):
        smc.cholesky(S)
    with pytest.raises(ValueError):
        smc.cholesky(np.zeros((8, 8)))


def test_weighted_mean_cov_matches_numpy():
    rng = np.random.default_rng(1)
    th = rng.random((300, 8)).astype(np.float32)
    Wt = rng.random(300)
    m, C = smc.weighted_mean_cov(th, Wt)
    np.testing.assert_allclose(m, np.average(th.astype(np.float64), axis=0, weights=Wt), rtol=1e-13)
    np.testing.assert_allclose(C, np.cov(th.astype(np.float64).T, aweights=Wt, bias=True),
                               rtol=1e-11, atol=1e-15)


def test_cumulative_and_normalise():
    w = np.random.default_rng(2).random(1000)
    np.testing.assert_array_equal(smc.cumulative(w), np.cumsum(w))
    Wn = smc.normalise(w)
    assert abs(Wn.sum() - 1.0) < 1e-12


def test_perturb_ancestor_frequencies_and_kernel_covariance():
    rng = np.random.default_rng(3)
    Np = 20
    prev = rng.random((Np, 8)).astype(np.float32)
    Wp = smc.normalise(rng.random(Np) ** 2)
    S = np.diag(rng.random(8) + 0.1)
    S[0, 1] = S[1, 0] = 0.05
    L = smc.cholesky(S)
    u, z = smc.proposal_draws(7, 0, 1, 0, 200_000)
    anc, cand = smc.perturb(prev, smc.cumulative(Wp), L, u, z)
    counts = np.bincount(anc, minlength=Np)
    chi = stats.chisquare(counts, Wp * anc.size)
    assert chi.pvalue > 1e-3
    # theta* - theta_anc ~ N(0, S) (up to float32 rounding)
    d = cand.astype(np.float64) - prev[anc].astype(np.float64)
    np.testing.assert_allclose(np.cov(d.T), S, atol=0.02)
    assert np.max(np.abs(d.mean(0))) < 0.01


def test_perturb_zero_weight_particles_never_drawn_and_top_edge():
    prev = np.arange(16, dtype=np.float32).reshape(2, 8)
    Wp = np.array([0.0, 1.0])
    L = np.eye(8) * 1e-3
    u = np.array([0.0, 0.5, 1.0 - 2.0 ** -53])
    anc, _ = smc.perturb(prev, smc.cumulative(Wp), L, u, np.zeros((3, 8)))
    assert list(anc) == [1, 1, 1]


def test_kernel_weights_match_scipy_mixture_density():
    rng = np.random.default_rng(4)
    prev = rng.random((15, 8))
    Wp = smc.normalise(rng.random(15))
    A = rng.standard_normal((8, 8)) * 0.2
    S = A @ A.T + 0.05 * np.eye(8)
    new = rng.random((40, 8))
    w = smc.kernel_weights(new, prev, Wp, S)
    q = np.array([sum(Wp[j] * stats.multivariate_normal(prev[j], S).pdf(x) for j in range(15))
                  for x in new])
    ratio = w * q  # = Gaussian normaliser, the same for every row
    np.testing.assert_allclose(ratio / ratio[0], np.ones(40), rtol=1e-10)
    norm = (2 * math.pi) ** -4 / math.sqrt(np.linalg.det(S))
    np.testing.assert_allclose(ratio, norm, rtol=1e-10)


def test_importance_weights_recover_the_prior_at_infinite_tolerance():
    """With eps = inf every in-box candidate is accepted: the weighted
    population must represent the uniform prior, whatever the previous one."""
    rng = np.random.default_rng(5)
    lo, hi = np.zeros(8), np.ones(8)
    Np = 200
    prev = rng.random((Np, 8))
    prev[:, :2] = rng.beta(2.0, 4.0, size=(Np, 2))  # two coordinates skewed low
    prev = prev.astype(np.float32)
    Wp = smc.normalise(np.ones(Np))
    _, cov = smc.weighted_mean_cov(prev, Wp)
    S = 2.0 * cov
    L = smc.cholesky(S)
    u, z = smc.proposal_draws(9, 0, 1, 0, 60_000)
    _, cand = smc.perturb(prev, smc.cumulative(Wp), L, u, z)
    ok = smc.in_box(cand, lo.astype(np.float32), hi.astype(np.float32))
    th = cand[ok].astype(np.float64)
    w = smc.kernel_weights(th, prev, Wp, S)
    Wn = smc.normalise(w)
    ess = 1.0 / np.sum(Wn ** 2)
    est = (Wn[:, None] * th).sum(0)
    se = math.sqrt(1.0 / 12.0) / math.sqrt(ess)
    assert ess > 1000
    assert np.all(np.abs(est - 0.5) < 4.5 * se), (est, se)
    # the unweighted candidates are far from uniform: the weights do the work
    assert np.all(np.abs(th.mean(0)[:2] - 0.5) > 8 * se)
    var = (Wn[:, None] * (th - est) ** 2).sum(0)
    assert np.all(np.abs(var - 1.0 / 12.0) < 0.1 / 12.0), var
    # a kernel width that differs from the proposal's biases the estimate
    w_bad = smc.normalise(smc.kernel_weights(th, prev, Wp, S / 2))
    assert np.max(np.abs((w_bad[:, None] * th).sum(0) - 0.5)) > 8 * se


def test_quantile_eps_order_statistic():
    d = np.array([5.0, 1.0, 3.0, 2.0, 4.0])
    assert smc.quantile_eps(d, 0.5, 0.0) == 3.0      # ceil(2.5) = 3rd smallest
    assert smc.quantile_eps(d, 0.2, 0.0) == 1.0
    assert smc.quantile_eps(d, 0.21, 0.0) == 2.0
    assert smc.quantile_eps(d, 0.5, 3.5) == 3.5      # floor at eps_min
    assert smc.quantile_eps(np.array([0.1]), 0.5, 0.0) == float(np.float32(0.1))


@pytest.fixture(scope="module")
def country():
    s = W.single_country()
    m = oracle.make_model(s.P, s.T)
    obs = oracle.observe(m, s.theta_true, s.obs_seed)
    eps0 = oracle.pilot_eps(oracle.distances(m, obs, 1, 20000), 0.02)
    return m, obs, eps0


def test_smc_invariants(country):
    m, obs, eps0 = country
    gens = smc.smc_abc(m, obs, seed=2, N=150, generations=4, alpha=0.5, eps0=eps0)
    assert len(gens) == 4
    assert gens[0].eps == float(np.float32(eps0))
    for t, g in enumerate(gens):
        assert g.idx.shape == (150,) and np.all(np.diff(g.idx) > 0)
        assert g.samples == g.idx[-1] + 1
        assert np.all(g.dist <= g.eps)
        assert np.all(smc.in_box(g.theta))
        assert abs(g.W.sum() - 1.0) < 1e-12 and np.all(g.W > 0)
        if t:
            assert g.eps == smc.quantile_eps(gens[t - 1].dist, 0.5, 0.0)
            assert g.eps <= gens[t - 1].eps
            assert g.in_support <= g.samples
    # generation 0 is plain rejection ABC: the first 150 accepted by index
    d0 = oracle.distances(m, obs, 2, int(gens[0].samples))
    np.testing.assert_array_equal(gens[0].idx, oracle.first_accepted(d0, gens[0].eps, 150))
    # the tolerance floor ends the run after the generation that reaches it
    floor = float(gens[1].eps) * 0.999
    g2 = smc.smc_abc(m, obs, seed=2, N=150, generations=6, alpha=0.3, eps0=eps0, eps_min=floor)
    assert g2[-1].eps == float(np.float32(floor)) and len(g2) < 6


def test_smc_targets_the_rejection_abc_posterior(country):
    """The weighted final population estimates the same ABC posterior as
    rejection ABC at the final tolerance (Sec. 2.2): means agree within the
    Monte Carlo error of both."""
    m, obs, eps0 = country
    gens = smc.smc_abc(m, obs, seed=3, N=500, generations=5, alpha=0.5, eps0=eps0)
    last = gens[-1]
    mean, cov = oracle.moments(last.theta, last.W)
    n = 1 << 21
    d = oracle.distances(m, obs, 11, n)
    acc = np.nonzero(d <= last.eps)[0]
    assert acc.size > 1000
    th = oracle.prior(n, 11)[acc]
    m2, c2 = oracle.moments(th)
    se = np.sqrt(np.diag(cov) / last.ess() + np.diag(c2) / acc.size)
    assert np.all(np.abs(mean - m2) < 4.5 * se), (mean - m2) / se
    # and SMC reached that tolerance with fewer simulations than rejection ABC
    sims = sum(g.in_support for g in gens)
    assert sims < n * 500 / acc.size
