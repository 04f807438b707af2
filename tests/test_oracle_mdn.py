"""Pins of the float64 mixture-density reference: its hand-derived gradient
against central finite differences, the mixture density's normalisation,
the loss as the negative log density of a known single Gaussian, and Adam
against a hand-worked first step."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import mdn


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for s in mdn.SHAPES:
        fan_in = s[0] if len(s) == 2 else 1
        parts.append(rng.uniform(-1, 1, size=s) * scale / math.sqrt(fan_in))
    return mdn.flatten(parts)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = _params(1)
    x = rng.standard_normal((6, mdn.N_IN))
    t = rng.standard_normal((6, mdn.D))
    _, g, _ = mdn.loss_and_grad(p, x, t)
    idx = rng.choice(p.size, size=60, replace=False)
    # include the output-layer bias entries of every block
    idx = np.concatenate([idx, p.size - np.array([1, 5, 70, 130, 136])])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mdn.loss(p + e, x, t) - mdn.loss(p - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_clamped_log_sigma_has_zero_gradient():
    rng = np.random.default_rng(2)
    p = _params(3)
    W1, b1, W2, b2, W3, b3 = mdn.unflatten(p)
    b3[mdn.K + mdn.K * mdn.D:] = 10.0  # every log sigma above the clamp
    x = rng.standard_normal((4, mdn.N_IN))
    t = rng.standard_normal((4, mdn.D))
    _, g, dout = mdn.loss_and_grad(p, x, t)
    assert np.all(dout[:, mdn.K + mdn.K * mdn.D:] == 0)


def test_mixture_density_integrates_to_one():
    rng = np.random.default_rng(4)
    out = rng.standard_normal(mdn.N_OUT) * 0.5
    # importance sampling from a broad Gaussian: E_g[q / g] = 1
    n = 400_000
    z = rng.standard_normal((n, mdn.D)) * 3.0
    logg = stats.norm.logpdf(z, scale=3.0).sum(1)
    logq = mdn.mixture_logpdf(np.repeat(out[None], n, 0), z)
    est = np.exp(logq - logg).mean()
    assert abs(est - 1.0) < 0.03, est


def test_single_component_reduces_to_gaussian():
    # one dominant component: the loss is the negative log of a diagonal normal
    out = np.zeros(mdn.N_OUT)
    out[0] = 50.0
    mu = np.linspace(-1, 1, mdn.D)
    ls = np.linspace(-0.5, 0.5, mdn.D)
    out[mdn.K:mdn.K + mdn.D] = mu
    out[mdn.K + mdn.K * mdn.D:mdn.K + mdn.K * mdn.D + mdn.D] = ls
    t = np.array([[0.3] * mdn.D])
    ref = stats.norm.logpdf(t[0], loc=mu, scale=np.exp(ls)).sum()
    assert math.isclose(mdn.mixture_logpdf(out[None], t)[0], ref, rel_tol=1e-12)


def test_mixture_sampler_moments():
    rng = np.random.default_rng(5)
    out = rng.standard_normal(mdn.N_OUT) * 0.4
    s = mdn.mixture_sample(out, 200_000, rng)
    logits, mu, ls = mdn.split_out(out[None])
    pi = np.exp(logits[0] - logits[0].max())
    pi /= pi.sum()
    m = (pi[:, None] * mu[0]).sum(0)
    assert np.allclose(s.mean(0), m, atol=0.02)


def test_adam_first_step_moves_by_lr():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    p1, m, v = mdn.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # bias-corrected first step is lr * sign(g) (eps negligible), 0 for g = 0
    np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), atol=1e-9)


def test_subsample_days():
    d = mdn.subsample_days(49)
    assert d[0] == 1 and d[-1] == 49 and len(d) == 32 and np.all(np.diff(d) >= 1)
    d = mdn.subsample_days(30)
    assert d[0] == 1 and d[-1] == 30 and np.all(np.diff(d) >= 0)
    assert mdn.subsample_days(200)[-1] == 200


LO = np.zeros(8)
HI = np.array([1, 100, 2, 1, 1, 1, 1, 2], dtype=np.float64)


def _row(seed, spread=0.5, shift=0.0):
    rng = np.random.default_rng(seed)
    out = rng.standard_normal(mdn.N_OUT) * spread
    out[mdn.K:mdn.K + mdn.K * mdn.D] += shift
    return out


@pytest.mark.parametrize("inflate,shift", [(1.0, 0.0), (3.0, 0.0), (1.5, 2.5)])
def test_truncated_proposal_integrates_to_one_on_the_box(inflate, shift):
    # E over uniform theta in the box of q(theta) * volume = integral of q = 1
    out = _row(5, shift=shift)
    rng = np.random.default_rng(6)
    n = 400_000
    th = LO + (HI - LO) * rng.random((n, 8))
    lq = mdn.truncated_logq(out, th, LO, HI, inflate)
    est = np.exp(lq + np.log(HI - LO).sum()).mean()
    se = np.exp(lq + np.log(HI - LO).sum()).std() / math.sqrt(n)
    assert abs(est - 1.0) < max(5 * se, 0.01), (est, se)
    # and the defensive mixture too
    lqd = mdn.defensive_logq(out, th, LO, HI, 0.3, inflate)
    assert abs(np.exp(lqd + np.log(HI - LO).sum()).mean() - 1.0) < max(5 * se, 0.01)


def test_truncated_proposal_single_component_is_scipy_truncnorm():
    out = np.zeros(mdn.N_OUT)
    out[0] = 60.0  # one component
    mu = np.linspace(-2.5, 2.5, mdn.D)      # some means outside the box in standardised units
    ls = np.linspace(-1.0, 0.8, mdn.D)
    out[mdn.K:mdn.K + mdn.D] = mu
    out[mdn.K + mdn.K * mdn.D:mdn.K + mdn.K * mdn.D + mdn.D] = ls
    s = (HI - LO) / math.sqrt(12.0)
    c = (LO + HI) / 2
    rng = np.random.default_rng(1)
    th = LO + (HI - LO) * rng.random((50, 8))
    got = mdn.truncated_logq(out, th, LO, HI, 1.7)
    sig = np.exp(ls + math.log(1.7))
    a = ((LO - c) / s - mu) / sig
    b = ((HI - c) / s - mu) / sig
    t = (th - c) / s
    ref = stats.truncnorm.logpdf(t, a, b, loc=mu, scale=sig).sum(1) - np.log(s).sum()
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_truncated_proposal_without_truncation_is_the_mixture():
    # components far inside a huge box: every mass is 1 and nothing changes
    out = _row(7, spread=0.2)
    out[mdn.K + mdn.K * mdn.D:] = -4.0  # narrow components
    lo, hi = -1e4 * np.ones(8), 1e4 * np.ones(8)
    s = (hi - lo) / math.sqrt(12.0)
    rng = np.random.default_rng(2)
    t = rng.standard_normal((20, 8)) * 0.05
    th = (lo + hi) / 2 + s * t
    got = mdn.truncated_logq(out, th, lo, hi, 1.0)
    ref = mdn.mixture_logpdf(np.repeat(out[None], 20, 0), t) - np.log(s).sum()
    np.testing.assert_allclose(got, ref, rtol=1e-12)


def test_proposal_with_no_mass_in_the_box_is_the_prior():
    out = np.zeros(mdn.N_OUT)
    out[mdn.K:mdn.K + mdn.K * mdn.D] = 60.0     # every mean far above the box
    out[mdn.K + mdn.K * mdn.D:] = -5.0          # narrow components
    Z = mdn.truncated_masses(out, LO, HI, 1.0)
    assert np.all(Z < 1e-30)
    th = LO + (HI - LO) * np.random.default_rng(3).random((5, 8))
    np.testing.assert_allclose(mdn.defensive_logq(out, th, LO, HI, 0.3), -np.log(HI - LO).sum())
