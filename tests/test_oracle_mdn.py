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
