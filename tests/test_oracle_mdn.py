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


# ---------------------------------------------------------------------------
# Feature extraction, parameter standardisation and Adam beyond one step.
# Each pin is computed without the function's own formula.
# ---------------------------------------------------------------------------

def _feature_days_exact(T):
    """The 32 feature days written out with exact rationals: day 1 + the
    nearest integer to k (T - 1) / 31, halves to even (Python's round on a
    Fraction), k = 0..31."""
    from fractions import Fraction

    return [1 + round(Fraction(k * (T - 1), 31)) for k in range(32)]


@pytest.mark.parametrize("T,days", [
    (32, list(range(1, 33))),            # one feature per day
    (63, [1 + 2 * k for k in range(32)]),  # every other day
    (94, [1 + 3 * k for k in range(32)]),  # every third day
])
def test_feature_days_closed_forms(T, days):
    assert mdn.subsample_days(T).tolist() == days


@pytest.mark.parametrize("T", [1, 2, 30, 31, 49, 72, 100, 200])
def test_feature_days_against_exact_rounding(T):
    assert mdn.subsample_days(T).tolist() == _feature_days_exact(T)


@pytest.mark.parametrize("T", [30, 49, 200])
def test_features_read_the_right_day_and_compartment(T):
    """A trajectory whose counts encode (day, compartment): compartment c of
    day t holds 10 t + c. Feature block b (A, R, D = compartments 2, 3, 4) at
    position k must decode to the k-th feature day and that compartment; day
    0 (the first row) and the other compartments must never be read."""
    n = 3
    traj = np.empty((n, T + 1, 6), dtype=np.int64)
    for t in range(T + 1):
        for c in range(6):
            traj[:, t, c] = 10 * t + c
    traj[:, 0, :] = -1            # day 0: log1p(-1) = -inf would show
    traj[:, :, 0] = -1            # S, I, Ru are never features
    traj[:, :, 1] = -1
    traj[:, :, 5] = -1
    f = mdn.features_from_traj(traj, T)
    assert f.shape == (n, 96)
    assert np.all(np.isfinite(f))
    code = np.rint(np.expm1(f)).astype(np.int64)  # back to the stored counts
    days = np.array(_feature_days_exact(T))
    for b, comp in enumerate((2, 3, 4)):
        np.testing.assert_array_equal(code[:, 32 * b:32 * (b + 1)], np.broadcast_to(10 * days + comp, (n, 32)))
    # log1p itself: a count of 1e9 gives log(1e9 + 1) to double precision
    traj[:, :, 2] = 10 ** 9
    f = mdn.features_from_traj(traj, T)
    assert math.isclose(f[0, 0], math.log(1e9 + 1.0), rel_tol=1e-15)


def test_theta_standardise_matches_the_uniform_closed_form():
    """Standardising by the prior's mean and sd maps U(lo, hi) to zero mean and
    unit variance: mean (lo + hi) / 2 and variance (hi - lo)^2 / 12 taken
    here from numerical integration of the uniform density, the box ends to
    -sqrt(3) and +sqrt(3), and a large uniform sample to mean 0, sd 1."""
    from scipy import integrate

    lo = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, ])
    hi = np.array([1.0, 100.0, 2.0, 1.0, 1.0, 1.0, 1.0, 2.0])
    lo2 = np.array([-3.0, 5.0, 0.25, 1e-3, -1.0, 10.0, 0.0, 0.5])
    hi2 = np.array([4.0, 6.0, 0.75, 2e-3, 1.0, 1000.0, 1e-6, 0.5 + 1e-3])
    for a_, b_ in ((lo, hi), (lo2, hi2)):
        for j in range(8):
            a, b = float(a_[j]), float(b_[j])
            dens = 1.0 / (b - a)
            m = integrate.quad(lambda x: x * dens, a, b)[0]
            v = integrate.quad(lambda x: (x - m) ** 2 * dens, a, b)[0]
            pts = np.array([[a] * 8, [b] * 8, [m] * 8, [m + math.sqrt(v)] * 8])
            t = mdn.theta_standardise(pts, a_, b_)[:, j]
            np.testing.assert_allclose(t, [-math.sqrt(3), math.sqrt(3), 0.0, 1.0], rtol=1e-9, atol=1e-9)
        rng = np.random.default_rng(11)
        u = a_ + (b_ - a_) * rng.random((400_000, 8))
        t = mdn.theta_standardise(u, a_, b_)
        # standard errors: 1/sqrt(n) for the mean, about 0.9/sqrt(n) for the sd
        assert np.all(np.abs(t.mean(0)) < 5 / math.sqrt(4e5))
        assert np.all(np.abs(t.std(0) - 1.0) < 5 / math.sqrt(4e5))


def test_adam_constant_gradient_moves_by_lr_every_step():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2 at every step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each of
    the first five steps moves every coordinate by lr * sign(g)."""
    p0 = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -4.0, 1e-3, 0.0])
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    lr = 0.01
    for step in range(1, 6):
        prev = p
        p, m, v = mdn.adam_step(p, g, m, v, step, lr=lr)
        np.testing.assert_allclose(p - prev, -lr * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8),
                                   rtol=1e-9, atol=1e-15)
        np.testing.assert_allclose(m, (1 - 0.9 ** step) * g, rtol=1e-12)
        np.testing.assert_allclose(v, (1 - 0.999 ** step) * g * g, rtol=1e-12)
    # five steps of lr sign(g), up to the eps of the denominator (1e-8 / |g|)
    np.testing.assert_allclose(p, p0 - 5 * lr * np.sign(g), atol=5 * lr * 1e-8 / 1e-3 * 1.01)


def test_adam_sign_flip_against_exact_arithmetic():
    """Two steps with gradient +g, then two with -g: the update of every step
    against the published recurrences evaluated in exact rational arithmetic
    (square roots in float64 from the exact second moment)."""
    from fractions import Fraction as F

    b1, b2, lr = F(9, 10), F(999, 1000), F(1, 100)
    gs = [F(1, 2), F(1, 2), F(-1, 2), F(-1, 2)]
    m = v = F(0)
    p_exact = F(1)
    p, mm, vv = np.array([1.0]), np.zeros(1), np.zeros(1)
    for t, g in enumerate(gs, start=1):
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p_exact -= lr * mh / F(math.sqrt(float(vh)) + 1e-8)
        p, mm, vv = mdn.adam_step(p, np.array([float(g)]), mm, vv, t, lr=float(lr))
        assert math.isclose(p[0], float(p_exact), rel_tol=1e-12), (t, p[0], float(p_exact))
    # the third step moves back by less than lr: m has not yet changed sign
    assert float(p_exact) < 1.0
