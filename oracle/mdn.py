"""Float64 numpy reference of the learned mixture-density proposal.

TEST INFRASTRUCTURE. Not part of the paper (which uses the prior as the
proposal); it follows the network the workload statement fixes: 96 inputs
(A, R, D at 32 evenly spaced days, log1p, standardised), two hidden layers of
256 with exact (erf) GELU, output an 8-component diagonal Gaussian mixture
over the standardised 8 parameters (8 logits, 8x8 means, 8x8 log standard
deviations clamped to [-7, 3]); trained by Adam on the mean negative
log-likelihood. Everything here is plain float64: a matrix product per layer,
the mixture density written out, hand-derived gradients (checked against
finite differences by the tests), Adam as published (Kingma & Ba 2015).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, logsumexp, ndtr

N_IN, N_H, K, D = 96, 256, 8, 8
N_OUT = K + 2 * K * D  # 136
LOGSIG_LO, LOGSIG_HI = -7.0, 3.0
LOG_2PI = math.log(2.0 * math.pi)

# parameter order of the flat vector: W1 [96,256], b1 [256], W2 [256,256], b2,
# W3 [256,136], b3 [136]; W stored [fan_in, fan_out] (row = input)
SHAPES = [(N_IN, N_H), (N_H,), (N_H, N_H), (N_H,), (N_H, N_OUT), (N_OUT,)]


def n_params() -> int:
    return int(sum(np.prod(s) for s in SHAPES))


def unflatten(p: np.ndarray):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    return out


def flatten(parts) -> np.ndarray:
    return np.concatenate([np.asarray(x, np.float64).ravel() for x in parts])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def split_out(out):
    """Network output rows -> (logits [n,K], mu [n,K,D], raw log sigma [n,K,D])."""
    logits = out[:, :K]
    mu = out[:, K:K + K * D].reshape(-1, K, D)
    ls = out[:, K + K * D:].reshape(-1, K, D)
    return logits, mu, ls


def forward(p, x):
    W1, b1, W2, b2, W3, b3 = unflatten(np.asarray(p, np.float64))
    z1 = x @ W1 + b1
    h1 = gelu(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu(z2)
    out = h2 @ W3 + b3
    return out, (x, z1, h1, z2, h2)


def mixture_logpdf(out, t):
    """log q(t | out) for rows of standardised parameters t [n, D]."""
    logits, mu, ls = split_out(out)
    lsc = np.clip(ls, LOGSIG_LO, LOGSIG_HI)
    logpi = logits - logsumexp(logits, axis=1, keepdims=True)
    u = (t[:, None, :] - mu) * np.exp(-lsc)
    comp = -0.5 * (u * u).sum(2) - lsc.sum(2) - 0.5 * D * LOG_2PI
    return logsumexp(logpi + comp, axis=1)


def mixture_logpdf_unclamped(out, t):
    """mixture_logpdf with the log sds taken as given (already clamped/shifted)."""
    logits, mu, ls = split_out(out)
    logpi = logits - logsumexp(logits, axis=1, keepdims=True)
    u = (t[:, None, :] - mu) * np.exp(-ls)
    comp = -0.5 * (u * u).sum(2) - ls.sum(2) - 0.5 * D * LOG_2PI
    return logsumexp(logpi + comp, axis=1)


def loss(p, x, t):
    out, _ = forward(p, x)
    return float(-mixture_logpdf(out, t).mean())


def loss_and_grad(p, x, t):
    """Mean NLL and its gradient w.r.t. the flat parameter vector."""
    W1, b1, W2, b2, W3, b3 = unflatten(np.asarray(p, np.float64))
    out, (x, z1, h1, z2, h2) = forward(p, x)
    n = x.shape[0]
    logits, mu, ls = split_out(out)
    lsc = np.clip(ls, LOGSIG_LO, LOGSIG_HI)
    inside = (ls > LOGSIG_LO) & (ls < LOGSIG_HI)
    logpi = logits - logsumexp(logits, axis=1, keepdims=True)
    sig_inv = np.exp(-lsc)
    u = (t[:, None, :] - mu) * sig_inv
    comp = -0.5 * (u * u).sum(2) - lsc.sum(2) - 0.5 * D * LOG_2PI
    L = logpi + comp
    lse = logsumexp(L, axis=1, keepdims=True)
    r = np.exp(L - lse)  # responsibilities
    pi = np.exp(logpi)
    d_logits = pi - r
    d_mu = -r[:, :, None] * u * sig_inv
    d_ls = -r[:, :, None] * (u * u - 1.0) * inside
    dout = np.concatenate([d_logits, d_mu.reshape(n, -1), d_ls.reshape(n, -1)], axis=1) / n
    gW3 = h2.T @ dout
    gb3 = dout.sum(0)
    dz2 = (dout @ W3.T) * gelu_grad(z2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * gelu_grad(z1)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(0)
    return float(-lse.mean()), flatten([gW1, gb1, gW2, gb2, gW3, gb3]), dout


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def subsample_days(T: int) -> np.ndarray:
    """The 32 feature days of a T-day series: d_k = 1 + round(k (T-1) / 31)
    (ties to even), k = 0..31; days repeat when T < 32."""
    k = np.arange(32, dtype=np.float64)
    return (1 + np.rint(k * (T - 1) / 31.0)).astype(np.int64)


def features_from_traj(traj, T):
    """Raw features [n, 96] = log1p(A, R, D) at the 32 subsampled days from
    trajectories [n, T+1, 6] (day 0 first)."""
    d = subsample_days(T)
    tr = np.asarray(traj, np.float64)
    return np.concatenate([np.log1p(tr[:, d, 2]), np.log1p(tr[:, d, 3]),
                           np.log1p(tr[:, d, 4])], axis=1)


def theta_standardise(theta, lo, hi):
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    c = (lo + hi) / 2
    s = (hi - lo) / math.sqrt(12.0)
    return (np.asarray(theta, np.float64) - c) / s


def mixture_sample(out_row, n, rng):
    """n draws (standardised) from the mixture of one output row."""
    logits, mu, ls = split_out(np.asarray(out_row, np.float64)[None])
    pi = np.exp(logits[0] - logsumexp(logits[0]))
    k = rng.choice(K, size=n, p=pi)
    sig = np.exp(np.clip(ls[0], LOGSIG_LO, LOGSIG_HI))
    return mu[0][k] + sig[k] * rng.standard_normal((n, D))


def truncated_masses(out_row, lo, hi, inflate=1.0):
    """Z [K, D]: the mass of component k's normal in dimension j (sd times
    `inflate`, standardised units) inside the box, computed on the side of the
    tail it lies in."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    c = (lo + hi) / 2
    s = (hi - lo) / math.sqrt(12.0)
    _, mu, ls = split_out(np.asarray(out_row, np.float64)[None])
    sig = np.exp(np.clip(ls[0], LOGSIG_LO, LOGSIG_HI) + math.log(inflate))
    a = (lo - c) / s
    b = (hi - c) / s
    al = (a[None, :] - mu[0]) / sig
    be = (b[None, :] - mu[0]) / sig
    upper = al >= 0
    lower = be <= 0
    Z = ndtr(be) - ndtr(al)
    Z = np.where(upper, ndtr(-al) - ndtr(-be), Z)
    Z = np.where(lower, ndtr(be) - ndtr(al), Z)
    return Z


def truncated_logq(out_row, theta, lo, hi, inflate=1.0):
    """log density (original units) of the mixture with every component
    truncated to the box dimension by dimension: component weights
    renormalised over the components whose masses are all >= 1e-30,
    log q = logsumexp_k [log w_k - sum_j log Z_kj + sum_j log N(t_j; mu_kj, sig_kj)]
            - sum_j log s_j."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    s = (hi - lo) / math.sqrt(12.0)
    t = theta_standardise(theta, lo, hi)
    logits, mu, ls = split_out(np.asarray(out_row, np.float64)[None])
    lsig = np.clip(ls[0], LOGSIG_LO, LOGSIG_HI) + math.log(inflate)
    Z = truncated_masses(out_row, lo, hi, inflate)
    keep = np.all(Z >= 1e-30, axis=1)
    lw = np.where(keep, logits[0], -np.inf)
    lw = lw - logsumexp(lw)
    u = (t[:, None, :] - mu[0][None]) / np.exp(lsig)[None]
    comp = (-0.5 * u * u - lsig[None] - 0.5 * LOG_2PI).sum(2) - np.log(np.where(keep, Z, 1.0)).sum(1)[None]
    return logsumexp(lw[None] + comp, axis=1) - np.log(s).sum()


def defensive_logq(out_row, theta, lo, hi, lam, inflate=1.0):
    """log of the defensive proposal density at theta (original units):
    (1 - lam) * truncated mixture (component sds times `inflate`) + lam * prior;
    the prior alone when every component is dropped."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    lq_prior = -np.log(hi - lo).sum()
    if not np.any(np.all(truncated_masses(out_row, lo, hi, inflate) >= 1e-30, axis=1)):
        # no component has mass in the box: the proposal is the prior
        return np.full(np.asarray(theta).reshape(-1, 8).shape[0], lq_prior)
    lq_mix = truncated_logq(out_row, theta, lo, hi, inflate)
    return np.logaddexp(np.log1p(-lam) + lq_mix, np.log(lam) + lq_prior) if lam > 0 else lq_mix
