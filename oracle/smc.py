"""Float64 reference of ABC-SMC (population Monte Carlo ABC).

TEST INFRASTRUCTURE. Only the test suite and the benchmark's CPU-baseline leg
may import this module; it shares nothing with the HIP implementation.

The paper names sequential Monte Carlo ABC (Sec. 2.2: a population refined
over a decreasing sequence of tolerances) as the refinement of rejection ABC,
without fixing an algorithm. This follows population Monte Carlo ABC
(Beaumont, Cornuet, Marin & Robert, Biometrika 2009), with the tolerance of
each generation set adaptively to a quantile of the previous generation's
distances (Del Moral, Doucet & Jasra, Stat. Comput. 2012; Drovandi & Pettitt,
Biometrics 2011):

  generation 0   rejection ABC from the prior at eps_0 (Sec. 2.2, eq. 7):
                 the first N accepted samples of the plain ABC stream, equal
                 weights.
  generation t   eps_t = max(eps_min, the ceil(alpha N)-th smallest float64
                 distance of generation t-1), rounded to float32;
                 Sigma_t = 2 x the weighted covariance of generation t-1;
                 candidate i: ancestor j drawn with probability W_j, theta* =
                 theta_j + L z (L L^T = Sigma_t, z standard normal), rounded to
                 float32; a candidate outside the prior box has prior density
                 zero and is rejected without simulation; otherwise it is
                 simulated and accepted iff its distance <= eps_t; the
                 population is the first N accepted candidates by index;
                 weights w_i = prior(theta_i) / sum_j W_j K(theta_i | theta_j)
                 with K the N(theta_j, Sigma_t) density, normalised. The prior
                 is uniform, so its density and the Gaussian normaliser are
                 common factors and drop out.

Everything is written out in plain float64 loops in the order stated in the
docstrings (means, covariances, the Cholesky factor, cumulative weights), so
that a reader can check each step.

Random numbers (Philox4x32-10, the counter layout of the rest of the oracle):
generation t >= 1 uses domain 7 and the series word series | (t << 16); on
that stream candidate i takes its proposal words from day 0, blocks 0..2, and
its simulation noise from days 1..T.
  ancestor uniform  u = (w0 * 2^21 + (w1 >> 11)) * 2^-53   (block 0, words 0, 1)
  normal pairs      (a, b) -> r = sqrt(-2 log((a + 1) 2^-32)), phi = 2 pi (b 2^-32),
                    (r cos phi, r sin phi)  [Box & Muller 1958]
                    pairs: block 0 words (2, 3), block 1 (0, 1), block 1 (2, 3),
                    block 2 (0, 1) -> z0..z7
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import DOMAIN_ABC, PRIOR_HI, PRIOR_LO, distances, philox, prior

DOMAIN_SMC = 7
TWO_PI = 2.0 * math.pi


def stream_series(series: int, gen: int) -> int:
    """Series word of generation `gen` >= 1 on the SMC stream."""
    return int(series) | (int(gen) << 16)


def _words(seed, domain, series, first, n, day, block):
    i = np.arange(first, first + n, dtype=np.uint64)
    ctr = np.empty((n, 4), dtype=np.uint32)
    ctr[:, 0] = (i & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    ctr[:, 1] = (i >> np.uint64(32)).astype(np.uint32)
    ctr[:, 2] = np.uint32(series)
    ctr[:, 3] = np.uint32((day << 8) | (domain << 4) | block)
    key = np.empty((n, 2), dtype=np.uint32)
    key[:, 0] = np.uint32(seed & 0xFFFFFFFF)
    key[:, 1] = np.uint32(seed >> 32)
    return philox(ctr, key).astype(np.uint64)


def proposal_draws(seed, series, gen, first, n):
    """(u [n] ancestor uniforms in [0, 1), z [n, 8] standard normals) of
    candidates first..first+n-1 of generation `gen`."""
    ss = stream_series(series, gen)
    b0 = _words(seed, DOMAIN_SMC, ss, first, n, 0, 0)
    b1 = _words(seed, DOMAIN_SMC, ss, first, n, 0, 1)
    b2 = _words(seed, DOMAIN_SMC, ss, first, n, 0, 2)
    u = ((b0[:, 0] << np.uint64(21)) | (b0[:, 1] >> np.uint64(11))).astype(np.float64) * 2.0 ** -53
    pairs = [(b0[:, 2], b0[:, 3]), (b1[:, 0], b1[:, 1]), (b1[:, 2], b1[:, 3]), (b2[:, 0], b2[:, 1])]
    z = np.empty((n, 8), dtype=np.float64)
    for p, (a, b) in enumerate(pairs):
        u1 = (a.astype(np.float64) + 1.0) * 2.0 ** -32
        r = np.sqrt(-2.0 * np.log(u1))
        phi = TWO_PI * (b.astype(np.float64) * 2.0 ** -32)
        z[:, 2 * p] = r * np.cos(phi)
        z[:, 2 * p + 1] = r * np.sin(phi)
    return u, z


def weighted_mean_cov(theta, W):
    """Weighted mean and covariance, sums over particles j = 0..N-1 in order:
    V = sum W_j;  m_a = (sum W_j theta_ja) / V;
    c_ab = (sum W_j ((theta_ja - m_a)(theta_jb - m_b))) / V."""
    th = np.asarray(theta, dtype=np.float64)
    W = [float(x) for x in W]
    N = th.shape[0]
    V = 0.0
    for j in range(N):
        V = V + W[j]
    m = [0.0] * 8
    for a in range(8):
        s = 0.0
        for j in range(N):
            s = s + W[j] * float(th[j, a])
        m[a] = s / V
    C = np.zeros((8, 8))
    for a in range(8):
        for b in range(a + 1):
            s = 0.0
            for j in range(N):
                s = s + W[j] * ((float(th[j, a]) - m[a]) * (float(th[j, b]) - m[b]))
            C[a, b] = C[b, a] = s / V
    return np.array(m), C


def cholesky(S):
    """Lower-triangular L with L L^T = S (Cholesky-Banachiewicz, row by row;
    within an entry the products L_ik L_jk are subtracted for k = 0, 1, ...).
    Raises ValueError when S is not positive definite."""
    n = S.shape[0]
    L = [[0.0] * n for _ in range(n)]
    for i in range(n):
        for j in range(i + 1):
            s = float(S[i, j])
            for k in range(j):
                s = s - L[i][k] * L[j][k]
            if i == j:
                if not s > 0.0:
                    raise ValueError("kernel covariance not positive definite")
                L[i][i] = math.sqrt(s)
            else:
                L[i][j] = s / L[j][j]
    return np.array(L)


def cumulative(W):
    """Running sums C_j = W_0 + ... + W_j, left to right."""
    out = np.empty(len(W))
    s = 0.0
    for j, x in enumerate(W):
        s = s + float(x)
        out[j] = s
    return out


def perturb(theta_prev, C, L, u, z):
    """Ancestor j = smallest index with C_j > u C_{N-1} (the last index if the
    product rounds up to C_{N-1}); theta* = theta_j + L z with, per row r,
    acc = theta_jr, then acc += L_rk z_k for k = 0..r; rounded to float32."""
    N = len(C)
    anc = np.searchsorted(C, u * C[-1], side="right")
    anc = np.minimum(anc, N - 1)
    base = np.asarray(theta_prev, dtype=np.float64)[anc]
    out = np.empty_like(base)
    for r in range(8):
        acc = base[:, r].copy()
        for k in range(r + 1):
            acc = acc + L[r, k] * z[:, k]
        out[:, r] = acc
    return anc, out.astype(np.float32)


def in_box(theta, lo=PRIOR_LO, hi=PRIOR_HI):
    th = np.asarray(theta, dtype=np.float32)
    return np.all((th >= lo) & (th <= hi), axis=1)


def kernel_weights(theta_new, theta_prev, W_prev, Sigma):
    """Unnormalised importance weights 1 / sum_j W_j exp(-q_ij / 2), q_ij the
    squared Mahalanobis distance (theta_i - theta_j)^T Sigma^-1 (theta_i - theta_j)."""
    tn = np.asarray(theta_new, dtype=np.float64)
    tp = np.asarray(theta_prev, dtype=np.float64)
    Wp = np.asarray(W_prev, dtype=np.float64)
    out = np.empty(tn.shape[0])
    for i in range(tn.shape[0]):
        d = tn[i][None, :] - tp
        q = np.einsum("jk,jk->j", d, np.linalg.solve(Sigma, d.T).T)
        out[i] = 1.0 / np.sum(Wp * np.exp(-0.5 * q))
    return out


def normalise(w):
    """W_j = w_j / (w_0 + ... + w_{N-1}), the sum taken left to right."""
    s = cumulative(w)[-1]
    return np.asarray(w, dtype=np.float64) / s


def quantile_eps(dist, alpha, eps_min):
    """max(eps_min, the ceil(alpha N)-th smallest distance), rounded to float32."""
    d = np.sort(np.asarray(dist, dtype=np.float64))
    k = max(1, int(math.ceil(alpha * d.size)))
    return float(np.float32(max(float(d[k - 1]), float(np.float32(eps_min)))))


@dataclasses.dataclass
class Generation:
    eps: float            # float32 value
    idx: np.ndarray       # [N] candidate indices (first N accepted)
    theta: np.ndarray     # [N, 8] float32
    W: np.ndarray         # [N] normalised weights
    dist: np.ndarray      # [N] float64 distances
    samples: int          # candidates consumed: idx[-1] + 1
    in_support: int       # candidates among them inside the prior box
    ancestors: np.ndarray | None = None
    Sigma: np.ndarray | None = None

    def ess(self) -> float:
        return float(1.0 / np.sum(self.W * self.W))


def smc_abc(model, obs, seed, N, generations, alpha, eps0, eps_min=0.0, series=0,
            chunk=1 << 14, max_samples=1 << 26, lo=PRIOR_LO, hi=PRIOR_HI):
    """Population Monte Carlo ABC as stated in the module docstring. Returns the
    list of generations (stops early after a generation at eps_min)."""
    gens = []
    # generation 0: plain rejection ABC on the ABC stream
    eps = float(np.float32(eps0))
    idx, dd = [], []
    first = 0
    while len(idx) < N:
        if first >= max_samples:
            raise RuntimeError("generation 0: quota not reached")
        d = distances(model, obs, seed, chunk, first=first, series=series, domain=DOMAIN_ABC,
                      lo=lo, hi=hi)
        acc = np.nonzero(d <= eps)[0]
        idx.extend((acc + first).tolist())
        dd.extend(d[acc].tolist())
        first += chunk
    idx = np.array(idx[:N], dtype=np.int64)
    th = np.concatenate([prior(1, seed, DOMAIN_ABC, series, int(i), lo, hi) for i in idx])
    W = normalise(np.ones(N))
    gens.append(Generation(eps, idx, th, W, np.array(dd[:N]), int(idx[-1]) + 1,
                           int(idx[-1]) + 1))
    for t in range(1, generations):
        prev = gens[-1]
        if eps_min > 0 and prev.eps <= float(np.float32(eps_min)):
            break
        eps = quantile_eps(prev.dist, alpha, eps_min)
        _, cov = weighted_mean_cov(prev.theta, prev.W)
        Sigma = 2.0 * cov
        L = cholesky(Sigma)
        C = cumulative(prev.W)
        ss = stream_series(series, t)
        idx, th, dd, anc_all = [], [], [], []
        first = 0
        valid_total = 0
        while len(idx) < N:
            if first >= max_samples:
                raise RuntimeError("generation %d: quota not reached" % t)
            u, z = proposal_draws(seed, series, t, first, chunk)
            anc, cand = perturb(prev.theta, C, L, u, z)
            ok = in_box(cand, lo, hi)
            d = distances(model, obs, seed, chunk, first=first, series=ss, theta=cand,
                          domain=DOMAIN_SMC, lo=lo, hi=hi)
            d[~ok] = np.inf
            acc = np.nonzero(d <= eps)[0]
            need = N - len(idx)
            take = acc[:need]
            idx.extend((take + first).tolist())
            th.append(cand[take])
            dd.extend(d[take].tolist())
            anc_all.extend(anc[take].tolist())
            last = int(take[-1]) + first if take.size else None
            if len(idx) == N:
                valid_total += int(ok[:last - first + 1].sum())
            else:
                valid_total += int(ok.sum())
            first += chunk
        idx = np.array(idx, dtype=np.int64)
        th = np.concatenate(th).astype(np.float32)
        w = kernel_weights(th, prev.theta, prev.W, Sigma)
        gens.append(Generation(eps, idx, th, normalise(w), np.array(dd), int(idx[-1]) + 1,
                               valid_total, np.array(anc_all), Sigma))
    return gens
