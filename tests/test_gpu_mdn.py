"""Learned mixture-density proposal on the GPU against the float64 numpy
reference (oracle/mdn.py, itself pinned by finite differences).

Bars: products run in bfloat16 with float32 accumulation, so network outputs
and gradients agree with float64 to a relative Frobenius error of a few
1e-3 (cosine >= 0.999); the loss to 1e-2 relative; importance weights to
float32 rounding of the same density; training pairs bit-exact in theta and
(T, P) and within float32-simulation error in the features.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import mdn as ref
from paper_2012_14332_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_14332_amd import abc

    abc.lib()
    return abc


def _rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for s in ref.SHAPES:
        if len(s) == 2:
            parts.append(rng.uniform(-1, 1, size=s) * scale / math.sqrt(s[0]))
        else:
            parts.append(rng.uniform(-0.1, 0.1, size=s))
    return ref.flatten(parts).astype(np.float32)


def _net_with(A, p, feats):
    net = A.Mdn(0)
    net.set_params(torch.from_numpy(p))
    net.fit_standardizer(feats)
    m, s = net.standardizer()
    x = (feats.cpu().numpy().astype(np.float64) - m.cpu().numpy()) / s.cpu().numpy()
    return net, x


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _cos(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("n", [1, 63, 333, 4096])
def test_forward_matches_reference(A, n):
    rng = np.random.default_rng(n)
    feats = torch.from_numpy(rng.uniform(0, 15, size=(max(n, 2), 96)).astype(np.float32)).cuda()
    p = _rand_params(1)
    net, x = _net_with(A, p, feats)
    out = net.forward(feats[:n]).cpu().numpy()
    want, _ = ref.forward(p.astype(np.float64), x[:n])
    assert _rel(out, want) < 1e-2, _rel(out, want)
    assert _cos(out, want) > 0.9999
    net.close()


@pytest.mark.parametrize("n", [513, 4096])
def test_loss_and_gradient_match_reference(A, n):
    rng = np.random.default_rng(7)
    feats = torch.from_numpy(rng.uniform(0, 15, size=(n, 96)).astype(np.float32)).cuda()
    theta = oracle.prior(n, seed=3)
    p = _rand_params(2)
    net, x = _net_with(A, p, feats)
    loss, g = net.loss_grad(feats, torch.from_numpy(theta).cuda())
    t = ref.theta_standardise(theta, W.PRIOR_LO, W.PRIOR_HI)
    loss_ref, g_ref, _ = ref.loss_and_grad(p.astype(np.float64), x, t)
    assert abs(float(loss.item()) - loss_ref) <= 1e-2 * abs(loss_ref) + 1e-3
    g = g.cpu().numpy()
    assert _cos(g, g_ref) > 0.999, _cos(g, g_ref)
    assert _rel(g, g_ref) < 3e-2, _rel(g, g_ref)
    # every parameter block on its own
    for part, part_ref in zip(ref.unflatten(g.astype(np.float64)), ref.unflatten(g_ref)):
        assert _cos(part, part_ref) > 0.995
    net.close()


def test_training_pairs_match_oracle(A):
    n = 600
    feats, theta, tp = A.simulate_features(n, seed=6, first=10)
    th = theta.cpu().numpy()
    np.testing.assert_array_equal(th, oracle.prior(n, seed=6, domain=2, first=10))
    tp = tp.cpu().numpy()
    f = feats.cpu().numpy()
    good = 0
    for i in range(n):
        w = oracle.stream_words(6, 2, 0, 10 + i, 0, 2)
        T = 30 + int(math.floor(((int(w[0]) >> 8) * 2.0 ** -24) * 171))
        P = int(np.rint(10 ** (5 + 4 * ((int(w[1]) >> 8) * 2.0 ** -24))))
        assert (tp[i, 0], tp[i, 1]) == (T, P)
        traj, _ = oracle.trajectory(oracle.make_model(P, T), th[i], 6, 2, 0, 10 + i)
        want = ref.features_from_traj(traj[None], T)[0]
        good += np.mean(np.abs(f[i] - want) <= 1e-3 * np.maximum(1, want)) == 1.0
    # float32 trajectories leave the float64 path at large counts; log1p
    # features move by ~1/count there
    assert good >= 0.9 * n, good


def test_training_reduces_loss(A):
    feats, theta, _ = A.simulate_features(1 << 17, seed=7)
    net = A.Mdn(1)
    net.fit_standardizer(feats)
    log, steps, ms = net.train(feats, theta, epochs=3, batch=4096, lr=1e-3, shuffle_seed=2)
    log = log.cpu().numpy()
    assert steps == 3 * 32 and np.all(np.isfinite(log))
    assert log[:4].mean() - log[-4:].mean() > 1.0, (log[:4], log[-4:])
    # the trained net's held-out loss matches its training loss level
    hf, ht, _ = A.simulate_features(4096, seed=8)
    loss, _ = net.loss_grad(hf, ht)
    assert float(loss.item()) < log[:4].mean() - 0.8
    net.close()


def _affine_perms(n, epochs, seed):
    """(a_e, c_e) of each epoch as abc_mdn_train draws them: splitmix64 from
    the shuffle seed, a_e uniform over the units mod n other than 0, c_e
    uniform mod n."""
    M = (1 << 64) - 1
    st = (seed * 0x9E3779B97F4A7C15 + 0x632BE59BD9B4E019) & M
    out = []

    def nxt():
        nonlocal st
        st = (st + 0x9E3779B97F4A7C15) & M
        z = st
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    for _ in range(epochs):
        while True:
            a = nxt() % n
            if a != 0 and math.gcd(a, n) == 1:
                break
        out.append((a, nxt() % n))
    return out


def test_training_steps_are_adam_on_each_batch(A):
    """The replayed training step against its definition: step k uses batch
    rows (a_e j + c_e) mod n, j = (k mod steps per epoch) batch + 0..batch-1, of
    epoch e = k / steps per epoch, logs that batch's loss, and makes one Adam
    update (t = k + 1) with the gradient loss_grad gives on that batch. The
    gradients are the same kernels on the same rows, so only the float32 Adam
    arithmetic may differ (contraction, powf): a wrong batch, update count or
    order moves parameters by ~lr."""
    n, batch, epochs, lr, seed = 192, 64, 2, 1e-3, 5
    feats, theta, _ = A.simulate_features(n, seed=9)
    net = A.Mdn(3)
    net.fit_standardizer(feats)
    p = net.get_params().cpu().numpy()
    log, steps, _ = net.train(feats, theta, epochs=epochs, batch=batch, lr=lr, shuffle_seed=seed)
    p_train = net.get_params().cpu().numpy()
    log = log.cpu().numpy()
    assert steps == epochs * (n // batch)
    ref_net = A.Mdn(3)
    ref_net.fit_standardizer(feats)
    b1, b2, eps, lr32 = np.float32(0.9), np.float32(0.999), np.float32(1e-8), np.float32(lr)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    spe = n // batch
    perms = _affine_perms(n, epochs, seed)
    for k in range(steps):
        a, c = perms[k // spe]
        j = (k % spe) * batch + np.arange(batch, dtype=np.int64)
        rows = torch.from_numpy((a * j + c) % n).cuda()
        ref_net.set_params(torch.from_numpy(p))
        loss, g = ref_net.loss_grad(feats[rows], theta[rows])
        loss = float(loss.item())
        assert abs(log[k] - loss) <= 1e-5 * abs(loss), (k, log[k], loss)
        g = g.cpu().numpy()
        t = k + 1
        m = b1 * m + (np.float32(1) - b1) * g
        v = b2 * v + (np.float32(1) - b2) * g * g
        mh = m / (np.float32(1) - b1 ** np.float32(t))
        vh = v / (np.float32(1) - b2 ** np.float32(t))
        p = (p - lr32 * mh / (np.sqrt(vh) + eps)).astype(np.float32)
    # a parameter whose float32 value differs by an ulp can round to another
    # bf16 copy, which moves later gradients by a bf16 ulp: a few 1e-6 at most
    err = np.abs(p_train - p)
    assert np.median(err) <= 1e-7 and err.max() <= 5e-5, (np.median(err), err.max(), int(err.argmax()))
    net.close()
    ref_net.close()


def test_sampler_weights_and_importance_identity(A):
    rng = np.random.default_rng(3)
    mix_row = (rng.standard_normal(136) * 0.4).astype(np.float32)
    mix_row[8 + 64:] -= 1.0  # narrower components
    mix = torch.from_numpy(mix_row).cuda()
    net = A.Mdn(0)
    n = 200_000
    th, w = net.sample(mix, n, seed=4, lam=0.05)
    th = th.cpu().numpy().astype(np.float64)
    w = w.cpu().numpy().astype(np.float64)
    lo, hi = W.PRIOR_LO.astype(np.float64), W.PRIOR_HI.astype(np.float64)
    assert np.all(th >= lo) and np.all(th <= hi)
    assert np.all(w > 0) and np.all(w <= 1 / 0.05 * (1 + 1e-5))
    # weights = prior / q with the reference density
    lq = ref.defensive_logq(mix_row.astype(np.float64), th[:2000], lo, hi, 0.05)
    w_ref = np.exp(-np.log(hi - lo).sum() - lq)
    np.testing.assert_allclose(w[:2000], w_ref, rtol=2e-4)
    # the same with inflated component widths
    th2, w2 = net.sample(mix, 3000, seed=5, lam=0.1, inflate=1.7)
    th2 = th2.cpu().numpy().astype(np.float64)
    lq2 = ref.defensive_logq(mix_row.astype(np.float64), th2, lo, hi, 0.1, inflate=1.7)
    np.testing.assert_allclose(w2.cpu().numpy(), np.exp(-np.log(hi - lo).sum() - lq2), rtol=2e-4)
    # self-normalised importance sampling recovers prior expectations
    est = (w[:, None] * th).sum(0) / w.sum()
    ess = w.sum() ** 2 / (w * w).sum()
    se = (hi - lo) / math.sqrt(12) / math.sqrt(ess)
    assert np.all(np.abs(est - (lo + hi) / 2) < 6 * se), (est, ess)
    # lambda = 1 is the prior itself: every weight is exactly 1
    _, w1 = net.sample(mix, 1000, seed=4, lam=1.0)
    assert torch.all(w1 == 1.0)
    # a mixture with no mass in the box falls back to the prior (weights 1)
    far = np.zeros(136, dtype=np.float32)
    far[8:8 + 64] = 60.0
    far[8 + 64:] = -5.0
    the, we = net.sample(torch.from_numpy(far).cuda(), 2000, seed=4, lam=0.2)
    assert torch.all(we == 1.0)
    the = the.cpu().numpy()
    assert np.all(the >= lo) and np.all(the <= hi)
    net.close()
