"""The posterior-agreement helper on the CPU with synthetic samplers whose
answer is known: two samplers of the same distribution agree once pooled to
the stated resolution (heavy tails included, which need many more runs); a
sampler whose sd is off by 10 % is caught; importance weights that correct a
tilted proposal make it agree."""
import numpy as np

from paper_2012_14332_amd import pipeline as P


def _sampler(draw, weight=None, q=2048):
    def run(seed, idxs):
        rng = np.random.default_rng(1000 * seed + 7)
        th = np.stack([draw(rng, q, j) for j in idxs])
        w = (np.stack([weight(t) for t in th]) if weight else np.ones((len(idxs), q)))
        return th, w
    return run


def _base(rng, q, j):
    return rng.normal(3.0 + j, 1.0 + 0.1 * j, size=(q, 8))


def _heavy(rng, q, j):  # Student t with 5 degrees of freedom: kurtosis 9
    return 2.0 + rng.standard_t(5, size=(q, 8))


def test_same_distribution_agrees_and_is_resolved():
    res = P.compare_posteriors([None] * 3, [None] * 3, _sampler(_base), _sampler(_base), quota=2048,
                               max_runs=64)
    for r in res:
        assert r["se_over_tol"] * 4 <= 1.0 and r["ess_b"] >= 1e4
        assert all(r["mean_ok"]) and all(r["sd_ok"])


def test_heavy_tails_need_more_runs():
    base = P.compare_posteriors([None], [None], _sampler(_base), _sampler(_base), quota=2048)
    heavy = P.compare_posteriors([None], [None], _sampler(_heavy), _sampler(_heavy), quota=2048,
                                 max_runs=200)
    assert heavy[0]["se_over_tol"] * 4 <= 1.0
    assert heavy[0]["runs_a"] + heavy[0]["runs_b"] > base[0]["runs_a"] + base[0]["runs_b"]
    assert all(heavy[0]["sd_ok"])


def test_wrong_sd_is_caught():
    wide = lambda rng, q, j: rng.normal(3.0 + j, 1.1 * (1.0 + 0.1 * j), size=(q, 8))
    res = P.compare_posteriors([None] * 2, [None] * 2, _sampler(_base), _sampler(wide), quota=2048)
    for r in res:
        assert not any(r["sd_ok"]) and r["sd_ratio"] > 1.5


def test_importance_weights_correct_a_tilted_proposal():
    # proposal N(3.5, 1) for target N(3, 1): weights N(3,1)/N(3.5,1)
    prop = lambda rng, q, j: rng.normal(3.5, 1.0, size=(q, 8))
    target = lambda rng, q, j: rng.normal(3.0, 1.0, size=(q, 8))
    wfun = lambda t: np.exp((-(t - 3.0) ** 2 + (t - 3.5) ** 2).sum(1) / 2)
    res = P.compare_posteriors([None], [None], _sampler(target), _sampler(prop, wfun), quota=4096,
                               max_runs=128)
    assert all(res[0]["mean_ok"]) and all(res[0]["sd_ok"])
    unweighted = P.compare_posteriors([None], [None], _sampler(target), _sampler(prop), quota=4096)
    assert not all(unweighted[0]["mean_ok"])


def test_running_pool_equals_the_pooled_summary():
    # the running sums give the summary of the concatenated runs
    rng = np.random.default_rng(3)
    pool, ths, ws = P._Pool(), [], []
    for r in range(7):
        th = rng.standard_t(5, size=(500, 8)) * (1.0 + np.arange(8)) + 40.0
        w = rng.gamma(0.5, size=500)
        pool.add(th, w)
        ths.append(th)
        ws.append(w)
    want = P._weighted_summary(np.concatenate(ths), np.concatenate(ws))
    got = pool.summary()
    for a, b in zip(got, want):
        np.testing.assert_allclose(a, b, rtol=1e-9)
