"""End-to-end parity of the plain rejection-ABC pass (float32 simulation,
compaction at eps (1 + w), float64 decision inside the band, float64
moments) against the FP64 oracle's accept rule dist <= eps (eq. 7).

Bar: the accepted index sets are identical except for samples whose oracle
distance lies within the tie band |d - eps| < 1e-5 eps; theta is bit-exact,
so the moments then agree to float64 rounding.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2012_14332_amd import workloads as W

pytestmark = pytest.mark.gpu

TIE = 1e-5


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_14332_amd import abc, pipeline

    abc.lib()
    return pipeline


def _check(P, s, n, q, band, first=0):
    from paper_2012_14332_amd import abc

    m = oracle.make_model(s.P, s.T)
    obs_ref = oracle.observe(m, s.theta_true, s.obs_seed, series=s.series_id)
    ser = P.observed_series(s)
    np.testing.assert_array_equal(ser.obs.cpu().numpy(), obs_ref)
    ref = oracle.distances(m, obs_ref, seed=11, n=n, first=first, series=s.series_id)
    eps = float(np.quantile(ref, q))
    run = P.PlainABC(ser, 11, eps, n, series=s.series_id, band_w=band, capacity=1 << 15)
    res = run.run(first, want_rechecked=True)
    c = res.n()
    got = set(res.idx[:c].cpu().numpy().tolist())
    want = set((np.nonzero(ref <= eps)[0] + first).tolist())
    diff = sorted(got ^ want)
    tie = [i for i in diff if abs(ref[i - first] - eps) < TIE * eps]
    assert diff == tie, "accept sets differ outside the tie band: %s" % [
        (i, ref[i - first], eps) for i in diff if i not in tie][:10]
    # float32 pass without the float64 band, for the record
    d32 = abc.simulate_distance(ser, n, 11, first=first, series=s.series_id).cpu().numpy()
    near = ref <= 2 * eps
    rel = np.abs(d32[near] - ref[near]) / ref[near]
    wrong32 = int(np.sum((d32 <= eps) != (ref <= eps)))
    print("%s: accepted %d, rechecked %d, fp32-only decision errors %d, near-eps fp32 rel err "
          "median %.1e max %.1e" % (s.name, c, int(res.rechecked.item()), wrong32,
                                    np.median(rel), rel.max()))
    if not diff:
        th = oracle.prior(n, seed=11, first=first, series=s.series_id)[np.nonzero(ref <= eps)[0]]
        np.testing.assert_array_equal(res.theta[:c].cpu().numpy(), th)
        rm, rc = oracle.moments(th)
        np.testing.assert_allclose(res.mean.cpu().numpy(), rm, rtol=1e-12)
        np.testing.assert_allclose(res.cov.cpu().numpy(), rc, rtol=1e-9, atol=1e-12)
    return wrong32


def test_plain_pass_country_T49(P):
    _check(P, W.three_countries()[0], 1_000_000, 1e-3, 0.02)


def test_plain_pass_country_T100_offset(P):
    _check(P, W.three_countries()[2], 300_000, 3e-3, 0.02, first=123_456)


def test_plain_pass_uneven_series(P):
    for s in W.uneven_series(64, 5)[:4]:
        _check(P, s, 200_000, 5e-3, 0.02)


def test_overflowed_pass_raises_instead_of_answering(P):
    from paper_2012_14332_amd import abc

    s = W.three_countries()[0]
    ser = P.observed_series(s)
    res = P.PlainABC(ser, 11, 1e30, 100_000, capacity=1000).run(0)
    with pytest.raises(abc.AbcError):
        res.n()
    ok = P.PlainABC(ser, 11, 1e30, 100_000, capacity=100_000).run(0)
    assert ok.n() == 100_000


def test_outputs_handed_across_streams_survive_early_release(P):
    """Compaction on stream B, band decision and moments on stream C that is
    held back behind a spin kernel, and every tensor dropped right after the
    calls while stream B allocates and overwrites new tensors of the same
    sizes: the rows stream C computes equal a one-stream pass, because the
    binding marks each tensor it hands to a call as in use on that call's
    stream."""
    from paper_2012_14332_amd import abc

    s = W.three_countries()[0]
    ser = P.observed_series(s)
    eps = P.pilot_eps(ser, 1, n=100_000, q=1e-3, series=0)
    n, first, w, cap = 1_000_000, 100_000, 0.02, 1 << 14
    ref = P.PlainABC(ser, 1, eps, n, series=0, band_w=w, capacity=cap).run(first)
    c_ref = ref.n()
    sB, sC = torch.cuda.Stream(), torch.cuda.Stream()
    dist = torch.empty(n, dtype=torch.float32, device="cuda")
    e_hi = eps * (1 + w)
    abc.simulate_distance(ser, n, 1, first=first, series=0, eps_exit=e_hi, out=dist)
    done = torch.cuda.Event()
    done.record()
    results = []
    for rep in range(3):
        with torch.cuda.stream(sB):
            sB.wait_event(done)
            idx, th, d, _, cnt = abc.accept_compact(dist, e_hi, cap, first=first, seed=1, series=0)
            ready = torch.cuda.Event()
            ready.record(sB)
        with torch.cuda.stream(sC):
            sC.wait_event(ready)
            torch.cuda._sleep(50_000_000)  # hold stream C back
            abc.recheck_band(ser, 1, eps, w, idx, th, d, cnt, series=0)
            mean, _ = abc.posterior_moments(th, n_dev=cnt)
            idx_c = idx.clone()
            cnt_c = cnt.clone()
        del idx, th, d, cnt
        with torch.cuda.stream(sB):
            junk = [torch.full((cap,), -3, dtype=torch.int64, device="cuda"),
                    torch.full((cap, 8), -3.0, device="cuda"), torch.full((cap,), -3.0, device="cuda"),
                    torch.full((1,), 7, dtype=torch.int64, device="cuda")]
        results.append((idx_c, cnt_c, mean, junk))
    torch.cuda.synchronize()
    for idx_c, cnt_c, mean, _ in results:
        assert int(cnt_c.item()) == c_ref
        assert torch.equal(idx_c[:c_ref], ref.idx[:c_ref])
        assert torch.equal(mean, ref.mean)
