"""Pins of the oracle's random numbers: Philox4x32-10, the prior draw (eq. 2)
and the per-day standard normals.

Each check compares the oracle with something other than itself: rocRAND's
Philox4x32-10 (an independent library implementation of the SC'11
generator), exact rational arithmetic, closed-form moments of the uniform and
normal laws, and the algebraic identity behind the Box-Muller pairs.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import pyref

ROCRAND_PROBE = r"""
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Eng : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};
int main() {
    Eng e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
"""


def _random_inputs(n, seed):
    rng = np.random.default_rng(seed)
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    # edge words
    ctr[0] = 0
    key[0] = 0
    ctr[1] = 0xFFFFFFFF
    key[1] = 0xFFFFFFFF
    return ctr, key


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_library():
    ctr, key = _random_inputs(512, 1)
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.cpp")
        exe = os.path.join(d, "probe")
        with open(src, "w") as f:
            f.write(ROCRAND_PROBE)
        subprocess.check_call(["hipcc", "-O1", "-I/opt/rocm/include", src, "-o", exe],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        inp = "\n".join(" ".join(str(int(x)) for x in list(c) + list(k))
                        for c, k in zip(ctr, key))
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()],
                   dtype=np.uint32)
    got = oracle.philox(ctr, key)
    np.testing.assert_array_equal(got, ref)


def test_philox_c_matches_python_integers():
    ctr, key = _random_inputs(256, 2)
    got = oracle.philox(ctr, key)
    for i in range(ctr.shape[0]):
        assert tuple(int(x) for x in got[i]) == pyref.philox(ctr[i], key[i])


def test_philox_bits_balanced():
    n = 1 << 15
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n, dtype=np.uint32)
    key = np.tile(np.array([7, 0], dtype=np.uint32), (n, 1))
    w = oracle.philox(ctr, key).ravel()
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(axis=0)
    # 4n samples per bit: sd = 0.5/sqrt(4n) ~ 1.4e-3; allow 6 sd
    assert np.all(np.abs(bits - 0.5) < 6 * 0.5 / math.sqrt(4 * n))
    # consecutive counters must not give correlated words
    a = w[0::4].astype(np.float64)
    b = w[1::4].astype(np.float64)
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(n)


def test_stream_layout_fields():
    # the counter layout: (i mod 2^32, i >> 32, series, day<<8 | domain<<4 | block)
    seed = (5 << 32) | 11
    i = (3 << 32) | 17
    got = oracle.stream_words(seed, 2, 9, i, 40, 1)
    ref = oracle.philox(np.array([[17, 3, 9, (40 << 8) | (2 << 4) | 1]], np.uint32),
                        np.array([[11, 5]], np.uint32))[0]
    np.testing.assert_array_equal(got, ref)


# --------------------------------------------------------------------------- prior


def test_prior_exact_rounding_default_and_custom_bounds():
    lo = np.array([0.1, -3.0, 0.0, 0.25, 0.0, 0.0, 0.3, 0.5], np.float32)
    hi = np.array([0.9, 7.5, 2.0, 0.75, 1.0, 1e-3, 1.0, 2.0], np.float32)
    for (l, h) in ((oracle.PRIOR_LO, oracle.PRIOR_HI), (lo, hi)):
        th = oracle.prior(64, seed=123, domain=1, series=4, first=1000, lo=l, hi=h)
        for j in range(th.shape[0]):
            ref = pyref.prior_theta(123, 1, 4, 1000 + j, l, h)
            np.testing.assert_array_equal(th[j], ref)


def test_prior_in_box_and_closed_form_moments():
    n = 200000
    th = oracle.prior(n, seed=99).astype(np.float64)
    lo = oracle.PRIOR_LO.astype(np.float64)
    hi = oracle.PRIOR_HI.astype(np.float64)
    assert np.all(th >= lo) and np.all(th < hi)
    mean_ref = (lo + hi) / 2
    var_ref = (hi - lo) ** 2 / 12
    se = np.sqrt(var_ref / n)
    assert np.all(np.abs(th.mean(0) - mean_ref) < 6 * se)
    # variance of a uniform estimate: sd ~ var * sqrt(0.8/n)
    assert np.all(np.abs(th.var(0) - var_ref) < 6 * var_ref * math.sqrt(0.8 / n))
    # KS against U(lo, hi) per coordinate
    for k in range(8):
        p = stats.kstest((th[:, k] - lo[k]) / (hi[k] - lo[k]), "uniform").pvalue
        assert p > 1e-4
    # coordinates independent
    c = np.corrcoef(th.T)
    assert np.all(np.abs(c - np.eye(8)) < 6 / math.sqrt(n))


def test_prior_streams_differ_by_series_sample_domain():
    a = oracle.prior(4, seed=1, domain=1, series=0)
    b = oracle.prior(4, seed=1, domain=1, series=1)
    c = oracle.prior(4, seed=1, domain=2, series=0)
    d = oracle.prior(4, seed=2, domain=1, series=0)
    for x in (b, c, d):
        assert not np.any(np.all(a == x, axis=1))
    # sample i of a longer range equals sample i drawn alone
    e = oracle.prior(1, seed=1, domain=1, series=0, first=3)
    np.testing.assert_array_equal(e[0], a[3])


# --------------------------------------------------------------------------- normals


def _collect_normals(n_samples, days, seed=5):
    z = np.empty((n_samples * len(days), 5))
    k = 0
    for i in range(n_samples):
        for t in days:
            z[k] = oracle.normals(seed, 1, 0, i, t)
            k += 1
    return z


def test_normals_match_python_restatement():
    for (i, t) in [(0, 1), (1, 1), (12345, 17), (2**33 + 5, 200)]:
        np.testing.assert_allclose(oracle.normals(9, 1, 3, i, t),
                                   pyref.normals(9, 1, 3, i, t), rtol=0, atol=1e-14)


def test_normals_standard_normal_and_independent():
    z = _collect_normals(4000, range(1, 11))
    n = z.shape[0]
    for k in range(5):
        assert abs(z[:, k].mean()) < 6 / math.sqrt(n)
        assert abs(z[:, k].var() - 1) < 6 * math.sqrt(2 / n)
        assert stats.kstest(z[:, k], "norm").pvalue > 1e-4
    c = np.corrcoef(z.T)
    assert np.all(np.abs(c - np.eye(5)) < 6 / math.sqrt(n))
    # squares uncorrelated too: a Box-Muller pair shares its radius, and only
    # a correct pairing of radius and angle makes the two squares independent
    c2 = np.corrcoef((z ** 2).T)
    assert np.all(np.abs(c2 - np.eye(5)) < 6 / math.sqrt(n))


def test_box_muller_radius_identity():
    # z1^2 + z2^2 = -2 ln u0 and z3^2 + z4^2 = -2 ln u2, with u from the 21-bit fields
    for (i, t) in [(0, 1), (77, 3), (9999, 48)]:
        w = oracle.stream_words(5, 1, 0, i, t, 0)
        u0 = ((int(w[0]) >> 11) + 0.5) / 2**21
        u2 = ((int(w[2]) >> 11) + 0.5) / 2**21
        z = oracle.normals(5, 1, 0, i, t)
        assert math.isclose(z[0] ** 2 + z[1] ** 2, -2 * math.log(u0), rel_tol=1e-13)
        assert math.isclose(z[2] ** 2 + z[3] ** 2, -2 * math.log(u2), rel_tol=1e-13)
        u4 = ((((int(w[0]) & 0x7FF) << 10) | (int(w[1]) & 0x3FF)) + 0.5) / 2**21
        u5 = ((((int(w[2]) & 0x7FF) << 10) | (int(w[3]) & 0x3FF)) + 0.5) / 2**21
        assert math.isclose(z[4], math.sqrt(-2 * math.log(u4)) * math.cos(2 * math.pi * u5),
                            rel_tol=1e-12, abs_tol=1e-12)
