"""The C ABI: libabc.so builds for gfx950, loads on a host without a GPU and
exports every entry point include/abc.h declares (no compute calls here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abc.h")
LIB = os.path.join(ROOT, "paper_2012_14332_amd", "libabc.so")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"ABC_API\s+[\w\s\*]+?\b(abc_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_2012_14332_amd import build

        build.build()
    return LIB


def test_header_declares_the_boundary():
    names = declared()
    for f in ("abc_sample_prior", "abc_simulate_distance", "abc_accept_compact",
              "abc_posterior_moments", "abc_simulate_record", "abc_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol(built):
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(abc_\w+)", out))
    missing = set(declared()) - exported
    assert not missing, missing


def test_library_loads_without_gpu(built):
    L = ctypes.CDLL(built)
    for f in declared():
        assert hasattr(L, f)
    L.abc_version.restype = ctypes.c_char_p
    assert L.abc_version().decode().startswith("abc-mi355x")


def test_host_validation_rejects_bad_arguments(built):
    """Argument errors are caught on the host before any HIP call."""
    from paper_2012_14332_amd import abc

    L = abc.lib()
    pr = abc.make_prior()
    st = abc.make_stream(1, 16, 0)  # domain out of range
    rc = L.abc_sample_prior(ctypes.byref(pr), ctypes.byref(st), 0, 10, None, None)
    assert rc == -1
    assert b"domain" in L.abc_last_error()
    st = abc.make_stream(1, 1, 0)
    bad = abc.make_prior(hi=(1, 100, 2, 1, 1, 1, 1, -1))
    rc = L.abc_sample_prior(ctypes.byref(bad), ctypes.byref(st), 0, 10, None, None)
    assert rc == -1
    ser = abc._Series(1000, 100, 0, 0, 0, None)  # T = 0
    md = abc._Model(1.0, 0)
    rc = L.abc_simulate_distance(ctypes.byref(ser), ctypes.byref(md), ctypes.byref(st), None,
                                 ctypes.byref(pr), 0, 10, float("inf"), None, None, None, None)
    assert rc == -1 and b"T = 0" in L.abc_last_error()
    ser = abc._Series(50, 100, 0, 0, 10, None)  # A0 > P
    rc = L.abc_simulate_record(ctypes.byref(ser), ctypes.byref(md), ctypes.byref(st), None, 0,
                               10, None, None)
    assert rc == -1
    ser = abc._Series(2**31, 100, 0, 0, 10, None)  # P beyond int32 state
    rc = L.abc_simulate_record(ctypes.byref(ser), ctypes.byref(md), ctypes.byref(st), None, 0,
                               10, None, None)
    assert rc == -1
    md = abc._Model(1.0, 0x100)  # unknown flag
    ser = abc._Series(1000, 100, 0, 0, 10, None)
    rc = L.abc_simulate_record(ctypes.byref(ser), ctypes.byref(md), ctypes.byref(st), None, 0,
                               10, None, None)
    assert rc == -1 and b"flags" in L.abc_last_error()
    # n = 0 is a no-op that needs no device pointers
    assert L.abc_sample_prior(ctypes.byref(pr), ctypes.byref(st), 0, 0, None, None) == 0


def test_host_validation_of_the_newer_entry_points(built):
    """Bad sizes and options of the nearest-k, bands, SMC, batched-proposal and
    tuning entry points are rejected on the host (ABC_EINVAL), no GPU needed."""
    from paper_2012_14332_amd import abc

    L = abc.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    pr = abc.make_prior()
    st = abc.make_stream(1, 1, 0)
    # nearest-k: k = 0, k > n, k > 4096
    for n, k in [(10, 0), (10, 11), (100000, 4097)]:
        assert L.abc_nearest_k(fake, None, ctypes.byref(pr), ctypes.byref(st), n, 0, k, fake, None,
                               None, None, None) == -1
    # bands: n > 8192, more than 16 quantiles, a quantile outside [0, 1]
    q = (ctypes.c_double * 17)(*([0.5] * 17))
    assert L.abc_trajectory_bands(fake, 8193, 10, q, 1, fake, None) == -1
    assert L.abc_trajectory_bands(fake, 10, 10, q, 17, fake, None) == -1
    qb = (ctypes.c_double * 1)(1.5)
    assert L.abc_trajectory_bands(fake, 10, 10, qb, 1, fake, None) == -1
    # SMC: population size and alpha out of range
    ser = abc._Series(1000000, 100, 0, 0, 10, 0x1000)
    md = abc._Model(1.0, 0)
    stats = abc._SmcGenStats()
    for cfg in (abc.smc_config(1, 10.0), abc.smc_config(8193, 10.0), abc.smc_config(100, 10.0, alpha=0.0),
                abc.smc_config(100, 10.0, chunk0=0)):
        assert L.abc_smc_generation(ctypes.byref(ser), ctypes.byref(md), ctypes.byref(pr), 1, 0, 0,
                                    None, None, None, 0, ctypes.byref(cfg), fake, fake, fake, fake,
                                    ctypes.byref(stats), None, None) == -1
    # ABC_FP64 is not an SMC mode
    md64 = abc._Model(1.0, abc.ABC_FP64)
    cfg = abc.smc_config(100, 10.0)
    assert L.abc_smc_generation(ctypes.byref(ser), ctypes.byref(md64), ctypes.byref(pr), 1, 0, 0,
                                None, None, None, 0, ctypes.byref(cfg), fake, fake, fake, fake,
                                ctypes.byref(stats), None, None) == -1
    # refill threshold
    assert L.abc_set_refill_min(65) == -1 and L.abc_set_refill_min(-1) == -1
    assert L.abc_get_refill_min() == 8
    # batch margin
    assert L.abc_set_batch_margin((1 << 20) + 1) == -1 and L.abc_set_batch_margin(-(1 << 20) - 1) == -1
    assert L.abc_set_batch_margin(-5) == 0 and L.abc_set_batch_margin(0) == 0
    # batched proposal: NULL proposal, lambda and inflate out of range
    bs = (abc._BatchSeries * 1)(abc._BatchSeries(1000000, 100, 0, 0, 10, 0x1000, 1.0, 0))
    bst = abc._BatchStats()
    assert L.abc_batch_run_weighted(bs, 1, ctypes.byref(pr), ctypes.byref(md), 1, 1, 10, 4096, 100,
                                    0.02, 1, 0, None, fake, fake, fake, fake, fake, fake, fake, fake,
                                    ctypes.byref(bst), None) == -1
    for lam, infl in [(1.5, 2.0), (0.5, 0.5), (0.5, 200.0)]:
        prop = abc._BatchProposal(0x1000, lam, infl, 5, 0)
        assert L.abc_batch_run_weighted(bs, 1, ctypes.byref(pr), ctypes.byref(md), 1, 1, 10, 4096,
                                        100, 0.02, 1, 0, ctypes.byref(prop), fake, fake, fake, fake,
                                        fake, fake, fake, fake, ctypes.byref(bst), None) == -1
    # the proposal's draws on the simulation's own domain would reuse its
    # day-1 noise words for theta: rejected
    prop = abc._BatchProposal(0x1000, 0.5, 2.0, 1, 0)
    assert L.abc_batch_run_weighted(bs, 1, ctypes.byref(pr), ctypes.byref(md), 1, 1, 10, 4096,
                                    100, 0.02, 1, 0, ctypes.byref(prop), fake, fake, fake, fake,
                                    fake, fake, fake, fake, ctypes.byref(bst), None) == -1
    assert b"equals the simulation domain" in L.abc_last_error()


def test_host_validation_of_limits_and_special_values(built):
    """The documented limits (T <= ABC_T_MAX, n <= 2^36), NaN or negative
    tolerances, misaligned buffers and capacity options are rejected on the
    host; eps = +INF is accepted where it means "no bound" or "accept all"."""
    from paper_2012_14332_amd import abc

    L = abc.lib()
    fake = ctypes.c_void_p(0x1000)      # never dereferenced: validation fails first
    odd = ctypes.c_void_p(0x1004)       # not 16-byte aligned
    pr = abc.make_prior()
    st = abc.make_stream(1, 1, 0)
    md = abc._Model(1.0, 0)
    sim = lambda ser, n, e, dist=fake: L.abc_simulate_distance(
        ctypes.byref(ser), ctypes.byref(md), ctypes.byref(st), None, ctypes.byref(pr), 0, n, e, dist,
        None, None, None)
    ser = abc._Series(1000000, 100, 0, 0, 1025, 0x1000)        # T beyond ABC_T_MAX
    assert sim(ser, 10, float("inf")) == -1 and b"T = 1025" in L.abc_last_error()
    ser = abc._Series(1000000, 100, 0, 0, 50, 0x1000)
    assert sim(ser, (1 << 36) + 1, float("inf")) == -1          # n beyond 2^36
    assert sim(ser, 10, float("nan")) == -1                     # NaN exit bound
    assert sim(ser, 10, -1.0) == -1                             # negative exit bound
    assert sim(ser, 0, float("inf"), None) == 0                 # n = 0: nothing to do
    # compaction: NaN tolerance; +INF is "accept every sample"
    cnt = fake
    assert L.abc_accept_compact(fake, None, None, ctypes.byref(pr), ctypes.byref(st), 10, 0,
                                float("nan"), 0, None, None, None, None, cnt, None) == -1
    # band decision: NaN or negative eps, band width outside [0, 1)
    for e, w in ((float("nan"), 0.02), (-1.0, 0.02), (1.0, 1.0), (1.0, -0.1)):
        assert L.abc_recheck_band(ctypes.byref(ser), ctypes.byref(md), ctypes.byref(st), e, w, 10,
                                  fake, fake, fake, None, fake, None, None) == -1
    # moments: theta must be 16-byte aligned, n_max >= 0
    assert L.abc_posterior_moments(odd, None, None, 10, fake, fake, None) == -1
    assert L.abc_posterior_moments(fake, None, None, -1, fake, fake, None) == -1
    # batched: candidate capacity below the quota or above 16384
    bs = (abc._BatchSeries * 1)(abc._BatchSeries(1000000, 100, 0, 0, 10, 0x1000, 1.0, 0))
    bst = abc._BatchStats()
    for cap in (99, 16385):
        assert L.abc_batch_run(bs, 1, ctypes.byref(pr), ctypes.byref(md), 1, 1, 100, 4096, 1000,
                               0.02, 1, cap, fake, fake, fake, fake, fake, fake, fake,
                               ctypes.byref(bst), None) == -1


def test_host_validation_of_the_multi_series_launch(built):
    """abc_simulate_distance_multi: job count, per-job series and sizes, and
    the float32-only options are checked on the host."""
    from paper_2012_14332_amd import abc

    L = abc.lib()
    pr = abc.make_prior()
    md = abc._Model(1.0, 0)
    ser = abc._Series(1000000, 100, 0, 0, 50, 0x1000)
    bad_ser = abc._Series(1000000, 100, 0, 0, 0, 0x1000)  # T = 0
    job = lambda s, n=10, e=1.0, d=0x1000: abc._SimJob(ctypes.pointer(s), 0, 0, 0, n, e, 0, d)
    arr = (abc._SimJob * 9)(*[job(ser) for _ in range(9)])
    run = lambda a, m, model=md: L.abc_simulate_distance_multi(a, m, ctypes.byref(model),
                                                               ctypes.byref(pr), 1, 1, None, None)
    assert run(arr, 0) == -1
    assert run(arr, 9) == -1                                    # more than ABC_MULTI_MAX
    assert run((abc._SimJob * 1)(job(bad_ser)), 1) == -1 and b"T = 0" in L.abc_last_error()
    assert run((abc._SimJob * 1)(job(ser, n=-1)), 1) == -1
    assert run((abc._SimJob * 1)(job(ser, e=float("nan"))), 1) == -1
    assert run((abc._SimJob * 1)(job(ser, d=None)), 1) == -1   # n > 0 needs dist
    assert run((abc._SimJob * 1)(job(ser)), 1, abc._Model(1.0, abc.ABC_FP64)) == -1
    assert run((abc._SimJob * 1)(job(ser, n=0, d=None)), 1) == 0  # nothing to do
