"""abc_accept_compact_noalloc through the C ABI: the same rows, distances,
weights and count as abc_accept_compact, on two calls in a row sharing the
library's fixed scratch (the second smaller, so stale tile words of the first
call must not leak into it), in both tile sizes and with theta re-drawn from
the prior; sizes beyond the fixed scratch are rejected on the host."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_14332_amd import abc

    return abc


def _outs(cap, weighted):
    o = {"idx": torch.full((cap,), -7, dtype=torch.int64, device="cuda"),
         "theta": torch.full((cap, 8), -7.0, dtype=torch.float32, device="cuda"),
         "dist": torch.full((cap,), -7.0, dtype=torch.float32, device="cuda"),
         "count": torch.full((1,), -7, dtype=torch.int64, device="cuda")}
    o["w"] = torch.full((cap,), -7.0, dtype=torch.float32, device="cuda") if weighted else None
    return o


def _call(abc, fn, dist, theta, weight, eps, first, o, seed=3, series=2):
    pr = abc.make_prior()
    st = abc.make_stream(seed, 1, series)
    p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    rc = fn(p(dist), p(theta), p(weight), ctypes.byref(pr), ctypes.byref(st), int(dist.shape[0]),
            int(first), float(eps), int(o["idx"].shape[0]), p(o["idx"]), p(o["theta"]), p(o["dist"]),
            p(o["w"]), p(o["count"]), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc


def _case(n, seed, with_theta):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    dist = torch.rand(n, generator=g, device="cuda")
    dist[torch.rand(n, generator=g, device="cuda") < 0.2] = float("inf")
    theta = torch.rand((n, 8), generator=g, device="cuda") if with_theta else None
    weight = torch.rand(n, generator=g, device="cuda") if with_theta else None
    return dist, theta, weight


def test_noalloc_equals_allocating_compaction_on_consecutive_calls(L):
    abc = L
    lib = abc.lib()
    # first a large input with big tiles, then a smaller one with small tiles
    # (fewer tiles than the first call left in the scratch), then one tile
    for n, eps, first, with_theta in [((1 << 25) + 4096 * 7 + 5, 2e-4, 10_000, True),
                                      (1_000_003, 1e-3, 77, True),
                                      (300_001, 5e-3, 1 << 33, False),
                                      (4095, 0.05, 0, True)]:
        dist, theta, weight = _case(n, n % 1000, with_theta)
        keep = int((dist <= eps).sum().item())
        cap = keep + 3
        print("n=%d eps=%g accepted=%d theta=%s" % (n, eps, keep, with_theta), flush=True)
        ref = _outs(cap, with_theta)
        got = _outs(cap, with_theta)
        assert _call(abc, lib.abc_accept_compact, dist, theta, weight, eps, first, ref) == 0
        assert _call(abc, lib.abc_accept_compact_noalloc, dist, theta, weight, eps, first, got) == 0
        torch.cuda.synchronize()
        assert int(got["count"].item()) == int(ref["count"].item()) == keep
        for k in ("idx", "theta", "dist", "w"):
            if ref[k] is not None:
                assert torch.equal(got[k], ref[k]), k
        # the kept indices are the brute-force ones
        want = torch.nonzero(dist <= eps).flatten().cpu().numpy() + first
        np.testing.assert_array_equal(got["idx"][:keep].cpu().numpy(), want)


def test_noalloc_overflow_count_and_limits(L):
    abc = L
    lib = abc.lib()
    dist, theta, weight = _case(200_000, 5, True)
    eps = 0.01
    keep = int((dist <= eps).sum().item())
    cap = keep // 2
    ref, got = _outs(cap, True), _outs(cap, True)
    assert _call(abc, lib.abc_accept_compact, dist, theta, weight, eps, 0, ref) == 0
    assert _call(abc, lib.abc_accept_compact_noalloc, dist, theta, weight, eps, 0, got) == 0
    torch.cuda.synchronize()
    assert int(got["count"].item()) == keep > cap
    for k in ("idx", "theta", "dist", "w"):
        assert torch.equal(got[k], ref[k]), k
    # n beyond the fixed scratch: rejected on the host, nothing enqueued
    big = (1 << 30) + 1
    pr = abc.make_prior()
    st = abc.make_stream(1, 1, 0)
    fake = ctypes.c_void_p(dist.data_ptr())
    rc = lib.abc_accept_compact_noalloc(fake, None, None, ctypes.byref(pr), ctypes.byref(st), big, 0,
                                        0.1, 0, None, None, None, None,
                                        ctypes.c_void_p(got["count"].data_ptr()), None)
    assert rc == -1 and b"ABC_NOALLOC_COMPACT_MAX_N" in lib.abc_last_error()
    # the binding with caller-provided outputs
    out = _outs(cap, True)
    abc.accept_compact_noalloc(dist, eps, out["idx"], out["theta"], out["count"], out_dist=out["dist"],
                               out_w=out["w"], theta=theta, weight=weight, seed=3, series=2)
    torch.cuda.synchronize()
    assert torch.equal(out["idx"], ref["idx"]) and int(out["count"].item()) == keep
