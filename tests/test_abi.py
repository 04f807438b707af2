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
