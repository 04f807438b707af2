"""ctypes binding of libabc.so (include/abc.h): argument marshalling only.

Every function takes torch CUDA (HIP) tensors as device buffers and enqueues
on ``torch.cuda.current_stream()``; nothing here computes. If the library is
missing the first call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libabc.so")

ABC_FP64 = 0x1
ABC_KAHAN = 0x2
ABC_NOISE_LITERAL = 0x4
ABC_DIST_RAW = 0x8
ABC_SUPPORT = 0x10
ABC_NO_BOUND = 0x20
T_MAX = 1024

PRIOR_LO = (0.0,) * 8
PRIOR_HI = (1.0, 100.0, 2.0, 1.0, 1.0, 1.0, 1.0, 2.0)


class AbcError(RuntimeError):
    pass


class _Prior(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_float * 8), ("hi", ctypes.c_float * 8)]


class _Stream(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("domain", ctypes.c_uint32),
                ("series", ctypes.c_uint32)]


class _Series(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int64), ("A0", ctypes.c_int32), ("R0", ctypes.c_int32),
                ("D0", ctypes.c_int32), ("T", ctypes.c_int32), ("obs", ctypes.c_void_p)]


class _Model(ctypes.Structure):
    _fields_ = [("noise_scale", ctypes.c_float), ("flags", ctypes.c_uint32)]


class _SimJob(ctypes.Structure):
    _fields_ = [("ser", ctypes.POINTER(_Series)), ("series", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("first", ctypes.c_uint64), ("n", ctypes.c_int64),
                ("eps_exit", ctypes.c_float), ("pad2", ctypes.c_uint32), ("dist", ctypes.c_void_p)]


class _BatchSeries(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int64), ("A0", ctypes.c_int32), ("R0", ctypes.c_int32),
                ("D0", ctypes.c_int32), ("T", ctypes.c_int32), ("obs", ctypes.c_void_p),
                ("eps", ctypes.c_float), ("series", ctypes.c_uint32)]


class _BatchStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("graph_replays", ctypes.c_int64),
                ("sample_days", ctypes.c_int64), ("rechecked", ctypes.c_int64),
                ("grid", ctypes.c_int32), ("block", ctypes.c_int32), ("spl", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("rounds_ms", ctypes.c_float),
                ("phases", ctypes.c_int32)]


_lib = None


class _BatchProposal(ctypes.Structure):
    _fields_ = [("mix", ctypes.c_void_p), ("lam", ctypes.c_float), ("inflate", ctypes.c_float),
                ("domain", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class _SmcConfig(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_int32), ("generations", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("eps0", ctypes.c_float), ("eps_min", ctypes.c_float),
                ("band_w", ctypes.c_float), ("pad", ctypes.c_int32), ("chunk0", ctypes.c_int64),
                ("chunk_max", ctypes.c_int64), ("max_samples", ctypes.c_int64)]


class _SmcGenStats(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_float), ("pad", ctypes.c_int32), ("samples", ctypes.c_int64),
                ("in_support", ctypes.c_int64), ("proposed", ctypes.c_int64),
                ("ess", ctypes.c_double)]


def lib():
    """Load libabc.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise AbcError("libabc.so not found at %s: build it with "
                           "`python -m paper_2012_14332_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, u64, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float
        P = ctypes.POINTER
        L.abc_sample_prior.argtypes = [P(_Prior), P(_Stream), u64, i64, vp, vp]
        L.abc_simulate_distance.argtypes = [P(_Series), P(_Model), P(_Stream), vp, P(_Prior), u64,
                                            i64, f32, vp, vp, vp, vp]
        L.abc_simulate_record.argtypes = [P(_Series), P(_Model), P(_Stream), vp, u64, i64, vp, vp]
        L.abc_accept_compact.argtypes = [vp, vp, vp, P(_Prior), P(_Stream), i64, u64, f32, i64,
                                         vp, vp, vp, vp, vp, vp]
        L.abc_accept_compact_noalloc.argtypes = L.abc_accept_compact.argtypes
        L.abc_posterior_moments.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        for f in ("abc_sample_prior", "abc_simulate_distance", "abc_simulate_record",
                  "abc_accept_compact", "abc_accept_compact_noalloc", "abc_posterior_moments"):
            getattr(L, f).restype = ctypes.c_int32
        L.abc_simulate_distance_multi.argtypes = [P(_SimJob), ctypes.c_int32, P(_Model), P(_Prior),
                                                  u64, ctypes.c_uint32, vp, vp]
        L.abc_simulate_distance_multi.restype = ctypes.c_int32
        L.abc_recheck_band.argtypes = [P(_Series), P(_Model), P(_Stream), f32, f32, i64, vp, vp,
                                       vp, vp, vp, vp, vp]
        L.abc_recheck_band.restype = ctypes.c_int32
        L.abc_batch_run.argtypes = [P(_BatchSeries), ctypes.c_int32, P(_Prior), P(_Model), u64,
                                    ctypes.c_uint32, ctypes.c_int32, i64, i64, f32,
                                    ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp,
                                    P(_BatchStats), vp]
        L.abc_batch_run.restype = ctypes.c_int32
        L.abc_mdn_param_count.restype = i64
        L.abc_mdn_create.argtypes = [P(_Prior), u64, P(vp)]
        L.abc_mdn_destroy.argtypes = [vp]
        L.abc_mdn_set_params.argtypes = [vp, vp, vp]
        L.abc_mdn_get_params.argtypes = [vp, vp, vp]
        L.abc_mdn_get_standardizer.argtypes = [vp, vp, vp, vp]
        L.abc_mdn_simulate_features.argtypes = [P(_Prior), u64, ctypes.c_uint32, ctypes.c_uint32,
                                                u64, i64, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                                vp, vp, vp, vp]
        L.abc_series_features.argtypes = [P(_Series), vp, vp]
        L.abc_mdn_fit_standardizer.argtypes = [vp, vp, i64, vp]
        L.abc_mdn_forward.argtypes = [vp, vp, i64, vp, vp]
        L.abc_mdn_loss_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.abc_mdn_train.argtypes = [vp, vp, vp, i64, ctypes.c_int32, ctypes.c_int32, f32, u64,
                                    vp, P(i64), P(f32), vp]
        L.abc_mdn_sample.argtypes = [vp, vp, f32, f32, P(_Stream), u64, i64, vp, vp, vp]
        for f in ("abc_mdn_create", "abc_mdn_destroy", "abc_mdn_set_params",
                  "abc_mdn_get_params", "abc_mdn_get_standardizer", "abc_mdn_simulate_features",
                  "abc_series_features", "abc_mdn_fit_standardizer", "abc_mdn_forward",
                  "abc_mdn_loss_grad", "abc_mdn_train", "abc_mdn_sample"):
            getattr(L, f).restype = ctypes.c_int32
        L.abc_batch_run_weighted.argtypes = [P(_BatchSeries), ctypes.c_int32, P(_Prior), P(_Model),
                                             u64, ctypes.c_uint32, ctypes.c_int32, i64, i64, f32,
                                             ctypes.c_int32, ctypes.c_int32, P(_BatchProposal),
                                             vp, vp, vp, vp, vp, vp, vp, vp, P(_BatchStats), vp]
        L.abc_batch_run_weighted.restype = ctypes.c_int32
        L.abc_smc_generation.argtypes = [P(_Series), P(_Model), P(_Prior), u64, ctypes.c_uint32,
                                         ctypes.c_int32, vp, vp, vp, ctypes.c_int32, P(_SmcConfig),
                                         vp, vp, vp, vp, P(_SmcGenStats), vp, vp]
        L.abc_smc_generation.restype = ctypes.c_int32
        L.abc_smc_run.argtypes = [P(_Series), P(_Model), P(_Prior), u64, ctypes.c_uint32,
                                  P(_SmcConfig), vp, vp, vp, vp, P(_SmcGenStats),
                                  ctypes.POINTER(ctypes.c_int32), vp]
        L.abc_smc_run.restype = ctypes.c_int32
        L.abc_nearest_k.argtypes = [vp, vp, P(_Prior), P(_Stream), i64, u64, ctypes.c_int32, vp, vp,
                                    vp, vp, vp]
        L.abc_nearest_k.restype = ctypes.c_int32
        L.abc_nearest_k_rows.argtypes = [vp, vp, vp, i64, ctypes.c_int32, vp, vp, vp, vp]
        L.abc_nearest_k_rows.restype = ctypes.c_int32
        L.abc_simulate_rows_f64.argtypes = [P(_Series), P(_Model), P(_Stream), vp, vp, i64, vp, vp]
        L.abc_simulate_rows_f64.restype = ctypes.c_int32
        L.abc_set_refill_min.argtypes = [ctypes.c_int32]
        L.abc_set_refill_min.restype = ctypes.c_int32
        L.abc_get_refill_min.argtypes = []
        L.abc_set_batch_margin.argtypes = [ctypes.c_int32]
        L.abc_set_batch_margin.restype = ctypes.c_int32
        L.abc_get_refill_min.restype = ctypes.c_int32
        L.abc_trajectory_bands.argtypes = [vp, i64, ctypes.c_int32, vp, ctypes.c_int32, vp, vp]
        L.abc_trajectory_bands.restype = ctypes.c_int32
        L.abc_set_launch_config.argtypes = [ctypes.c_int32] * 3
        L.abc_set_launch_config.restype = ctypes.c_int32
        L.abc_get_launch_config.argtypes = [ctypes.POINTER(ctypes.c_int32)] * 3
        L.abc_get_launch_config.restype = ctypes.c_int32
        L.abc_last_error.restype = ctypes.c_char_p
        L.abc_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise AbcError("libabc status %d: %s" % (rc, lib().abc_last_error().decode()))


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t: Optional[torch.Tensor]):
    """Device address of a contiguous device tensor that the library call about to
    be made uses on the current stream. The tensor is marked as in use by that
    stream (record_stream), so torch's caching allocator does not hand its memory
    to other work before the call's kernels have finished, even when the tensor
    came from another stream and the caller drops it right after the call
    (a no-op for tensors allocated on the current stream)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise AbcError("expected a device tensor")
    if not t.is_contiguous():
        raise AbcError("expected a contiguous tensor")
    t.record_stream(torch.cuda.current_stream(t.device))
    return ctypes.c_void_p(t.data_ptr())


def make_prior(lo: Sequence[float] = PRIOR_LO, hi: Sequence[float] = PRIOR_HI) -> _Prior:
    return _Prior((ctypes.c_float * 8)(*lo), (ctypes.c_float * 8)(*hi))


def make_stream(seed: int, domain: int = 1, series: int = 0) -> _Stream:
    return _Stream(int(seed), int(domain), int(series))


class DeviceSeries:
    """An observed series whose [3, T] int32 counts live in device memory."""

    def __init__(self, P: int, T: int, obs: Optional[torch.Tensor] = None, A0: int = 100,
                 R0: int = 0, D0: int = 0, device="cuda"):
        self.P, self.T, self.A0, self.R0, self.D0 = int(P), int(T), int(A0), int(R0), int(D0)
        if obs is not None:
            obs = obs.to(device=device, dtype=torch.int32).contiguous()
            if tuple(obs.shape) != (3, self.T):
                raise AbcError("obs must have shape [3, T]")
        self.obs = obs

    def c(self) -> _Series:
        return _Series(self.P, self.A0, self.R0, self.D0, self.T,
                       None if self.obs is None else self.obs.data_ptr())


def sample_prior(n: int, seed: int, domain: int = 1, series: int = 0, first: int = 0,
                 prior: Optional[_Prior] = None, out: Optional[torch.Tensor] = None,
                 device="cuda") -> torch.Tensor:
    theta = out if out is not None else torch.empty((n, 8), dtype=torch.float32, device=device)
    pr = prior or make_prior()
    st = make_stream(seed, domain, series)
    _check(lib().abc_sample_prior(ctypes.byref(pr), ctypes.byref(st), int(first), int(n),
                                  _dptr(theta), _stream_handle()))
    return theta


def simulate_distance(ser: DeviceSeries, n: int, seed: int, *, theta: Optional[torch.Tensor] = None,
                      first: int = 0, domain: int = 1, series: int = 0,
                      eps_exit: float = math.inf, flags: int = 0, noise_scale: float = 1.0,
                      prior: Optional[_Prior] = None, out: Optional[torch.Tensor] = None,
                      want64: bool = False, days: Optional[torch.Tensor] = None,
                      device="cuda"):
    """Distances of samples first..first+n-1 ([n] float32; + float64 copy if want64).
    days: optional int64 [1] device tensor that accumulates the sample-days simulated."""
    dist = out if out is not None else torch.empty(n, dtype=torch.float32, device=device)
    d64 = torch.empty(n, dtype=torch.float64, device=device) if want64 else None
    pr = prior or make_prior()
    st = make_stream(seed, domain, series)
    md = _Model(float(noise_scale), int(flags))
    cs = ser.c()
    _check(lib().abc_simulate_distance(ctypes.byref(cs), ctypes.byref(md), ctypes.byref(st),
                                       _dptr(theta), ctypes.byref(pr), int(first), int(n),
                                       float(eps_exit), _dptr(dist), _dptr(d64), _dptr(days),
                                       _stream_handle()))
    return (dist, d64) if want64 else dist


def simulate_distance_multi(jobs, seed: int, *, domain: int = 1, flags: int = 0,
                            noise_scale: float = 1.0, prior: Optional[_Prior] = None,
                            days: Optional[torch.Tensor] = None, device="cuda"):
    """One launch for several series. jobs: sequence of dicts with keys ser
    (DeviceSeries), n, and optionally series (stream series id, default the job's
    position), first (0), eps_exit (+INF), out (float32 [n] device tensor).
    Returns the list of distance tensors, each equal to simulate_distance's for
    that job."""
    m = len(jobs)
    arr = (_SimJob * max(m, 1))()
    sers, outs = [], []
    for j, jb in enumerate(jobs):
        n = int(jb["n"])
        out = jb.get("out")
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.float32, device=device)[:n]
        cs = jb["ser"].c()
        sers.append(cs)
        outs.append(out)
        arr[j] = _SimJob(ctypes.pointer(cs), int(jb.get("series", j)), 0, int(jb.get("first", 0)), n,
                         float(jb.get("eps_exit", math.inf)), 0,
                         _dptr(out) if n > 0 else None)
    pr = prior or make_prior()
    md = _Model(float(noise_scale), int(flags))
    _check(lib().abc_simulate_distance_multi(arr, m, ctypes.byref(md), ctypes.byref(pr), int(seed),
                                             int(domain), _dptr(days), _stream_handle()))
    return outs


def simulate_record(ser: DeviceSeries, theta: torch.Tensor, seed: int, *, first: int = 0,
                    domain: int = 1, series: int = 0, flags: int = 0, noise_scale: float = 1.0,
                    device="cuda") -> torch.Tensor:
    n = theta.shape[0]
    traj = torch.empty((n, ser.T + 1, 6), dtype=torch.int32, device=device)
    st = make_stream(seed, domain, series)
    md = _Model(float(noise_scale), int(flags))
    cs = ser.c()
    _check(lib().abc_simulate_record(ctypes.byref(cs), ctypes.byref(md), ctypes.byref(st),
                                     _dptr(theta), int(first), int(n), _dptr(traj),
                                     _stream_handle()))
    return traj


def accept_compact(dist: torch.Tensor, eps: float, capacity: int, *,
                   theta: Optional[torch.Tensor] = None, weight: Optional[torch.Tensor] = None,
                   first: int = 0, seed: int = 0, domain: int = 1, series: int = 0,
                   prior: Optional[_Prior] = None, device="cuda"):
    """Returns (idx int64 [cap], theta [cap,8], dist [cap], w [cap] or None, count int64 [1]);
    only the first min(count, cap) rows are valid."""
    n = dist.shape[0]
    cap = int(capacity)
    out_idx = torch.empty(max(cap, 1), dtype=torch.int64, device=device)
    out_th = torch.empty((max(cap, 1), 8), dtype=torch.float32, device=device)
    out_d = torch.empty(max(cap, 1), dtype=torch.float32, device=device)
    out_w = torch.empty(max(cap, 1), dtype=torch.float32, device=device) if weight is not None else None
    count = torch.empty(1, dtype=torch.int64, device=device)
    pr = prior or make_prior()
    st = make_stream(seed, domain, series)
    _check(lib().abc_accept_compact(_dptr(dist), _dptr(theta), _dptr(weight), ctypes.byref(pr),
                                    ctypes.byref(st), int(n), int(first), float(eps), cap,
                                    _dptr(out_idx), _dptr(out_th), _dptr(out_d), _dptr(out_w),
                                    _dptr(count), _stream_handle()))
    return out_idx, out_th, out_d, out_w, count


def accept_compact_noalloc(dist: torch.Tensor, eps: float, out_idx: torch.Tensor,
                           out_theta: torch.Tensor, out_count: torch.Tensor, *,
                           out_dist: Optional[torch.Tensor] = None,
                           out_w: Optional[torch.Tensor] = None,
                           theta: Optional[torch.Tensor] = None,
                           weight: Optional[torch.Tensor] = None, first: int = 0, seed: int = 0,
                           domain: int = 1, series: int = 0, prior: Optional[_Prior] = None):
    """accept_compact into caller-provided outputs (capacity = out_idx rows), with the
    library's fixed scratch instead of an allocation."""
    pr = prior or make_prior()
    st = make_stream(seed, domain, series)
    _check(lib().abc_accept_compact_noalloc(_dptr(dist), _dptr(theta), _dptr(weight),
                                            ctypes.byref(pr), ctypes.byref(st), int(dist.shape[0]),
                                            int(first), float(eps), int(out_idx.shape[0]),
                                            _dptr(out_idx), _dptr(out_theta), _dptr(out_dist),
                                            _dptr(out_w), _dptr(out_count), _stream_handle()))


def recheck_band(ser: DeviceSeries, seed: int, eps: float, band_w: float, idx: torch.Tensor,
                 theta: torch.Tensor, dist: torch.Tensor, count: torch.Tensor, *,
                 weight: Optional[torch.Tensor] = None, domain: int = 1, series: int = 0,
                 flags: int = 0, noise_scale: float = 1.0, want_rechecked: bool = False):
    """Float64 decision of the in-band candidate rows; edits the rows and count in place."""
    st = make_stream(seed, domain, series)
    md = _Model(float(noise_scale), int(flags))
    cs = ser.c()
    nre = torch.zeros(1, dtype=torch.int32, device=idx.device) if want_rechecked else None
    _check(lib().abc_recheck_band(ctypes.byref(cs), ctypes.byref(md), ctypes.byref(st),
                                  float(eps), float(band_w), int(idx.shape[0]), _dptr(idx),
                                  _dptr(theta), _dptr(dist), _dptr(weight), _dptr(count),
                                  _dptr(nre), _stream_handle()))
    return nre


def posterior_moments(theta: torch.Tensor, weight: Optional[torch.Tensor] = None,
                      n_dev: Optional[torch.Tensor] = None, device="cuda"):
    n_max = theta.shape[0]
    mean = torch.empty(8, dtype=torch.float64, device=device)
    cov = torch.empty((8, 8), dtype=torch.float64, device=device)
    _check(lib().abc_posterior_moments(_dptr(theta), _dptr(weight), _dptr(n_dev), int(n_max),
                                       _dptr(mean), _dptr(cov), _stream_handle()))
    return mean, cov


def set_launch_config(spl: int = 0, block: int = 0, blocks_per_cu: int = 0):
    """Launch shape of the float32 simulate kernel for this thread (0 = default)."""
    _check(lib().abc_set_launch_config(int(spl), int(block), int(blocks_per_cu)))


def get_launch_config():
    v = [ctypes.c_int32() for _ in range(3)]
    _check(lib().abc_get_launch_config(*[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def batch_run(sers, eps, seed: int, quota: int, *, series_ids=None, round_size: int = 1 << 22,
              max_samples: int = 1 << 40, band_w: float = 0.02, rounds_per_graph: int = 4,
              domain: int = 1, noise_scale: float = 1.0, prior: Optional[_Prior] = None,
              cand_capacity: int = 0, device="cuda", check: bool = True, mix=None,
              lam: float = 0.05, inflate: float = 1.5, prop_domain: int = 5):
    """Batched persistent ABC over DeviceSeries `sers` with tolerances `eps` until each has
    `quota` accepted samples. With `mix` (device [m,136] network outputs) theta comes from
    the learned proposal and the result carries importance weights `w`. Returns a dict of
    device tensors and the run statistics."""
    m = len(sers)
    ids = list(range(m)) if series_ids is None else list(series_ids)
    arr = (_BatchSeries * m)()
    for j, (ser, e) in enumerate(zip(sers, eps)):
        arr[j] = _BatchSeries(ser.P, ser.A0, ser.R0, ser.D0, ser.T, ser.obs.data_ptr(), float(e),
                              int(ids[j]))
    out = {
        "idx": torch.full((m, quota), -1, dtype=torch.int64, device=device),
        "theta": torch.zeros((m, quota, 8), dtype=torch.float32, device=device),
        "dist": torch.zeros((m, quota), dtype=torch.float32, device=device),
        "count": torch.zeros(m, dtype=torch.int64, device=device),
        "used": torch.zeros(m, dtype=torch.int64, device=device),
        "mean": torch.zeros((m, 8), dtype=torch.float64, device=device),
        "cov": torch.zeros((m, 8, 8), dtype=torch.float64, device=device),
    }
    st = _BatchStats()
    pr = prior or make_prior()
    md = _Model(float(noise_scale), 0)
    if mix is None:
        rc = lib().abc_batch_run(arr, m, ctypes.byref(pr), ctypes.byref(md), int(seed), int(domain),
                                 int(quota), int(round_size), int(max_samples), float(band_w),
                                 int(rounds_per_graph), int(cand_capacity), _dptr(out["idx"]),
                                 _dptr(out["theta"]),
                                 _dptr(out["dist"]), _dptr(out["count"]), _dptr(out["used"]),
                                 _dptr(out["mean"]), _dptr(out["cov"]), ctypes.byref(st),
                                 _stream_handle())
    else:
        mix = mix.contiguous()
        if tuple(mix.shape) != (m, 136):
            raise AbcError("mix must have shape [m, 136]")
        out["w"] = torch.zeros((m, quota), dtype=torch.float32, device=device)
        prop = _BatchProposal(mix.data_ptr(), float(lam), float(inflate), int(prop_domain), 0)
        rc = lib().abc_batch_run_weighted(arr, m, ctypes.byref(pr), ctypes.byref(md), int(seed),
                                          int(domain), int(quota), int(round_size),
                                          int(max_samples), float(band_w), int(rounds_per_graph),
                                          int(cand_capacity), ctypes.byref(prop), _dptr(out["idx"]),
                                          _dptr(out["theta"]), _dptr(out["w"]), _dptr(out["dist"]),
                                          _dptr(out["count"]), _dptr(out["used"]),
                                          _dptr(out["mean"]), _dptr(out["cov"]), ctypes.byref(st),
                                          _stream_handle())
    out["status"] = rc
    out["stats"] = {k: getattr(st, k) for k, _ in _BatchStats._fields_}
    if check:
        _check(rc)
    return out


def simulate_features(n: int, seed: int, *, domain: int = 2, series: int = 0, first: int = 0,
                      T_lo: int = 30, T_hi: int = 200, log10P_lo: float = 5.0,
                      log10P_hi: float = 9.0, A0: int = 100, prior: Optional[_Prior] = None,
                      device="cuda"):
    """(features [n,96], theta [n,8], TP [n,2]) training pairs drawn by the simulator."""
    feats = torch.empty((n, 96), dtype=torch.float32, device=device)
    theta = torch.empty((n, 8), dtype=torch.float32, device=device)
    tp = torch.empty((n, 2), dtype=torch.int32, device=device)
    pr = prior or make_prior()
    _check(lib().abc_mdn_simulate_features(ctypes.byref(pr), int(seed), int(domain), int(series),
                                           int(first), int(n), int(T_lo), int(T_hi),
                                           float(log10P_lo), float(log10P_hi), int(A0),
                                           _dptr(feats), _dptr(theta), _dptr(tp),
                                           _stream_handle()))
    return feats, theta, tp


def series_features(ser: DeviceSeries, device="cuda") -> torch.Tensor:
    out = torch.empty(96, dtype=torch.float32, device=device)
    cs = ser.c()
    _check(lib().abc_series_features(ctypes.byref(cs), _dptr(out), _stream_handle()))
    return out


class Mdn:
    """Handle of the learned mixture-density proposal (device memory owned by libabc)."""

    def __init__(self, init_seed: int = 0, prior: Optional[_Prior] = None):
        self.prior = prior or make_prior()
        h = ctypes.c_void_p()
        _check(lib().abc_mdn_create(ctypes.byref(self.prior), int(init_seed), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().abc_mdn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def param_count() -> int:
        return int(lib().abc_mdn_param_count())

    def set_params(self, p: torch.Tensor):
        p = p.to(dtype=torch.float32, device="cuda").contiguous()
        assert p.numel() == self.param_count()
        _check(lib().abc_mdn_set_params(self.h, _dptr(p), _stream_handle()))

    def get_params(self) -> torch.Tensor:
        out = torch.empty(self.param_count(), dtype=torch.float32, device="cuda")
        _check(lib().abc_mdn_get_params(self.h, _dptr(out), _stream_handle()))
        return out

    def standardizer(self):
        m = torch.empty(96, dtype=torch.float32, device="cuda")
        s = torch.empty(96, dtype=torch.float32, device="cuda")
        _check(lib().abc_mdn_get_standardizer(self.h, _dptr(m), _dptr(s), _stream_handle()))
        return m, s

    def fit_standardizer(self, feats: torch.Tensor):
        _check(lib().abc_mdn_fit_standardizer(self.h, _dptr(feats), int(feats.shape[0]),
                                              _stream_handle()))

    def forward(self, feats: torch.Tensor) -> torch.Tensor:
        feats = feats.contiguous()
        n = feats.shape[0]
        out = torch.empty((n, 136), dtype=torch.float32, device="cuda")
        _check(lib().abc_mdn_forward(self.h, _dptr(feats), int(n), _dptr(out), _stream_handle()))
        return out

    def loss_grad(self, feats: torch.Tensor, theta: torch.Tensor):
        n = feats.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        grad = torch.empty(self.param_count(), dtype=torch.float32, device="cuda")
        _check(lib().abc_mdn_loss_grad(self.h, _dptr(feats.contiguous()), _dptr(theta.contiguous()),
                                       int(n), _dptr(loss), _dptr(grad), _stream_handle()))
        return loss, grad

    def train(self, feats: torch.Tensor, theta: torch.Tensor, *, epochs: int = 20,
              batch: int = 4096, lr: float = 1e-3, shuffle_seed: int = 0):
        n = feats.shape[0]
        steps = (n // batch) * epochs
        log = torch.zeros(steps, dtype=torch.float32, device="cuda")
        st = ctypes.c_int64()
        ms = ctypes.c_float()
        _check(lib().abc_mdn_train(self.h, _dptr(feats), _dptr(theta), int(n), int(epochs),
                                   int(batch), float(lr), int(shuffle_seed), _dptr(log),
                                   ctypes.byref(st), ctypes.byref(ms), _stream_handle()))
        return log, int(st.value), float(ms.value)

    def sample(self, mix: torch.Tensor, n: int, seed: int, *, lam: float = 0.05,
               inflate: float = 1.0, domain: int = 5, series: int = 0, first: int = 0):
        theta = torch.empty((n, 8), dtype=torch.float32, device="cuda")
        w = torch.empty(n, dtype=torch.float32, device="cuda")
        st = make_stream(seed, domain, series)
        _check(lib().abc_mdn_sample(self.h, _dptr(mix.contiguous()), float(lam), float(inflate),
                                    ctypes.byref(st),
                                    int(first), int(n), _dptr(theta), _dptr(w), _stream_handle()))
        return theta, w


def nearest_k(dist: torch.Tensor, k: int, *, theta: Optional[torch.Tensor] = None, first: int = 0,
              seed: int = 0, domain: int = 1, series: int = 0, prior: Optional[_Prior] = None,
              device="cuda"):
    """The k samples with the smallest distances (ties to the lower index), in index order:
    (idx [k] int64, theta [k,8], dist [k], kth [1] = k-th smallest distance)."""
    n = int(dist.shape[0])
    out_idx = torch.empty(k, dtype=torch.int64, device=device)
    out_th = torch.empty((k, 8), dtype=torch.float32, device=device)
    out_d = torch.empty(k, dtype=torch.float32, device=device)
    kth = torch.empty(1, dtype=torch.float32, device=device)
    pr = prior or make_prior()
    st = make_stream(seed, domain, series)
    _check(lib().abc_nearest_k(_dptr(dist), _dptr(theta), ctypes.byref(pr), ctypes.byref(st), n,
                               int(first), int(k), _dptr(out_idx), _dptr(out_th), _dptr(out_d),
                               _dptr(kth), _stream_handle()))
    return out_idx, out_th, out_d, kth


def nearest_k_rows(dist64: torch.Tensor, idx: torch.Tensor, theta: torch.Tensor, k: int,
                   device="cuda"):
    """k rows with the smallest (float64 distance, index), in index order."""
    n = int(dist64.shape[0])
    out_idx = torch.empty(k, dtype=torch.int64, device=device)
    out_th = torch.empty((k, 8), dtype=torch.float32, device=device)
    out_d = torch.empty(k, dtype=torch.float64, device=device)
    _check(lib().abc_nearest_k_rows(_dptr(dist64), _dptr(idx), _dptr(theta), n, int(k),
                                    _dptr(out_idx), _dptr(out_th), _dptr(out_d), _stream_handle()))
    return out_idx, out_th, out_d


def simulate_rows_f64(ser: DeviceSeries, seed: int, idx: torch.Tensor, theta: torch.Tensor, *,
                      domain: int = 1, series: int = 0, flags: int = 0, noise_scale: float = 1.0,
                      device="cuda") -> torch.Tensor:
    """Float64 distances of rows (sample idx[q], theta[q])."""
    n = int(idx.shape[0])
    out = torch.empty(n, dtype=torch.float64, device=device)
    st = make_stream(seed, domain, series)
    md = _Model(float(noise_scale), int(flags))
    cs = ser.c()
    _check(lib().abc_simulate_rows_f64(ctypes.byref(cs), ctypes.byref(md), ctypes.byref(st),
                                       _dptr(idx), _dptr(theta), n, _dptr(out), _stream_handle()))
    return out


def smc_config(n_particles: int, eps0: float, *, generations: int = 5, alpha: float = 0.5,
               eps_min: float = 0.0, band_w: float = 0.02, chunk0: int = 1 << 14,
               chunk_max: int = 1 << 20, max_samples: int = 1 << 34) -> _SmcConfig:
    return _SmcConfig(int(n_particles), int(generations), float(alpha), float(eps0), float(eps_min),
                      float(band_w), 0, int(chunk0), int(chunk_max), int(max_samples))


def _gen_stats(st: _SmcGenStats) -> dict:
    return {k: getattr(st, k) for k, _ in _SmcGenStats._fields_ if k != "pad"}


def smc_generation(ser: DeviceSeries, cfg: _SmcConfig, seed: int, gen: int, prev=None, *,
                   series: int = 0, flags: int = 0, noise_scale: float = 1.0,
                   prior: Optional[_Prior] = None, want_ancestors: bool = False, device="cuda"):
    """One ABC-SMC generation. prev = (theta [Np,8] f32, w [Np] f64, dist [Np] f64) device
    tensors for gen >= 1. Returns a dict of device tensors + the generation statistics."""
    N = cfg.n_particles
    out = {"idx": torch.empty(N, dtype=torch.int64, device=device),
           "theta": torch.empty((N, 8), dtype=torch.float32, device=device),
           "w": torch.empty(N, dtype=torch.float64, device=device),
           "dist": torch.empty(N, dtype=torch.float64, device=device),
           "ancestors": torch.empty(N, dtype=torch.int32, device=device) if want_ancestors else None}
    pt, pw, pd = prev if prev is not None else (None, None, None)
    np_ = 0 if prev is None else int(pt.shape[0])
    st = _SmcGenStats()
    pr = prior or make_prior()
    md = _Model(float(noise_scale), int(flags))
    cs = ser.c()
    _check(lib().abc_smc_generation(ctypes.byref(cs), ctypes.byref(md), ctypes.byref(pr), int(seed),
                                    int(series), int(gen), _dptr(pt), _dptr(pw), _dptr(pd), np_,
                                    ctypes.byref(cfg), _dptr(out["idx"]), _dptr(out["theta"]),
                                    _dptr(out["w"]), _dptr(out["dist"]), ctypes.byref(st),
                                    _dptr(out["ancestors"]), _stream_handle()))
    out["stats"] = _gen_stats(st)
    return out


def smc_run(ser: DeviceSeries, cfg: _SmcConfig, seed: int, *, series: int = 0, flags: int = 0,
            noise_scale: float = 1.0, prior: Optional[_Prior] = None, device="cuda"):
    """All generations of ABC-SMC; returns a list of per-generation dicts (views)."""
    G, N = cfg.generations, cfg.n_particles
    idx = torch.empty((G, N), dtype=torch.int64, device=device)
    th = torch.empty((G, N, 8), dtype=torch.float32, device=device)
    w = torch.empty((G, N), dtype=torch.float64, device=device)
    d = torch.empty((G, N), dtype=torch.float64, device=device)
    stats = (_SmcGenStats * G)()
    done = ctypes.c_int32(0)
    pr = prior or make_prior()
    md = _Model(float(noise_scale), int(flags))
    cs = ser.c()
    _check(lib().abc_smc_run(ctypes.byref(cs), ctypes.byref(md), ctypes.byref(pr), int(seed),
                             int(series), ctypes.byref(cfg), _dptr(idx), _dptr(th), _dptr(w), _dptr(d),
                             stats, ctypes.byref(done), _stream_handle()))
    return [{"idx": idx[t], "theta": th[t], "w": w[t], "dist": d[t], "stats": _gen_stats(stats[t])}
            for t in range(done.value)]


def set_refill_min(lanes: int):
    _check(lib().abc_set_refill_min(int(lanes)))


def get_refill_min() -> int:
    return int(lib().abc_get_refill_min())


def set_batch_margin(margin: int):
    """First target of batch_run's float32 accepts: quota + margin (0: default)."""
    _check(lib().abc_set_batch_margin(int(margin)))


def trajectory_bands(traj: torch.Tensor, quantiles=(0.05, 0.5, 0.95)) -> torch.Tensor:
    """Per-day, per-compartment quantiles [nq, T+1, 6] of trajectories [n, T+1, 6]."""
    n, T1, _ = traj.shape
    q = (ctypes.c_double * len(quantiles))(*quantiles)
    out = torch.empty((len(quantiles), T1, 6), dtype=torch.float32, device=traj.device)
    _check(lib().abc_trajectory_bands(_dptr(traj.contiguous()), int(n), int(T1 - 1), q,
                                      len(quantiles), _dptr(out), _stream_handle()))
    return out


def version() -> str:
    return lib().abc_version().decode()
