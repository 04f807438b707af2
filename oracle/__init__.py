"""FP64 CPU oracle for the rejection-ABC hot path (arXiv 2012.14332).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the HIP implementation in ``paper_2012_14332_amd`` and never imports it.

Layers:
  * ``abc_oracle.c`` (built to ``liboracle.so``): Philox4x32-10, the prior
    draw (eq. 2), the tau-leap model of Sec. 2.1 (eqs. 3-5) and the distance
    of Sec. 2.2, all in double precision, one trajectory at a time.
  * this module: ctypes bindings plus the accept rule (Sec. 2.2, eq. 7), the
    posterior moments and the pilot tolerance, in numpy float64.
  * ``pyref.py``: a pure-Python re-statement of the same definitions, used
    only to cross-check the C code on tiny inputs.
  * ``mdn.py``: the float64 numpy reference of the mixture-density proposal.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "abc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Paper prior, eq. (2): U(0, [1, 100, 2, 1, 1, 1, 1, 2]) over
# theta = [alpha0, alpha, n, beta, gamma, delta, eta, kappa] (eq. 1).
PRIOR_LO = np.zeros(8, dtype=np.float32)
PRIOR_HI = np.array([1, 100, 2, 1, 1, 1, 1, 2], dtype=np.float32)

DOMAIN_OBS = 0
DOMAIN_ABC = 1


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class Model(ctypes.Structure):
    """Mirror of ``oracle_model`` in abc_oracle.c."""

    _fields_ = [
        ("P", ctypes.c_int64),
        ("A0", ctypes.c_int64),
        ("R0", ctypes.c_int64),
        ("D0", ctypes.c_int64),
        ("T", ctypes.c_int32),
        ("noise_mode", ctypes.c_int32),
        ("dist_mode", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("noise_scale", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        u64, u32, i64, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_void_p
        _lib.oracle_philox.argtypes = [p, p, i64, p]
        _lib.oracle_stream_words.argtypes = [u64, u32, u32, u64, u32, u32, p]
        _lib.oracle_prior.argtypes = [p, p, u64, u32, u32, u64, i64, p]
        _lib.oracle_normals.argtypes = [u64, u32, u32, u64, u32, p]
        _lib.oracle_trajectory.argtypes = [ctypes.POINTER(Model), p, u64, u32, u32, u64, p, p]
        _lib.oracle_trajectory.restype = ctypes.c_double
        _lib.oracle_distances.argtypes = [ctypes.POINTER(Model), p, p, p, u64, u32, u32, u64,
                                          i64, p, p]
        _lib.oracle_record.argtypes = [ctypes.POINTER(Model), p, u64, u32, u32, u64, i64, p]
        _lib.oracle_num_threads.restype = ctypes.c_int
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def make_model(P, T, A0=100, R0=0, D0=0, noise_scale=1.0, noise_mode=0, dist_mode=0) -> Model:
    return Model(int(P), int(A0), int(R0), int(D0), int(T), int(noise_mode), int(dist_mode), 0,
                 float(noise_scale))


# ----------------------------------------------------------------------------
# Random numbers
# ----------------------------------------------------------------------------

def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Philox4x32-10 of counters [n,4] under keys [n,2] (uint32) -> [n,4]."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.empty_like(ctr)
    lib().oracle_philox(_ptr(ctr), _ptr(key), ctr.shape[0], _ptr(out))
    return out


def stream_words(seed, domain, series, sample, day, block) -> np.ndarray:
    w = np.empty(4, dtype=np.uint32)
    lib().oracle_stream_words(seed, domain, series, sample, day, block, _ptr(w))
    return w


def normals(seed, domain, series, sample, day) -> np.ndarray:
    z = np.empty(5, dtype=np.float64)
    lib().oracle_normals(seed, domain, series, sample, day, _ptr(z))
    return z


# ----------------------------------------------------------------------------
# Prior, model, distance
# ----------------------------------------------------------------------------

def prior(n, seed, domain=DOMAIN_ABC, series=0, first=0, lo=PRIOR_LO, hi=PRIOR_HI) -> np.ndarray:
    """theta [n,8] float32 drawn from U(lo, hi) (eq. 2) on the stated stream."""
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    hi = np.ascontiguousarray(hi, dtype=np.float32)
    th = np.empty((int(n), 8), dtype=np.float32)
    lib().oracle_prior(_ptr(lo), _ptr(hi), seed, domain, series, first, int(n), _ptr(th))
    return th


def trajectory(model: Model, theta, seed, domain=DOMAIN_ABC, series=0, sample=0, obs=None):
    """(traj [(T+1),6] int64 of S,I,A,R,D,Ru; distance or None)."""
    th = np.ascontiguousarray(theta, dtype=np.float32).reshape(8)
    traj = np.empty((model.T + 1, 6), dtype=np.int64)
    ob = None if obs is None else np.ascontiguousarray(obs, dtype=np.int32).reshape(3, model.T)
    d = lib().oracle_trajectory(ctypes.byref(model), _ptr(th), seed, domain, series, sample,
                                _ptr(ob), _ptr(traj))
    return traj, (None if obs is None else d)


def record(model: Model, theta, seed, domain=DOMAIN_ABC, series=0, first=0) -> np.ndarray:
    """Trajectories [n, T+1, 6] int64 for theta [n,8]."""
    th = np.ascontiguousarray(theta, dtype=np.float32).reshape(-1, 8)
    out = np.empty((th.shape[0], model.T + 1, 6), dtype=np.int64)
    lib().oracle_record(ctypes.byref(model), _ptr(th), seed, domain, series, first, th.shape[0],
                        _ptr(out))
    return out


def observe(model: Model, theta_true, seed, series=0, sample=0) -> np.ndarray:
    """Synthetic observed series [3,T] int32 (A,R,D, days 1..T) from one run at theta_true
    on the observation stream (domain 0)."""
    traj, _ = trajectory(model, theta_true, seed, DOMAIN_OBS, series, sample)
    return np.ascontiguousarray(traj[1:, 2:5].T.astype(np.int32))


def distances(model: Model, obs, seed, n, first=0, series=0, theta=None, domain=DOMAIN_ABC,
              lo=PRIOR_LO, hi=PRIOR_HI) -> np.ndarray:
    """Distance (Sec. 2.2) of samples first..first+n-1; theta [n,8] or None (prior draw)."""
    ob = np.ascontiguousarray(obs, dtype=np.int32).reshape(3, model.T)
    th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float32).reshape(-1, 8)
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    hi = np.ascontiguousarray(hi, dtype=np.float32)
    out = np.empty(int(n), dtype=np.float64)
    lib().oracle_distances(ctypes.byref(model), _ptr(th), _ptr(lo), _ptr(hi), seed, domain,
                           series, first, int(n), _ptr(ob), _ptr(out))
    return out


# ----------------------------------------------------------------------------
# Accept rule, tolerance, moments (numpy float64)
# ----------------------------------------------------------------------------

def accept(dist, eps) -> np.ndarray:
    """Indices (ascending) of samples with dist <= eps (Sec. 2.2, eq. 7)."""
    return np.nonzero(np.asarray(dist) <= eps)[0]


def nearest(dist, k) -> np.ndarray:
    """Indices of the k smallest distances; ties go to the lower index."""
    d = np.asarray(dist)
    order = np.lexsort((np.arange(d.size), d))
    return np.sort(order[:k])


def pilot_eps(dist, q) -> float:
    """Tolerance that a fraction q of the pilot samples fall under: the
    ceil(q*n)-th smallest pilot distance."""
    d = np.sort(np.asarray(dist, dtype=np.float64))
    k = max(1, int(np.ceil(q * d.size)))
    return float(d[k - 1])


def first_accepted(dist, eps, quota) -> np.ndarray:
    """The first `quota` accepted sample indices in index order."""
    return accept(dist, eps)[:quota]


def moments(theta, weight=None):
    """Posterior mean [8] and covariance [8,8] of accepted theta in float64.

    Unweighted: the unbiased (n-1) sample covariance. Weighted (importance
    weights w): mean = sum w theta / V1, cov = sum w (theta-mean)(theta-mean)^T
    / (V1 - V2/V1) with V1 = sum w, V2 = sum w^2 (reliability weights).
    Plain two-pass definition: mean first, then centred products.
    """
    th = np.asarray(theta, dtype=np.float64).reshape(-1, 8)
    w = np.ones(th.shape[0]) if weight is None else np.asarray(weight, dtype=np.float64)
    v1 = w.sum()
    v2 = (w * w).sum()
    mean = (w[:, None] * th).sum(axis=0) / v1
    c = th - mean
    cov = (w[:, None, None] * c[:, :, None] * c[:, None, :]).sum(axis=0) / (v1 - v2 / v1)
    return mean, cov
