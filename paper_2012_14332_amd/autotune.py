"""Launch-shape autotuner for the float32 simulate kernels.

Sweeps samples per lane (SPL), workgroup size and resident workgroups per CU,
times each shape with HIP events on short runs of the real workload, and
keeps the fastest. Results never depend on the shape (every random number is
fixed by the sample's counter), so the tuner only trades speed. Choices are
cached as JSON per (device, kernel, T bucket) in $ABC_TUNE_CACHE (default
~/.cache/abc_mi355x/tune.json).
"""
from __future__ import annotations

import itertools
import json
import math
import os
from typing import Dict, List, Sequence, Tuple

import torch

from . import abc

SPL_PLAIN = (1, 2, 4, 8)
SPL_BATCH = (1, 2, 4)
BLOCKS = (64, 128, 256, 512, 1024)
PER_CU = (1, 2, 4, 8)


def cache_path() -> str:
    return os.environ.get("ABC_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "abc_mi355x", "tune.json"))


def _load() -> Dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, rec: Dict):
    data = _load()
    data[key] = rec
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(data, f, indent=1)
        os.replace(path + ".tmp", path)
    except OSError:
        pass  # a read-only home only loses the cache


def t_bucket(T: int) -> int:
    return 1 << max(5, math.ceil(math.log2(max(T, 1))))


def device_key() -> str:
    return torch.cuda.get_device_name(0).replace(" ", "_")


def shapes(spls: Sequence[int]) -> List[Tuple[int, int, int]]:
    return [(s, b, c) for s, b, c in itertools.product(spls, BLOCKS, PER_CU) if b <= 1024 // s]


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    best = math.inf
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune_plain(ser: abc.DeviceSeries, eps_exit: float, n: int = 4_000_000, seed: int = 1,
               reps: int = 3, use_cache: bool = True) -> Dict:
    """Fastest shape of the plain kernel on n samples of `ser` with early exit at eps_exit."""
    key = "%s|plain|T%d" % (device_key(), t_bucket(ser.T))
    if use_cache:
        rec = _load().get(key)
        if rec:
            abc.set_launch_config(*rec["shape"])
            return rec
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    table = []
    for sh in shapes(SPL_PLAIN):
        abc.set_launch_config(*sh)
        ms = _time(lambda: abc.simulate_distance(ser, n, seed, eps_exit=eps_exit, out=out), reps)
        table.append((ms, sh))
    table.sort()
    rec = {"shape": list(table[0][1]), "ms": table[0][0], "n": n,
           "table": [[round(ms, 4)] + list(sh) for ms, sh in table]}
    abc.set_launch_config(*rec["shape"])
    _store(key, rec)
    return rec


def tune_batch(sers, eps, seed: int = 1, quota: int = 1000, round_size: int = 1 << 22,
               rounds: int = 4, use_cache: bool = True) -> Dict:
    """Fastest shape of the batched kernel over `rounds` rounds of the real batch."""
    key = "%s|batch|T%d|m%d" % (device_key(), t_bucket(max(s.T for s in sers)), len(sers))
    if use_cache:
        rec = _load().get(key)
        if rec:
            abc.set_launch_config(*rec["shape"])
            return rec
    table = []
    for sh in shapes(SPL_BATCH):
        abc.set_launch_config(*sh)
        best = math.inf
        for _ in range(2):
            o = abc.batch_run(sers, eps, seed, quota, round_size=round_size,
                              max_samples=rounds * round_size // len(sers), rounds_per_graph=1,
                              cand_capacity=4096, check=False)
            if o["status"] not in (0, -5):
                best = math.inf
                break
            st = o["stats"]
            best = min(best, st["rounds_ms"] / max(st["rounds"], 1))
        table.append((best, sh))
    table.sort()
    if not math.isfinite(table[0][0]):
        raise abc.AbcError("autotune: no launch shape ran the batch")
    rec = {"shape": list(table[0][1]), "ms_per_round": table[0][0],
           "table": [[round(ms, 4)] + list(sh) for ms, sh in table]}
    abc.set_launch_config(*rec["shape"])
    _store(key, rec)
    return rec
