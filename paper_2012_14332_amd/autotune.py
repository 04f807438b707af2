"""Launch-shape autotuner for the float32 simulate kernels.

Sweeps samples per lane (SPL), workgroup size and resident workgroups per CU,
then the lane-refill threshold at the best shape, times each setting with HIP
events on short runs of the real workload, and keeps the fastest; for the
batched quota run it also picks the round size from whole timed runs. Results
never depend on these choices (every random number is fixed by the sample's
counter, and each series keeps its first accepts by sample index), so the
tuner only trades speed. Choices are cached as JSON per (device, kernel,
T bucket) in $ABC_TUNE_CACHE (default ~/.cache/abc_mi355x/tune.json).
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
SPL_BATCH = (1, 2, 4, 8)
BLOCKS = (64, 128, 256, 512, 1024)
PER_CU = (1, 2, 4, 8)
REFILL = (1, 4, 8, 16, 24)
ROUND_SIZES = (1 << 21, 1 << 22, 1 << 23, 1 << 24, 1 << 25)


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
               reps: int = 3, use_cache: bool = True, flags: int = 0) -> Dict:
    """Fastest shape of the plain kernel on n samples of `ser` with early exit at
    eps_exit (model flags `flags`)."""
    key = "%s|plain|T%d|f%d|%s" % (device_key(), t_bucket(ser.T), flags,
                                   "exit" if math.isfinite(eps_exit) else "full")
    if use_cache:
        rec = _load().get(key)
        if rec and "refill" in rec:
            _apply(rec)
            return rec
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    run = lambda: abc.simulate_distance(ser, n, seed, eps_exit=eps_exit, flags=flags, out=out)
    table = []
    for sh in shapes(SPL_PLAIN):
        abc.set_launch_config(*sh)
        table.append((_time(run, reps), sh))
    table.sort()
    abc.set_launch_config(*table[0][1])
    rtable = []
    for lanes in REFILL:
        abc.set_refill_min(lanes)
        rtable.append((_time(run, reps), lanes))
    rtable.sort()
    rec = {"shape": list(table[0][1]), "refill": rtable[0][1], "ms": rtable[0][0], "n": n,
           "table": [[round(ms, 4)] + list(sh) for ms, sh in table],
           "refill_table": [[round(ms, 4), lanes] for ms, lanes in rtable]}
    _apply(rec)
    _store(key, rec)
    return rec


def _apply(rec: Dict):
    abc.set_launch_config(*rec["shape"])
    abc.set_refill_min(rec.get("refill", 0))


def tune_batch(sers, eps, seed: int = 1, quota: int = 1000, round_size: int = 1 << 22,
               rounds: int = 4, use_cache: bool = True, **run_kw) -> Dict:
    """Fastest shape of the batched kernel over `rounds` rounds of the real batch.
    run_kw goes to abc.batch_run (mix, lam, inflate: the learned proposal's
    round kernel, which is tuned and cached separately)."""
    key = "%s|batch|T%d|m%d%s" % (device_key(), t_bucket(max(s.T for s in sers)), len(sers),
                                  "|mix" if run_kw.get("mix") is not None else "")
    if use_cache:
        rec = _load().get(key)
        if rec and "refill" in rec:
            _apply(rec)
            return rec

    def per_round() -> float:
        best = math.inf
        for _ in range(2):
            o = abc.batch_run(sers, eps, seed, quota, round_size=round_size,
                              max_samples=rounds * round_size // len(sers), rounds_per_graph=1,
                              cand_capacity=4096, check=False, **run_kw)
            if o["status"] not in (0, -5):
                return math.inf
            st = o["stats"]
            best = min(best, st["rounds_ms"] / max(st["rounds"], 1))
        return best

    table = []
    for sh in shapes(SPL_BATCH):
        abc.set_launch_config(*sh)
        table.append((per_round(), sh))
    table.sort()
    if not math.isfinite(table[0][0]):
        raise abc.AbcError("autotune: no launch shape ran the batch")
    abc.set_launch_config(*table[0][1])
    rtable = []
    for lanes in REFILL:
        abc.set_refill_min(lanes)
        rtable.append((per_round(), lanes))
    rtable.sort()
    rec = {"shape": list(table[0][1]), "refill": rtable[0][1], "ms_per_round": rtable[0][0],
           "table": [[round(ms, 4)] + list(sh) for ms, sh in table],
           "refill_table": [[round(ms, 4), lanes] for ms, lanes in rtable]}
    _apply(rec)
    _store(key, rec)
    return rec


def tune_round_size(sers, eps, seed: int = 1, quota: int = 1000,
                    sizes: Sequence[int] = ROUND_SIZES, reps: int = 2, use_cache: bool = True,
                    **run_kw) -> Dict:
    """Round size of the batched quota run, at the launch shape in force.
    Larger rounds pay the per-round tail (lanes idle at the end of a round)
    less often but simulate more samples past each series' quota; the fastest
    whole quota run wins. run_kw goes to abc.batch_run."""
    key = "%s|round|T%d|m%d|q%d%s" % (device_key(), t_bucket(max(s.T for s in sers)), len(sers),
                                      quota, "|mix" if run_kw.get("mix") is not None else "")
    if use_cache:
        rec = _load().get(key)
        if rec and "round_size" in rec:
            return rec
    table = []
    for rs in sizes:
        best, used = math.inf, 0
        for _ in range(reps):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            o = abc.batch_run(sers, eps, seed, quota, round_size=rs, **run_kw)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            if ms < best:
                best, used = ms, int(o["used"].sum().item())
        table.append((best, int(rs), used))
    table.sort()
    rec = {"round_size": table[0][1], "ms": round(table[0][0], 3),
           "table": [[round(ms, 3), rs, used] for ms, rs, used in table]}
    _store(key, rec)
    return rec
