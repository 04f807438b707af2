"""The launch-shape autotuner: its sweep space and JSON cache on the CPU, and
on the GPU that it picks a shape from that space, caches it per key, and --
since every random number is fixed by the sample's counter -- that the tuned
shape changes no result."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2012_14332_amd import autotune
from paper_2012_14332_amd import workloads as W


def test_shapes_fit_the_workgroup_limit():
    for spls in (autotune.SPL_PLAIN, autotune.SPL_BATCH):
        sh = autotune.shapes(spls)
        assert sh and len(set(sh)) == len(sh)
        assert all(b * s <= 1024 and s in spls and c in autotune.PER_CU for s, b, c in sh)
        # every admissible combination is swept
        want = {(s, b, c) for s in spls for b in autotune.BLOCKS for c in autotune.PER_CU
                if b * s <= 1024}
        assert set(sh) == want


def test_t_buckets_are_powers_of_two_from_32():
    assert [autotune.t_bucket(T) for T in (1, 32, 33, 49, 64, 100, 200, 1024)] == \
        [32, 32, 64, 64, 64, 128, 256, 1024]


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("ABC_TUNE_CACHE", str(tmp_path / "sub" / "tune.json"))
    assert autotune._load() == {}
    autotune._store("a", {"shape": [1, 512, 2], "refill": 8})
    autotune._store("b", {"shape": [2, 256, 4], "refill": 16})
    data = autotune._load()
    assert data["a"]["shape"] == [1, 512, 2] and data["b"]["refill"] == 16
    (tmp_path / "sub" / "tune.json").write_text("{not json")
    assert autotune._load() == {}          # a damaged cache is ignored, not fatal


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_14332_amd import abc

    abc.lib()
    yield abc
    abc.set_launch_config(0, 0, 0)
    abc.set_refill_min(0)


@pytest.mark.gpu
def test_tune_plain_picks_a_swept_shape_and_changes_no_result(A, tmp_path, monkeypatch):
    monkeypatch.setenv("ABC_TUNE_CACHE", str(tmp_path / "tune.json"))
    s = W.three_countries()[1]
    obs = oracle.observe(oracle.make_model(s.P, s.T), s.theta_true, s.obs_seed)
    ser = A.DeviceSeries(s.P, s.T, torch.from_numpy(obs))
    A.set_launch_config(0, 0, 0)
    A.set_refill_min(0)
    full = A.simulate_distance(ser, 200_003, 4).cpu().numpy()
    eps = float(np.quantile(full, 0.01))
    ref = A.simulate_distance(ser, 200_003, 4, eps_exit=eps).cpu().numpy()
    rec = autotune.tune_plain(ser, eps, n=200_000, reps=1, use_cache=True)
    assert tuple(rec["shape"]) in autotune.shapes(autotune.SPL_PLAIN)
    assert rec["refill"] in autotune.REFILL
    assert A.get_launch_config() == tuple(rec["shape"]) and A.get_refill_min() == rec["refill"]
    np.testing.assert_array_equal(A.simulate_distance(ser, 200_003, 4, eps_exit=eps).cpu().numpy(),
                                  ref)
    # a second call is served from the cache
    A.set_launch_config(0, 0, 0)
    again = autotune.tune_plain(ser, eps, n=200_000, reps=1, use_cache=True)
    assert again == rec and A.get_launch_config() == tuple(rec["shape"])
    # full trajectories of the raw distance are a key of their own
    raw = autotune.tune_plain(ser, math.inf, n=200_000, reps=1, use_cache=True, flags=A.ABC_DIST_RAW)
    assert len(autotune._load()) == 2 and tuple(raw["shape"]) in autotune.shapes(autotune.SPL_PLAIN)


@pytest.mark.gpu
def test_tune_batch_changes_no_result(A, tmp_path, monkeypatch):
    monkeypatch.setenv("ABC_TUNE_CACHE", str(tmp_path / "tune.json"))
    ss = W.uneven_series(64, 5)[:4]
    sers = [A.DeviceSeries(s.P, s.T, torch.from_numpy(
        oracle.observe(oracle.make_model(s.P, s.T), s.theta_true, s.obs_seed, series=s.series_id)))
        for s in ss]
    eps = []
    for j, (s, ser) in enumerate(zip(ss, sers)):
        d = A.simulate_distance(ser, 100_000, 9, series=j).cpu().numpy()
        eps.append(float(np.quantile(d, 2e-3)))
    A.set_launch_config(0, 0, 0)
    A.set_refill_min(0)
    kw = dict(round_size=1 << 18, series_ids=list(range(4)))
    ref = A.batch_run(sers, eps, 3, 50, **kw)
    rec = autotune.tune_batch(sers, eps, seed=3, quota=50, round_size=1 << 18, rounds=2,
                              use_cache=False)
    assert tuple(rec["shape"]) in autotune.shapes(autotune.SPL_BATCH)
    got = A.batch_run(sers, eps, 3, 50, **kw)
    for k in ("idx", "theta", "count", "used"):
        np.testing.assert_array_equal(got[k].cpu().numpy(), ref[k].cpu().numpy(), err_msg=k)


@pytest.mark.gpu
def test_tune_round_size_picks_a_swept_size_and_changes_no_result(A, tmp_path, monkeypatch):
    """The round-size sweep keeps one of its sizes and caches it; every size
    yields the same accepted rows (each series' first accepts by index)."""
    monkeypatch.setenv("ABC_TUNE_CACHE", str(tmp_path / "tune.json"))
    ss = W.uneven_series(64, 5)[:4]
    sers = [A.DeviceSeries(s.P, s.T, torch.from_numpy(
        oracle.observe(oracle.make_model(s.P, s.T), s.theta_true, s.obs_seed, series=s.series_id)))
        for s in ss]
    eps = []
    for j, (s, ser) in enumerate(zip(ss, sers)):
        d = A.simulate_distance(ser, 100_000, 9, series=j).cpu().numpy()
        eps.append(float(np.quantile(d, 2e-3)))
    A.set_launch_config(0, 0, 0)
    A.set_refill_min(0)
    sizes = (1 << 16, 1 << 18, 1 << 20)
    rec = autotune.tune_round_size(sers, eps, seed=3, quota=50, sizes=sizes, reps=1,
                                   series_ids=list(range(4)))
    assert rec["round_size"] in sizes and sorted(r[1] for r in rec["table"]) == list(sizes)
    assert rec["ms"] == min(r[0] for r in rec["table"])
    assert autotune.tune_round_size(sers, eps, seed=3, quota=50, sizes=sizes) == rec  # cached
    outs = [A.batch_run(sers, eps, 3, 50, round_size=rs, series_ids=list(range(4))) for rs in sizes]
    for o in outs[1:]:
        for k in ("idx", "theta", "count"):
            np.testing.assert_array_equal(o[k].cpu().numpy(), outs[0][k].cpu().numpy(), err_msg=k)
