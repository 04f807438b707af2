#!/usr/bin/env python3
"""Benchmark of the plain rejection-ABC hot path on one MI355X.

Workload (one step): three synthetic countries run separately -- P = 6e7,
8.3e7, 3.3e8 with T = 49, 72, 100 days, observed series from one model run
at the Italy / New Zealand / USA parameter averages (observation seeds 2-4)
-- 1e7 fresh prior samples per country per step at a fixed eps, the
distance that a fraction 1e-4 of a 1e5-sample pilot falls under. Per country
and step: float32 simulate+distance with the prior drawn in-kernel and early
exit, ballot compaction, float64 decision of the borderline band, float64
posterior mean/covariance. Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "accepted ABC samples/s at fixed ε (sim-days/s, VALU %); plain vs learned proposal"
# Algorithmic work of the float32 simulate kernel, counted class by class in
# its gfx950 assembly (the blocks of one simulated day, and the block that
# prepares one sample in a wave's ring). One simulated day: 158 VALU
# instructions -- 22 transcendental, 16 v_mad_u64_u32 (Philox), 18
# conversions, 54 integer/bit, 15 FMA, 16 multiplies, 5 adds, 8
# compares/selects, 4 moves -- not counting the 10 of the lower-bound lookup
# (an optimisation, not the method's work). One sample: 120 (the prior draw's
# two Philox calls, theta, the rates, the initial state, the hoisted Philox
# words; 13 register moves not counted).
FP32_FLOP_PER_SAMPLE_DAY = 73     # FMA 2, add / multiply / transcendental 1
FP32_FLOP_PER_SAMPLE = 25
# VALU issue in instruction slots: a SIMD issues one wave64 VALU instruction
# per quad-cycle. A transcendental occupies its wave for 2 quad-cycles (a
# single-wave probe: v_log/v_exp/v_sqrt/v_rcp/v_sin 2.0, v_fma_f32 and
# v_mad_u64_u32 1.0), but with several waves per SIMD other waves issue
# beside it (SQ_ACTIVE_INST_VALU, which counts it twice, exceeds the SIMD's
# quad-cycles at eight waves per SIMD), so the issue model counts every
# instruction once and the transcendental unit as a resource of its own.
ISSUE_PER_SAMPLE_DAY = 158
ISSUE_PER_SAMPLE = 120
# The batched round kernel's day step has no bound lookup either.
BATCH_ISSUE_PER_SAMPLE_DAY = ISSUE_PER_SAMPLE_DAY
# Issue peak in lane-instructions/s: 256 CUs x 4 SIMDs x 64 lanes x 2.4e9 / 4.
ISSUE_PEAK_T = 256 * 4 * 64 * 2.4e9 / 4 / 1e12
FP32_PEAK_TFLOPS = 157.3
SIM_SOURCES = ["paper_2012_14332_amd/csrc/simulate.hip", "paper_2012_14332_amd/csrc/multi.hip",
               "paper_2012_14332_amd/csrc/bound.hpp", "paper_2012_14332_amd/csrc/model.hpp",
               "paper_2012_14332_amd/csrc/philox.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_simulate_multi_f32_traffic.json")


def note(text):
    """Progress line on stderr (the JSON result is the only line on stdout)."""
    print("bench: " + text, file=sys.stderr, flush=True)


def sim_source_hash():
    h = hashlib.sha256()
    for p in SIM_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per launch of the simulate kernel from the committed PMC
    summary, or None when the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != sim_source_hash():
        return None
    return rec.get("bytes_per_launch")


VALU_FILE = os.path.join(ROOT, "profiles", "k_simulate_multi_f32_valu.json")


def valu_counters():
    """VALU counters of the simulate kernel from the committed PMC summary
    (busy fraction, lane utilisation, counter FP32 FLOP per sample-day), or
    None when the kernel sources changed since they were taken."""
    try:
        with open(VALU_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != sim_source_hash():
        return None
    return {k: v for k, v in rec.items() if k != "source_hash"}


def cpu_baseline(countries, eps, first, n_sample, reps=3):
    """The FP64 oracle on the host cores, on the first n_sample indices of each
    country's main range, at the same eps; `reps` runs, the median reported."""
    import numpy as np

    import oracle

    models = []
    for s in countries:
        m = oracle.make_model(s.P, s.T)
        models.append((m, oracle.observe(m, s.theta_true, s.obs_seed, series=s.series_id)))
    runs = []
    for r in range(reps):
        t_total = 0.0
        acc = 0
        days = 0
        for c, ((m, obs), s, e) in enumerate(zip(models, countries, eps)):
            t0 = time.perf_counter()
            d = oracle.distances(m, obs, seed=1, n=n_sample, first=first, series=c)
            t_total += time.perf_counter() - t0
            acc += int(np.sum(d <= e))
            days += n_sample * s.T
        runs.append((acc / t_total, t_total, acc, days))
    rates = [r[0] for r in runs]
    med = sorted(runs, key=lambda r: r[0])[len(runs) // 2]
    return {
        "value": float(np.median(rates)),
        "unit": "accepted samples/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": "%d prior samples of each country (indices %d..%d), same eps; %d accepted in "
                  "%.2f s (median of %d runs); %.3e trajectories/s, %.3e sample-days/s (no early "
                  "exit)" % (n_sample, first, first + n_sample - 1, med[2], med[1], reps,
                             3 * n_sample / med[1], med[3] / med[1]),
        "runs_accepted_per_s": [round(x, 2) for x in rates],
    }


def single_country_leg(args):
    """The single-country workload: 1e5 prior samples of the P = 1e7, T = 49
    series, the 100 nearest kept (float32 simulation of every day, device
    nearest-k, float64 decision of the band around the 100th distance,
    float64 moments). Timed per run on the host clock around device
    synchronisation, median and IQR of the repetitions."""
    import numpy as np
    import torch

    from paper_2012_14332_amd import pipeline as PL
    from paper_2012_14332_amd import workloads as W

    s = W.single_country()
    ser = PL.observed_series(s)
    n, k = 100_000, 100
    run = PL.NearestABC(ser, 1, n, k)
    res = run.run(0)  # warm-up; also the run the parity tests check
    ms = []
    for r in range(max(args.reps, 10)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = run.run((r + 1) * n)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    med = float(np.median(ms))
    return {
        "workload": "%s: %d prior samples, the %d nearest kept (float64 decision)" % (s.name, n, k),
        "ms_per_run_median": med,
        "ms_per_run_iqr": [float(np.percentile(ms, 25)), float(np.percentile(ms, 75))],
        "runs": len(ms),
        "kept_per_s": k / (med * 1e-3),
        "trajectories_per_s": n / (med * 1e-3),
        "sim_days_per_s": n * s.T / (med * 1e-3),
        "float64_rows_last_run": int(res.candidates),
    }


def batched_leg(args):
    """The 64-uneven-series workload: one persistent launch per round of 2^22
    samples, rounds planned on the device and overlapping on two streams,
    until every series has 1000 accepted samples; launch shape from the
    autotuner."""
    import numpy as np
    import torch

    from paper_2012_14332_amd import abc, autotune
    from paper_2012_14332_amd import pipeline as PL
    from paper_2012_14332_amd import workloads as W

    ss = W.uneven_series(64, 5)
    sers = [PL.observed_series(s) for s in ss]
    eps = [PL.pilot_eps(ser, 2, n=args.pilot, q=args.q, series=j) for j, ser in enumerate(sers)]
    tune = autotune.tune_batch(sers, eps, seed=2, quota=args.quota, round_size=1 << 22,
                               use_cache=False)
    runs = []
    for rep in range(args.batch_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = abc.batch_run(sers, eps, 2, args.quota, round_size=1 << 22, rounds_per_graph=4,
                          cand_capacity=4 * args.quota)
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t0, o))
    wall, o = min(runs, key=lambda r: r[0])
    st = o["stats"]
    acc = int(o["count"].sum().item())
    used = int(o["used"].sum().item())
    nominal = int(sum(int(o["used"][j].item()) * s.T for j, s in enumerate(ss)))
    # the same quota run with the round size the autotuner picks from whole
    # timed runs (the workload above fixes 2^22); the accepted sets are the same
    rt = autotune.tune_round_size(sers, eps, seed=2, quota=args.quota, use_cache=False,
                                  cand_capacity=4 * args.quota)
    truns = []
    for rep in range(args.batch_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ot = abc.batch_run(sers, eps, 2, args.quota, round_size=rt["round_size"],
                           rounds_per_graph=4, cand_capacity=4 * args.quota)
        torch.cuda.synchronize()
        truns.append((time.perf_counter() - t0, ot))
    twall, ot = min(truns, key=lambda r: r[0])
    same = all(torch.equal(ot[k], o[k]) for k in ("idx", "count"))
    tuned_round = {"round_size": rt["round_size"],
                   "accepted_per_s": int(ot["count"].sum().item()) / twall, "wall_s": twall,
                   "samples": int(ot["used"].sum().item()), "rounds": ot["stats"]["rounds"],
                   "same_accepted_sets": bool(same),
                   "table_ms_round_samples": rt["table"]}
    return {
        "workload": "64 synthetic series, T uniform in [30,200], P log-uniform in [1e5,1e9], "
                    "theta_true from the prior (seed 5); eps_j = 1e-4 pilot quantile; rounds of "
                    "2^22 samples until every series has %d accepted" % args.quota,
        "accepted_per_s": acc / wall,
        "wall_s": wall,
        "accepted": acc,
        "samples": used,
        "trajectories_per_s": used / wall,
        "sim_days_per_s_effective": st["sample_days"] / wall,
        "sim_days_per_s_nominal": nominal / wall,
        "rounds": st["rounds"],
        "graph_replays": st["graph_replays"],
        "rounds_ms": st["rounds_ms"],
        # algorithmic VALU issue (lane-instructions) of the round kernels over the
        # replays' wall time (host waits between replays included, so a lower
        # bound on the kernel's own fraction)
        "issue_frac_rounds_lower_bound": (BATCH_ISSUE_PER_SAMPLE_DAY * st["sample_days"] +
                                          ISSUE_PER_SAMPLE * used) /
                                         (st["rounds_ms"] * 1e-3) / (ISSUE_PEAK_T * 1e12),
        "refill_min": tune.get("refill"),
        "rechecked_fp64": st["rechecked"],
        "autotuned_round": tuned_round,
        "launch_shape": [st["spl"], st["block"], st["grid"]],
        "lds_bytes": st["lds_bytes"],
        "autotune_best_ms_per_round": tune["ms_per_round"],
        "autotune_top": tune["table"][:5],
        "reps": [round(r[0], 4) for r in runs],
        "_eps": eps,
        "_used": [int(x) for x in o["used"].cpu().numpy()],
    }


def learned_leg(args, batched):
    """Learned proposal: 1e6 (theta, x) pairs from the prior, the mixture-density
    network trained 20 epochs (Adam, lr 1e-3, batch 4096) on the GPU, then
    importance-weighted ABC on the same 64 series at the same eps, compared
    with plain ABC (the batched leg's run) on accepted samples/s, effective
    sample size and the posterior mean/sd criterion."""
    import numpy as np
    import torch

    from paper_2012_14332_amd import abc, autotune
    from paper_2012_14332_amd import pipeline as PL
    from paper_2012_14332_amd import workloads as W

    net, log, steps, train_ms, data_ms = PL.train_proposal(
        n_pairs=args.mdn_pairs, epochs=args.mdn_epochs, batch=4096, lr=1e-3, seed=6)
    log = log.cpu().numpy()
    ss = W.uneven_series(64, 5)
    sers = [PL.observed_series(s) for s in ss]
    eps = batched["_eps"]
    # one forward pass for all 64 observed series
    torch.cuda.synchronize()
    tf0 = time.perf_counter()
    feats = torch.stack([abc.series_features(ser) for ser in sers])
    mix = net.forward(feats).contiguous()
    torch.cuda.synchronize()
    train_total_s = (data_ms + train_ms) * 1e-3 + (time.perf_counter() - tf0)
    Q = args.quota
    kw = dict(round_size=1 << 22, rounds_per_graph=4, cand_capacity=4 * Q, mix=mix, lam=args.lam,
              inflate=args.inflate)
    # the proposal's round kernel has its own register budget: tune its shape
    # too, and give the plain kernels their shape back afterwards
    prev_shape, prev_refill = abc.get_launch_config(), abc.get_refill_min()
    tune = autotune.tune_batch(sers, eps, seed=2, quota=Q, round_size=1 << 22, use_cache=False,
                               mix=mix, lam=args.lam, inflate=args.inflate)
    abc.batch_run(sers, eps, 2, Q, **kw)  # warm-up (scratch, code paths)
    walls = []
    for rep in range(args.batch_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lb = abc.batch_run(sers, eps, 2, Q, **kw)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    wall = min(walls)
    acc = int(lb["count"].clamp(max=Q).sum().item())
    # the same run with the round size the autotuner picks (the workload fixes 2^22)
    rt = autotune.tune_round_size(sers, eps, seed=2, quota=Q, use_cache=False,
                                  **{k: v for k, v in kw.items() if k != "round_size"})
    twalls = []
    for rep in range(args.batch_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lt = abc.batch_run(sers, eps, 2, Q, **dict(kw, round_size=rt["round_size"]))
        torch.cuda.synchronize()
        twalls.append(time.perf_counter() - t0)
    tacc_s = int(lt["count"].clamp(max=Q).sum().item()) / min(twalls)
    plain_t = batched["autotuned_round"]["accepted_per_s"]
    tuned_round = {"round_size": rt["round_size"], "accepted_per_s": tacc_s,
                   "wall_s": min(twalls), "plain_accepted_per_s_tuned_round": plain_t,
                   "gain_accepted_per_s": tacc_s / plain_t,
                   "same_accepted_sets": bool(torch.equal(lt["idx"], lb["idx"]) and
                                              torch.equal(lt["count"], lb["count"])),
                   "table_ms_round_samples": rt["table"]}
    w = lb["w"].double().cpu().numpy()
    ess_series = w.sum(1) ** 2 / (w * w).sum(1)
    ess = float(ess_series.sum())
    used = lb["used"].cpu().numpy()
    samples = int(used.sum())
    # posterior comparison against plain ABC at the same eps: both sides pool
    # runs of Qc accepted per series on further seeds until the learned ESS is
    # >= 1e4 and the 5 % criterion is resolved at four standard errors (the
    # posteriors of some series are heavy-tailed, so their sds need far more
    # samples than 1e4 to be known to 5 %)
    Qc = args.compare_quota
    # candidates (d <= eps (1 + w)) per accept can approach 2 where the
    # distance distribution is steep near eps: 4x headroom, within the 8192
    # rows the finalisation sorts in LDS
    cap_c = min(4 * Qc, 8192)

    def sampler(runs_kw):
        def run(seed, idxs):
            o = abc.batch_run([sers[j] for j in idxs], [eps[j] for j in idxs], seed, Qc,
                              series_ids=idxs, round_size=1 << 22, cand_capacity=cap_c,
                              **({k: (v[idxs].contiguous() if k == "mix" else v)
                                  for k, v in runs_kw.items()}))
            th = o["theta"].cpu().numpy().astype(np.float64)
            w = (o["w"].double().cpu().numpy() if "w" in o else np.ones((len(idxs), Qc)))
            return th, w
        return run

    torch.cuda.synchronize()
    tc0 = time.perf_counter()
    cmp_ = PL.compare_posteriors(sers, eps, sampler({}),
                                 sampler(dict(mix=mix, lam=args.lam, inflate=args.inflate)),
                                 quota=Qc, seeds_a=args.compare_seeds_plain,
                                 seeds_b=args.compare_seeds_learned, max_runs=args.compare_max_runs,
                                 time_limit_s=args.compare_time_s, progress=note)
    compare_s = time.perf_counter() - tc0
    worst_mu = np.array([r["mean_ratio"] for r in cmp_])
    worst_sd = np.array([r["sd_ratio"] for r in cmp_])
    ok_mu = np.array([r["mean_ok"] for r in cmp_])
    ok_sd = np.array([r["sd_ok"] for r in cmp_])
    ess_c = np.array([r["ess_b"] for r in cmp_])
    pn = np.array([r["ess_a"] for r in cmp_])
    gains = [(Q / u) / (Q / pu) for u, pu in zip(used, batched["_used"])]
    net.close()
    abc.set_launch_config(*prev_shape)
    abc.set_refill_min(prev_refill)
    return {
        "workload": "1e6 training pairs (T ~ U[30,200], P log-uniform [1e5,1e9], theta from the "
                    "prior), 20 epochs Adam lr 1e-3 batch 4096 (BF16 MFMA, FP32 accumulation); "
                    "importance-weighted ABC on the 64 uneven series at the batched leg's eps, "
                    "quota %d each; defensive weight %.2f, proposal sd x%.1f" % (Q, args.lam, args.inflate),
        "train_steps": steps,
        "train_ms": train_ms,
        "train_step_us": 1e3 * train_ms / max(steps, 1),
        "data_ms": data_ms,
        "loss_first_last": [float(log[:10].mean()), float(log[-10:].mean())],
        "path": "batched persistent kernel with per-series proposal rows (abc_batch_run_weighted)",
        "launch_shape": tune["shape"],
        "refill_min": tune["refill"],
        "autotune_top": tune["table"][:5],
        "accepted_per_s": acc / wall,
        # end to end: the training pairs, the 20 epochs and the one forward pass
        # of the series' features counted in the learned run's time
        "train_total_s": train_total_s,
        "accepted_per_s_incl_training": acc / (wall + train_total_s),
        # accepted samples per series set beyond which the trained proposal
        # pays for its training at these rates
        "break_even_accepted": (train_total_s / (1.0 / batched["accepted_per_s"] - wall / acc)
                                if acc / wall > batched["accepted_per_s"] else None),
        "ess_per_s": ess / wall,
        "plain_accepted_per_s": batched["accepted_per_s"],
        "gain_accepted_per_s": (acc / wall) / batched["accepted_per_s"],
        "autotuned_round": tuned_round,
        "gain_ess_per_s": (ess / wall) / batched["accepted_per_s"],
        "acceptance_rate_gain_median": float(np.median(gains)),
        "acceptance_rate_gain_range": [float(np.min(gains)), float(np.max(gains))],
        "ess_median": float(np.median(ess_series)),
        "wall_s": wall,
        "samples": samples,
        "posterior_check": "runs of %d accepted per series pooled on further seeds until the learned "
                           "ESS >= 1e4 and every difference's standard error (from the samples' second "
                           "and fourth moments) is <= 1/4 of its 5%% tolerance, at most %d runs a side"
                           % (Qc, args.compare_max_runs),
        "posterior_check_s": compare_s,
        "posterior_check_plain_n": int(pn.min()),
        "posterior_check_runs_max": [int(max(r["runs_a"] for r in cmp_)),
                                     int(max(r["runs_b"] for r in cmp_))],
        "posterior_check_resolved_series": int(sum(r["se_over_tol"] * 4 <= 1.0 for r in cmp_)),
        "posterior_check_se_over_tol_max": float(max(r["se_over_tol"] for r in cmp_)),
        "posterior_check_unresolved_series": [j for j, r in enumerate(cmp_) if r["se_over_tol"] * 4 > 1.0],
        "posterior_check_runs_per_series": [[int(r["runs_a"]), int(r["runs_b"])] for r in cmp_],
        "posterior_check_ess_median": float(np.median(ess_c)),
        "posterior_check_ess_min": float(ess_c.min()),
        "posterior_worst_mean_over_tol_per_series": [round(float(x), 3) for x in worst_mu],
        "posterior_worst_sd_over_tol_per_series": [round(float(x), 3) for x in worst_sd],
        "posterior_mean_within_5pct": float(ok_mu.mean()),
        "posterior_sd_within_5pct": float(ok_sd.mean()),
        "posterior_both_within_5pct_series": int(np.sum(ok_mu.all(1) & ok_sd.all(1))),
    }


def smc_leg(args):
    """ABC-SMC on the first country: N particles, adaptive quantile tolerances
    from the pilot quantile eps0; compared with rejection ABC at the final
    tolerance (its acceptance rate measured on a plain pass)."""
    import torch

    from paper_2012_14332_amd import abc
    from paper_2012_14332_amd import pipeline as PL
    from paper_2012_14332_amd import workloads as W

    s = W.three_countries()[0]
    ser = PL.observed_series(s)
    eps0 = PL.pilot_eps(ser, 3, n=args.pilot, q=args.smc_q0, series=0)
    N, G = args.smc_particles, args.smc_generations
    cfg = abc.smc_config(N, eps0, generations=G, alpha=args.smc_alpha, chunk0=1 << 16,
                         chunk_max=1 << 22)
    abc.smc_run(ser, abc.smc_config(N, eps0, generations=2, alpha=args.smc_alpha,
                                    chunk0=1 << 16, chunk_max=1 << 22), 4)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = abc.smc_run(ser, cfg, 3)
    torch.cuda.synchronize()
    smc_s = time.perf_counter() - t0
    gens = [o["stats"] for o in outs]
    eps_final = float(gens[-1]["eps"])
    sims = sum(g["in_support"] for g in gens)
    proposed = sum(g["proposed"] for g in gens)
    # rejection ABC at the final tolerance: acceptance rate and speed of a plain pass
    n_chunk = args.smc_rejection_samples
    run = PL.PlainABC(ser, 3, eps_final, n_chunk, series=0, band_w=args.band, capacity=1 << 20)
    run.run(0)
    torch.cuda.synchronize()
    acc = n_rej = 0
    rej_s = 0.0
    while acc < 200 and n_rej < (1 << 33):
        t0 = time.perf_counter()
        acc += run.run(n_rej).n()
        rej_s += time.perf_counter() - t0
        n_rej += n_chunk
    rate = acc / n_rej
    need = N / rate if acc else float("inf")
    return {
        "workload": "%s: N = %d particles, %d generations, alpha %.2f, eps0 = pilot quantile %.0e; "
                    "rejection ABC at the final eps for comparison (%d samples)" % (
                        s.name, N, len(gens), args.smc_alpha, args.smc_q0, n_rej),
        "generations": [{"eps": g["eps"], "samples": g["samples"], "in_support": g["in_support"],
                         "proposed": g["proposed"], "ess": round(g["ess"], 1)} for g in gens],
        "wall_s": smc_s,
        "eps_final": eps_final,
        "simulations": sims,
        "proposals": proposed,
        "rejection_accept_rate_at_eps_final": rate,
        "rejection_samples_for_N": need,
        "rejection_s_for_N": need * rej_s / n_rej,
        "simulation_gain": need / sims if sims else None,
        "wall_gain": (need * rej_s / n_rej) / smc_s,
    }


def paper_style_leg(args):
    """Like-for-like with the paper's per-run figures (Sec. 4: T = 49, raw-count
    distance, full trajectories, no early exit): simulator throughput of the
    single synthetic country in trajectories/s and simulated days/s, next to
    the paper's 2x Mk1 IPU, V100 and 2-socket Xeon numbers (other hardware,
    real data; context only)."""
    import torch

    from paper_2012_14332_amd import abc, autotune
    from paper_2012_14332_amd import pipeline as PL
    from paper_2012_14332_amd import workloads as W

    s = W.single_country()
    ser = PL.observed_series(s)
    n = 10_000_000
    # full trajectories favour another shape than early exit does: tune it
    prev_shape, prev_refill = abc.get_launch_config(), abc.get_refill_min()
    tune = autotune.tune_plain(ser, math.inf, flags=abc.ABC_DIST_RAW, use_cache=False)
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    run = lambda f: abc.simulate_distance(ser, n, 1, first=f, flags=abc.ABC_DIST_RAW, out=out)
    run(0)
    torch.cuda.synchronize()
    reps = 5
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        run((r + 1) * n)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    traj = n / sec
    abc.set_launch_config(*prev_shape)
    abc.set_refill_min(prev_refill)
    paper = {"2x_Mk1_IPU": 4.25e7, "V100": 5.68e6, "2x_Xeon_Gold_6248": 1.38e6}
    return {
        "workload": "%s, raw-count distance, all %d days simulated (no early exit), %d samples per "
                    "launch, %d launches" % (s.name, s.T, n, reps),
        "trajectories_per_s": traj,
        "sim_days_per_s": traj * s.T,
        "launch_shape": tune["shape"],
        "paper_trajectories_per_s": paper,
        "ratio_to_paper": {k: traj / v for k, v in paper.items()},
    }


HBM_PEAK_GBS = 8000.0


def hbm_leg(args):
    """Bandwidth of the two HBM-bound passes, each on inputs larger than the
    256 MB last-level cache, timed with HIP events on the launch stream:
    accept-compaction of 4e8 float32 distances at an acceptance of 1e-4
    (theta of the accepted rows re-drawn from their counters), and the float64
    posterior moments of 1e8 theta rows, unweighted and weighted. The sizes
    keep each call several hundred microseconds long, well above the host's
    per-call launch cost, so back-to-back calls keep the GPU busy.
    Algorithmic bytes: 4 B per distance read plus 44 B per accepted row
    written (index, theta, distance); 32 B per theta row (+ 4 B weight)."""
    import torch

    from paper_2012_14332_amd import abc

    g = torch.Generator(device="cuda")
    g.manual_seed(17)
    n_c, q = 400_000_000, 1e-4
    dist = torch.rand(n_c, generator=g, device="cuda", dtype=torch.float32)
    eps = q                      # uniform distances: a fraction q falls at or below q
    cap = 1 << 16
    n_m = 100_000_000
    theta = torch.rand((n_m, 8), generator=g, device="cuda", dtype=torch.float32)
    w = torch.rand(n_m, generator=g, device="cuda", dtype=torch.float32)
    stream = torch.cuda.current_stream()

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out

    ms_c, res = timed(lambda: abc.accept_compact(dist, eps, cap, seed=3))
    acc = int(res[4].item())
    bytes_c = 4.0 * n_c + 44.0 * min(acc, cap)
    ms_m, _ = timed(lambda: abc.posterior_moments(theta))
    ms_w, _ = timed(lambda: abc.posterior_moments(theta, weight=w))
    bytes_m, bytes_w = 32.0 * n_m, 36.0 * n_m

    def rec(ms, b, **kw):
        gbs = b / (ms * 1e-3) / 1e9
        return dict(kw, ms=ms, algorithmic_bytes=b, GB_per_s=gbs, frac_of_hbm_peak=gbs / HBM_PEAK_GBS)

    return {
        "compact": rec(ms_c, bytes_c, n=n_c, accepted=acc),
        "moments": rec(ms_m, bytes_m, rows=n_m),
        "moments_weighted": rec(ms_w, bytes_w, rows=n_m),
        "peak_GB_per_s": HBM_PEAK_GBS,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # a first process on a box with only a few warm-up steps has run its whole
    # timed region a third slower (host side; the kernels themselves at full
    # speed); about 0.4 s of warm-up steps avoided it
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--samples", type=int, default=10_000_000, help="prior samples per country per step")
    ap.add_argument("--reps", type=int, default=10, help="timed K-step regions (the first is `value`)")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-single", action="store_true", help="skip the single-country nearest-100 leg")
    ap.add_argument("--per-series-launches", action="store_true",
                    help="one simulate launch per country instead of one for all three")
    ap.add_argument("--band", type=float, default=0.02)
    ap.add_argument("--pilot", type=int, default=100_000)
    ap.add_argument("--q", type=float, default=1e-4)
    ap.add_argument("--cpu-samples", type=int, default=1_000_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--launch", type=str, default="", help="spl,block,blocks_per_cu")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--quota", type=int, default=1000)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-only", action="store_true",
                    help="only train the learned proposal's network and report its timings")
    ap.add_argument("--mdn-pairs", type=int, default=1_000_000)
    ap.add_argument("--mdn-epochs", type=int, default=20)
    ap.add_argument("--lam", type=float, default=0.5)
    ap.add_argument("--inflate", type=float, default=8.0)
    ap.add_argument("--compare-quota", type=int, default=2048)
    ap.add_argument("--compare-seeds-plain", type=int, nargs="+", default=[2, 3, 4])
    ap.add_argument("--compare-seeds-learned", type=int, nargs="+", default=[2, 3, 4, 5])
    ap.add_argument("--compare-max-runs", type=int, default=8000)
    ap.add_argument("--compare-time-s", type=float, default=240.0,
                    help="wall-time bound on the posterior check's pooling")
    ap.add_argument("--refill-min", type=int, default=0, help="lane-refill threshold (0 = default)")
    ap.add_argument("--no-smc", action="store_true")
    ap.add_argument("--no-hbm", action="store_true", help="skip the compaction/moments bandwidth leg")
    ap.add_argument("--smc-particles", type=int, default=4096)
    ap.add_argument("--smc-generations", type=int, default=16)
    ap.add_argument("--smc-alpha", type=float, default=0.5)
    ap.add_argument("--smc-q0", type=float, default=1e-2)
    ap.add_argument("--smc-rejection-samples", type=int, default=1 << 26)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (scales HBM byte counters)")
    args = ap.parse_args()

    if args.train_only:
        import torch

        from paper_2012_14332_amd import abc
        from paper_2012_14332_amd import pipeline as PL

        assert torch.cuda.is_available(), "bench.py needs a GPU"
        torch.cuda.set_device(0)
        abc.lib()
        net, loss_log, steps, train_ms, data_ms = PL.train_proposal(
            n_pairs=args.mdn_pairs, epochs=args.mdn_epochs, batch=4096, lr=1e-3, seed=6)
        loss_log = loss_log.cpu().numpy()
        net.close()
        # one step's products at batch 4096: three forward (x W1, h1 W2, h2 W3)
        # and five backward (dW3, dZ2, dW2, dZ1, dW1; no gradient w.r.t. x)
        flop = 2 * 4096 * (2 * 96 * 256 + 3 * 256 * 256 + 3 * 256 * 136)
        print(json.dumps({"workload": "learned-proposal training: %d pairs, %d epochs, batch 4096"
                          % (args.mdn_pairs, args.mdn_epochs), "steps": steps, "train_ms": train_ms,
                          "step_us": 1e3 * train_ms / max(steps, 1), "data_ms": data_ms,
                          "gemm_gflop_per_step": flop / 1e9,
                          "loss_first_last": [float(loss_log[:10].mean()), float(loss_log[-10:].mean())]}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the ABC path is built for one device's share "
              "(see the sharding notes); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2012_14332_amd import abc
    from paper_2012_14332_amd import pipeline as PL
    from paper_2012_14332_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    abc.lib()
    if args.launch:
        abc.set_launch_config(*[int(x) for x in args.launch.split(",")])
    elif not args.per_series_launches:
        # two 1024-thread workgroups per CU (eight wavefronts per SIMD at the
        # kernel's 57 VGPRs); each gets half the LDS, so the bound tables are
        # coarser in time than at one workgroup per CU, but the step is
        # fastest here (same-box sweep of (spl, block, workgroups/CU): ms per
        # step 1.73 at (1, 1024, 2), 1.78 at (1, 512, 2), 1.99 at (1, 1024, 1))
        abc.set_launch_config(1, 1024, 2)
    if args.refill_min:
        abc.set_refill_min(args.refill_min)
    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    countries = W.three_countries()
    sers = [PL.observed_series(s) for s in countries]
    eps = [PL.pilot_eps(ser, 1, n=args.pilot, q=args.q, series=c) for c, ser in enumerate(sers)]
    N = args.samples
    first0 = args.pilot  # main-run indices follow the pilot prefix
    runs = [PL.PlainABC(ser, 1, e, N, series=c, band_w=args.band) for c, (ser, e) in
            enumerate(zip(sers, eps))]
    # One step: a single launch simulates all three countries' samples (their
    # 64-sample chunks form one queue, so the launch ends with one tail); then
    # stream B compacts each country's distances and one stream C per country
    # makes its float64 band decision and moments. The distance buffers are
    # double-buffered by step parity, so the next step's launch never waits on
    # this step's compactions; those and the band decisions run beside it.
    # (--per-series-launches: one launch per country, each country's compaction
    # overlapping the next country's launch.)
    sA = torch.cuda.current_stream()
    sB = torch.cuda.Stream()
    sCs = [torch.cuda.Stream() for _ in runs]
    days = torch.zeros(1, dtype=torch.int64, device="cuda")
    bufs = [[torch.empty(N, dtype=torch.float32, device="cuda") for _ in runs] for _ in range(2)]
    compacted = {}  # (parity, country) -> event after the buffer's last compaction

    def finish_country(c, r, first, dist, ready, par, keep):
        e_hi = r.eps * (1 + r.band_w)
        with torch.cuda.stream(sB):
            sB.wait_event(ready)
            idx, th, d, _, cnt = abc.accept_compact(dist, e_hi, r.cap, first=first,
                                                    seed=r.seed, series=c)
            compacted[(par, c)] = torch.cuda.Event()
            compacted[(par, c)].record(sB)
        sC = sCs[c]
        with torch.cuda.stream(sC):
            sC.wait_event(compacted[(par, c)])
            abc.recheck_band(r.ser, r.seed, r.eps, r.band_w, idx, th, d, cnt, series=c)
            mean, cov = abc.posterior_moments(th, n_dev=cnt)
        # each step's accepted count, and the latest rows for the last-step
        # check; earlier outputs are released (the binding marks every tensor
        # it hands to a stream as in use there, so the caching allocator
        # reuses a block only after that stream's work on it), which keeps a
        # steady-state step free of device allocations
        keep["cnt"].append((c, cnt))
        keep["last"][c] = (idx, cnt, mean)

    def step(s, keep, ev):
        first = first0 + s * N
        par = s % 2
        for c in range(len(runs)):
            if (par, c) in compacted:
                sA.wait_event(compacted[(par, c)])  # the buffer is free once compacted
        if not args.per_series_launches:
            jobs = [{"ser": r.ser, "n": N, "first": first, "series": c,
                     "eps_exit": r.eps * (1 + r.band_w), "out": bufs[par][c]}
                    for c, r in enumerate(runs)]
            if ev is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e0.record(sA)
            abc.simulate_distance_multi(jobs, 1, days=days if ev is not None else None)
            if ev is not None:
                e1 = torch.cuda.Event(enable_timing=True)
                e1.record(sA)
                ev.append((e0, e1, -1))
            simulated = torch.cuda.Event()
            simulated.record(sA)
            for c, r in enumerate(runs):
                finish_country(c, r, first, bufs[par][c], simulated, par, keep)
            return
        for c, r in enumerate(runs):
            if ev is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e0.record(sA)
            abc.simulate_distance(r.ser, N, r.seed, first=first, series=c,
                                  eps_exit=r.eps * (1 + r.band_w), out=bufs[par][c],
                                  days=days if ev is not None else None)
            if ev is not None:
                e1 = torch.cuda.Event(enable_timing=True)
                e1.record(sA)
                ev.append((e0, e1, c))
            simulated = torch.cuda.Event()
            simulated.record(sA)
            finish_country(c, r, first, bufs[par][c], simulated, par, keep)

    def timed_region(s0, ev):
        """K steps from step s0, bracketed by device synchronisation."""
        keep = {"cnt": [], "last": {}}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(s0, s0 + args.steps):
            step(s, keep, ev)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, sum(int(k[1].item()) for k in keep["cnt"]), keep

    # warm-up: the last K steps run exactly as a timed region does (launch
    # events, sample-day count, outputs kept until the region ends), with the
    # result discarded, so the first timed region finds the caching allocator
    # already grown for that overlap of steps; the earlier ones keep nothing
    # (the binding's record_stream holds each output's block until its stream
    # is done with it)
    rehearse = args.warmup >= args.steps
    for s in range(args.warmup - args.steps if rehearse else args.warmup):
        step(s, {"cnt": [], "last": {}}, None)
    if rehearse:
        timed_region(args.warmup - args.steps, [])
    torch.cuda.synchronize()
    ev = []
    days.zero_()
    wall, accepted, keep = timed_region(args.warmup, ev)
    note("timed region: %.3f ms per step" % (wall / args.steps * 1e3))
    # further repetitions of the same K-step region on fresh sample ranges
    # (median and interquartile range, as the paper repeats its runs)
    rep_rates, rep_ms = [accepted / wall], [wall / args.steps * 1e3]
    for r in range(1, args.reps):
        w_r, a_r = timed_region(args.warmup + r * args.steps, None)[:2]
        rep_rates.append(a_r / w_r)
        rep_ms.append(w_r / args.steps * 1e3)
    # the last step of the first region again, one country at a time on one
    # stream: the pipelined step must have accepted exactly the same rows
    last_first = first0 + (args.warmup + args.steps - 1) * N
    same_rows = True
    for c, r in enumerate(runs):
        idx_c, cnt_c, _ = keep["last"][c]
        ref = r.run(last_first)
        n_ref, n_got = int(ref.count.item()), int(cnt_c.item())
        same_rows &= n_ref == n_got and torch.equal(ref.idx[:n_ref], idx_c[:n_got])
    torch.cuda.synchronize()
    sim_ms = [a.elapsed_time(b) for a, b, _ in ev]
    eff_days = int(days.item())
    nominal_days = args.steps * N * sum(s.T for s in countries)
    traj = args.steps * N * len(countries)
    launches = len(sim_ms)
    avg_ms = float(np.mean(sim_ms))
    days_per_launch = eff_days / launches
    samples_per_launch = N * len(countries) // (launches // args.steps)
    # One launch over its average duration (HIP events on the launch stream).
    # Algorithmic work from the assembly count (FP32 FLOP, VALU instructions);
    # measured work from the committed PMC summary of the same kernel, workload
    # and launch shape (FP32 FLOP = 64 (add + mul + trans + 2 fma), issued
    # lane-instructions = 64 SQ_INSTS_VALU), scaled per sample-day to this
    # launch.
    flop_launch = FP32_FLOP_PER_SAMPLE_DAY * days_per_launch + FP32_FLOP_PER_SAMPLE * samples_per_launch
    issue_launch = ISSUE_PER_SAMPLE_DAY * days_per_launch + ISSUE_PER_SAMPLE * samples_per_launch
    flops_alg = flop_launch / (avg_ms * 1e-3) / 1e12
    issue_alg = issue_launch / (avg_ms * 1e-3) / 1e12
    shape = list(abc.get_launch_config())
    valu_pmc = valu_counters() if not args.per_series_launches else None
    if valu_pmc and valu_pmc.get("launch_config") != shape:
        valu_pmc = None  # taken at another launch shape
    traffic = traffic_per_launch() if not args.per_series_launches else None
    if valu_pmc:
        flop_meas = valu_pmc["fp32_flop_per_sample_day"] * days_per_launch
        qc_meas = valu_pmc["valu_lane_inst_per_sample_day"] * days_per_launch
        flops = flop_meas / (avg_ms * 1e-3) / 1e12
        issue_meas = qc_meas / (avg_ms * 1e-3) / 1e12
        # the FP32 FLOP rate this instruction mix reaches with every VALU
        # issue slot of the device busy
        mix_ceiling = flop_meas / qc_meas * ISSUE_PEAK_T
        flop_source = "PMC counters (profiles/k_simulate_multi_f32_valu.json)"
    else:
        flops, issue_meas = flops_alg, None
        mix_ceiling = flop_launch / issue_launch * ISSUE_PEAK_T
        flop_source = "static assembly count (counters not taken for these sources)"
    per_country = {}
    for c, s in enumerate(countries):
        n_c = sum(int(k[1].item()) for k in keep["cnt"] if k[0] == c)
        per_country[s.name] = {"eps": eps[c], "accepted": n_c,
                               "posterior_mean_last_step": [round(float(x), 5) for x in
                                                            keep["last"][c][2].cpu().numpy()]}
    out = {
        "metric": METRIC,
        "value": accepted / wall,
        "unit": "accepted samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": "plain rejection ABC, 3 synthetic countries run separately (P=6e7/8.3e7/"
                        "3.3e8, T=49/72/100, 100 active at day 0), 1e7 prior samples per country "
                        "per step, eps = 1e-4 quantile of a 1e5-sample pilot",
            "samples_per_step": N * len(countries),
            "eps": eps,
            "band_w": args.band,
            "launch_config": list(abc.get_launch_config()),
            "refill_min": abc.get_refill_min(),
        },
        "value_median": float(np.median(rep_rates)),
        "value_iqr": [float(np.percentile(rep_rates, 25)), float(np.percentile(rep_rates, 75))],
        "ms_per_step_median": float(np.median(rep_ms)),
        "repetitions": {"n": len(rep_rates), "steps_each": args.steps,
                        "accepted_per_s": [round(x, 1) for x in rep_rates],
                        "ms_per_step": [round(x, 4) for x in rep_ms]},
        "trajectories_per_s": traj / wall,
        "last_step_rows_match_single_stream": bool(same_rows),
        "sim_days_per_s_effective": eff_days / wall,
        "sim_days_per_s_nominal": nominal_days / wall,
        "simulate_kernel_ms_avg": avg_ms,
        "roofline": {
            "bound": "alu",
            "kernel": "k_simulate_f32" if args.per_series_launches else "k_simulate_multi_f32",
            "achieved": flops,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": flops / FP32_PEAK_TFLOPS,
            "traffic": traffic,
            "achieved_source": flop_source,
            "sample_days_per_launch": days_per_launch,
            "samples_per_launch": samples_per_launch,
            "launch_ms": avg_ms,
            # the kernel is bound by VALU issue; FP32 arithmetic is a
            # fraction of its instruction mix (Philox integer work, conversions)
            "mix_ceiling_tflops": mix_ceiling,
            "mix_ceiling_frac": mix_ceiling / FP32_PEAK_TFLOPS,
            "frac_of_mix_ceiling": flops / mix_ceiling,
            "issue": {"unit": "T lane-instructions/s", "peak": ISSUE_PEAK_T,
                      "measured": issue_meas,
                      "busy_frac": issue_meas / ISSUE_PEAK_T if issue_meas else None,
                      "algorithmic": issue_alg,
                      "algorithmic_frac": issue_alg / ISSUE_PEAK_T,
                      "algorithmic_share_of_issued": issue_alg / issue_meas if issue_meas else None,
                      "trans_unit_busy_frac": valu_pmc.get("trans_unit_busy_frac") if valu_pmc else None,
                      "inst_per_sample_day": ISSUE_PER_SAMPLE_DAY,
                      "inst_per_sample": ISSUE_PER_SAMPLE},
            "algorithmic_fp32": {"achieved": flops_alg, "frac": flops_alg / FP32_PEAK_TFLOPS,
                                 "flop_per_sample_day": FP32_FLOP_PER_SAMPLE_DAY,
                                 "flop_per_sample": FP32_FLOP_PER_SAMPLE},
            "valu_counters": valu_pmc,
        },
        "per_country": per_country,
    }
    if not args.no_batched:
        # the batched legs tune their own shapes; the float32 simulate kernel
        # of the later legs gets the main step's shape back
        main_shape, main_refill = abc.get_launch_config(), abc.get_refill_min()
        out["batched"] = batched_leg(args)
        note("batched leg done")
        if not args.no_learned:
            out["learned"] = learned_leg(args, out["batched"])
            note("learned leg done")
        out["batched"].pop("_eps", None)
        abc.set_launch_config(*main_shape)
        abc.set_refill_min(main_refill)
        out["batched"].pop("_used", None)
    if not args.no_smc:
        out["smc"] = smc_leg(args)
        note("smc leg done")
    out["paper_style"] = paper_style_leg(args)
    note("paper-style leg done")
    if not args.no_hbm:
        out["hbm_passes"] = hbm_leg(args)
        note("hbm leg done")
    if not args.no_single:
        out["single_country"] = single_country_leg(args)
        note("single-country leg done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(countries, eps, first0, args.cpu_samples, args.cpu_reps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
