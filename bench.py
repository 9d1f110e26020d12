#!/usr/bin/env python3
"""Throughput of the persistent call-auction engine on one MI355X.

One benchmark step = one cae_step call of S = 1000 steps over the fixed standard workload
(1024 markets, L = 256 ticks, A = 1024 agents, offsets +-16, quantities 1..100, seed 1):
1.049e9 agent events, every row of the hot path (orders, aggregation, curves, clearing,
allocation, statistics, persistent loop) inside one launch.  Inputs are resident on the GPU
before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--verbose] [--detail PATH]

Prints ONE compact JSON line on stdout, last: the headline, its roofline (VALU issue and LDS
atomics), the oracle's CPU baseline and one short summary per leg.  Every leg's full detail goes
to a JSON file (--detail, default gpurun_out/bench_detail.json); diagnostics go to stderr, the
autotuner's per-candidate timings only with --verbose.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "agent events/s on 1 MI355X + roofline %; surrogate vs exact sweep speedup at ≤5% err"

# --- roofline of the engine kernel (plain integer VALU issue; LDS second) ----------------------
# Peak: 256 CUs x 4 SIMDs x 16 lanes = 64 lane-slots per CU per clock at the 2.4 GHz peak
# engine clock; a slot is one lane of one full-rate 32-bit VALU instruction (v_add_u32 issues
# one wave64 instruction per clock per CU when saturated).
N_CU, LANES_PER_CU, CLOCK_HZ = 256, 64, 2.4e9
PEAK_SLOTS = N_CU * LANES_PER_CU * CLOCK_HZ  # 3.93e13 slots/s
# Issue costs in full-rate slots, measured on MI355X by paper_2606_21784_amd/ubench.py at 16
# waves per CU (summary keys mad_in_mix_slots, bitop3_slots, mul_hi_slots): the Philox product
# v_mad_u64_u32 inside Philox rounds (1.14; 1.34 alone), the three-input xor v_bitop3_b32 (1.07)
# and v_mul_hi_u32 (1.29).
COST = {"mad_u64_u32": 1.14, "xor3": 1.07, "mul_hi_u32": 1.29, "alu": 1.0}
# Least VALU work per agent event that this generator and these order rules need, counted from
# the definitions (not from compiled code):
#  * Philox4x32-10 with counter (step, agent, market, 0): 20 products and 20 three-input xors,
#    of which 4 products and 2 xors do not depend on the agent (the agent word enters round 1
#    through an xor), so they are computed once per market-step: 16 products and 18 xors;
#  * 2 range reductions (multiply-high for the offset and the quantity; the quantity's +1 rides
#    in the 64-bit multiply-add's addend);
#  * 1 op for the order's book word: the side bit and the offset index in one funnel shift
#    (v_alignbit_b32); the reference price and the clamp to the grid apply per offset bin, not
#    per agent, when the orders are binned by offset as in the overlapped schedule;
#  * clearing, per tick and step: the two cumulative sums (2), and per side the unmatched part
#    max(D - V*, 0) in one saturating subtract and the fill as its difference to the next tick
#    (2 + 2): 6 ops per tick, i.e. 6 L / A per event.
PHILOX_PRODUCTS, PHILOX_XORS, RANGE_MULHI, ORDER_OPS, CLEAR_OPS_PER_TICK = 16, 18, 2, 1, 6
# LDS: one ds_add_u32 per event, at the rate ubench.py measures in the engine's aggregation
# pattern (addresses in a 66-word window; lds_window_lane_atomics_per_clk_cu), plus the
# clearing's pass over the book, 4 L / A words per event (read and write each tick's (bid, ask)
# pair once per step), at the rate of that access form (lds_rw_b64_lane_words_per_clk_cu).
LDS_LANE_ATOMICS_PER_CLK_CU = 8.2
LDS_RW_WORDS_PER_CLK_CU = 107.7
LDS_WORDS_PER_TICK = 4


def slots_per_event(L, A):
    return (PHILOX_PRODUCTS * COST["mad_u64_u32"] + PHILOX_XORS * COST["xor3"]
            + RANGE_MULHI * COST["mul_hi_u32"] + ORDER_OPS * COST["alu"]
            + CLEAR_OPS_PER_TICK * COST["alu"] * L / A)


def lds_clocks_per_event(L, A):
    """CU clocks of LDS work per event: the order's atomic and the clearing's share of words."""
    return 1.0 / LDS_LANE_ATOMICS_PER_CLK_CU + LDS_WORDS_PER_TICK * L / A / LDS_RW_WORDS_PER_CLK_CU


def valu_ceiling(L, A):
    return PEAK_SLOTS / slots_per_event(L, A)


def lds_ceiling(L, A):
    return N_CU * CLOCK_HZ / lds_clocks_per_event(L, A)


def ceiling_events_per_s(L, A):
    """R = min(VALU ceiling, LDS ceiling) for a market of L ticks and A agents."""
    return min(valu_ceiling(L, A), lds_ceiling(L, A))


def ensemble_ceiling(descs):
    """Ceiling of a whole ensemble: the time each market's events need at its own ceiling,
    summed (work of different shapes adds up on one chip)."""
    import numpy as np
    A = descs["A"].astype(np.float64)
    L = descs["L"].astype(np.float64)
    t = sum(a / ceiling_events_per_s(l, a) for l, a in zip(L.tolist(), A.tolist()))
    return float(A.sum()) / t


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "engine_fixed_M1024_L256_A1024_S1000.traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2606_21784_amd", "csrc", "cae_engine.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when the
    kernel source changed after the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != kernel_source_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_threads():
    """Threads for the multi-threaded oracle: the host's CPUs available to this process, at most
    16 (one GPU's share of the host).  Returns (threads, nproc)."""
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return max(1, min(nproc, 16)), nproc


def cpu_baseline(w, n_markets, n_markets_1t):
    """The oracle (plain sequential C, one market at a time per thread) on the host cores: one
    thread on the first n_markets_1t markets, then `cpu_threads()` threads on the first n_markets
    markets (all steps).  Returns (record, states, books) of the multi-threaded run."""
    import numpy as np

    import oracle
    nthreads, nproc = cpu_threads()
    rows = {}
    for key, n, th in (("one_thread", n_markets_1t, 1), ("threads", n_markets, nthreads)):
        descs = w["descs"][:n]
        t0 = time.perf_counter()
        st, bk = oracle.run(descs, w["seed"], w["S"], nthreads=th)
        dt = time.perf_counter() - t0
        ev = float(np.sum(descs["A"].astype(np.float64))) * w["S"]
        rows[key] = {"events_per_s": ev / dt, "ns_per_event": 1e9 * dt / ev, "threads": th,
                     "markets": n, "events": ev, "wall_s": dt}
    mt = rows["threads"]
    rec = {"value": mt["events_per_s"], "unit": "agent-events/s", "cores": nthreads, "kind": "oracle",
           "ns_per_event": mt["ns_per_event"], "nproc": nproc,
           "one_thread": {"value": rows["one_thread"]["events_per_s"],
                          "ns_per_event": rows["one_thread"]["ns_per_event"],
                          "markets": rows["one_thread"]["markets"]},
           "sample": "%s, all %d steps: %d of %d markets on %d threads (%.3g events, %.1f s); "
                     "%d markets on 1 thread (%.3g events, %.1f s)" %
                     (w["name"], w["S"], n, len(w["descs"]), nthreads, mt["events"], mt["wall_s"],
                      rows["one_thread"]["markets"], rows["one_thread"]["events"],
                      rows["one_thread"]["wall_s"])}
    return rec, st, bk


def uneven_leg(reps=2):
    """Markets of uneven L and A in one autotuned persistent launch, against one launch per
    size class (same kernel, same market streams) on the same stream."""
    import numpy as np
    import torch

    from paper_2606_21784_amd import autotune, engine, workloads
    w = workloads.uneven()
    d, S = w["descs"], w["S"]
    events = float(d["A"].astype(np.float64).sum()) * S

    def timed(ensembles, n):
        """Best wall time of n rounds; each round rewinds the ensembles to their opening state
        (outside the timed region) and launches S steps on every ensemble back to back."""
        opening = [(e.read_state(), e.read_books()) for e in ensembles]
        best = None
        for _ in range(n):
            for e, (st, bk) in zip(ensembles, opening):
                e.write_state(st, bk)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for e in ensembles:
                e.step(S)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    t0 = time.perf_counter()
    tn = autotune.tune(d, seed=w["seed"], log=log if VERBOSE else None)
    tune_s = time.perf_counter() - t0
    ens = engine.Ensemble(d, w["seed"], tuning=tn)
    t_batched = timed([ens], reps)
    sched = ens.tuning()
    ens.close()
    ens = engine.Ensemble(d, w["seed"])
    t_default = timed([ens], reps)
    ens.close()
    groups = autotune.per_size_groups(d)
    parts = []
    for c, idx in groups.items():
        wpm = tn["waves_per_market"][c]
        pipe = tn.get("pipelined", {}).get(c, 0)
        ovl = tn.get("overlap", {}).get(c, 0)
        parts.append(engine.Ensemble(d[idx], w["seed"], market_ids=idx,
                                     tuning={"waves_per_group": max(4 if not pipe else 8, wpm),
                                             "waves_per_market": {c: wpm},
                                             "pipelined": {c: pipe} if pipe else {},
                                             "overlap": {c: ovl} if ovl else {}}))
    t_split = timed(parts, reps)
    for e in parts:
        e.close()
    out = {"workload": w["name"], "markets": len(d), "events": events,
           "batched_ms": 1e3 * t_batched, "batched_events_per_s": events / t_batched,
           "untuned_batched_ms": 1e3 * t_default,
           "per_size_launches": len(groups), "per_size_ms": 1e3 * t_split,
           "per_size_events_per_s": events / t_split, "speedup_vs_per_size": t_split / t_batched,
           "ceiling_frac": events / t_batched / ensemble_ceiling(d),
           "schedule": {"waves_per_group": sched["waves_per_group"],
                        "groups_per_cu": sched["groups_per_cu"], "flags": sched["flags"],
                        "waves_per_market": {str(k): v for k, v in sched["waves_per_market"].items()},
                        "overlap": {str(k): v for k, v in sched["overlap"].items()}},
           "tune_s": tune_s}
    log("uneven: batched %.1f ms (untuned %.1f), per-size %d launches %.1f ms, tuning flags %d" %
        (out["batched_ms"], out["untuned_batched_ms"], len(groups), out["per_size_ms"], sched["flags"]))
    return out


def ablation_leg(reps=3):
    """The paper's ablation (section IV-I): the naive one-thread-per-market engine (book in
    global memory, serial clearing) against the persistent engine, on the fixed workload and on
    the paper's own fixed-workload shape (8192 markets, A = 256, L = 128, 500 steps; offsets
    +-8 and quantities 1..10 here, the paper's values being unstated)."""
    import numpy as np

    from paper_2606_21784_amd import engine, workloads
    out = {}
    for w in (workloads.fixed(), workloads.paper_fixed()):
        d, S = w["descs"], w["S"]
        events = float(d["A"].astype(np.float64).sum()) * S
        row = {}
        for kind in ("persistent", "naive"):
            ens = engine.Ensemble(d, w["seed"])
            st, bk = ens.read_state(), ens.read_books()
            best = None
            for _ in range(reps if kind == "persistent" else 1):
                ens.write_state(st, bk)
                (ens.step if kind == "persistent" else ens.step_naive)(S)
                ms = ens.last_step_ms()
                best = ms if best is None else min(best, ms)
            row[kind + "_ms"] = best
            row[kind + "_events_per_s"] = events / (best * 1e-3)
            ens.close()
        row["speedup"] = row["naive_ms"] / row["persistent_ms"]
        out[w["name"]] = row
        log("ablation %s: persistent %.2f ms, naive %.1f ms (%.1fx)" %
            (w["name"], row["persistent_ms"], row["naive_ms"], row["speedup"]))
    return out


# The paper's own results on an RTX 5090 for its shapes (its agent parameters and generator
# differ from this engine's): Table III (market and agent sweeps), Table IV (fixed workload),
# and the median per-step latency of section IV-I.
PAPER_MARKET_SWEEP = {64: 3.61e9, 256: 1.35e10, 1024: 3.69e10, 4096: 4.73e10, 16384: 5.39e10}
PAPER_AGENT_SWEEP = {16: 8.41e9, 64: 2.84e10, 256: 5.16e10, 1024: 5.47e10}
PAPER_FIXED = 5.203e10
PAPER_STEP_LATENCY_US = 22.1


def tuned_time(w, reps=2):
    """Autotuned schedule, then the best of `reps` timed launches of S steps (rewinding the
    state between launches, outside the timed region).  Returns (ms, events/s, schedule)."""
    import numpy as np

    from paper_2606_21784_amd import autotune, engine
    d, S = w["descs"], w["S"]
    events = float(d["A"].astype(np.float64).sum()) * S
    tn = autotune.tune(d, seed=w["seed"])
    ens = engine.Ensemble(d, w["seed"], tuning=tn)
    st, bk = ens.read_state(), ens.read_books()
    times = []
    for _ in range(reps):
        ens.write_state(st, bk)
        ens.step(S)
        times.append(ens.last_step_ms())
    used = ens.tuning()
    ens.close()
    ms = min(times)
    frac = events / (ms * 1e-3) / ensemble_ceiling(d)
    sched = {"waves_per_group": used["waves_per_group"],
             "waves_per_market": sorted(set(used["waves_per_market"].values())),
             "pipelined": bool(used["pipelined"]),
             "overlap": sorted(set(used["overlap"].values())),
             "pack": sorted(set(used["pack"].values())), "flags": used["flags"]}
    sched["ceiling_frac"] = frac
    return ms, events / (ms * 1e-3), sched, times


def sweeps_leg():
    """The paper's sweep shapes and latency figure, and the 10000-step market-count sweep."""
    import numpy as np

    from paper_2606_21784_amd import workloads
    out = {"paper_market_sweep": {}, "paper_agent_sweep": {}, "market_sweep": {}}
    for M in workloads.PAPER_SWEEP_M:
        ms, ev, sched, _ = tuned_time(workloads.paper_market_sweep(M))
        out["paper_market_sweep"][str(M)] = {"ms": ms, "events_per_s": ev, "schedule": sched,
                                             "paper_rtx5090_events_per_s": PAPER_MARKET_SWEEP[M]}
        log("paper market sweep M=%d: %.3f ms, %.3g events/s" % (M, ms, ev))
    for A in workloads.PAPER_SWEEP_A:
        ms, ev, sched, _ = tuned_time(workloads.paper_agent_sweep(A))
        out["paper_agent_sweep"][str(A)] = {"ms": ms, "events_per_s": ev, "schedule": sched,
                                            "paper_rtx5090_events_per_s": PAPER_AGENT_SWEEP[A]}
        log("paper agent sweep A=%d: %.3f ms, %.3g events/s" % (A, ms, ev))
    w = workloads.paper_fixed()
    ms, ev, sched, _ = tuned_time(w)
    out["paper_fixed"] = {"workload": w["name"], "ms": ms, "events_per_s": ev, "schedule": sched,
                          "paper_rtx5090_events_per_s": PAPER_FIXED}
    # per-step latency: wall time of a launch / its steps, 11 launches, median (section IV-I)
    w = workloads.paper_market_sweep(4096)
    _, _, sched, times = tuned_time(w, reps=11)
    lat = [1e3 * t / w["S"] for t in times]
    out["step_latency"] = {"workload": w["name"], "median_us": float(np.median(lat)),
                           "min_us": float(np.min(lat)), "max_us": float(np.max(lat)),
                           "paper_rtx5090_median_us": PAPER_STEP_LATENCY_US, "schedule": sched}
    log("step latency %s: median %.2f us" % (w["name"], out["step_latency"]["median_us"]))
    for M in workloads.MARKET_SWEEP_M:
        ms, ev, sched, _ = tuned_time(workloads.market_sweep(M), reps=1)
        out["market_sweep"][str(M)] = {"ms": ms, "events_per_s": ev, "schedule": sched,
                                       "step_latency_us": 1e3 * ms / 10000}
        log("market sweep M=%d: %.1f ms, %.3g events/s" % (M, ms, ev))
    return out


# Marketable-order probability of the mid-price model in the dynamics leg (the paper names
# P_mkt without a value).
DYN_P_MKT = 0.05


def dynamics_leg():
    """The agent-mix sweep of section IV-J (alpha_mom 0..0.70, makers 0.15, 64 markets of each
    mix, 1000 steps, L = 128, K = 8, Q = 10) for A in {16, 64, 256, 1024}: one traced launch
    of all 3840 markets per agent model (autotuned schedule), then the stylized facts from the
    recorded series."""
    from paper_2606_21784_amd import dynamics, engine
    from paper_2606_21784_amd._lib import MODEL_LAST, MODEL_MID
    dynamics.run_sweep(A_values=(16,), alphas=(0.0,), markets=4, S=10)  # load / warm up
    out = {"paper_rtx5090": "12.8e6-event sweep in under 0.25 s (section IV-J)"}
    for name, flags in (("last_tick", engine.model_flags(MODEL_LAST)),
                        ("mid_price_pmkt%.2f" % DYN_P_MKT, engine.model_flags(MODEL_MID, DYN_P_MKT))):
        report, timing = dynamics.run_sweep(flags=flags, tuning="auto")
        out[name] = {
            "timing": timing, "facts_A256": dynamics.facts(report, A=256),
            "sweep": {str(A): {k: report[A][k] for k in ("alpha_mom", "tick_change_std",
                                                         "price_std", "excess_kurtosis",
                                                         "mean_volume", "mean_spread")}
                      for A in report},
            "acf_A256_alpha015": {k: report[256][k][3] for k in ("acf_r", "acf_abs_r")}}
        log("dynamics %s: %d markets x %d steps, %.3g events in %.2f ms (%.3g events/s)" %
            (name, timing["markets"], timing["steps"], timing["events"], timing["kernel_ms"],
             timing["events_per_s"]))
    return out


def leg_summaries(detail):
    """One short record per leg for the result line (the full detail goes to the detail file)."""
    out = {}
    r = lambda x, n=4: float("%.*g" % (n, x))
    if "ablation" in detail:
        a = detail["ablation"]
        out["ablation_naive_vs_persistent"] = {k: r(v["speedup"], 3) for k, v in a.items()}
    if "sweeps" in detail:
        sw = detail["sweeps"]
        ms = sw["market_sweep"]
        out["market_sweep_L512_A4096_S10000"] = {
            "M": [int(k) for k in ms], "events_per_s": [r(v["events_per_s"], 3) for v in ms.values()],
            "ceiling_frac": [r(v["schedule"]["ceiling_frac"], 3) for v in ms.values()]}
        pm = sw["paper_market_sweep"]
        out["paper_market_sweep_A256_L128_S500"] = {
            "M": [int(k) for k in pm], "events_per_s": [r(v["events_per_s"], 3) for v in pm.values()]}
        pa = sw["paper_agent_sweep"]
        out["paper_agent_sweep_M8192_L128_S500"] = {
            "A": [int(k) for k in pa], "events_per_s": [r(v["events_per_s"], 3) for v in pa.values()],
            "ceiling_frac": [r(v["schedule"]["ceiling_frac"], 3) for v in pa.values()]}
        pf = sw["paper_fixed"]
        out["paper_fixed_M8192_A256_L128_S500"] = {"ms": r(pf["ms"]), "events_per_s": r(pf["events_per_s"], 3)}
        out["step_latency_M4096_A256_us"] = r(sw["step_latency"]["median_us"], 3)
    if "dynamics" in detail:
        dy = detail["dynamics"]
        out["dynamics_M3840_L128_S1000"] = {k: {"kernel_ms": r(v["timing"]["kernel_ms"]),
                                                "events_per_s": r(v["timing"]["events_per_s"], 3)}
                                            for k, v in dy.items() if isinstance(v, dict)}
    if "uneven" in detail:
        u = detail["uneven"]
        out["uneven_M8192_S2000"] = {"batched_ms": r(u["batched_ms"]), "per_size_ms": r(u["per_size_ms"]),
                                     "per_size_launches": u["per_size_launches"],
                                     "speedup": r(u["speedup_vs_per_size"], 3),
                                     "events_per_s": r(u["batched_events_per_s"], 3),
                                     "ceiling_frac": r(u["ceiling_frac"], 3)}
    if "surrogate" in detail:
        sg = detail["surrogate"]
        names = ("mean_spread", "logret_variance", "mean_volume")
        out["surrogate_65536_draws"] = {
            "speedup": r(sg["speedup"], 4), "exact_s": r(sg["exact_test_sweep_s"]),
            "surrogate_s": r(sg["surrogate_test_sweep_s"], 3),
            "mean_rel_err": [r(sg["surrogate_rel_err"][k]["mean"], 3) for k in names],
            "p95_rel_err": [r(sg["surrogate_rel_err"][k]["p95"], 3) for k in names],
            "noise_floor_mean": [r(sg["mc_noise_rel_diff"][k]["mean"], 3) for k in names],
            "linear_mean_rel_err": [r(sg["linear_predictor_rel_err"][k]["mean"], 3) for k in names]}
    return out


VERBOSE = False


def main():
    global VERBOSE
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-markets", type=int, default=1024,
                    help="markets of the fixed workload the multi-threaded oracle runs")
    ap.add_argument("--cpu-markets-1t", type=int, default=32,
                    help="markets of the fixed workload the one-thread oracle runs")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven-ensemble leg (batched launch vs per-size launches)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the calibration-surrogate leg (65536-draw sweep, training, scoring)")
    ap.add_argument("--no-sweeps", action="store_true",
                    help="skip the sweep leg (paper shapes, step latency, market-count sweep)")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the naive-engine ablation leg")
    ap.add_argument("--no-dynamics", action="store_true",
                    help="skip the agent-mix dynamics leg (traced sweep, stylized facts)")
    ap.add_argument("--verbose", action="store_true",
                    help="log the autotuner's per-candidate timings and training progress")
    ap.add_argument("--detail", default=os.path.join(ROOT, "gpurun_out", "bench_detail.json"),
                    help="file for every leg's full detail (JSON)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="after timing, copy 1 GiB device-to-device (counter calibration)")
    ap.add_argument("--schedule", default=None,
                    help="run the headline in this schedule instead of the autotuner's: "
                         "waves_per_group,waves_per_market,overlap (e.g. 8,4,4), so that separate "
                         "profiler passes all time the same code")
    ap.add_argument("--steps-per-call", type=int, default=0,
                    help="auction steps per launch instead of the workload's 1000 (for the HBM "
                         "check that traffic does not grow with S; the result line then names "
                         "another workload)")
    args = ap.parse_args()
    VERBOSE = args.verbose
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this engine has no multi-GPU path (markets would be "
              "sharded with no communication); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_21784_amd import engine, workloads
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)

    w = workloads.fixed()
    if args.steps_per_call:
        w = dict(w, S=args.steps_per_call,
                 name=w["name"].replace("_S%d" % w["S"], "_S%d" % args.steps_per_call))
    d = w["descs"]
    M, L, A, S = len(d), int(d["L"][0]), int(d["A"][0]), w["S"]
    events = float(np.sum(d["A"].astype(np.float64))) * S
    from paper_2606_21784_amd import autotune
    # a few untimed launches first, so that the autotuner's probes do not start on a cold GPU
    warm = engine.Ensemble(d, w["seed"])
    for _ in range(5):
        warm.step(S)
    torch.cuda.synchronize()
    warm.close()
    t0 = time.perf_counter()
    if args.schedule:
        g, wpm, ovl = (int(x) for x in args.schedule.split(","))
        c = int(autotune.classes_of(d)[0])  # the fixed workload is one size class
        tn = {"waves_per_group": g, "waves_per_market": {c: wpm}, "overlap": {c: ovl} if ovl else {}}
    else:
        tn = autotune.tune(d, seed=w["seed"], log=log if VERBOSE else None)
    tune_s = time.perf_counter() - t0
    ens = engine.Ensemble(d, w["seed"], tuning=tn)
    sched = ens.tuning()
    sched = {"waves_per_group": sched["waves_per_group"], "groups_per_cu": sched["groups_per_cu"],
             "waves_per_market": sorted(set(sched["waves_per_market"].values())),
             "pipelined": bool(sched["pipelined"]), "overlap": sorted(set(sched["overlap"].values())),
             "autotune_s": round(tune_s, 2), "pinned": bool(args.schedule)}
    log("schedule:", json.dumps(sched))

    first_bk = None  # books after the first launch, checked against the oracle below
    for i in range(args.warmup):
        ens.step(S)
        if i == 0:
            first_bk = ens.read_books()
    torch.cuda.synchronize()
    snap_st, snap_bk = ens.read_state(), ens.read_books()
    guard = (2**32 - 1) // (A * int(d["Q"][0]))

    # Launches are queued back to back (no host wait inside the timed region).  The kernel time
    # comes from HIP events recorded on the engine's own stream around the timed launches,
    # divided by their number (it includes the few microseconds between consecutive launches);
    # the library's per-launch events give the last launch of each chunk alone.
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    kern_total = 0.0
    last_ms = []
    wall = 0.0
    done = 0
    while done < args.steps:
        chunk = min(args.steps - done, max(1, guard // S - args.warmup - 1))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(ens.stream)
        for _ in range(chunk):
            ens.step(S)
        ev1.record(ens.stream)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        kern_total += ev0.elapsed_time(ev1)
        last_ms.append(ens.last_step_ms())
        done += chunk
        if done < args.steps:  # rewind outside the timed region (32-bit book guard)
            ens.write_state(snap_st, snap_bk)
    value = events * args.steps / wall
    kms = kern_total / args.steps
    log("wall %.3f ms/step, kernel %.3f ms (last launch alone %.3f), %.4g events/s" %
        (1e3 * wall / args.steps, kms, min(last_ms), value))

    if args.copy_calib:
        x = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")

    w_ev = slots_per_event(L, A)
    rate = events / (kms * 1e-3)  # kernel-time events/s
    achieved = rate * w_ev
    lds_busy = rate * lds_clocks_per_event(L, A) / (N_CU * CLOCK_HZ)  # fraction of LDS clocks
    roof = {"bound": "alu" if valu_ceiling(L, A) <= lds_ceiling(L, A) else "lds",
            "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
            "unit": "TOP/s", "frac": achieved / PEAK_SLOTS, "traffic": measured_traffic(),
            "kernel": "cae_engine_kernel<%d,false,false,false>" % max(1, L // 64), "kernel_ms": kms,
            "kernel_ms_last_launch": min(last_ms), "slots_per_event": round(w_ev, 3),
            "lds": {"frac": lds_busy, "ceiling_events_per_s": lds_ceiling(L, A),
                    "clocks_per_event": lds_clocks_per_event(L, A)},
            "ceiling_events_per_s": ceiling_events_per_s(L, A),
            "ceiling_frac": rate / ceiling_events_per_s(L, A)}

    result = {
        "metric": METRIC, "value": value, "unit": "agent-events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w["name"], "markets": M, "L": L, "A": A,
                   "steps_per_call": S, "K": int(d["K"][0]), "Q": int(d["Q"][0]),
                   "seed": w["seed"], "events_per_step": events, "parallelism": "none",
                   "schedule": sched},
        "roofline": roof,
    }
    if not args.no_cpu:
        cb, rst, rbk = cpu_baseline(w, args.cpu_markets, args.cpu_markets_1t)
        # the benchmarked kernel is the correct one: its first call matches the oracle
        n = args.cpu_markets
        if first_bk is not None:
            cb["gpu_matches_oracle"] = bool(np.array_equal(first_bk[:n * 2 * L], rbk))
        result["cpu_baseline"] = cb
        log("cpu baseline: %.3g events/s on %d threads (%.1f ns/event), %.3g on 1 thread" %
            (cb["value"], cb["cores"], cb["ns_per_event"], cb["one_thread"]["value"]))
    ens.close()
    detail = {}
    if not args.no_ablation:
        detail["ablation"] = ablation_leg()
    if not args.no_sweeps:
        detail["sweeps"] = sweeps_leg()
    if not args.no_dynamics:
        detail["dynamics"] = dynamics_leg()
    if not args.no_uneven:
        detail["uneven"] = uneven_leg()
    if not args.no_surrogate:
        from paper_2606_21784_amd import surrogate
        rep, _, _ = surrogate.run(log=log if VERBOSE else None)
        detail["surrogate"] = rep
        log("surrogate: speedup %.0f, mean rel err %s" %
            (rep["speedup"], {k: round(v["mean"], 4) for k, v in rep["surrogate_rel_err"].items()}))
    result["legs"] = leg_summaries(detail)
    result["detail_file"] = os.path.relpath(args.detail, ROOT)
    try:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
        with open(args.detail, "w") as f:
            json.dump(dict(result, detail=detail), f, indent=1)
    except OSError as e:
        log("could not write %s: %s" % (args.detail, e))
    line = json.dumps(result, separators=(",", ":"))
    print(line, flush=True)
    if len(line) > 4096:
        log("warning: the result line is %d characters" % len(line))


if __name__ == "__main__":
    main()
