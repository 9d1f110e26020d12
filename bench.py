#!/usr/bin/env python3
"""Throughput of the persistent call-auction engine on one MI355X.

One benchmark step = one cae_step call of S = 1000 steps over the fixed standard workload
(1024 markets, L = 256 ticks, A = 1024 agents, offsets +-16, quantities 1..100, seed 1):
1.049e9 agent events, every row of the hot path (orders, aggregation, curves, clearing,
allocation, statistics, persistent loop) inside one launch.  Inputs are resident on the GPU
before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--copy-calib]

Prints ONE JSON line on stdout (diagnostics go to stderr).
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

# --- roofline of the engine kernel (plain integer ALU work) --------------------------------
# Peak: 256 CUs x 4 SIMDs x 16 lanes = 64 lane-slots per CU per clock at the 2.4 GHz peak
# engine clock, for full-rate 32-bit VALU operations.
N_CU, LANES_PER_CU, CLOCK_HZ = 256, 64, 2.4e9
PEAK_SLOTS = N_CU * LANES_PER_CU * CLOCK_HZ  # 3.93e13 slots/s
# Issue cost in full-rate slots on gfx950, measured at saturation by
# paper_2606_21784_amd/ubench.py (one workgroup of 16 waves per CU, wave64 instructions per clock
# per CU): v_add/v_xor/v_bitop3 1.0, v_mul_hi_u32 1/0.824 = 1.21, v_mad_u64_u32 1/0.792 = 1.26.
COST = {"mad_u64_u32": 1.26, "mul_hi_u32": 1.21, "alu": 1.0}
# Algorithmic work per agent event, from the generator and order rules (not from compiled
# code): Philox4x32-10 with counter (step, agent, market, 0) needs 16 agent-dependent
# 32x32->64 products and 18 agent-dependent three-input xors; 2 multiply-high range
# reductions; 5 ops to form the tick (add, clamp), the quantity and the book address.
# Clearing costs 10 ops per tick per step, i.e. 10 L / A per event.
PHILOX_PRODUCTS, PHILOX_XORS, RANGE_MULHI, ORDER_OPS, CLEAR_OPS_PER_TICK = 16, 18, 2, 5, 10


def slots_per_event(L, A):
    return (PHILOX_PRODUCTS * COST["mad_u64_u32"] + PHILOX_XORS * COST["alu"]
            + RANGE_MULHI * COST["mul_hi_u32"] + ORDER_OPS * COST["alu"]
            + CLEAR_OPS_PER_TICK * COST["alu"] * L / A)


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


def cpu_baseline(w, n_markets):
    import numpy as np

    import oracle
    descs = w["descs"][:n_markets]
    nthreads = min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    st, bk = oracle.run(descs, w["seed"], w["S"], nthreads=nthreads)
    dt = time.perf_counter() - t0
    ev = float(np.sum(descs["A"].astype(np.float64))) * w["S"]
    return {"value": ev / dt, "unit": "agent-events/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d of %d markets of %s, all %d steps (%.3g events, %.1f s wall)" %
                      (n_markets, len(w["descs"]), w["name"], w["S"], ev, dt)}, st, bk


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
    tn = autotune.tune(d, seed=w["seed"], log=log)
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
           "schedule": {"waves_per_group": sched["waves_per_group"],
                        "groups_per_cu": sched["groups_per_cu"],
                        "waves_per_market": {str(k): v for k, v in sched["waves_per_market"].items()},
                        "overlap": {str(k): v for k, v in sched["overlap"].items()}},
           "tune_s": tune_s}
    log("uneven: batched %.1f ms (untuned %.1f), per-size %d launches %.1f ms" %
        (out["batched_ms"], out["untuned_batched_ms"], len(groups), out["per_size_ms"]))
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
    sched = {"waves_per_group": used["waves_per_group"],
             "waves_per_market": sorted(set(used["waves_per_market"].values())),
             "pipelined": bool(used["pipelined"]),
             "overlap": sorted(set(used["overlap"].values()))}
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-markets", type=int, default=1024)
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
    ap.add_argument("--copy-calib", action="store_true",
                    help="after timing, copy 1 GiB device-to-device (counter calibration)")
    args = ap.parse_args()
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
    d = w["descs"]
    M, L, A, S = len(d), int(d["L"][0]), int(d["A"][0]), w["S"]
    events = float(np.sum(d["A"].astype(np.float64))) * S
    from paper_2606_21784_amd import autotune
    t0 = time.perf_counter()
    tn = autotune.tune(d, seed=w["seed"])
    tune_s = time.perf_counter() - t0
    ens = engine.Ensemble(d, w["seed"], tuning=tn)
    sched = ens.tuning()
    sched = {"waves_per_group": sched["waves_per_group"], "groups_per_cu": sched["groups_per_cu"],
             "waves_per_market": sorted(set(sched["waves_per_market"].values())),
             "pipelined": bool(sched["pipelined"]), "overlap": sorted(set(sched["overlap"].values())),
             "autotune_s": tune_s}
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
    achieved = events * w_ev / (kms * 1e-3)
    traffic = measured_traffic()
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
            "unit": "Tslot/s", "frac": achieved / PEAK_SLOTS, "traffic": traffic,
            "kernel": "cae_engine_kernel<%d, false, false>" % max(1, L // 64), "kernel_ms": kms,
            "kernel_ms_last_launch": min(last_ms),
            "slots_per_event": w_ev, "events_per_launch": events,
            "roofline_events_per_s": PEAK_SLOTS / w_ev}

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
        cb, rst, rbk = cpu_baseline(w, args.cpu_markets)
        result["cpu_baseline"] = cb
        # the benchmarked kernel is the correct one: its first call matches the oracle
        n = args.cpu_markets
        if first_bk is not None:
            ok = np.array_equal(first_bk[:n * 2 * L], rbk)
            result["cpu_baseline"]["gpu_matches_oracle"] = ok
    ens.close()
    if not args.no_ablation:
        result["ablation"] = ablation_leg()
    if not args.no_sweeps:
        result["sweeps"] = sweeps_leg()
    if not args.no_dynamics:
        result["dynamics"] = dynamics_leg()
    if not args.no_uneven:
        result["uneven"] = uneven_leg()
    if not args.no_surrogate:
        from paper_2606_21784_amd import surrogate
        rep, _, _ = surrogate.run(log=log)
        result["surrogate"] = rep
        log("surrogate: speedup %.0f, mean rel err %s" %
            (rep["speedup"], {k: round(v["mean"], 4) for k, v in rep["surrogate_rel_err"].items()}))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
