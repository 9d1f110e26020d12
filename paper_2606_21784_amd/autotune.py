"""Autotuner for the persistent engine's schedule.

The engine's schedule has these knobs (``cae_tuning`` in include/cae.h):
  * waves per market, per size class (class = L bucket x A bucket): how many wave64s generate
    one market's orders; the rest of the workgroup's waves belong to other markets;
  * pipelined, per size class: markets run in pairs that share all of a workgroup's waves in
    alternating phases (one wave clears one market while the others generate the other's);
  * overlap, per size class (lock-step classes, either agent model): the market's other waves
    generate the next step's orders while one wave clears, the clearing wave taking overlap - 1
    rows of 64 agents after its clearing;
  * pack, per size class (small last-tick markets in an ensemble of books of at most 128
    ticks): P = 2 or 4 markets share one wave, 64 / P lanes each (up to 8 ticks per lane);
  * waves per workgroup: how many markets of one class share a workgroup (in lock-step when a
    market spans more than one wave) and therefore how the workgroup's LDS is partitioned into
    market slices;
  * the resident workgroups per CU that the persistent grid is sized for;
  * a priority boost (tuning flag bit 1): in a mixed ensemble the waves of the costliest
    markets, which hold the launch's critical path, issue one priority level above the rest.

``tune`` times candidates on the GPU through the C ABI (short launches on copies of the
ensemble's own markets), keeps the fastest per class, then picks waves-per-workgroup on the
whole ensemble.  Results can be cached as JSON keyed by GPU architecture and size class.
"""
import json
import os
import time

import numpy as np

from . import engine

WPM_CANDIDATES = (1, 2, 4, 8, 16)
PIPE_GROUPS = (4, 8)
PACK_CANDIDATES = (2, 4)
PACK_MAX_L = 128  # packing applies in ensembles whose books have at most this many ticks
GROUP_CANDIDATES = (4, 8, 16)
# A candidate within this fraction of the fastest counts as a tie; ties go to the schedule
# with fewer waves per market, which leaves the whole ensemble more freedom of group size.
TIE = 0.02
# Whole-ensemble stage: classes holding at least HEAVY_SHARE of the events (at most MAX_HEAVY
# of them) try up to MAX_RUNNERS of their schedules within RUNNER_UP of their probe's fastest.
HEAVY_SHARE, MAX_HEAVY, MAX_RUNNERS, RUNNER_UP = 0.1, 4, 3, 0.25
# The overlapped schedule is also probed at the second fastest plain width within this fraction.
OVL_SECOND = 0.3
# cae_tuning flag: the costliest markets' waves issue one priority level above the others'.
BOOST = 2


def classes_of(descs):
    return np.array([engine.size_class(int(L), int(A)) for L, A in zip(descs["L"], descs["A"])])


def _time_launch(descs, seed, tuning, S, reps=3):
    """Best kernel time (ms) of `reps` launches of S steps, each from the same opening state
    (rewound outside the timed region) after one untimed launch."""
    ens = engine.Ensemble(descs, seed, tuning=tuning)
    try:
        st, bk = ens.read_state(), ens.read_books()
        ens.step(S)
        ens.last_step_ms()
        best = None
        for _ in range(reps):
            ens.write_state(st, bk)
            ens.step(S)
            ms = ens.last_step_ms()
            best = ms if best is None else min(best, ms)
        return best
    finally:
        ens.close()


# Probe launches are sized to about this many agent events (roughly a millisecond), so that
# launch overhead and timer resolution stay below the differences between candidates.
PROBE_EVENTS = 5e8
# The whole-ensemble stages (workgroup size, runner-up schedules, priority boost) decide between
# schedules a few percent apart, so their probes run four times longer.
ENSEMBLE_PROBE_EVENTS = 2e9


def probe_steps(descs, S_min=20, S_max=1000, events=PROBE_EVENTS):
    """Steps per probe launch: about `events` agent events, within [S_min, S_max] and within
    the 32-bit book guard ((S + 1) A Q < 2^32 for the untimed launch plus one timed one)."""
    per_step = float(descs["A"].astype(np.float64).sum())
    S = int(np.clip(round(events / max(per_step, 1.0)), S_min, S_max))
    guard = (2**32 - 1) // int((descs["A"].astype(np.int64) * descs["Q"].astype(np.int64)).max())
    return int(max(1, min(S, guard // 2 - 1)))


def _pick(timings):
    """The schedule kept from a class's probe timings (w, pipelined, G, overlap, ms, pack): the
    fewest waves per market among the near-fastest (plain candidates come first, in increasing
    order of waves per market).  The overlapped candidates are one family, represented by its
    fastest member: the tie margin prefers a narrower schedule, not the first of several
    clearing shares that differ by noise."""
    fastest = min(x[4] for x in timings)
    ovl = [x for x in timings if x[3]]
    family = [x for x in timings if not x[3]] + ([min(ovl, key=lambda x: x[4])] if ovl else [])
    return next(x for x in family if x[4] <= fastest * (1.0 + TIE))


def _probe_set(descs, idx, min_markets, rng):
    """Markets of one class for probing: the class's own descriptors, replicated or sampled so
    that the probe fills the GPU (min_markets) without exceeding it by much."""
    if len(idx) >= min_markets:
        pick = np.sort(rng.choice(idx, min_markets, replace=False))
    else:
        pick = np.resize(idx, min_markets)
    return np.ascontiguousarray(descs[pick])


def tune(descs, seed=0, S_probe=None, min_markets=None, cache=None, arch="gfx950", log=None):
    """Return a tuning dict for ``engine.Ensemble(..., tuning=...)``.

    descs: the ensemble's market descriptors; S_probe: steps per timed probe launch (default:
    sized by probe_steps); min_markets: fewest markets in a class probe (default 4 per CU; a
    probe holds the class's own markets, at most 32 per CU, so that it sees the occupancy the
    ensemble will have); cache: optional JSON path.
    """
    rng = np.random.default_rng(0)
    cached = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            cached = json.load(f).get(arch, {})
    ncu = engine.device_info()["num_cu"]
    if min_markets is None:
        min_markets = 4 * ncu
    cls = classes_of(descs)
    wpm = {}
    pipe_c = {}
    ovl_c = {}
    pack_c = {}
    small_books = int(descs["L"].max()) <= PACK_MAX_L
    runners = {}   # class -> [(waves per market, pipelined, overlap, pack)] near its fastest
    timings_c = {}  # class -> every probed (waves per market, pipelined, G, overlap, ms, pack)
    cost = {}
    t0 = time.perf_counter()
    for c in sorted(set(cls.tolist())):
        key = str(c)
        if key in cached:
            wpm[c] = int(cached[key]["waves_per_market"])
            pipe_c[c] = bool(cached[key].get("pipelined", False))
            ovl_c[c] = int(cached[key].get("overlap", 0))
            pack_c[c] = int(cached[key].get("pack", 0))
            cost[c] = float(cached[key]["ns_per_market_step"])
            continue
        idx = np.nonzero(cls == c)[0]
        # the class's own markets: a class that is the whole ensemble is probed as it is, a
        # small class of a mixed ensemble is replicated up to min_markets
        n = min(len(idx) if len(idx) == len(descs) else max(len(idx), min_markets), 32 * ncu)
        probe = _probe_set(descs, idx, n, rng)
        Sp = S_probe or probe_steps(probe)
        events = float(probe["A"].astype(np.float64).sum()) * Sp
        # packed candidates first (the narrowest schedules): small last-tick Philox markets
        packable = (small_books and int(probe["flags"].max()) == 0)
        cands = [(1, False, G, 0, P) for P in PACK_CANDIDATES for G in (4, 8)
                 if packable and int(probe["L"].max()) <= 512 // P]
        cands += [(w, False, max(4, w), 0, 0) for w in WPM_CANDIDATES] + [(1, True, G, 0, 0) for G in PIPE_GROUPS]
        timings = []

        def run(w, pipe, G, k, P=0):
            tn = {"waves_per_group": G, "waves_per_market": {int(c): w}}
            if pipe:
                tn["pipelined"] = {int(c): 1}
            if k:
                tn["overlap"] = {int(c): k}
            if P:
                tn["pack"] = {int(c): P}
            ms = _time_launch(probe, seed, tn, Sp)
            if log:
                mode = ("pipelined G=%d" % G) if pipe else (("packed %d per wave G=%d" % (P, G)) if P else
                                                            "wpm %2d" % w + (" overlap %d" % k if k else ""))
                log("class %2d (L<=%4d, A~2^%d) %s: %.3f ms, %.3g events/s" %
                    (c, 64 << (c // 8), 6 + c % 8, mode, ms, events / (ms * 1e-3)))
            timings.append((w, pipe, G, k, ms, P))
            return ms

        for w, pipe, G, k, P in cands:
            run(w, pipe, G, k, P)
        # overlapped lock-step at the fastest plain lock-step width (and at the second fastest
        # when it is within OVL_SECOND of it: a long clearing, as for books of 1024 ticks, can
        # favour more generating waves), one or two markets per workgroup: the clearing wave
        # takes from none to all of an even share of the market's rows of 64 agents (at most 5
        # steps)
        plain = sorted((x for x in timings if x[0] >= 2 and not x[1] and not x[5]), key=lambda x: x[4])
        widths = [plain[0][0]] + [x[0] for x in plain[1:2] if x[4] <= plain[0][4] * (1.0 + OVL_SECOND)]
        rows = -(-int(probe["A"].max()) // 64)
        for w in widths:
            even = rows // w
            for G in sorted({max(4, w), min(16, 2 * max(4, w))}):
                for share in sorted({min(even, (even * j + 3) // 4) for j in range(5)}):
                    run(w, False, G, share + 1)
        fastest = min(x[4] for x in timings)
        best = _pick(timings)
        timings_c[c] = list(timings)
        wpm[c] = best[0]
        pipe_c[c] = best[1]
        ovl_c[c] = best[3]
        pack_c[c] = best[5]
        # runners-up for the whole-ensemble stage: the class's other schedules within
        # RUNNER_UP of its fastest, fastest first (one per kind of schedule)
        seen = {(best[0], best[1], best[3], best[5])}
        runners[c] = []
        for x in sorted(timings, key=lambda x: x[4]):
            kind = (x[0], x[1], x[3], x[5])
            if x[4] <= fastest * (1.0 + RUNNER_UP) and kind not in seen and len(runners[c]) < MAX_RUNNERS:
                seen.add(kind)
                runners[c].append(kind)
        # per market-step cost when the class fills the GPU alone
        cost[c] = best[4] * 1e6 / (len(probe) * Sp) * ncu
        cached[key] = {"waves_per_market": wpm[c], "pipelined": bool(pipe_c[c]), "overlap": ovl_c[c],
                       "pack": pack_c[c], "ns_per_market_step": cost[c]}
    # waves per workgroup on the whole ensemble: at each candidate size every class runs the
    # fastest of its probed schedules that fits a workgroup of that size (classes taken from
    # the cache are clamped to it)
    def fitting(c, G):
        if c in timings_c:
            fit = [x for x in timings_c[c] if x[0] <= G and (not x[1] or x[2] == G)]
            if fit:
                x = _pick(fit)
                return x[0], x[1], x[3], x[5]
        return min(wpm[c], G), pipe_c[c] and G >= 2, ovl_c.get(c, 0), pack_c[c]

    # two rounds over the sizes, keeping each size's best, so that a drift of the clocks during
    # the stage does not favour the sizes timed last
    best_g = None
    g_ms = {}
    for _ in range(2):
        for G in GROUP_CANDIDATES:
            sel = {c: fitting(c, G) for c in wpm}
            tn = {"waves_per_group": G, "waves_per_market": {int(c): v[0] for c, v in sel.items()},
                  "pipelined": {int(c): 1 for c, v in sel.items() if v[1]},
                  "overlap": {int(c): v[2] for c, v in sel.items() if v[2]},
                  "pack": {int(c): v[3] for c, v in sel.items() if v[3]}}
            ms = _time_launch(descs, seed, tn, S_probe or probe_steps(descs, events=ENSEMBLE_PROBE_EVENTS))
            g_ms[G] = min(ms, g_ms.get(G, ms))
            if log:
                log("waves_per_group %2d: %.3f ms" % (G, ms))
            if best_g is None or g_ms[G] < best_g[1]:
                best_g = (G, g_ms[G], sel)
    for c, v in best_g[2].items():
        wpm[c], pipe_c[c], ovl_c[c], pack_c[c] = v
    # whole-ensemble stage: a class's own probe fills the GPU with that class alone, while in a
    # small mixed ensemble its markets share the chip with the others and the longest chains of
    # steps set the launch's end.  For the classes that carry most of the events, each runner-up
    # schedule of the class is tried in the whole ensemble and kept if it is faster by more than
    # the tie margin.
    G = best_g[0]
    S_ens = S_probe or probe_steps(descs, events=ENSEMBLE_PROBE_EVENTS)

    def ensemble_tuning():
        return {"waves_per_group": G, "waves_per_market": {int(c): w for c, w in wpm.items()},
                "pipelined": {int(c): 1 for c, p in pipe_c.items() if p},
                "overlap": {int(c): k for c, k in ovl_c.items() if k},
                "pack": {int(c): P for c, P in pack_c.items() if P}}

    work = {c: float(descs["A"][cls == c].astype(np.float64).sum()) for c in set(cls.tolist())}
    total = sum(work.values())
    heavy = [c for c in sorted(work, key=lambda c: -work[c]) if work[c] >= HEAVY_SHARE * total][:MAX_HEAVY]
    if len(work) > 1 and any(runners.get(c) for c in heavy):  # one class: its probe was the ensemble
        current = _time_launch(descs, seed, ensemble_tuning(), S_ens)
        for c in heavy:
            for w, pipe, k, P in runners.get(c, []):
                if w > G or (pipe and G < 2):
                    continue
                keep = (wpm[c], pipe_c[c], ovl_c.get(c, 0), pack_c[c])
                wpm[c], pipe_c[c], ovl_c[c], pack_c[c] = w, pipe, k, P
                ms = _time_launch(descs, seed, ensemble_tuning(), S_ens)
                if log:
                    log("ensemble: class %2d as (wpm %d, pipelined %d, overlap %d, pack %d): %.3f ms (current %.3f)" %
                        (c, w, pipe, k, P, ms, current))
                if ms < current * (1.0 - TIE):
                    current = ms
                else:
                    wpm[c], pipe_c[c], ovl_c[c], pack_c[c] = keep
    # priority boost for the costliest markets (tuning flag bit 1): in a mixed ensemble every
    # market runs the same steps, so the markets with the most work per step hold the launch's
    # critical path; kept only if the whole ensemble runs faster by more than the tie margin
    flags = 0
    if len(work) > 1:
        base = dict(ensemble_tuning(), class_cost_ns=cost)
        t_base = _time_launch(descs, seed, base, S_ens)
        t_boost = _time_launch(descs, seed, dict(base, flags=BOOST), S_ens)
        if log:
            log("ensemble: priority boost %.3f ms (without %.3f)" % (t_boost, t_base))
        if t_boost < t_base * (1.0 - TIE):
            flags = BOOST
    if cache:
        allc = {}
        if os.path.exists(cache):
            with open(cache) as f:
                allc = json.load(f)
        allc[arch] = cached
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(allc, f, indent=1, sort_keys=True)
    result = {"waves_per_group": best_g[0], "flags": flags,
              "waves_per_market": {int(c): int(w) for c, w in wpm.items()},
              "pipelined": {int(c): 1 for c, p in pipe_c.items() if p},
              "overlap": {int(c): int(k) for c, k in ovl_c.items() if k},
              "pack": {int(c): int(P) for c, P in pack_c.items() if P},
              "class_cost_ns": {int(c): float(v) for c, v in cost.items()},
              "tune_seconds": time.perf_counter() - t0}
    return result


def per_size_groups(descs):
    """Indices of the markets of each size class (the per-size-launch baseline runs one
    launch per group)."""
    cls = classes_of(descs)
    return {int(c): np.nonzero(cls == c)[0] for c in sorted(set(cls.tolist()))}
