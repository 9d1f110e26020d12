"""Calibration surrogate: agent-population parameters -> ensemble statistics.

The exact path is the engine: for a parameter vector theta = (noise fraction, momentum
fraction, offset width, mean quantity) an ensemble of markets is stepped and its statistics
are pooled (mean post-auction spread, log-return variance, mean volume per step).  The
surrogate is a 4 -> 256 -> 256 -> 3 perceptron trained on the GPU with libcae's bfloat16
matrix-core kernels on ensembles the engine generated.  Its inputs are the engine's own market
parameters derived from theta (noise and momentum shares after rounding to agents, the integer
offset half-width K and the integer quantity bound Q, each scaled to [-1, 1]); its outputs are
the logarithms of the three statistics, centred; it is trained with a Huber loss in log space,
which matches the relative-error criterion.  The engine remains the fallback (``exact_stats``)
and the reference that measures the surrogate's error on held-out parameters.
"""
import time

import numpy as np

from . import engine, workloads

STAT_NAMES = ("mean_spread", "logret_variance", "mean_volume")
THETA_LO = np.array([0.0, 0.0, 2.0, 5.0])
THETA_HI = np.array([1.0, 1.0, 32.0, 100.0])


def pooled(states, S_total):
    """Pool per-market statistics in market order: mean spread over steps where both sides
    exist, population variance of the per-step log return, mean executed volume per step."""
    n = float(len(states) * S_total)
    ns = float(np.sum(states["n_spread"].astype(np.float64)))
    spread = float(np.sum(states["sum_spread"].astype(np.float64))) / ns if ns > 0 else np.nan
    mr = float(np.sum(states["sum_r"])) / n
    var = float(np.sum(states["sum_r2"])) / n - mr * mr
    vol = float(np.sum(states["sum_vol"].astype(np.float64))) / n
    return spread, var, vol


def exact_stats(theta, draw_ids, seed=workloads.CALIB_SEED, S=workloads.CALIB_S,
                markets_per_draw=workloads.CALIB_MARKETS, chunk_draws=8192, timing=None, tuning=None):
    """Exact statistics of every parameter row (the engine, one launch per chunk).

    theta: (n, 4); draw_ids: (n,) global draw index of each row (market index of replica r of
    draw d is d * markets_per_draw + r, so any subset reproduces the full sweep's markets).
    tuning: the engine's schedule (see ``sweep_tuning``), None for the default one.
    Returns (n, 3) float64.  If timing is a list, the kernel milliseconds of each launch are
    appended to it."""
    theta = np.atleast_2d(theta)
    draw_ids = np.asarray(draw_ids, dtype=np.int64)
    out = np.zeros((len(theta), 3))
    for c0 in range(0, len(theta), chunk_draws):
        th = theta[c0:c0 + chunk_draws]
        ids = draw_ids[c0:c0 + chunk_draws]
        d = workloads.calibration_markets(th, markets_per_draw=markets_per_draw)
        mids = (ids[:, None] * markets_per_draw + np.arange(markets_per_draw)[None, :]).ravel()
        ens = engine.Ensemble(d, seed, market_ids=mids.astype(np.uint32), tuning=tuning)
        ens.step(S)
        if timing is not None:
            timing.append(ens.last_step_ms())
        st = ens.read_state()
        ens.close()
        out[c0:c0 + len(th)] = pooled_rows(st.reshape(len(th), markets_per_draw), S)
    return out


def sweep_tuning(seed=workloads.CALIB_SEED, markets_per_draw=workloads.CALIB_MARKETS, n_probe=4096):
    """The autotuner's schedule for the calibration sweep's markets (one size class: L = 256,
    A = 1024), probed on a chunk of draws; the exact sweep runs in it."""
    from . import autotune
    theta = workloads.calibration_params(n_probe, seed=6)
    d = workloads.calibration_markets(theta, markets_per_draw=markets_per_draw)
    return autotune.tune(d, seed=seed)


def _schedule_summary(tn):
    if not tn:
        return "default"
    return {"waves_per_group": tn.get("waves_per_group"),
            "waves_per_market": sorted(set(tn.get("waves_per_market", {}).values())),
            "overlap": sorted(set(tn.get("overlap", {}).values()))}


def pooled_rows(states, S_total):
    """``pooled`` for every row of a (draws, markets) array of states."""
    n = float(states.shape[1] * S_total)
    ns = states["n_spread"].astype(np.float64).sum(axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        spread = states["sum_spread"].astype(np.float64).sum(axis=1) / ns
    mr = states["sum_r"].sum(axis=1) / n
    var = states["sum_r2"].sum(axis=1) / n - mr * mr
    vol = states["sum_vol"].astype(np.float64).sum(axis=1) / n
    return np.stack([spread, var, vol], axis=1)


def features(theta):
    """The engine's parameters of each draw (n_noise/A, n_mom/A, K, Q), scaled to [-1, 1] by
    their ranges (K in [2, 32], Q in [9, 199])."""
    d = workloads.calibration_markets(np.atleast_2d(theta), markets_per_draw=1)
    A = float(workloads.CALIB_A)
    f = np.stack([d["n_noise"] / A, d["n_mom"] / A, (d["K"] - 2.0) / 30.0, (d["Q"] - 9.0) / 190.0],
                 axis=1)
    return (2.0 * f - 1.0).astype(np.float32)


class TargetScaler:
    """log of each statistic, centred on the training mean (scaled by the training deviation
    if standardize)."""

    def __init__(self, Y, standardize=False):
        L = np.log(Y)
        self.mu = L.mean(axis=0)
        self.sd = L.std(axis=0) + 1e-12 if standardize else np.ones(L.shape[1])

    def fwd(self, Y):
        return ((np.log(Y) - self.mu) / self.sd).astype(np.float32)

    def inv(self, Z):
        return np.exp(np.asarray(Z, dtype=np.float64) * self.sd + self.mu)


def train(net, X, Z, epochs=300, batch=1024, lr=3e-3, lr_min=1e-5, seed=0, huber_delta=0.05, log=None,
          timing=None):
    """Adam on the Huber loss (huber_delta; None: squared error) of the log targets, cosine
    learning rate.  Each step is one ``cae_mlp_train_step`` call (two launches) on the rows a
    per-epoch device permutation selects.  If timing is a dict, the mean wall time per step
    (host launch rate, measured over the whole run) is stored in it."""
    import torch
    n = len(X)
    xd = torch.from_numpy(np.ascontiguousarray(X)).to(net.device)
    zd = torch.from_numpy(np.ascontiguousarray(Z)).to(net.device)
    g = torch.Generator(device=net.device)
    g.manual_seed(seed)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    step = 0
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, device=net.device, generator=g).to(torch.int32)
        for b in range(steps_per_epoch):
            rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * step / total))
            net.train_step_fused(xd, zd, float(rate), idx=perm[b * batch:(b + 1) * batch],
                                 huber_delta=huber_delta)
            step += 1
        if ep % max(1, epochs // 10) == 0 or ep == epochs - 1:
            hist.append((ep, float(net.loss.item())))
            if log:
                log("epoch %d loss %.5f" % hist[-1])
    torch.cuda.synchronize()
    if timing is not None:
        timing["steps"] = step
        timing["us_per_step"] = 1e6 * (time.perf_counter() - t0) / max(step, 1)
    return hist


def predict(net, X, scaler, batch=None):
    import torch
    xd = torch.from_numpy(np.ascontiguousarray(X)).to(net.device)
    return scaler.inv(net.predict(xd).cpu().numpy())


def rel_err(pred, exact):
    return np.abs(pred - exact) / np.abs(exact)


def linear_baseline(Xtr, Ztr, Xte, scaler):
    """Least squares on the scaled parameters (with intercept), in the same log space."""
    A = np.hstack([Xtr.astype(np.float64), np.ones((len(Xtr), 1))])
    coef, *_ = np.linalg.lstsq(A, Ztr.astype(np.float64), rcond=None)
    return scaler.inv(np.hstack([Xte.astype(np.float64), np.ones((len(Xte), 1))]) @ coef)


def summary(err):
    return {name: {"mean": float(np.mean(err[:, k])), "p95": float(np.percentile(err[:, k], 95)),
                   "max": float(np.max(err[:, k]))} for k, name in enumerate(STAT_NAMES)}


def generate(n_draws=65536, markets_per_draw=workloads.CALIB_MARKETS, S=workloads.CALIB_S,
             seed=workloads.CALIB_SEED):
    """Exact statistics of the whole sweep: training draws, then the held-out draws in launches
    of their own (that held-out sweep is what the surrogate replaces, and it is timed)."""
    import torch
    theta = workloads.calibration_params(n_draws)
    ids = np.arange(n_draws)
    tr, te = workloads.test_split(n_draws)
    tn = sweep_tuning(seed, markets_per_draw)
    t0 = time.perf_counter()
    Ytr = exact_stats(theta[tr], ids[tr], seed, S, markets_per_draw, tuning=tn)
    gen_s = time.perf_counter() - t0
    kern = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Yte = exact_stats(theta[te], ids[te], seed, S, markets_per_draw, timing=kern, tuning=tn)
    exact_wall = time.perf_counter() - t0
    return {"theta": theta, "ids": ids, "tr": tr, "te": te, "Ytr": Ytr, "Yte": Yte,
            "markets_per_draw": markets_per_draw, "S": S, "seed": seed, "generate_train_s": gen_s,
            "exact_test_sweep_s": sum(kern) * 1e-3, "exact_test_sweep_wall_s": exact_wall,
            "tuning": tn}


def fit_and_evaluate(data, epochs=300, hidden=256, batch=1024, lr=3e-3, huber_delta=0.05, noise_draws=256,
                     log=None):
    """Train on the training draws, score the held-out draws against their exact statistics,
    compare with predictors that use no network, and time the surrogate's held-out sweep."""
    import torch
    from . import mlp
    theta, ids, tr, te = data["theta"], data["ids"], data["tr"], data["te"]
    Ytr, Yte = data["Ytr"], data["Yte"]
    ok_tr = np.all(np.isfinite(Ytr) & (Ytr > 0), axis=1)
    ok_te = np.all(np.isfinite(Yte) & (Yte > 0), axis=1)
    Xtr, Xte = features(theta[tr][ok_tr]), features(theta[te][ok_te])
    scaler = TargetScaler(Ytr[ok_tr])
    Ztr = scaler.fwd(Ytr[ok_tr])
    net = mlp.MLP(4, hidden, 3, max_batch=8192, seed=0)
    t0 = time.perf_counter()
    ttime = {}
    hist = train(net, Xtr, Ztr, epochs=epochs, batch=batch, lr=lr, huber_delta=huber_delta, log=log, timing=ttime)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    pred = predict(net, Xte, scaler)
    err = rel_err(pred, Yte[ok_te])
    # predictors without the network: the training mean, and least squares on the parameters
    mean_pred = np.tile(scaler.inv(np.zeros((1, 3))), (len(Xte), 1))
    lin_pred = linear_baseline(Xtr, Ztr, Xte, scaler)
    # Monte-Carlo noise floor: held-out draws re-simulated with another engine seed
    te_ok = te[ok_te]
    sub = np.arange(min(noise_draws, len(te_ok)))
    Yalt = exact_stats(theta[te_ok[sub]], ids[te_ok[sub]], data["seed"] + 1000, data["S"],
                       data["markets_per_draw"], tuning=data.get("tuning"))
    noise = rel_err(Yalt, Yte[ok_te][sub])
    # surrogate sweep of the held-out parameters (device resident; events on its stream)
    xd = torch.from_numpy(Xte).to(net.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(7):
        e0.record()
        net.predict(xd)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    sur_s = float(np.median(times))
    rep = {
        "draws": len(theta), "markets_per_draw": data["markets_per_draw"], "steps": data["S"],
        "train_draws": int(ok_tr.sum()), "test_draws": int(ok_te.sum()),
        "dropped_draws": int((~ok_tr).sum() + (~ok_te).sum()),
        "exact_test_sweep_s": data["exact_test_sweep_s"],
        "exact_test_sweep_wall_s": data["exact_test_sweep_wall_s"],
        "exact_schedule": _schedule_summary(data.get("tuning")),
        "surrogate_test_sweep_s": sur_s, "speedup": data["exact_test_sweep_s"] / sur_s,
        "test_events": float(len(te) * data["markets_per_draw"] * workloads.CALIB_A * data["S"]),
        "surrogate_rel_err": summary(err),
        "mean_predictor_rel_err": summary(rel_err(mean_pred, Yte[ok_te])),
        "linear_predictor_rel_err": summary(rel_err(lin_pred, Yte[ok_te])),
        "mc_noise_rel_diff": summary(noise),
        "generate_train_s": data["generate_train_s"], "train_s": train_s,
        "train_steps": ttime.get("steps"), "train_us_per_step": ttime.get("us_per_step"),
        "train_loss": hist[-1][1], "epochs": epochs, "batch": batch, "lr": lr, "hidden": hidden,
        "huber_delta": huber_delta,
    }
    return rep, net, scaler


def _log_dist(Y, Yt):
    return np.mean(np.abs(np.log(Y) - np.log(Yt)), axis=-1)


def calibration_demo(net, scaler, data, n_targets=16, n_candidates=65536, verify=4, seed=55):
    """Calibration: find parameters whose exact statistics match a target.  Targets are held-out
    draws' exact statistics.  Surrogate-driven: rank n_candidates random parameter vectors by
    the surrogate, verify the best `verify` with the engine, keep the exactly best.
    Exact-only: evaluate candidates with the engine only, as many as fit in the same wall time.
    Reported distance: mean |log stat - log target| of the chosen parameters' exact statistics."""
    import torch
    te = data["te"]
    ok = np.all(np.isfinite(data["Yte"]) & (data["Yte"] > 0), axis=1)
    rng = np.random.default_rng(seed)
    tgt = rng.choice(np.nonzero(ok)[0], n_targets, replace=False)
    cand = workloads.calibration_params(n_candidates, seed=seed)
    Xc = torch.from_numpy(features(cand)).to(net.device)
    base = 10_000_000  # generator market ids of candidate draws, away from the sweep's ids
    sur_d, exact_d, n_exact, t_sur = [], [], [], []
    for k, ti in enumerate(tgt):
        Yt = data["Yte"][ti]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = scaler.inv(net.predict(Xc).cpu().numpy())
        best = np.argsort(_log_dist(P, Yt[None, :]))[:verify]
        Yv = exact_stats(cand[best], base + best, data["seed"], data["S"], data["markets_per_draw"],
                         tuning=data.get("tuning"))
        dv = _log_dist(Yv, Yt[None, :])
        t_budget = time.perf_counter() - t0
        sur_d.append(float(dv.min()))
        t_sur.append(t_budget)
        # exact-only search with the same wall time: grow the batch while it fits the budget
        n, best_exact = verify, np.inf
        while True:
            t0 = time.perf_counter()
            Ye = exact_stats(cand[:n], base + np.arange(n), data["seed"], data["S"], data["markets_per_draw"],
                             tuning=data.get("tuning"))
            dt = time.perf_counter() - t0
            if dt > t_budget and n > verify:
                break
            best_exact = float(_log_dist(Ye, Yt[None, :]).min())
            used = n
            if dt > t_budget:
                break
            n *= 2
        exact_d.append(best_exact)
        n_exact.append(used)
    return {"targets": int(n_targets), "candidates": int(n_candidates), "verified": int(verify),
            "surrogate_search_s_mean": float(np.mean(t_sur)),
            "surrogate_dist_mean": float(np.mean(sur_d)), "surrogate_dist_median": float(np.median(sur_d)),
            "exact_only_candidates_mean": float(np.mean(n_exact)),
            "exact_only_dist_mean": float(np.mean(exact_d)), "exact_only_dist_median": float(np.median(exact_d)),
            "surrogate_better_on": int(np.sum(np.array(sur_d) < np.array(exact_d)))}


def run(n_draws=65536, epochs=300, log=None, demo=True, **kw):
    data = generate(n_draws)
    rep, net, scaler = fit_and_evaluate(data, epochs=epochs, log=log, **kw)
    if demo:
        rep["calibration"] = calibration_demo(net, scaler, data)
    return rep, net, scaler
