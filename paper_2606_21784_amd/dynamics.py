"""Market-dynamics experiments on the traced engine (the paper's section IV-J).

The paper sweeps the fraction of momentum agents alpha_mom from 0 to 0.70 in steps of 0.05, with
the market-maker fraction fixed at 0.15 and noise traders making up the rest, runs 64
independent markets of every mix for 1000 steps and reads four stylized facts from the price
and volume series: volatility rising with alpha_mom, fat-tailed returns (positive excess
kurtosis), trading volume per step, and volatility clustering (autocorrelation of returns
negative at lag 1 and near zero after, autocorrelation of absolute returns positive and slowly
decaying) at alpha_mom = 0.15.

Here every mix of the sweep (and, for the agent-density dimension, every population size A) is
one ensemble stepped by a single traced launch (``Ensemble.step_traced``); the statistics are
reductions over the recorded series, computed on the device in float64.  Prices are ticks;
the log return of a step is ln(L + last_t) - ln(L + last_{t-1}), the engine's own return.
"""
import time

import numpy as np

from . import engine, workloads

ALPHA_MOM = tuple(round(0.05 * i, 2) for i in range(15))  # 0.00 .. 0.70
MAKER_FRACTION = 0.15
ACF_LAGS = 20


def composition_descs(A=256, L=128, K=8, Q=10, markets=64, alphas=ALPHA_MOM,
                      maker=MAKER_FRACTION, h=2, flags=0):
    """Descriptors of the composition sweep: `markets` markets of every alpha_mom, in sweep
    order.  n_mom = round(alpha A), n_maker = round(maker A), the rest noise traders; flags
    selects the agent model (``engine.model_flags``)."""
    rows = []
    for al in alphas:
        n_mom = int(round(al * A))
        n_mk = int(round(maker * A))
        n_noise = A - n_mom - n_mk
        if n_noise < 0:
            raise ValueError("alpha_mom %.2f + maker %.2f exceed 1" % (al, maker))
        rows.append(workloads.uniform(markets, L, A, K, Q, n_noise=n_noise, n_mom=n_mom, h=h,
                                      flags=flags))
    return np.concatenate(rows)


def series_stats(price, volume, L, opening, groups, lags=ACF_LAGS):
    """Stylized facts of traced series, pooled per group of markets.

    price, volume: (M, S) integer tensors (ticks after each step; volume of each step);
    L: grid size (scalar, or per market); opening: (M,) tick before the first step;
    groups: number of consecutive equal-size market groups.  Returns a dict of float64
    tensors of shape (groups,) (ACFs: (groups, lags)):
      price_std      mean over the group's markets of the standard deviation of the price
                     level (ticks) over the steps;
      tick_change_std  standard deviation of the per-step price change (ticks), pooled;
      return_std     standard deviation of the per-step log return, pooled;
      excess_kurtosis  m4 / m2^2 - 3 of the pooled log returns (central moments);
      mean_volume    mean volume per step; trade_fraction: share of steps that traded;
      acf_r, acf_abs_r  autocorrelation of r and |r| at lags 1..lags: per market
                     sum_t x_t x_{t+k} / sum_t x_t^2 of the demeaned series, averaged over the
                     group's markets whose series is not constant.
    """
    import torch
    p = price.to(torch.float64)
    M, S = p.shape
    dev = p.device
    Lt = torch.as_tensor(L, dtype=torch.float64, device=dev).reshape(-1, 1).expand(M, 1)
    p0 = torch.as_tensor(opening, dtype=torch.float64, device=dev).reshape(M, 1)
    prev = torch.cat([p0, p[:, :-1]], dim=1)
    r = torch.log(Lt + p) - torch.log(Lt + prev)
    dp = p - prev
    g = groups
    per = M // g
    if per * g != M:
        raise ValueError("markets do not split into %d equal groups" % g)

    def pooled(x):
        return x.reshape(g, per * S)

    def cmoment(x, k):
        xc = x - x.mean(dim=1, keepdim=True)
        return (xc ** k).mean(dim=1)

    rp = pooled(r)
    m2 = cmoment(rp, 2)
    m4 = cmoment(rp, 4)
    kurt = torch.where(m2 > 0, m4 / torch.clamp(m2, min=1e-300) ** 2 - 3.0,
                       torch.full_like(m2, float("nan")))
    out = {
        "price_std": p.std(dim=1, unbiased=False).reshape(g, per).mean(dim=1),
        "tick_change_std": cmoment(pooled(dp), 2).sqrt(),
        "return_std": m2.sqrt(),
        "excess_kurtosis": kurt,
        "mean_volume": pooled(volume.to(torch.float64)).mean(dim=1),
        "trade_fraction": pooled((volume != 0).to(torch.float64)).mean(dim=1),
    }

    def acf(x):
        xc = x - x.mean(dim=1, keepdim=True)
        den = (xc * xc).sum(dim=1)
        ok = den > 0
        ks = []
        for k in range(1, lags + 1):
            num = (xc[:, :-k] * xc[:, k:]).sum(dim=1)
            ks.append(torch.where(ok, num / torch.clamp(den, min=1e-300), torch.zeros_like(num)))
        a = torch.stack(ks, dim=1).reshape(g, per, lags)
        n = ok.reshape(g, per).sum(dim=1, keepdim=True).to(torch.float64)
        return a.sum(dim=1) / torch.clamp(n, min=1.0)

    out["acf_r"] = acf(r)
    out["acf_abs_r"] = acf(r.abs())
    return out


def run_sweep(A_values=(16, 64, 256, 1024), alphas=ALPHA_MOM, markets=64, S=1000, L=128, K=8,
              Q=10, seed=6, tuning=None, flags=0):
    """The composition sweep for every population size in A_values, all in one traced launch.

    tuning: a schedule for engine.Ensemble, None for the default one, or "auto" for the
    autotuner's (probed on untraced launches of the same markets).  Returns (report, timing):
    report[A][key] = list over alphas; timing = launch time and events of the whole sweep."""
    import torch
    descs = np.concatenate([composition_descs(A, L, K, Q, markets, alphas, flags=flags)
                            for A in A_values])
    if isinstance(tuning, str) and tuning == "auto":
        from . import autotune
        tuning = autotune.tune(descs, seed=seed)
    ens = engine.Ensemble(descs, seed, tuning=tuning)
    used = ens.tuning()
    opening = torch.from_numpy(ens.read_state()["last"].astype(np.int64)).to(ens.device)
    t0 = time.perf_counter()
    price, volume = ens.step_traced(S)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = ens.last_step_ms()
    st = ens.read_state()
    ens.close()
    pr = price.to(torch.int64) & 0xFFFFFFFF
    vo = volume.to(torch.int64) & 0xFFFFFFFF
    stats = series_stats(pr, vo, L, opening, groups=len(A_values) * len(alphas))
    ng = len(alphas)
    report = {}
    spread = (st["sum_spread"].astype(np.float64).reshape(-1, markets).sum(1)
              / np.maximum(1, st["n_spread"].astype(np.float64).reshape(-1, markets).sum(1)))
    for j, A in enumerate(A_values):
        sl = slice(j * ng, (j + 1) * ng)
        rep = {"alpha_mom": list(alphas)}
        for k, v in stats.items():
            rep[k] = v[sl].cpu().numpy().tolist()
        rep["mean_spread"] = spread[sl].tolist()
        report[int(A)] = rep
    events = float(descs["A"].astype(np.float64).sum()) * S
    timing = {"markets": int(len(descs)), "steps": int(S), "events": events,
              "kernel_ms": kernel_ms, "wall_ms": 1e3 * wall,
              "events_per_s": events / (kernel_ms * 1e-3),
              "schedule": {"waves_per_group": used["waves_per_group"],
                           "waves_per_market": sorted(set(used["waves_per_market"].values())),
                           "overlap": sorted(set(used["overlap"].values())),
                           "flags": used["flags"]}}
    return report, timing


def facts(report, A=256, standard_alpha=0.15):
    """The four stylized facts read off one population size's sweep (booleans and values)."""
    rep = report[A]
    al = np.array(rep["alpha_mom"])
    j = int(np.argmin(np.abs(al - standard_alpha)))
    vol = np.array(rep["tick_change_std"])
    acf_r = np.array(rep["acf_r"][j])
    acf_a = np.array(rep["acf_abs_r"][j])
    return {
        "volatility_low_high": [float(vol[0]), float(vol.max())],
        "volatility_increases": bool(vol[-1] > vol[0]),
        "excess_kurtosis_min": float(np.nanmin(rep["excess_kurtosis"])),
        "fat_tails": bool(np.nanmin(rep["excess_kurtosis"]) > 0),
        "volume_low_high": [float(rep["mean_volume"][0]), float(max(rep["mean_volume"]))],
        "acf_r_lag1": float(acf_r[0]), "acf_abs_r_lag1": float(acf_a[0]),
        "acf_r_lags2_20_mean_abs": float(np.mean(np.abs(acf_r[1:]))),
        "acf_abs_r_lags2_20_mean": float(np.mean(acf_a[1:])),
        "volatility_clustering": bool(acf_a[0] > 0 and np.mean(acf_a[1:]) > np.mean(np.abs(acf_r[1:]))),
    }
