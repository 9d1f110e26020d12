"""Stylized-fact statistics of traced series (the paper's section IV-J experiments): checked on
CPU tensors against numpy / scipy definitions, and on the oracle's own traces of a small
composition sweep (no GPU needed)."""
import numpy as np
import pytest
import scipy.stats

import oracle as O
from paper_2606_21784_amd import dynamics


def _synthetic(M=6, S=300, L=128, seed=0):
    rng = np.random.default_rng(seed)
    steps = rng.integers(-3, 4, (M, S)) * (rng.random((M, S)) < 0.7)
    p = np.clip(L // 2 + np.cumsum(steps, axis=1), 0, L - 1)
    v = rng.integers(0, 50, (M, S)) * (steps != 0)
    return p.astype(np.int64), v.astype(np.int64)


def test_series_stats_match_numpy_and_scipy():
    import torch
    M, S, L, g = 6, 300, 128, 2
    p, v = _synthetic(M, S, L)
    opening = np.full(M, L // 2)
    out = dynamics.series_stats(torch.from_numpy(p), torch.from_numpy(v), L,
                                torch.from_numpy(opening), groups=g, lags=5)
    prev = np.hstack([opening[:, None], p[:, :-1]])
    r = np.log(L + p) - np.log(L + prev)
    dp = p - prev
    per = M // g
    for j in range(g):
        sl = slice(j * per, (j + 1) * per)
        np.testing.assert_allclose(out["price_std"][j], np.std(p[sl], axis=1).mean(), rtol=1e-12)
        np.testing.assert_allclose(out["tick_change_std"][j], np.std(dp[sl]), rtol=1e-12)
        np.testing.assert_allclose(out["return_std"][j], np.std(r[sl]), rtol=1e-12)
        np.testing.assert_allclose(out["excess_kurtosis"][j],
                                   scipy.stats.kurtosis(r[sl].ravel(), fisher=True, bias=True),
                                   rtol=1e-9)
        np.testing.assert_allclose(out["mean_volume"][j], v[sl].mean(), rtol=1e-12)
        np.testing.assert_allclose(out["trade_fraction"][j], (v[sl] != 0).mean(), rtol=1e-12)
        for key, x in (("acf_r", r[sl]), ("acf_abs_r", np.abs(r[sl]))):
            acfs = []
            for row in x:
                xc = row - row.mean()
                full = np.correlate(xc, xc, mode="full")[S - 1:]
                acfs.append(full[1:6] / full[0])
            np.testing.assert_allclose(out[key][j], np.mean(acfs, axis=0), rtol=1e-9, atol=1e-15)


def test_acf_special_cases():
    """An alternating price gives lag-1 return autocorrelation -(S-1)/S-like reversal and a
    constant |r| series is excluded (no variance); a constant price has no kurtosis."""
    import torch
    S, L = 200, 64
    alt = np.where(np.arange(S) % 2 == 0, 33, 32)[None, :]
    const = np.full((1, S), 32)
    p = np.vstack([alt, const]).astype(np.int64)
    v = np.ones_like(p)
    out = dynamics.series_stats(torch.from_numpy(p), torch.from_numpy(v), L,
                                torch.tensor([32, 32]), groups=2, lags=3)
    assert out["acf_r"][0, 0] < -0.98 and out["acf_r"][0, 1] > 0.97
    assert out["acf_abs_r"][0, 0] == 0.0  # |r| of the alternating walk is constant: excluded
    assert bool(torch.isnan(out["excess_kurtosis"][1])) and float(out["acf_r"][1, 0]) == 0.0


def test_composition_descs():
    d = dynamics.composition_descs(A=256, markets=4)
    assert len(d) == 15 * 4
    a = np.repeat(np.array(dynamics.ALPHA_MOM), 4)
    np.testing.assert_array_equal(d["n_mom"], np.rint(a * 256).astype(np.uint32))
    assert np.all(d["A"] - d["n_noise"] - d["n_mom"] == round(0.15 * 256))


def test_oracle_sweep_stats_are_sane():
    """On the oracle's traces of a small sweep: positive volume, returns bounded by ln 2, every
    series starting from the opening price."""
    import torch
    alphas = (0.0, 0.35, 0.7)
    d = dynamics.composition_descs(A=64, markets=4, alphas=alphas)
    st, bk, pr, vo = O.run(d, 6, 150, trace=True)
    out = dynamics.series_stats(torch.from_numpy(pr.astype(np.int64)),
                                torch.from_numpy(vo.astype(np.int64)), 128,
                                torch.full((len(d),), 64), groups=len(alphas))
    assert np.all(out["mean_volume"].numpy() > 0)
    assert np.all(out["return_std"].numpy() < np.log(2))
    tot = out["mean_volume"].numpy() * 4 * 150
    np.testing.assert_allclose(tot, st["sum_vol"].reshape(3, 4).sum(1).astype(np.float64))


def _facts_on_oracle(flags, alphas=(0.0, 0.15, 0.7), A=256, markets=8, S=1000):
    import torch
    d = dynamics.composition_descs(A=A, markets=markets, alphas=alphas, flags=flags)
    st, bk, pr, vo = O.run(d, 6, S, trace=True)
    out = dynamics.series_stats(torch.from_numpy(pr.astype(np.int64)),
                                torch.from_numpy(vo.astype(np.int64)), 128,
                                torch.full((len(d),), 64), groups=len(alphas))
    return {k: v.numpy() for k, v in out.items()}


def test_reproduced_facts_last_tick_model():
    """What the agent-mix sweep of section IV-J reproduces in the last-tick model: volatility
    (tick-change s.d. and price-level s.d.) and volume per step rise from alpha_mom = 0 to 0.7.
    Not reproduced here, so not asserted: fat tails and volatility clustering (they depend on
    constants the paper does not state)."""
    f = _facts_on_oracle(0)
    assert f["tick_change_std"][-1] > 1.2 * f["tick_change_std"][0]
    assert f["price_std"][-1] > 2.0 * f["price_std"][0]
    assert f["mean_volume"][-1] > 1.5 * f["mean_volume"][0]


def test_reproduced_facts_mid_price_model():
    """The paper's own agent rules (mid-price reference, marketable orders with P_mkt = 0.05):
    volatility and volume rise with alpha_mom, and returns reverse at lag 1 at the standard mix
    alpha_mom = 0.15 (negative lag-1 autocorrelation, as the paper reports)."""
    from paper_2606_21784_amd._lib import MODEL_MID
    from paper_2606_21784_amd.engine import model_flags
    f = _facts_on_oracle(model_flags(MODEL_MID, 0.05))
    assert f["tick_change_std"][-1] > 1.05 * f["tick_change_std"][0]
    assert f["price_std"][-1] > 2.0 * f["price_std"][0]
    assert f["mean_volume"][-1] > 1.5 * f["mean_volume"][0]
    assert f["acf_r"][1][0] < -0.2
