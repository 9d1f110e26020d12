"""Calibration surrogate end to end at a reduced size: the engine generates the sweep, the
project's kernels train the network, the engine scores it.  The network must beat the
predictors that use no network, and the engine's pooled statistics must equal the oracle's."""
import numpy as np
import pytest

import oracle
from paper_2606_21784_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sur():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_21784_amd import surrogate
    return surrogate


def test_exact_statistics_match_oracle():
    SG = _sur()
    theta = W.calibration_params(40)[[3, 17, 29]]
    ids = np.array([3, 17, 29])
    Y = SG.exact_stats(theta, ids, seed=5, S=200, markets_per_draw=4)
    for k in range(3):
        d = W.calibration_markets(theta[k:k + 1], markets_per_draw=4)
        mids = ids[k] * 4 + np.arange(4)
        st, _ = oracle.run(d, 5, 200, ids=mids)
        ref = oracle.pooled_stats(st, 200)
        np.testing.assert_allclose(Y[k], ref, rtol=1e-9)


def test_exact_statistics_sweep_schedule_full_steps():
    """The calibration sweep's exact statistics as the sweep computes them: 64 markets per draw,
    2000 steps, in the autotuner's schedule for the sweep (the one the timed held-out sweep
    runs), three draws against the oracle's pooled statistics."""
    SG = _sur()
    tn = SG.sweep_tuning()
    theta = W.calibration_params(100)[[9, 19, 58]]
    ids = np.array([9, 19, 58])
    Y = SG.exact_stats(theta, ids, tuning=tn)
    S, mpd = W.CALIB_S, W.CALIB_MARKETS
    for k in range(3):
        d = W.calibration_markets(theta[k:k + 1], markets_per_draw=mpd)
        st, _ = oracle.run(d, W.CALIB_SEED, S, ids=ids[k] * mpd + np.arange(mpd))
        np.testing.assert_allclose(Y[k], oracle.pooled_stats(st, S), rtol=1e-9)


def test_surrogate_beats_networkless_predictors():
    SG = _sur()
    data = SG.generate(n_draws=2048, markets_per_draw=16, S=400)
    rep, net, scaler = SG.fit_and_evaluate(data, epochs=120, noise_draws=64)
    s, lin, mean = (rep[k] for k in ("surrogate_rel_err", "linear_predictor_rel_err",
                                     "mean_predictor_rel_err"))
    print("surrogate", s, "linear", lin, "mean", mean, "speedup", rep["speedup"], flush=True)
    for name in ("logret_variance", "mean_volume"):
        assert s[name]["mean"] < 0.5 * lin[name]["mean"], (name, s[name], lin[name])
        assert s[name]["mean"] < 0.5 * mean[name]["mean"], (name, s[name], mean[name])
    # the spread is nearly linear in the parameters: the network still beats both, by less
    assert s["mean_spread"]["mean"] < 0.8 * lin["mean_spread"]["mean"], (s["mean_spread"], lin["mean_spread"])
    assert s["mean_spread"]["mean"] < 0.8 * mean["mean_spread"]["mean"], (s["mean_spread"], mean["mean_spread"])
    assert rep["speedup"] > 10
    # calibration: the parameters the surrogate picks (and the engine verifies) reproduce the
    # targets' exact statistics closer than an exact-only search in the same wall time
    demo = SG.calibration_demo(net, scaler, data, n_targets=2, n_candidates=2048, verify=2)
    print("calibration", demo, flush=True)
    assert demo["surrogate_dist_mean"] < 0.1, demo
    assert demo["surrogate_dist_mean"] < demo["exact_only_dist_mean"], demo
