"""Pin of the ensemble outputs the calibration sweep reads (section IV-J: mean post-auction
spread, variance of the log return, mean volume), pooled over markets and steps.

The per-step values of two markets over three steps are written out by hand; the expected
outputs come from those lists (the spread over the steps where both sides are quoted, the
population variance of all M*S returns via the statistics module, the volume per market and
step), not from the per-market sums the oracle pools.  A spread divided by M*S, a variance
with an n - 1 divisor, or a volume divided by S alone each fail here.
"""
import math
import statistics
from fractions import Fraction

import numpy as np
import pytest

# market -> per-step (volume, spread or None when a side is empty, log return)
STEPS = {
    0: [(5, 2, 0.5), (0, None, -0.25), (7, 4, 0.25)],
    1: [(1, None, 0.0), (2, None, 0.0), (4, None, 0.5)],  # never quoted on both sides
}
S_TOTAL = 3


def _states(orc, steps):
    st = np.zeros(len(steps), orc.STATE_DTYPE)
    for m, rows in steps.items():
        st[m]["steps_done"] = len(rows)
        st[m]["sum_vol"] = sum(v for v, _, _ in rows)
        st[m]["n_trade"] = sum(1 for v, _, _ in rows if v > 0)
        st[m]["sum_spread"] = sum(s for _, s, _ in rows if s is not None)
        st[m]["n_spread"] = sum(1 for _, s, _ in rows if s is not None)
        st[m]["sum_r"] = math.fsum(r for _, _, r in rows)
        st[m]["sum_r2"] = math.fsum(r * r for _, _, r in rows)
    return st


def _expected(steps):
    spreads = [s for rows in steps.values() for _, s, _ in rows if s is not None]
    returns = [Fraction(r) for rows in steps.values() for _, _, r in rows]
    vols = [v for rows in steps.values() for v, _, _ in rows]
    spread = Fraction(sum(spreads), len(spreads)) if spreads else None
    return spread, statistics.pvariance(returns), Fraction(sum(vols), len(vols))


def test_hand_values():
    """The hand case's expected outputs, written as exact fractions."""
    spread, var, vol = _expected(STEPS)
    assert spread == 3                      # (2 + 4) / 2 quoted steps
    assert var == Fraction(11, 144)         # mean 1/6; squared deviations sum to 66/144
    assert vol == Fraction(19, 6)           # 19 shares over 2 markets x 3 steps


def test_oracle_pooled_stats(orc):
    spread, var, vol = orc.pooled_stats(_states(orc, STEPS), S_TOTAL)
    e_spread, e_var, e_vol = _expected(STEPS)
    assert spread == pytest.approx(float(e_spread), rel=1e-15)
    assert var == pytest.approx(float(e_var), rel=1e-12)
    assert vol == pytest.approx(float(e_vol), rel=1e-15)
    # the wrong readings a slip would give are far from the pinned values
    assert abs(spread - 6.0 / 6.0) > 1.0                    # spread / (M*S)
    assert abs(var - float(e_var) * 6.0 / 5.0) > 1e-3        # n - 1 divisor
    assert abs(vol - 19.0 / 3.0) > 1.0                      # volume / S only


def test_oracle_pooled_stats_no_quotes(orc):
    """No step with both sides quoted: the mean spread is undefined (NaN), the rest is not."""
    steps = {0: STEPS[1]}
    spread, var, vol = orc.pooled_stats(_states(orc, steps), S_TOTAL)
    _, e_var, e_vol = _expected(steps)
    assert math.isnan(spread)
    assert var == pytest.approx(float(e_var), rel=1e-12)
    assert vol == pytest.approx(float(e_vol), rel=1e-15)


def test_surrogate_pooling_matches_hand_values(orc):
    """The product's host-side pooling of engine states (per draw, markets in order) gives the
    same hand values."""
    from paper_2606_21784_amd import surrogate
    st = _states(orc, STEPS)
    e_spread, e_var, e_vol = _expected(STEPS)
    rows = surrogate.pooled_rows(st.reshape(1, 2), S_TOTAL)
    np.testing.assert_allclose(rows[0], [float(e_spread), float(e_var), float(e_vol)], rtol=1e-12)
    two = np.stack([st, st])  # two draws with identical markets pool identically
    np.testing.assert_allclose(surrogate.pooled_rows(two, S_TOTAL),
                               np.tile(rows[0], (2, 1)), rtol=0)
    np.testing.assert_allclose(surrogate.pooled(st, S_TOTAL), rows[0], rtol=1e-12)
