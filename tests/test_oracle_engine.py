"""Pins of the oracle's agent orders, step loop and statistics.

Whole trajectories have no printed values in the paper (its Table II uses another generator
and unstated agent parameters), so they are pinned by properties that any correct engine has:
step-split invariance, independence of markets, invariance under the order in which agents
are aggregated, and the clearing invariants at every step.  The agent rules (section III-C)
are pinned by their closed-form distributions and by hand cases; the statistics by a hand
case with known values.
"""
import math

import numpy as np
import pytest
from scipy import stats


def test_noise_orders_distribution(orc):
    """Offsets are uniform on {-K..K}, quantities on {1..Q}, sides a fair coin."""
    L, A, K, Q = 256, 4096, 16, 100
    d = orc.market(L, A, K, Q)
    sides, offs, qtys = [], [], []
    for s in range(8):
        side, tick, qty = orc.orders(d, 5, 1, s, 128, 128)
        sides.append(side)
        offs.append(tick.astype(int) - 128)
        qtys.append(qty)
    side, off, qty = map(np.concatenate, (sides, offs, qtys))
    assert off.min() == -K and off.max() == K
    assert qty.min() == 1 and qty.max() == Q
    assert set(np.unique(side)) == {0, 1}
    for x, lo, n in ((off, -K, 2 * K + 1), (qty, 1, Q), (side, 0, 2)):
        obs = np.bincount(x - lo, minlength=n)
        starts = np.array([-(-(v << 32) // n) for v in range(n + 1)], dtype=np.float64)
        starts[-1] = 2.0**32
        exp = np.diff(starts) / 2.0**32 * len(x)
        chi2 = ((obs - exp) ** 2 / exp).sum()
        assert 1.0 - stats.chi2.cdf(chi2, n - 1) > 1e-4
    # side and offset come from different words: independent
    tab = np.zeros((2, 2 * K + 1))
    np.add.at(tab, (side, off + K), 1)
    assert stats.chi2_contingency(tab)[1] > 1e-4


def test_noise_orders_clamped_to_grid(orc):
    L, A, K, Q = 64, 2048, 8, 10
    d = orc.market(L, A, K, Q)
    for last in (0, 3, 60, 63):
        side, tick, qty = orc.orders(d, 0, 0, 11, last, last)
        assert tick.min() >= 0 and tick.max() <= L - 1
        lo, hi = max(0, last - K), min(L - 1, last + K)
        assert tick.min() == lo and tick.max() == hi
        # every offset that falls off the grid lands on the edge tick
        if last - K < 0:
            frac = np.mean(tick == 0)
            assert abs(frac - (K - last + 1) / (2 * K + 1)) < 0.05


def test_momentum_and_maker_rules(orc):
    L, A, K, Q, h = 64, 300, 8, 10, 3
    d = orc.market(L, A, K, Q, n_noise=100, n_mom=100, h=h)
    mom = slice(100, 200)
    mk = np.arange(200, 300)
    for s in (4, 5):
        # price went up: every momentum agent buys one tick above the reference
        side, tick, qty = orc.orders(d, 2, 9, s, 30, 29)
        assert np.all(side[mom] == orc.BUY) and np.all(tick[mom] == 31)
        # price went down: they sell one tick below
        side, tick, qty = orc.orders(d, 2, 9, s, 30, 31)
        assert np.all(side[mom] == orc.SELL) and np.all(tick[mom] == 29)
        # unchanged: a fair coin, still one tick away in the side's direction
        side, tick, qty = orc.orders(d, 2, 9, s, 30, 30)
        buys = side[mom] == orc.BUY
        assert 0 < buys.sum() < 100
        assert np.all(tick[mom][buys] == 31) and np.all(tick[mom][~buys] == 29)
        # makers alternate with the parity of agent index + step, h ticks from the reference
        want_buy = ((mk + s) % 2) == 0
        assert np.all((side[200:] == orc.BUY) == want_buy)
        assert np.all(tick[200:][want_buy] == 30 - h)
        assert np.all(tick[200:][~want_buy] == 30 + h)
        assert qty.min() >= 1 and qty.max() <= Q
    # clamping at the grid edges
    side, tick, qty = orc.orders(d, 2, 9, 4, 0, 1)
    assert np.all(tick[mom] == 0)
    side, tick, qty = orc.orders(d, 2, 9, 4, 63, 62)
    assert np.all(tick[mom] == 63)
    side, tick, qty = orc.orders(d, 2, 9, 4, 1, 1)
    assert np.all(tick[200:][side[200:] == orc.BUY] == 0)


def test_initial_state(orc):
    for L in (1, 5, 64, 1024):
        st = orc.initial_state(orc.market(L, 8, 1, 1))
        assert st["last"][0] == L // 2 and st["prev"][0] == L // 2
        assert st["steps_done"][0] == 0 and st["n_trade"][0] == 0


def test_stats_hand_case(orc):
    """Three finished steps on L = 4 with hand-computed statistics."""
    L = 4
    lnp = np.log(np.array([4.0, 5.0, 6.0, 7.0]))
    st = orc.initial_state(orc.market(L, 1, 1, 1))  # last = prev = 2
    # step 1: traded 5 at tick 2; residual bid at 0, ask at 3 -> spread 3; price unchanged
    orc.update_stats([1, 0, 0, 0], [0, 0, 0, 3], 2, 5, lnp, st)
    # step 2: nothing traded; residual only a bid -> no spread
    orc.update_stats([2, 0, 0, 0], [0, 0, 0, 0], 0, 0, lnp, st)
    # step 3: traded 4 at tick 3; bid at 1, ask at 3 -> spread 2; return ln 7 - ln 6
    orc.update_stats([0, 1, 0, 0], [0, 0, 0, 1], 3, 4, lnp, st)
    s = st[0]
    assert s["last"] == 3 and s["prev"] == 2 and s["steps_done"] == 3
    assert s["n_trade"] == 2 and s["sum_vol"] == 9 and s["sum_px"] == 5
    assert s["sum_spread"] == 5 and s["n_spread"] == 2
    r = math.log(7.0) - math.log(6.0)
    assert s["sum_r"] == r and s["sum_r2"] == r * r


def _python_step(orc, d, m, seed, st, bid, ask):
    """One step assembled from the oracle's pieces, checking every clearing invariant."""
    L = int(d["L"][0])
    s = int(st["steps_done"][0])
    if int(d["flags"][0]) & 0xFF == orc.MODEL_MID:
        hb, la = np.nonzero(bid)[0], np.nonzero(ask)[0]
        ref2 = int(hb.max() + la.min()) if len(hb) and len(la) else 2 * int(st["last"][0])
        side, tick, qty = orc.orders_mid(d, m, seed, s, ref2, int(st["ref2"][0]))
    else:
        ref2 = 2 * int(st["last"][0])
        side, tick, qty = orc.orders(d, m, seed, s, int(st["last"][0]), int(st["prev"][0]))
    b = bid.astype(np.int64).copy()
    a = ask.astype(np.int64).copy()
    np.add.at(b, tick[side == orc.BUY], qty[side == orc.BUY])
    np.add.at(a, tick[side == orc.SELL], qty[side == orc.SELL])
    p, v, nb, na = orc.clear(b, a)
    fb, fs = b - nb.astype(np.int64), a - na.astype(np.int64)
    assert fb.sum() == v and fs.sum() == v and fb.min() >= 0 and fs.min() >= 0
    D = np.cumsum(b[::-1])[::-1]
    S = np.cumsum(a)
    assert v == np.minimum(D, S).max()
    if v:
        assert v == min(D[p], S[p]) and np.all(np.minimum(D, S)[:p] < v)
    hb, la = np.nonzero(nb)[0], np.nonzero(na)[0]
    if len(hb) and len(la):
        assert hb.max() < la.min()
    orc.update_stats(nb, na, p, v, orc.log_prices(L), st)
    st["ref2"] = ref2
    return nb, na


@pytest.mark.parametrize("cfg", [(64, 128, 8, 10, 128, 0, 2), (32, 40, 4, 7, 20, 10, 1),
                                 (8, 33, 3, 5, 11, 11, 2)])
def test_trajectory_invariants_and_assembly(orc, cfg):
    L, A, K, Q, nn, nm, h = cfg
    d = orc.market(L, A, K, Q, n_noise=nn, n_mom=nm, h=h)
    m, seed, S = 3, 77, 40
    st = orc.initial_state(d)
    bid = np.zeros(L, np.uint32)
    ask = np.zeros(L, np.uint32)
    for _ in range(S):
        bid, ask = _python_step(orc, d, m, seed, st, bid, ask)
    st2, bk2 = orc.market_run(d, m, seed, S)
    assert st2.tobytes() == st.tobytes()
    assert bk2.tolist() == bid.tolist() + ask.tolist()


def test_step_split_invariance(orc):
    d = orc.market(64, 128, 8, 10)
    st_a, bk_a = orc.market_run(d, 1, 0, 100)
    st_b, bk_b = orc.market_run(d, 1, 0, 37)
    st_b, bk_b = orc.market_run(d, 1, 0, 63, state=st_b, book=bk_b)
    assert st_a.tobytes() == st_b.tobytes()
    assert np.array_equal(bk_a, bk_b)


def test_market_independence(orc):
    descs = np.concatenate([orc.market(64, 128, 8, 10) for _ in range(4)])
    st, bk = orc.run(descs, 0, 50)
    for m in range(4):
        s1, b1 = orc.market_run(descs[m:m + 1], m, 0, 50)
        assert s1.tobytes() == st[m:m + 1].tobytes()
        assert np.array_equal(b1, bk[m * 128:(m + 1) * 128])
    # a sampled sub-ensemble with explicit market ids reproduces the same slices
    st2, bk2 = orc.run(descs[[3, 1]], 0, 50, ids=[3, 1])
    assert st2[0].tobytes() == st[3].tobytes() and st2[1].tobytes() == st[1].tobytes()


def test_agent_order_invariance(orc):
    d = orc.market(64, 100, 8, 10, n_noise=60, n_mom=20, h=2)
    rng = np.random.default_rng(3)
    s1, b1 = orc.market_run(d, 2, 5, 60)
    s2, b2 = orc.market_run(d, 2, 5, 60, agent_order=rng.permutation(100))
    assert s1.tobytes() == s2.tobytes() and np.array_equal(b1, b2)


def test_seed_and_market_change_the_stream(orc):
    d = orc.market(64, 128, 8, 10)
    _, b0 = orc.market_run(d, 0, 0, 20)
    _, b1 = orc.market_run(d, 1, 0, 20)
    _, b2 = orc.market_run(d, 0, 1, 20)
    _, b3 = orc.market_run(d, 0, 1 << 32, 20)
    assert not np.array_equal(b0, b1) and not np.array_equal(b0, b2)
    assert not np.array_equal(b2, b3)


def test_overflow_guard(orc):
    d = orc.market(8, 1 << 16, 1, 1 << 15)  # 2^31 per step
    orc.market_run(d, 0, 0, 1)
    with pytest.raises(ValueError):
        orc.market_run(d, 0, 0, 2)


def test_paper_scale_sanity(orc):
    """At the paper's shape (L = 128, A = 256) the price stays near the centre and volume per
    step is of the order of the quantity posted near the reference (section IV, Table II
    reports a mean clearing tick of 63.94 for its own agent mix)."""
    d = np.concatenate([orc.market(128, 256, 8, 10) for _ in range(16)])
    st, _ = orc.run(d, 0, 200)
    mean_px = st["sum_px"].sum() / st["n_trade"].sum()
    assert 44 < mean_px < 84
    assert st["n_trade"].min() > 150


def test_trace_records_each_step(orc):
    """The traced run records, per step, the reference tick after the step and the volume
    executed in it: it equals a step-by-step assembly, and the series reproduce the running
    statistics (trades, volume, price sum, log-return sums in step order) exactly."""
    descs = np.concatenate([orc.market(32, 40, 4, 7, n_noise=20, n_mom=10, h=1),
                            orc.market(64, 128, 8, 10), orc.market(5, 9, 1, 3, n_noise=0, n_mom=9)])
    S, seed = 60, 9
    st, bk, pr, vo = orc.run(descs, seed, S, trace=True)
    st0, bk0 = orc.run(descs, seed, S)
    assert st.tobytes() == st0.tobytes() and np.array_equal(bk, bk0)
    L0 = int(descs["L"][0])
    s = orc.initial_state(descs[:1])
    bid, ask = np.zeros(L0, np.uint32), np.zeros(L0, np.uint32)
    for t in range(S):
        v_before = int(s["sum_vol"][0])
        bid, ask = _python_step(orc, descs[:1], 0, seed, s, bid, ask)
        assert pr[0, t] == s["last"][0] and vo[0, t] == int(s["sum_vol"][0]) - v_before
    for i in range(len(descs)):
        L = int(descs["L"][i])
        assert vo[i].sum() == st["sum_vol"][i]
        assert (vo[i] > 0).sum() == st["n_trade"][i]
        assert pr[i][vo[i] > 0].astype(np.uint64).sum() == st["sum_px"][i]
        ref = np.concatenate([[L // 2], pr[i][:-1]]).astype(np.int64)
        assert np.all(pr[i][vo[i] == 0] == ref[vo[i] == 0])  # no trade: price unchanged
        lnp = orc.log_prices(L)
        acc, acc2 = 0.0, 0.0
        for x in lnp[pr[i]] - lnp[ref]:
            acc, acc2 = acc + x, acc2 + x * x
        assert acc == st["sum_r"][i] and acc2 == st["sum_r2"][i]
    # series of a split run concatenate to the series of the whole run
    st1, bk1, p1, v1 = orc.run(descs, seed, 25, trace=True)
    _, _, p2, v2 = orc.run(descs, seed, S - 25, states=st1, book=bk1, trace=True)
    assert np.array_equal(np.hstack([p1, p2]), pr) and np.array_equal(np.hstack([v1, v2]), vo)


def _words(orc, d, m, seed, a, s):
    if (int(d["flags"][0]) >> 8) & 0xFF == orc.GEN_SPLITMIX:
        return orc.splitmix_words([m * int(d["A"][0]) + a], [s], seed)[0]
    return orc.philox([s, a, m, 0], [seed & 0xFFFFFFFF, seed >> 32])


def _exact_mid_order(orc, d, m, seed, a, s, mid2, mid2_prev):
    """The paper's mid-price agent rules (section III-C) evaluated in exact rationals."""
    from fractions import Fraction as F
    L, K, Q = int(d["L"][0]), int(d["K"][0]), int(d["Q"][0])
    nn, nm, h = int(d["n_noise"][0]), int(d["n_mom"][0]), int(d["h"][0])
    p_mkt = F(int(d["flags"][0]) >> 16, 65536)
    w = _words(orc, d, m, seed, a, s)
    u = [F(int(x), 2**32) for x in w]
    mid, mid_prev = F(mid2, 2), F(mid2_prev, 2)
    coin = orc.BUY if u[0] < F(1, 2) else orc.SELL
    rnd = lambda x: math.floor(x + F(1, 2))
    mkt = u[3] < p_mkt
    if a < nn:
        side, price = coin, rnd(mid + K * (2 * u[1] - 1))
    elif a < nn + nm:
        side = orc.BUY if mid > mid_prev else orc.SELL if mid < mid_prev else coin
        price = rnd(mid + (1 if side == orc.BUY else -1))
    else:
        side = orc.BUY if (a + s) % 2 == 0 else orc.SELL
        price = rnd(mid - h if side == orc.BUY else mid + h)
        mkt = False
    if mkt:
        price = L - 1 if side == orc.BUY else 0
    return side, min(max(price, 0), L - 1), 1 + (int(w[2]) * Q >> 32)


@pytest.mark.parametrize("L,K,h,p16,mid2,mid2_prev", [
    (128, 8, 2, 0, 129, 129), (128, 8, 2, 6554, 128, 130), (128, 8, 2, 6554, 131, 127),
    (10, 9, 4, 32768, 1, 0), (10, 9, 4, 65535, 17, 18), (64, 1, 1, 0, 0, 0),
    (1024, 1023, 30, 1000, 2045, 3)])
def test_mid_model_orders_exact(orc, L, K, h, p16, mid2, mid2_prev):
    d = orc.market(L, 300, K, 17, n_noise=150, n_mom=90, h=h, flags=orc.model_flags(orc.MODEL_MID, p16))
    for s in (0, 7):
        side, tick, qty = orc.orders_mid(d, 5, 1234567890123, s, mid2, mid2_prev)
        for a in range(300):
            assert (side[a], tick[a], qty[a]) == _exact_mid_order(orc, d, 5, 1234567890123, a, s,
                                                                  mid2, mid2_prev), (a, s)


def test_mid_model_hand_values(orc):
    """Best bid 3, best ask 6 -> mid 4.5: makers with h = 2 post round(2.5) = 3 and round(6.5)
    = 7; momentum after a rise buys at round(5.5) = 6, after a fall sells at round(3.5) = 4."""
    d = orc.market(10, 4, 2, 1, n_noise=0, n_mom=2, h=2, flags=orc.model_flags(orc.MODEL_MID))
    side, tick, _ = orc.orders_mid(d, 0, 0, 0, 9, 8)  # mid rose from 4 to 4.5
    assert list(side[:2]) == [orc.BUY, orc.BUY] and list(tick[:2]) == [6, 6]
    assert (side[2], tick[2]) == (orc.BUY, 3) and (side[3], tick[3]) == (orc.SELL, 7)
    side, tick, _ = orc.orders_mid(d, 0, 0, 0, 9, 10)  # mid fell from 5 to 4.5
    assert list(side[:2]) == [orc.SELL, orc.SELL] and list(tick[:2]) == [4, 4]


@pytest.mark.parametrize("cfg", [(64, 128, 8, 10, 60, 40, 2, 6554), (32, 40, 4, 7, 20, 10, 1, 0),
                                 (8, 33, 3, 5, 11, 11, 2, 30000)])
def test_mid_model_assembly_and_invariants(orc, cfg):
    """Mid-price model: the oracle's steps equal an assembly from its pieces, with the
    reference read from the resting book at the start of each step; every clearing
    invariant holds."""
    L, A, K, Q, nn, nm, h, p16 = cfg
    d = orc.market(L, A, K, Q, n_noise=nn, n_mom=nm, h=h, flags=orc.model_flags(orc.MODEL_MID, p16))
    m, seed, S = 2, 99, 50
    st = orc.initial_state(d)
    bid, ask = np.zeros(L, np.uint32), np.zeros(L, np.uint32)
    for _ in range(S):
        bid, ask = _python_step(orc, d, m, seed, st, bid, ask)
    st2, bk2 = orc.market_run(d, m, seed, S)
    assert st2.tobytes() == st.tobytes()
    assert bk2.tolist() == bid.tolist() + ask.tolist()
    st3, bk3 = orc.market_run(d, m, seed, 21)
    st3, bk3 = orc.market_run(d, m, seed, S - 21, state=st3, book=bk3)
    assert st3.tobytes() == st2.tobytes() and np.array_equal(bk3, bk2)


def test_model_flags_validated(orc):
    with pytest.raises(ValueError):
        orc.market_run(orc.market(16, 8, 2, 3, flags=orc.model_flags(orc.MODEL_LAST, 5)), 0, 0, 1)
    with pytest.raises(ValueError):
        orc.market_run(orc.market(16, 8, 2, 3, flags=2), 0, 0, 1)


def test_splitmix64_known_answers(orc):
    """The first outputs of the reference SplitMix64 stream from state 0."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64_state0.json")))
    for k, v in enumerate(g["outputs"]):
        assert orc.splitmix64((k + 1) * 0x9E3779B97F4A7C15) == int(v, 16)


def test_splitmix_words_are_stream_positions(orc):
    """Channel c of agent gid at step s is the high half of stream output gid*2^34 + 4s + c;
    the words are uniform (chi-square over 64 bins)."""
    seed = 0x1234_5678_9ABC_DEF0
    gid = np.array([0, 1, 7, 2**20 + 3, 2**29 - 1], np.uint64)
    st = np.array([0, 5, 2**31, 17, 999], np.uint32)
    w = orc.splitmix_words(gid, st, seed)
    for i in range(len(gid)):
        for c in range(4):
            k = (int(gid[i]) << 34) + (int(st[i]) << 2) + c
            assert w[i, c] == orc.splitmix64(seed + (k + 1) * 0x9E3779B97F4A7C15) >> 32
    n = 40000
    w = orc.splitmix_words(np.arange(n, dtype=np.uint64), np.full(n, 3, np.uint32), 7)
    for c in range(4):
        counts = np.bincount(w[:, c] >> 26, minlength=64)
        assert stats.chisquare(counts).pvalue > 1e-4


@pytest.mark.parametrize("model", ["last", "mid"])
def test_splitmix_generator_orders(orc, model):
    """Orders drawn from the SplitMix64 reading follow the same rules: the mid-price model
    against exact rationals, the last-tick model against the closed-form mapping."""
    if model == "mid":
        d = orc.market(128, 300, 8, 17, n_noise=150, n_mom=90, h=2,
                       flags=orc.model_flags(orc.MODEL_MID, 6554, orc.GEN_SPLITMIX))
        side, tick, qty = orc.orders_mid(d, 9, 77, 4, 129, 127)
        for a in range(300):
            assert (side[a], tick[a], qty[a]) == _exact_mid_order(orc, d, 9, 77, a, 4, 129, 127)
    else:
        d = orc.market(128, 300, 8, 17, flags=orc.model_flags(gen=orc.GEN_SPLITMIX))
        side, tick, qty = orc.orders(d, 9, 77, 4, 64, 64)
        w = orc.splitmix_words(9 * 300 + np.arange(300, dtype=np.uint64), np.full(300, 4, np.uint32), 77)
        off = ((w[:, 1].astype(np.uint64) * 17) >> 32).astype(np.int64) - 8
        np.testing.assert_array_equal(tick, np.clip(64 + off, 0, 127))
        np.testing.assert_array_equal(side, (w[:, 0] >= 2**31).astype(np.uint32))
        np.testing.assert_array_equal(qty, 1 + ((w[:, 2].astype(np.uint64) * 17) >> 32))
    st, bk = orc.market_run(d, 9, 77, 40)
    st2, bk2 = orc.market_run(d, 9, 78, 40)
    assert not np.array_equal(bk, bk2)
