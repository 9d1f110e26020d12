"""Pins of the oracle's uniform-price clearing (paper Eq. 1-2, section II-A, section IV-C).

The oracle forms D and S by running sums, picks the first maximiser of min(D, S) and fills
bids top-down and asks bottom-up.  It is checked against
  * the paper's printed L = 5 example (every intermediate value),
  * an independent unit-share formulation on every book with L <= 4 and per-tick
    quantities 0..3 (the executed volume is the largest k such that the k-th highest bid
    unit is priced at or above the k-th lowest ask unit; the residual book drops exactly
    those units), with p* found by summing D and S directly at every price,
  * invariants on random larger books.
"""
import itertools
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_worked_example_section_iv_c(orc):
    with open(os.path.join(HERE, "golden", "worked_example_l5.json")) as f:
        g = json.load(f)
    p, v, nb, na = orc.clear(g["BUY"], g["SELL"])
    assert p == g["p_star"] and v == g["volume"]
    assert nb.tolist() == g["new_bid"]
    assert na.tolist() == g["new_ask"]
    # the printed intermediate curves, from their definitions
    L = g["L"]
    D = [sum(g["BUY"][q] for q in range(p_, L)) for p_ in range(L)]
    S = [sum(g["SELL"][q] for q in range(0, p_ + 1)) for p_ in range(L)]
    assert D == g["D_cum"] and S == g["S_cum"]
    assert [min(d, s) for d, s in zip(D, S)] == g["V"]


def _unit_share_clear(bid, ask):
    """Independent formulation: match unit shares by price priority."""
    L = len(bid)
    bu = sorted([p for p in range(L) for _ in range(bid[p])], reverse=True)
    au = sorted([p for p in range(L) for _ in range(ask[p])])
    k = 0
    while k < min(len(bu), len(au)) and bu[k] >= au[k]:
        k += 1
    D = [sum(bid[q] for q in range(p, L)) for p in range(L)]
    S = [sum(ask[q] for q in range(0, p + 1)) for p in range(L)]
    V = [min(d, s) for d, s in zip(D, S)]
    assert max(V) == k  # the two definitions of executable volume agree
    pstar = V.index(k)
    nb = np.bincount(bu[k:], minlength=L) if len(bu) > k else np.zeros(L, int)
    na = np.bincount(au[k:], minlength=L) if len(au) > k else np.zeros(L, int)
    return pstar, k, nb, na


@pytest.mark.parametrize("L", [1, 2, 3, 4])
def test_exhaustive_small_books(orc, L):
    vals = range(4)
    books = np.array([list(c) for c in itertools.product(vals, repeat=2 * L)], np.uint32)
    books = books.reshape(-1, 2, L)
    ps, vs, res = orc.clear_batch(books)
    for i in range(len(books)):
        bid, ask = books[i, 0].tolist(), books[i, 1].tolist()
        p, k, nb, na = _unit_share_clear(bid, ask)
        assert vs[i] == k
        if k > 0:
            assert ps[i] == p
        else:
            assert ps[i] == 0
        assert res[i, 0].tolist() == nb.tolist(), (bid, ask)
        assert res[i, 1].tolist() == na.tolist(), (bid, ask)
        D = [sum(bid[q:]) for q in range(L)]
        S = [sum(ask[:q + 1]) for q in range(L)]
        _check_best_quotes(D, S, k, res[i, 0], res[i, 1])


def _check_best_quotes(D, S, v, nb, na):
    """The best quotes after the fill follow from the curves alone: the unmatched demand
    max(D(q) - V*, 0) falls with q and the residual bids are its drops, so the best bid is the
    highest tick with D > V*; the best ask is the lowest tick with S > V*.  (The engine's
    clearing takes them as these counts of ticks instead of scanning the residual.)"""
    D = np.asarray(D, np.int64)
    S = np.asarray(S, np.int64)
    L = len(D)
    hb = np.nonzero(np.asarray(nb))[0]
    la = np.nonzero(np.asarray(na))[0]
    nd = int(np.sum(D > v))  # the ticks with D > V* are a prefix of the book
    ns = int(np.sum(S <= v))  # the ticks with S <= V* too
    assert np.all(D[:nd] > v) and np.all(S[:ns] <= v)
    assert (hb.max() if len(hb) else None) == (nd - 1 if nd else None)
    assert (la.min() if len(la) else None) == (ns if ns < L else None)


def _check_invariants(bid, ask, p, v, nb, na):
    bid = np.asarray(bid, np.int64)
    ask = np.asarray(ask, np.int64)
    nb = np.asarray(nb, np.int64)
    na = np.asarray(na, np.int64)
    L = len(bid)
    D = np.cumsum(bid[::-1])[::-1]
    S = np.cumsum(ask)
    V = np.minimum(D, S)
    assert v == V.max()
    assert v == min(D[p], S[p]) or v == 0
    assert np.all(V[:p] < v) or v == 0
    fb, fs = bid - nb, ask - na
    assert np.all(fb >= 0) and np.all(fs >= 0)
    assert fb.sum() == v and fs.sum() == v  # conservation of shares
    if v > 0:
        assert np.all(fb[:p] == 0)  # no bid below the clearing price trades
        assert np.all(fs[p + 1:] == 0)  # no ask above it trades
    else:
        assert np.all(fb == 0) and np.all(fs == 0)
    # residual book is not crossed
    hb = np.nonzero(nb)[0]
    la = np.nonzero(na)[0]
    if len(hb) and len(la):
        assert hb.max() < la.min()
    _check_best_quotes(D, S, v, nb, na)
    # price priority: a bid level is touched only if every better level is fully filled
    for q in range(L):
        if fb[q] > 0:
            assert np.all(nb[q + 1:] == 0)
        if fs[q] > 0:
            assert np.all(na[:q] == 0)
    # closed form of the fill: fill_b(q) = min(D(q), V) - min(D(q+1), V), same for asks
    Dn = np.append(D[1:], 0)
    Sp = np.insert(S[:-1], 0, 0)
    np.testing.assert_array_equal(fb, np.minimum(D, v) - np.minimum(Dn, v))
    np.testing.assert_array_equal(fs, np.minimum(S, v) - np.minimum(Sp, v))


@pytest.mark.parametrize("L,seed", [(5, 0), (16, 1), (64, 2), (256, 3), (1024, 4)])
def test_invariants_random_books(orc, L, seed):
    rng = np.random.default_rng(seed)
    for trial in range(60):
        kind = trial % 4
        if kind == 0:  # dense
            bid = rng.integers(0, 50, L)
            ask = rng.integers(0, 50, L)
        elif kind == 1:  # sparse, narrow window as in the engine
            bid = np.zeros(L, np.int64)
            ask = np.zeros(L, np.int64)
            c = rng.integers(0, L)
            w = max(1, L // 16)
            for _ in range(40):
                t = int(np.clip(c + rng.integers(-w, w + 1), 0, L - 1))
                (bid if rng.random() < 0.5 else ask)[t] += rng.integers(1, 101)
        elif kind == 2:  # uncrossed: nothing trades
            cut = rng.integers(1, L + 1)
            bid = np.where(np.arange(L) < cut - 1, rng.integers(0, 9, L), 0)
            ask = np.where(np.arange(L) >= cut, rng.integers(0, 9, L), 0)
        else:  # ties in V across several prices
            bid = np.zeros(L, np.int64)
            ask = np.zeros(L, np.int64)
            bid[rng.integers(L // 2, L)] = 7
            ask[rng.integers(0, L // 2 + 1)] = 7
        p, v, nb, na = orc.clear(bid, ask)
        _check_invariants(bid, ask, p, v, nb, na)


def test_no_trade_leaves_book(orc):
    bid = [3, 2, 0, 0, 0, 0]
    ask = [0, 0, 0, 1, 4, 0]
    p, v, nb, na = orc.clear(bid, ask)
    assert v == 0 and p == 0
    assert nb.tolist() == bid and na.tolist() == ask


def test_tie_goes_to_lowest_tick(orc):
    # V = [0, 5, 5, 5, 0]: bids at 3, asks at 1 -> every p in 1..3 executes 5
    bid = [0, 0, 0, 5, 0]
    ask = [0, 5, 0, 0, 0]
    p, v, nb, na = orc.clear(bid, ask)
    assert (p, v) == (1, 5)
    assert nb.tolist() == [0] * 5 and na.tolist() == [0] * 5
