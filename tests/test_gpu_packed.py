"""Packed small markets (P = 2 or 4 markets per wave, one lane segment each, for the orders and
the clearing) against the oracle, bit for bit: ragged populations and grids within a wave,
every agent class, segment counts that leave part of the last wave empty, traces, step splits,
and mixed with unpacked markets, mid-price and SplitMix64 markets in one launch.  Through the
C ABI."""
import numpy as np
import pytest

import oracle as O
from paper_2606_21784_amd import workloads as W

pytestmark = pytest.mark.gpu

INT_FIELDS = ["last", "prev", "steps_done", "n_trade", "sum_vol", "sum_px", "sum_spread",
              "n_spread", "ref2", "reserved"]


def _engine():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_21784_amd import engine
    return engine


def _pack_all(P, G=4):
    return {"waves_per_group": G, "pack": {c: P for c in range(40)}}


def _check(descs, seed, steps, tuning, expect_pack=True):
    E = _engine()
    ens = E.Ensemble(descs, seed, tuning=tuning)
    used = ens.tuning()
    if expect_pack:
        assert used["pack"], "no class was packed"
    for S in steps:
        ens.step(S)
    st, bk = ens.read_state(), ens.read_books()
    ens.close()
    rst, rbk = O.run(descs, seed, sum(steps))
    np.testing.assert_array_equal(bk, rbk)
    for f in INT_FIELDS:
        np.testing.assert_array_equal(st[f], rst[f], err_msg=f)
    for f in ("sum_r", "sum_r2"):
        np.testing.assert_allclose(st[f], rst[f], rtol=1e-6, atol=1e-300, err_msg=f)
    return used


@pytest.mark.parametrize("P", [2, 4])
@pytest.mark.parametrize("G", [1, 4, 8])
def test_packed_uniform(P, G):
    """37 markets (not a multiple of G P) of 16 agents on 64 ticks."""
    d = W.uniform(37, 64, 16, 8, 10)
    _check(d, 21, [50], _pack_all(P, G))


@pytest.mark.parametrize("P", [2, 4])
@pytest.mark.parametrize("cfg", [
    # L, A, K, Q, n_noise, n_mom, h
    (1, 1, 0, 1, 1, 0, 0),
    (5, 7, 2, 3, 3, 2, 1),
    (32, 16, 4, 10, 8, 4, 2),
    (64, 17, 8, 100, 17, 0, 2),
    (64, 33, 30, 7, 10, 13, 5),
    (64, 100, 3, 50, 40, 40, 2),
    (48, 127, 64, 9, 0, 127, 3),
])
def test_packed_ragged_and_mixed_agents(P, cfg):
    L, A, K, Q, nn, nm, h = cfg
    d = W.uniform(11, L, A, K, Q, n_noise=nn, n_mom=nm, h=h)
    _check(d, 77, [40], _pack_all(P))


def test_packed_books_of_128_ticks():
    """Two markets per wave on 128-tick books (4 ticks per lane of a 32-lane segment), with
    prices driven to the book edges by offsets wider than the book."""
    d = np.concatenate([W.uniform(9, 128, 16, 8, 10), W.uniform(9, 100, 40, 200, 5, n_noise=30, n_mom=5, h=3),
                        W.uniform(5, 128, 64, 16, 100)])
    _check(d, 5, [30, 1, 19], _pack_all(2, 8))


@pytest.mark.parametrize("G", [4, 16])
def test_packed_four_books_of_128_ticks(G):
    """Four markets per wave on books of up to 128 ticks (8 ticks per lane of a 16-lane
    segment): the agent-sweep shape (A = 16, L = 128), books of 65..128 ticks next to smaller
    ones in the same waves, mixed agent classes, and offsets wider than the book."""
    d = np.concatenate([W.uniform(23, 128, 16, 8, 10),
                        W.uniform(7, 97, 16, 300, 7, n_noise=9, n_mom=4, h=3),
                        W.uniform(5, 65, 33, 8, 100, n_noise=20, n_mom=0, h=2),
                        W.uniform(6, 40, 16, 2, 5)])
    used = _check(d, 12, [40, 7], _pack_all(4, G))
    assert set(used["pack"].values()) == {4}


@pytest.mark.parametrize("budget", [6500, 2000])
def test_packed_lds_budget_not_whole_waves(budget):
    """An LDS budget that fits 5 packed 128-tick books (4 per wave) keeps items of whole waves
    (4 books), and one that fits only one book still runs: every slot of an item's waves has its
    LDS, the empty segments of a wave included."""
    d = W.uniform(13, 128, 16, 8, 10)
    tn = dict(_pack_all(4, 8), max_lds_bytes=budget)
    _check(d, 31, [25, 4], tn)


def test_packed_populations_differ_within_a_wave():
    """Markets of one size class (A below 128) with different populations and grids share waves."""
    rng = np.random.default_rng(3)
    n = 45
    d = np.zeros(n, W.MARKET_DTYPE)
    d["L"] = rng.choice([8, 33, 64], n)
    d["A"] = rng.integers(1, 128, n)
    d["K"] = rng.integers(0, 12, n)
    d["Q"] = rng.integers(1, 101, n)
    d["n_noise"] = d["A"] // 2
    d["n_mom"] = d["A"] // 4
    d["h"] = np.minimum(2, d["L"] - 1)
    _check(d, 9, [33], _pack_all(4))


def test_packed_mixed_with_unpacked_and_other_models():
    """Packed last-tick markets in one launch with unpacked larger populations, mid-price and
    SplitMix64 markets (which never pack) and lock-step / overlapped classes."""
    mid, smx = O.model_flags(O.MODEL_MID, 3000), O.model_flags(O.MODEL_LAST, 0, O.GEN_SPLITMIX)
    d = np.concatenate([W.uniform(13, 64, 16, 8, 10, n_noise=10, n_mom=3, h=2),
                        W.uniform(6, 128, 24, 8, 10, flags=mid),
                        W.uniform(5, 64, 20, 8, 10, flags=smx),
                        W.uniform(4, 128, 700, 8, 10, n_noise=400, n_mom=200, h=2),
                        W.uniform(3, 128, 2000, 8, 10)])
    tn = {"waves_per_group": 8, "pack": {c: 4 for c in range(40)},
          "waves_per_market": {c: 4 for c in range(8, 16) if c % 8 >= 3},
          "overlap": {c: 3 for c in range(8, 16) if c % 8 >= 3}}
    used = _check(d, 31, [25, 15], tn)
    assert used["overlap"]


def test_packed_traced_series():
    import torch
    E = _engine()
    d = np.concatenate([W.uniform(10, 64, 16, 8, 10, n_noise=12, n_mom=2), W.uniform(3, 128, 300, 8, 10)])
    ens = E.Ensemble(d, 44, tuning=_pack_all(4))
    assert ens.tuning()["pack"]
    pr, vo = ens.step_traced(60)
    torch.cuda.synchronize()
    st, bk = ens.read_state(), ens.read_books()
    ens.close()
    rst, rbk, rpr, rvo = O.run(d, 44, 60, trace=True)
    np.testing.assert_array_equal(pr.cpu().numpy().view(np.uint32), rpr)
    np.testing.assert_array_equal(vo.cpu().numpy().view(np.uint32).astype(np.uint64), rvo)
    np.testing.assert_array_equal(bk, rbk)


def test_packing_needs_small_books_and_resumes_exactly():
    """A book above 128 ticks in the ensemble turns packing off (reported as such); a packed
    ensemble resumed from a checkpoint continues bit for bit."""
    E = _engine()
    d = np.concatenate([W.uniform(6, 64, 16, 8, 10), W.uniform(2, 256, 16, 8, 10)])
    used = _check(d, 8, [20], _pack_all(4), expect_pack=False)
    assert not used["pack"]
    d = W.uniform(21, 64, 16, 8, 10, n_noise=9, n_mom=5)
    rst, rbk = O.run(d, 6, 70)
    a = E.Ensemble(d, 6, tuning=_pack_all(2))
    a.step(31)
    st, bk = a.read_state(), a.read_books()
    a.close()
    b = E.Ensemble(d, 6, tuning=_pack_all(4))
    b.write_state(st, bk)
    b.step(39)
    np.testing.assert_array_equal(b.read_books(), rbk)
    np.testing.assert_array_equal(b.read_state()["n_spread"], rst["n_spread"])
    b.close()


def test_packed_many_launches():
    """Many short launches: the work queue resets after every packed launch."""
    E = _engine()
    d = W.uniform(300, 64, 16, 8, 10)
    ens = E.Ensemble(d, 2, tuning=_pack_all(4, 4))
    for _ in range(12):
        ens.step(3)
    bk = ens.read_books()
    ens.close()
    _, rbk = O.run(d, 2, 36)
    np.testing.assert_array_equal(bk, rbk)


def _segment_books(L, seg, rng):
    """Books whose crossing of demand and supply lands on the edges of the ticks a lane of a
    seg-lane segment owns, on the first and last tick or nowhere, with ties over a plateau,
    separated and one-sided books, and large quantities.  Returns (n, 2, L) uint32."""
    tpl = 1
    while seg * tpl < L:
        tpl *= 2
    edges = sorted({q for e in range(0, L + 1, tpl) for q in (e - 1, e, e + 1) if 0 <= q < L})
    out = []
    for q in edges:
        for below in (0, 1, 2):
            b = np.zeros((2, L), np.uint64)
            b[1, : q + 1] = 3
            b[0, q:] = 2
            b[0, q] += below * 3 * q
            out.append(b)
        b = np.zeros((2, L), np.uint64)  # a plateau of equal volume over [q, top]
        b[0, L - 1] = 7
        b[1, q] = 7
        out.append(b)
        b = np.zeros((2, L), np.uint64)  # separated: nothing trades
        b[0, :q] = 5
        b[1, q:] = 5
        out.append(b)
    for side in (0, 1):
        b = np.zeros((2, L), np.uint64)
        b[side] = rng.integers(0, 9, L)
        out.append(b)
    for _ in range(12):
        b = np.zeros((2, L), np.uint64)  # sparse, often on lane edges, some large quantities
        for side in (0, 1):
            k = int(rng.integers(1, 5))
            pool = edges if rng.random() < 0.5 else list(range(L))
            b[side, rng.choice(pool, size=k)] += rng.choice([1, 2, 5, (1 << 29) // k], size=k).astype(np.uint64)
        out.append(b)
    return np.stack(out).astype(np.uint32)


@pytest.mark.parametrize("P", [2, 4])
def test_packed_clearing_structured_books(P):
    """The packed clearing (one lane segment per book, DPP-row reductions for 16-lane segments)
    on books built to cross on the edges of a lane's ticks, on the first or last tick or nowhere,
    with ties, with nothing to trade, one-sided and with large quantities: each market starts
    from such a book (cae_write_state) and steps once with one agent of one share, against the
    oracle started from the same state."""
    E = _engine()
    rng = np.random.default_rng(40 + P)
    for L in (1, 2, 7, 15, 16, 17, 31, 32, 33, 48, 63, 64, 65, 100, 127, 128):
        if L > 512 // P:
            continue
        books = _segment_books(L, 64 // P, rng)
        n = books.shape[0]
        d = W.uniform(n, L, 1, 0, 1, h=min(2, L - 1))
        st = np.zeros(n, O.STATE_DTYPE)
        st["last"] = rng.integers(0, L, n)
        st["prev"] = rng.integers(0, L, n)
        st["ref2"] = 2 * st["last"]
        st["steps_done"] = books.reshape(n, -1).astype(np.uint64).sum(axis=1) + 1  # the book's shares fit
        bk = books.reshape(-1)
        ens = E.Ensemble(d, 3, tuning=_pack_all(P))
        assert set(ens.tuning()["pack"].values()) == {P}, L
        ens.write_state(st, bk)
        ens.step(1)
        gst, gbk = ens.read_state(), ens.read_books()
        ens.close()
        rst, rbk = O.run(d, 3, 1, states=st, book=bk)
        np.testing.assert_array_equal(gbk, rbk, err_msg="L=%d" % L)
        for f in INT_FIELDS:
            np.testing.assert_array_equal(gst[f], rst[f], err_msg="L=%d %s" % (L, f))
        for f in ("sum_r", "sum_r2"):
            np.testing.assert_allclose(gst[f], rst[f], rtol=1e-6, atol=1e-300, err_msg=f)
