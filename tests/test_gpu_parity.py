"""GPU engine vs CPU oracle: bit-exact books, states and integer statistics; floating-point
statistics within 1e-6 relative (they are computed in the same order from the same table, so
in practice they are bit-equal too).  Every call goes through the C ABI."""
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


def _run_gpu(descs, seed, steps, tuning=None):
    E = _engine()
    ens = E.Ensemble(descs, seed, tuning=tuning)
    for S in steps:
        ens.step(S)
    st, bk = ens.read_state(), ens.read_books()
    tn = ens.tuning()
    ens.close()
    return st, bk, tn


def _assert_states(gpu, ref, rtol=1e-6):
    for f in INT_FIELDS:
        np.testing.assert_array_equal(gpu[f], ref[f], err_msg=f)
    for f in ("sum_r", "sum_r2"):
        np.testing.assert_allclose(gpu[f], ref[f], rtol=rtol, atol=1e-300, err_msg=f)


def _assert_books(descs, gpu_book, ref_book, ids=None):
    L = descs["L"].astype(np.int64)
    off = np.zeros(len(L), np.int64)
    off[1:] = np.cumsum(2 * L)[:-1]
    if ids is None:
        np.testing.assert_array_equal(gpu_book, ref_book)
        return
    roff = 0
    for i in ids:
        n = 2 * int(L[i])
        np.testing.assert_array_equal(gpu_book[off[i]:off[i] + n], ref_book[roff:roff + n],
                                      err_msg="market %d" % i)
        roff += n


def test_smoke_workload_full():
    w = W.smoke()
    st, bk, _ = _run_gpu(w["descs"], w["seed"], [w["S"]])
    rst, rbk = O.run(w["descs"], w["seed"], w["S"])
    _assert_books(w["descs"], bk, rbk)
    _assert_states(st, rst)
    assert (st["sum_r"] == rst["sum_r"]).all() and (st["sum_r2"] == rst["sum_r2"]).all()


@pytest.mark.parametrize("wpm,G", [(1, 1), (1, 4), (2, 2), (2, 8), (4, 4), (8, 8), (16, 16)])
def test_schedule_invariance(wpm, G):
    """Every waves-per-market / waves-per-workgroup choice gives the oracle's books."""
    descs = W.uniform(6, 64, 128, 8, 10)
    tn = {"waves_per_group": G, "waves_per_market": {c: wpm for c in range(40)}}
    st, bk, used = _run_gpu(descs, 0, [60], tuning=tn)
    assert used["waves_per_group"] == G
    rst, rbk = O.run(descs, 0, 60)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)


@pytest.mark.parametrize("cfg", [
    # L, A, K, Q, n_noise, n_mom, h  -- ragged sizes, one-lane grids, mixed agent classes
    (1, 1, 0, 1, 1, 0, 0),
    (3, 65, 2, 7, 65, 0, 1),
    (100, 1000, 9, 33, 500, 300, 3),
    (257, 777, 16, 100, 300, 300, 5),
    (1000, 130, 40, 5, 0, 130, 7),
    (1024, 3000, 64, 100, 1000, 1000, 2),
    (64, 64, 8, 10, 0, 0, 2),
])
def test_ragged_and_mixed_markets(cfg):
    L, A, K, Q, nn, nm, h = cfg
    descs = W.uniform(5, L, A, K, Q, n_noise=nn, n_mom=nm, h=h)
    st, bk, _ = _run_gpu(descs, 12345, [40])
    rst, rbk = O.run(descs, 12345, 40)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)


def test_mixed_sizes_one_launch():
    rng = np.random.default_rng(7)
    n = 40
    L = rng.choice([1, 17, 64, 100, 128, 256, 300, 512, 1000, 1024], n)
    A = rng.integers(1, 3000, n)
    d = np.zeros(n, W.MARKET_DTYPE)
    d["L"], d["A"], d["K"], d["Q"] = L, A, np.maximum(1, L // 16), rng.integers(1, 101, n)
    d["n_noise"] = A // 2
    d["n_mom"] = A // 4
    d["h"] = np.minimum(2, L - 1)
    st, bk, _ = _run_gpu(d, 99, [30])
    rst, rbk = O.run(d, 99, 30)
    _assert_books(d, bk, rbk)
    _assert_states(st, rst)


def test_step_split_and_resume():
    E = _engine()
    descs = W.uniform(8, 128, 300, 8, 20, n_noise=200, n_mom=50)
    rst, rbk = O.run(descs, 5, 100)
    ens = E.Ensemble(descs, 5)
    ens.step(37)
    mid_st, mid_bk = ens.read_state(), ens.read_books()
    ens.step(63)
    _assert_books(descs, ens.read_books(), rbk)
    _assert_states(ens.read_state(), rst)
    # checkpoint resume into a fresh ensemble
    ens2 = E.Ensemble(descs, 5)
    ens2.write_state(mid_st, mid_bk)
    ens2.step(63)
    _assert_books(descs, ens2.read_books(), rbk)
    _assert_states(ens2.read_state(), rst)
    ens.close()
    ens2.close()


@pytest.mark.parametrize("tuning", [None, {"waves_per_group": 4, "waves_per_market": {c: 4 for c in range(40)},
                                     "overlap": {c: 4 for c in range(40)}}])
def test_zero_steps_and_single_market(tuning):
    """A single market, and cae_step(0), which must leave books and states untouched (also
    between launches that continue the same market)."""
    E = _engine()
    descs = W.uniform(1, 256, 1024, 16, 100)
    ens = E.Ensemble(descs, 21, tuning=tuning)
    st0, bk0 = ens.read_state(), ens.read_books()
    ens.step(0)
    _assert_books(descs, ens.read_books(), bk0)
    _assert_states(ens.read_state(), st0)
    ens.step(30)
    ens.step(0)
    ens.step(20)
    rst, rbk = O.run(descs, 21, 50)
    _assert_books(descs, ens.read_books(), rbk)
    _assert_states(ens.read_state(), rst)
    ens.close()


def test_overflow_guard_refuses_launch():
    E = _engine()
    from paper_2606_21784_amd import _lib
    descs = W.uniform(2, 64, 2**16, 4, 2**15)  # 2^31 per step
    ens = E.Ensemble(descs, 0)
    ens.step(1)
    with pytest.raises(_lib.CaeError) as ei:
        ens.step(1)
    assert ei.value.code == _lib.CAE_EOVERFLOW
    st = ens.read_state()
    assert (st["steps_done"] == 1).all()
    ens.close()


def test_write_state_rejects_bad_input():
    E = _engine()
    from paper_2606_21784_amd import _lib
    descs = W.uniform(2, 64, 16, 4, 5)
    ens = E.Ensemble(descs, 0)
    st, bk = ens.read_state(), ens.read_books()
    bad = st.copy()
    bad["last"][0] = 64
    with pytest.raises(_lib.CaeError):
        ens.write_state(bad, bk)
    with pytest.raises(_lib.CaeError):
        ens.write_state(st[:1], bk)
    with pytest.raises(_lib.CaeError):
        ens.write_state(st, bk[:-1])
    # a book holding more shares than steps_done steps can have added (the overflow guard's
    # premise): at 0 steps any share is too many; after 3 steps at most 3 A Q = 240 per market
    fat = bk.copy()
    fat[5] = 1
    with pytest.raises(_lib.CaeError, match="shares"):
        ens.write_state(st, fat)
    st3 = st.copy()
    st3["steps_done"] = 3
    ok = bk.copy()
    ok[0], ok[64 + 1] = 120, 120  # market 0: 240 shares over its two sides
    ens.write_state(st3, ok)
    ok[2 * 64 + 7] = 241  # market 1: one share too many on one side
    with pytest.raises(_lib.CaeError, match="market 1"):
        ens.write_state(st3, ok)
    ens.close()


def test_clear_worked_example_and_random_books():
    import json
    import os
    import torch
    E = _engine()
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example_l5.json")))
    book = torch.tensor(g["BUY"] + g["SELL"], dtype=torch.int32, device="cuda")
    ps, vs = E.clear_books(book, 5, 1)
    torch.cuda.synchronize()
    assert int(ps[0]) == g["p_star"] and int(vs[0]) == g["volume"]
    res = book.cpu().numpy()
    assert res[:5].tolist() == g["new_bid"] and res[5:].tolist() == g["new_ask"]
    rng = np.random.default_rng(11)
    for L in (1, 2, 5, 63, 64, 65, 128, 200, 256, 511, 512, 1000, 1024):
        n = 37
        books = rng.integers(0, 60, size=(n, 2, L)).astype(np.uint32)
        books[::3] = 0  # empty books
        books[1::5, 0, : L // 2] = 0  # one-sided
        rp, rv, rres = O.clear_batch(books)
        dev = torch.from_numpy(books.reshape(-1).view(np.int32).copy()).cuda()
        ps, vs = E.clear_books(dev, L, n)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ps.cpu().numpy().view(np.uint32), rp)
        np.testing.assert_array_equal(vs.cpu().numpy().view(np.uint32).astype(np.uint64), rv)
        np.testing.assert_array_equal(dev.cpu().numpy().view(np.uint32).reshape(n, 2, L), rres)


def _structured_books(L, rng):
    """Books built to land the crossing of D and S on chosen ticks: at the edges of the ticks
    a lane owns, at the first and last tick, nowhere (the top tick's bids exceed every ask),
    with ties over a plateau of ticks, separated (nothing trades) and one-sided books, and a
    few large quantities.  Returns (n, 2, L) uint32."""
    tpl = 1
    while 64 * tpl < L:
        tpl *= 2
    edges = sorted({q for e in range(0, L + 1, tpl) for q in (e - 1, e, e + 1) if 0 <= q < L})
    out = []

    def book():
        return np.zeros((2, L), np.uint64)

    for q in edges:
        # asks up to q, bids from q: the crossing at q with S(q-1) below, equal to and above D(q)
        for below in (0, 1, 2):
            b = book()
            b[1, : q + 1] = 3
            b[0, q:] = 2
            b[0, q] += below * 3 * q
            out.append(b)
        b = book()  # a plateau: V is the same on every tick of [q, top]
        b[0, L - 1] = 7
        b[1, q] = 7
        out.append(b)
        b = book()  # separated: every bid below every ask, nothing trades
        b[0, :q] = 5
        b[1, q:] = 5
        out.append(b)
    for _ in range(4):
        b = book()  # no crossing below the top tick: its bids exceed all asks
        b[1, : L] = rng.integers(0, 4, L)
        b[0, L - 1] = b[1].sum() + 1 + rng.integers(0, 3)
        out.append(b)
        b = book()  # crossing at the first tick: its asks exceed all bids
        b[0, :] = rng.integers(0, 4, L)
        b[1, 0] = b[0].sum() + rng.integers(0, 3)
        out.append(b)
    for side in (0, 1):
        b = book()
        b[side] = rng.integers(0, 9, L)
        out.append(b)
    for _ in range(40):
        b = book()  # sparse: a few ticks per side, often on lane edges, some large quantities
        for side in (0, 1):
            k = int(rng.integers(1, 5))
            pool = edges if rng.random() < 0.5 else list(range(L))
            qs = rng.choice(pool, size=k)
            big = (1 << 31) // (4 * max(1, k))
            b[side, qs] += rng.choice([1, 2, 5, big], size=k).astype(np.uint64)
        out.append(b)
    books = np.stack(out)
    assert books.sum(axis=2).max() < (1 << 32)
    return books.astype(np.uint32)


def test_clear_structured_books():
    """cae_clear on books whose crossing of demand and supply falls on lane edges, on the first
    and last tick or nowhere, with ties and with nothing to trade, for every ticks-per-lane
    width, against the oracle."""
    import torch
    E = _engine()
    rng = np.random.default_rng(12)
    for L in (1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 512, 700, 1023, 1024):
        books = _structured_books(L, rng)
        n = books.shape[0]
        rp, rv, rres = O.clear_batch(books)
        dev = torch.from_numpy(books.reshape(-1).view(np.int32).copy()).cuda()
        ps, vs = E.clear_books(dev, L, n)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ps.cpu().numpy().view(np.uint32), rp, err_msg="L=%d" % L)
        np.testing.assert_array_equal(vs.cpu().numpy().view(np.uint32).astype(np.uint64), rv,
                                      err_msg="L=%d" % L)
        np.testing.assert_array_equal(dev.cpu().numpy().view(np.uint32).reshape(n, 2, L), rres,
                                      err_msg="L=%d" % L)


@pytest.fixture(scope="module")
def fixed_reference():
    w = W.fixed()
    return w, O.run(w["descs"], w["seed"], w["S"])


@pytest.mark.parametrize("schedule", ["autotuned", "default"])
def test_fixed_workload_full_parity(schedule, fixed_reference):
    """The fixed workload at full size (1024 x 1024 agents x 1000 steps, L = 256), every market
    against the oracle: in the launch configuration the benchmark times (the autotuner's
    schedule, overlapped lock-step on MI355X) and in the default one."""
    w, (rst, rbk) = fixed_reference
    tn = None
    if schedule == "autotuned":
        _engine()
        from paper_2606_21784_amd import autotune
        tn = autotune.tune(w["descs"], seed=w["seed"])
    st, bk, used = _run_gpu(w["descs"], w["seed"], [w["S"]], tuning=tn)
    if tn is not None:
        assert used["waves_per_group"] == tn["waves_per_group"]
        assert used["overlap"] == tn["overlap"]
    _assert_books(w["descs"], bk, rbk)
    _assert_states(st, rst)


def _tuned(descs, seed):
    _engine()
    from paper_2606_21784_amd import autotune
    return autotune.tune(descs, seed=seed)


@pytest.mark.parametrize("schedule", ["autotuned", "default"])
def test_market_sweep_sampled(schedule):
    """Market-count sweep at its full step count (10000 steps, L = 512, A = 4096), smallest
    and a mid-size M, in the benchmark's autotuned schedule and the default one; sampled
    markets re-simulated alone by the oracle."""
    for M in (16, 1024):
        w = W.market_sweep(M)
        tn = _tuned(w["descs"], w["seed"]) if schedule == "autotuned" else None
        st, bk, _ = _run_gpu(w["descs"], w["seed"], [w["S"]], tuning=tn)
        ids = [0, M // 2, M - 1]
        rst, rbk = O.run(w["descs"][ids], w["seed"], w["S"], ids=ids)
        _assert_books(w["descs"], bk, rbk, ids=ids)
        _assert_states(st[ids], rst)


@pytest.mark.parametrize("M", [4096, 65536])
def test_market_sweep_large_sampled(M):
    """Market-count sweep at large M in the schedule the benchmark times there (the autotuner's,
    chosen for this M), full 10000 steps; four markets (first, a third, the middle, last)
    re-simulated alone by the oracle and compared bit for bit, and every market's statistics
    checked for the invariants that hold at any size."""
    w = W.market_sweep(M)
    tn = _tuned(w["descs"], w["seed"])
    st, bk, used = _run_gpu(w["descs"], w["seed"], [w["S"]], tuning=tn)
    assert used["waves_per_group"] == tn["waves_per_group"]
    ids = [0, M // 3, M // 2, M - 1]
    rst, rbk = O.run(w["descs"][ids], w["seed"], w["S"], ids=ids)
    _assert_books(w["descs"], bk, rbk, ids=ids)
    _assert_states(st[ids], rst)
    L = int(w["descs"]["L"][0])
    assert (st["steps_done"] == w["S"]).all()
    assert (st["last"] < L).all() and (st["prev"] < L).all()
    assert (st["n_trade"] <= w["S"]).all() and (st["n_spread"] <= w["S"]).all()
    assert (st["sum_px"] <= st["n_trade"] * (L - 1)).all()
    # residual books are never crossed: highest bid below lowest ask in every market
    b = bk.reshape(M, 2, L)
    has_b, has_a = (b[:, 0] > 0).any(1), (b[:, 1] > 0).any(1)
    hb = np.where(has_b, L - 1 - np.argmax(b[:, 0, ::-1] > 0, axis=1), -1)
    la = np.where(has_a, np.argmax(b[:, 1] > 0, axis=1), L)
    assert (hb < la).all()


@pytest.mark.slow
@pytest.mark.parametrize("schedule", ["autotuned", "default"])
def test_uneven_ensemble_sampled(schedule):
    """The 8192-market uneven ensemble at full size in the benchmark's autotuned schedule and
    the default one; sampled markets (the largest and smallest A among them) against the
    oracle."""
    w = W.uneven()
    d = w["descs"]
    tn = _tuned(d, w["seed"]) if schedule == "autotuned" else None
    st, bk, _ = _run_gpu(d, w["seed"], [w["S"]], tuning=tn)
    A = d["A"].astype(np.int64)
    rng = np.random.default_rng(1)
    ids = sorted(set([int(np.argmax(A)), int(np.argmin(A))] +
                     rng.choice(len(d), 10, replace=False).tolist()))
    rst, rbk = O.run(d[ids], w["seed"], w["S"], ids=ids)
    _assert_books(d, bk, rbk, ids=ids)
    _assert_states(st[ids], rst)
    # every market traded at least once and no book is crossed
    assert (st["n_trade"] > 0).all()


def test_per_size_launches_and_shards_match_one_batched_launch():
    """Markets keep their generator index when split into per-size-class launches or shards, so
    every split reproduces the single batched launch bit for bit (and the oracle)."""
    E = _engine()
    from paper_2606_21784_amd import autotune
    w = W.uneven(M=300)
    d = w["descs"].copy()
    d["A"] = np.minimum(d["A"], 3000)
    d["n_noise"] = d["A"] // 2
    d["n_mom"] = d["A"] // 4
    S = 60
    ens = E.Ensemble(d, w["seed"])
    ens.step(S)
    st, bk = ens.read_state(), ens.read_books()
    ens.close()
    off = np.zeros(len(d), np.int64)
    off[1:] = np.cumsum(2 * d["L"].astype(np.int64))[:-1]
    groups = list(autotune.per_size_groups(d).values())
    halves = [np.arange(0, 150), np.arange(150, 300)]
    for split in (groups, halves):
        for idx in split:
            sub = E.Ensemble(d[idx], w["seed"], market_ids=idx)
            sub.step(S)
            sst, sbk = sub.read_state(), sub.read_books()
            sub.close()
            _assert_states(sst, st[idx])
            pos = 0
            for i in idx:
                n = 2 * int(d["L"][i])
                np.testing.assert_array_equal(sbk[pos:pos + n], bk[off[i]:off[i] + n])
                pos += n
    ids = [0, 7, 299]
    rst, rbk = O.run(d[ids], w["seed"], S, ids=ids)
    _assert_books(d, bk, rbk, ids=ids)
    _assert_states(st[ids], rst)


def test_autotuned_schedule_is_exact():
    E = _engine()
    from paper_2606_21784_amd import autotune
    w = W.uneven(M=200)
    d = w["descs"].copy()
    d["A"] = np.minimum(d["A"], 2000)
    d["n_noise"] = d["A"]
    tn = autotune.tune(d, seed=w["seed"], S_probe=8, min_markets=64)
    assert tn["waves_per_group"] in autotune.GROUP_CANDIDATES
    assert set(tn["waves_per_market"].values()) <= set(autotune.WPM_CANDIDATES)
    ens = E.Ensemble(d, w["seed"], tuning=tn)
    used = ens.tuning()
    assert used["waves_per_group"] == tn["waves_per_group"]
    ens.step(25)
    st, bk = ens.read_state(), ens.read_books()
    ens.close()
    rst, rbk = O.run(d, w["seed"], 25)
    _assert_books(d, bk, rbk)
    _assert_states(st, rst)


def test_queue_resets_between_launches():
    """Many short launches in a row (the on-device work queue is reset by the last workgroup of
    each launch) give the same result as one long launch."""
    E = _engine()
    descs = W.uniform(50, 64, 96, 8, 10, n_noise=60, n_mom=20)
    ens = E.Ensemble(descs, 3, tuning={"waves_per_group": 4, "groups_per_cu": 1})
    for _ in range(20):
        ens.step(3)
    st, bk = ens.read_state(), ens.read_books()
    ens.close()
    rst, rbk = O.run(descs, 3, 60)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)


@pytest.mark.parametrize("G", [2, 3, 4, 8, 16])
def test_pipelined_pairs_exact(G):
    """Pipelined pairs (one wave clears one market while the others generate the other's
    orders), including an odd market left alone, give the oracle's books."""
    descs = W.uniform(7, 100, 300, 9, 20, n_noise=150, n_mom=90, h=3)
    tn = {"waves_per_group": G, "pipelined": {c: 1 for c in range(40)}}
    st, bk, used = _run_gpu(descs, 21, [33, 17], tuning=tn)
    assert used["pipelined"] and used["waves_per_group"] == G
    rst, rbk = O.run(descs, 21, 50)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)


def test_pipelined_mixed_with_other_modes():
    rng = np.random.default_rng(17)
    n = 60
    L = rng.choice([5, 64, 128, 256, 512, 1000], n)
    A = rng.integers(1, 5000, n)
    d = np.zeros(n, W.MARKET_DTYPE)
    d["L"], d["A"], d["K"], d["Q"] = L, A, np.maximum(1, L // 16), rng.integers(1, 60, n)
    d["n_noise"] = A // 2
    d["n_mom"] = A // 3
    d["h"] = np.minimum(2, L - 1)
    from paper_2606_21784_amd import engine
    cls = [engine.size_class(int(a), int(b)) for a, b in zip(L, A)]
    tn = {"waves_per_group": 8,
          "waves_per_market": {c: (1 if c % 3 == 0 else 4) for c in set(cls)},
          "pipelined": {c: 1 for c in set(cls) if c % 3 == 1}}
    st, bk, _ = _run_gpu(d, 77, [25], tuning=tn)
    rst, rbk = O.run(d, 77, 25)
    _assert_books(d, bk, rbk)
    _assert_states(st, rst)


@pytest.mark.parametrize("wpm,G,k", [(2, 2, 1), (2, 8, 2), (4, 4, 1), (4, 4, 2), (4, 8, 5),
                                     (8, 8, 3), (16, 16, 1), (4, 4, 200)])
def test_overlapped_lockstep_exact(wpm, G, k):
    """Lock-step markets that generate the next step's orders during the clearing (clearing
    wave taking k - 1 rows of agents, from none to all of them) give the oracle's books, over
    calls of 33, 1 and 17 steps."""
    descs = W.uniform(7, 100, 700, 9, 20, n_noise=350, n_mom=190, h=3)
    tn = {"waves_per_group": G, "waves_per_market": {c: wpm for c in range(40)},
          "overlap": {c: k for c in range(40)}}
    st, bk, used = _run_gpu(descs, 21, [33, 1, 17], tuning=tn)
    assert set(used["overlap"].values()) == {k}
    rst, rbk = O.run(descs, 21, 51)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)


@pytest.mark.parametrize("cfg", [
    # L, A, K, Q, n_noise, n_mom, h  -- clamped offsets, agents fewer than a wave, one class only
    (1, 1, 0, 1, 1, 0, 0),
    (3, 65, 2, 7, 65, 0, 1),
    (100, 1000, 9, 33, 500, 300, 3),
    (257, 777, 16, 100, 300, 300, 5),
    (1000, 130, 40, 5, 0, 130, 7),
    (1024, 3000, 64, 100, 1000, 1000, 2),
    (64, 64, 8, 10, 0, 0, 2),
    (64, 40, 100, 10, 40, 0, 1),
    (512, 5000, 1022, 50, 5000, 0, 1),
    (512, 900, 1023, 50, 300, 300, 1),
])
def test_overlapped_ragged_markets(cfg):
    """Overlapped lock-step on ragged shapes, offsets wider than the book, momentum-only and
    maker-only populations, and K past the bin limit (those markets run plain lock-step)."""
    L, A, K, Q, nn, nm, h = cfg
    descs = W.uniform(5, L, A, K, Q, n_noise=nn, n_mom=nm, h=h)
    tn = {"waves_per_group": 8, "waves_per_market": {c: 4 for c in range(40)},
          "overlap": {c: 2 for c in range(40)}}
    st, bk, _ = _run_gpu(descs, 12345, [40, 3], tuning=tn)
    rst, rbk = O.run(descs, 12345, 43)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)


@pytest.mark.parametrize("L,K,nn,nm", [(256, 16, 1024, 0), (256, 16, 300, 700), (128, 8, 200, 800),
                                        (64, 4, 100, 900), (200, 30, 500, 500)])
def test_overlapped_small_books_near_the_edges(L, K, nn, nm):
    """Overlapped markets with books of up to 4 ticks per lane add the order bins inside the
    clearing unless the offset window leaves the book; momentum-heavy populations drive the
    price to the edges, so both ways run, within one market and across steps."""
    A = 1024
    descs = W.uniform(12, L, A, K, 50, n_noise=nn, n_mom=nm, h=3)
    tn = {"waves_per_group": 8, "waves_per_market": {c: 4 for c in range(40)},
          "overlap": {c: 4 for c in range(40)}}
    st, bk, _ = _run_gpu(descs, 2024, [70, 33], tuning=tn)
    rst, rbk, rpr, _ = O.run(descs, 2024, 103, trace=True)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)
    if L <= 200:
        # the trend carried the prices to within K of an edge for some steps and not for others
        near = (rpr < K) | (rpr > L - 1 - K)
        assert near.any() and not near.all()


def test_overlapped_mixed_with_other_modes():
    """Overlapped, plain lock-step, single-wave and pipelined classes in one launch."""
    rng = np.random.default_rng(19)
    n = 60
    L = rng.choice([5, 64, 128, 256, 512, 1000], n)
    A = rng.integers(1, 5000, n)
    d = np.zeros(n, W.MARKET_DTYPE)
    d["L"], d["A"], d["K"], d["Q"] = L, A, np.maximum(1, L // 16), rng.integers(1, 60, n)
    d["n_noise"] = A // 2
    d["n_mom"] = A // 3
    d["h"] = np.minimum(2, L - 1)
    from paper_2606_21784_amd import engine
    cls = sorted(set(engine.size_class(int(a), int(b)) for a, b in zip(L, A)))
    tn = {"waves_per_group": 8,
          "waves_per_market": {c: (1 if c % 4 == 0 else 4) for c in cls},
          "pipelined": {c: 1 for c in cls if c % 4 == 1},
          "overlap": {c: 1 + c % 3 for c in cls if c % 4 in (0, 2, 3)}}
    st, bk, used = _run_gpu(d, 77, [25, 6], tuning=tn)
    # reported only where it applies: lock-step classes that are not pipelined
    assert sorted(used["overlap"]) == [c for c in cls if c % 4 in (2, 3)]
    rst, rbk = O.run(d, 77, 31)
    _assert_books(d, bk, rbk)
    _assert_states(st, rst)


def test_priority_boost_is_exact():
    """Tuning flag bit 1 raises the issue priority of the costliest items (here the overlapped
    markets of 1024 agents among single-wave markets of 16 to 256): the same books and
    statistics as the oracle, in the same mixed launch with and without it."""
    from paper_2606_21784_amd import engine
    parts = []
    for A in (16, 64, 256, 1024):
        parts.append(W.uniform(6, 128, A, 8, 10, n_noise=A - A // 4 - A // 8, n_mom=A // 4, h=2))
    d = np.concatenate(parts)
    cls = sorted(set(engine.size_class(int(a), int(b)) for a, b in zip(d["L"], d["A"])))
    big = engine.size_class(128, 1024)
    base = {"waves_per_group": 4, "waves_per_market": {c: (4 if c == big else 1) for c in cls},
            "overlap": {big: 3}}
    rst, rbk = O.run(d, 31, 120)
    for flags in (0, 2):
        st, bk, used = _run_gpu(d, 31, [70, 50], tuning=dict(base, flags=flags))
        assert used["flags"] == flags
        _assert_books(d, bk, rbk)
        _assert_states(st, rst)
    # the same mix with half the markets on the mid-price model (the instantiation that may meet
    # it runs its own overlapped loop)
    d2 = d.copy()
    d2["flags"][::2] = O.model_flags(O.MODEL_MID, 3277)
    rst2, rbk2 = O.run(d2, 32, 120)
    for flags in (0, 2):
        st, bk, used = _run_gpu(d2, 32, [64, 56], tuning=dict(base, flags=flags))
        _assert_books(d2, bk, rbk2)
        _assert_states(st, rst2)


@pytest.mark.parametrize("k", [1, 3, 9])
def test_overlap_with_mid_price_and_splitmix_markets(k):
    """The overlapped schedule with last-tick and mid-price markets (marketable orders
    included), Philox and SplitMix64 generators, side by side; mid-price markets with K past
    510 run plain lock-step.  Exact against the oracle."""
    mid, smx = O.model_flags(O.MODEL_MID, 3000), O.model_flags(O.MODEL_LAST, 0, O.GEN_SPLITMIX)
    d = np.concatenate([W.uniform(3, 128, 600, 8, 10, n_noise=300, n_mom=200, h=2),
                        W.uniform(3, 128, 600, 8, 10, n_noise=300, n_mom=200, h=2, flags=mid),
                        W.uniform(2, 128, 600, 8, 10, n_noise=300, n_mom=200, h=2, flags=smx),
                        W.uniform(2, 128, 600, 8, 10, n_noise=300, n_mom=200, h=2,
                                  flags=O.model_flags(O.MODEL_MID, 20000, O.GEN_SPLITMIX)),
                        W.uniform(2, 1024, 700, 600, 10, n_noise=300, n_mom=200, h=2, flags=mid),
                        W.uniform(2, 200, 900, 0, 7, n_noise=500, n_mom=300, h=1, flags=mid)])
    tn = {"waves_per_group": 8, "waves_per_market": {c: 4 for c in range(40)},
          "overlap": {c: k for c in range(40)}}
    st, bk, used = _run_gpu(d, 5, [20, 1, 9], tuning=tn)
    assert set(used["overlap"].values()) == {k}
    rst, rbk = O.run(d, 5, 30)
    _assert_books(d, bk, rbk)
    _assert_states(st, rst)


@pytest.mark.parametrize("cfg", [(64, 128, 8, 10, 128, 0, 2), (100, 300, 9, 20, 150, 90, 3),
                                 (1024, 700, 40, 50, 200, 300, 2), (1, 5, 0, 3, 2, 2, 0)])
def test_naive_engine_is_bit_identical(cfg):
    """The naive one-thread-per-market ablation engine gives the persistent engine's books."""
    E = _engine()
    L, A, K, Q, nn, nm, h = cfg
    descs = W.uniform(70, L, A, K, Q, n_noise=nn, n_mom=nm, h=h)
    ens = E.Ensemble(descs, 8)
    ens.step_naive(20)
    ens.step(10)
    ens.step_naive(10)
    st, bk = ens.read_state(), ens.read_books()
    ens.close()
    rst, rbk = O.run(descs, 8, 40)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("mode", ["lockstep", "single", "pipelined", "overlapped"])
def test_traced_series_match_oracle(mode):
    """cae_step_traced writes each market's per-step price and volume series equal to the
    oracle's, in every schedule mode; untraced calls leave their columns alone and tracing does
    not change books or states."""
    import torch
    E = _engine()
    descs = W.uniform(9, 100, 300, 9, 20, n_noise=150, n_mom=90, h=3)
    tn = {"lockstep": {"waves_per_group": 4, "waves_per_market": {c: 2 for c in range(40)}},
          "single": {"waves_per_group": 4, "waves_per_market": {c: 1 for c in range(40)}},
          "pipelined": {"waves_per_group": 4, "pipelined": {c: 1 for c in range(40)}},
          "overlapped": {"waves_per_group": 4, "waves_per_market": {c: 4 for c in range(40)},
                         "overlap": {c: 2 for c in range(40)}}}[mode]
    ens = E.Ensemble(descs, 21, tuning=tn)
    pr = torch.full((9, 80), -1, dtype=torch.int32, device="cuda")
    vo = torch.full((9, 80), -1, dtype=torch.int32, device="cuda")
    ens.step_traced(30, out=(pr, vo), col=0)
    ens.step(20)
    ens.step_traced(30, out=(pr, vo), col=50)
    p2, v2 = ens.step_traced(7)
    _, v3 = ens.step_traced(5, price=False)
    st, bk = ens.read_state(), ens.read_books()
    ens.close()
    rst, rbk, rpr, rvo = O.run(descs, 21, 92, trace=True)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)
    p, v = _u32(pr), _u32(vo)
    assert rvo.max() < 2**32
    for a, b in ((0, 30), (50, 80)):
        np.testing.assert_array_equal(p[:, a:b], rpr[:, a:b])
        np.testing.assert_array_equal(v[:, a:b], rvo[:, a:b].astype(np.uint32))
    assert np.all(p[:, 30:50] == 0xFFFFFFFF) and np.all(v[:, 30:50] == 0xFFFFFFFF)
    np.testing.assert_array_equal(_u32(p2), rpr[:, 80:87])
    np.testing.assert_array_equal(_u32(v2), rvo[:, 80:87].astype(np.uint32))
    np.testing.assert_array_equal(_u32(v3), rvo[:, 87:92].astype(np.uint32))


def test_traced_mixed_sizes_and_modes():
    """Traced series of markets of mixed L and A in one launch, with single-wave, lock-step and
    pipelined classes side by side."""
    import torch
    E = _engine()
    rng = np.random.default_rng(23)
    n = 40
    L = rng.choice([5, 64, 128, 256, 512, 1000], n)
    A = rng.integers(1, 3000, n)
    d = np.zeros(n, W.MARKET_DTYPE)
    d["L"], d["A"], d["K"], d["Q"] = L, A, np.maximum(1, L // 16), rng.integers(1, 60, n)
    d["n_noise"] = A // 2
    d["n_mom"] = A // 3
    d["h"] = np.minimum(2, L - 1)
    cls = [E.size_class(int(a), int(b)) for a, b in zip(L, A)]
    tn = {"waves_per_group": 8,
          "waves_per_market": {c: (1 if c % 3 == 0 else 4) for c in set(cls)},
          "pipelined": {c: 1 for c in set(cls) if c % 3 == 1},
          "overlap": {c: 2 for c in set(cls) if c % 6 == 2}}
    ens = E.Ensemble(d, 78, tuning=tn)
    pr, vo = ens.step_traced(40)
    torch.cuda.synchronize()
    ens.close()
    _, _, rpr, rvo = O.run(d, 78, 40, trace=True)
    np.testing.assert_array_equal(_u32(pr), rpr)
    np.testing.assert_array_equal(_u32(vo), rvo.astype(np.uint32))


def test_traced_rejects_short_rows():
    import ctypes as C
    E = _engine()
    from paper_2606_21784_amd import _lib
    import torch
    descs = W.uniform(3, 64, 64, 4, 5)
    ens = E.Ensemble(descs, 1)
    buf = torch.zeros((3, 8), dtype=torch.int32, device="cuda")
    rc = _lib.lib().cae_step_traced(ens.handle, 10, C.c_void_p(buf.data_ptr()), None, 8)
    assert rc == _lib.CAE_EINVAL
    with pytest.raises(ValueError):
        ens.step_traced(5, out=(buf, None), col=4)
    st = ens.read_state()
    ens.close()
    assert np.all(st["steps_done"] == 0)


def _mid(p_mkt):
    return O.model_flags(O.MODEL_MID, int(round(p_mkt * 65536)))


@pytest.mark.parametrize("mode", ["lockstep", "single", "pipelined", "overlapped"])
@pytest.mark.parametrize("p_mkt", [0.0, 0.05, 0.6])
def test_mid_model_matches_oracle(mode, p_mkt):
    """The mid-price agent model (section III-C's rules, marketable orders with P_mkt): books,
    states (with the momentum memory ref2) and traces equal the oracle's in every schedule mode,
    across split calls."""
    import torch
    E = _engine()
    descs = W.uniform(9, 100, 300, 9, 20, n_noise=150, n_mom=90, h=3, flags=_mid(p_mkt))
    tn = {"lockstep": {"waves_per_group": 4, "waves_per_market": {c: 2 for c in range(40)}},
          "single": {"waves_per_group": 4, "waves_per_market": {c: 1 for c in range(40)}},
          "pipelined": {"waves_per_group": 4, "pipelined": {c: 1 for c in range(40)}},
          "overlapped": {"waves_per_group": 4, "waves_per_market": {c: 4 for c in range(40)},
                         "overlap": {c: 2 for c in range(40)}}}[mode]
    ens = E.Ensemble(descs, 31, tuning=tn)
    ens.step(13)
    pr, vo = ens.step_traced(40)
    ens.step(7)
    st, bk = ens.read_state(), ens.read_books()
    ens.close()
    rst, rbk = O.run(descs, 31, 13)
    rst, rbk, rpr, rvo = O.run(descs, 31, 40, states=rst, book=rbk, trace=True)
    rst, rbk = O.run(descs, 31, 7, states=rst, book=rbk)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)
    np.testing.assert_array_equal(_u32(pr), rpr)
    np.testing.assert_array_equal(_u32(vo), rvo.astype(np.uint32))


def test_models_mixed_in_one_launch():
    """Last-tick and mid-price markets of mixed sizes in one launch, every schedule mode."""
    E = _engine()
    rng = np.random.default_rng(29)
    n = 48
    L = rng.choice([5, 64, 128, 256, 512, 1000], n)
    A = rng.integers(1, 3000, n)
    d = np.zeros(n, W.MARKET_DTYPE)
    d["L"], d["A"], d["K"], d["Q"] = L, A, np.maximum(1, L // 16), rng.integers(1, 60, n)
    d["n_noise"] = A // 2
    d["n_mom"] = A // 3
    d["h"] = np.minimum(2, L - 1)
    d["flags"] = np.where(rng.random(n) < 0.5, 0, [_mid(x) for x in rng.choice([0.0, 0.1], n)])
    cls = [E.size_class(int(a), int(b)) for a, b in zip(L, A)]
    tn = {"waves_per_group": 8,
          "waves_per_market": {c: (1 if c % 3 == 0 else 4) for c in set(cls)},
          "pipelined": {c: 1 for c in set(cls) if c % 3 == 1},
          "overlap": {c: 1 + c % 4 for c in set(cls) if c % 3 == 2}}
    st, bk, _ = _run_gpu(d, 41, [11, 19], tuning=tn)
    rst, rbk = O.run(d, 41, 30)
    _assert_books(d, bk, rbk)
    _assert_states(st, rst)


@pytest.mark.parametrize("p_mkt", [0.0, 0.2])
def test_naive_engine_mid_model(p_mkt):
    E = _engine()
    descs = W.uniform(70, 128, 256, 8, 10, n_noise=100, n_mom=100, h=2, flags=_mid(p_mkt))
    ens = E.Ensemble(descs, 12)
    ens.step_naive(15)
    ens.step(10)
    ens.step_naive(5)
    st, bk = ens.read_state(), ens.read_books()
    ens.close()
    rst, rbk = O.run(descs, 12, 30)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)


def test_mid_model_many_launch_starts():
    """Each launch reads the mid-price reference of its first step from the book before any
    wave adds orders: many short launches of lock-step mid-price markets equal the oracle."""
    rng = np.random.default_rng(31)
    n = 48
    L = rng.choice([64, 100, 256, 1000, 1024], n)
    A = rng.integers(200, 3000, n)
    d = np.zeros(n, W.MARKET_DTYPE)
    d["L"], d["A"], d["K"], d["Q"] = L, A, np.maximum(1, L // 16), rng.integers(1, 40, n)
    d["n_noise"] = A // 2
    d["n_mom"] = A // 3
    d["h"] = 2
    d["flags"] = _mid(0.05)
    for G, wpm, k in ((16, 4, 0), (8, 2, 0), (4, 4, 0), (8, 4, 2), (16, 8, 1)):
        tn = {"waves_per_group": G, "waves_per_market": {c: wpm for c in range(40)}}
        if k:
            tn["overlap"] = {c: k for c in range(40)}
        st, bk, _ = _run_gpu(d, 53, [3] * 12 + [5], tuning=tn)
        rst, rbk = O.run(d, 53, 41)
        _assert_books(d, bk, rbk)
        _assert_states(st, rst)


@pytest.mark.parametrize("mode", ["lockstep", "single", "pipelined", "overlapped"])
@pytest.mark.parametrize("model", ["last", "mid"])
def test_splitmix_generator_matches_oracle(mode, model):
    """Markets that select the SplitMix64 generator (section III-G) give the oracle's books,
    states and traces in every schedule mode, next to Philox markets in the same launch."""
    E = _engine()
    flags = (O.model_flags(O.MODEL_MID, 3277, O.GEN_SPLITMIX) if model == "mid"
             else O.model_flags(gen=O.GEN_SPLITMIX))
    descs = W.uniform(10, 100, 300, 9, 20, n_noise=150, n_mom=90, h=3, flags=flags)
    descs["flags"][::3] = 0  # some Philox markets in the same launch
    tn = {"lockstep": {"waves_per_group": 4, "waves_per_market": {c: 2 for c in range(40)}},
          "single": {"waves_per_group": 4, "waves_per_market": {c: 1 for c in range(40)}},
          "pipelined": {"waves_per_group": 4, "pipelined": {c: 1 for c in range(40)}},
          "overlapped": {"waves_per_group": 4, "waves_per_market": {c: 4 for c in range(40)},
                         "overlap": {c: 2 for c in range(40)}}}[mode]
    ens = E.Ensemble(descs, 0xDEADBEEF12345, tuning=tn, market_ids=np.arange(10) * 7 + 3)
    ens.step(11)
    pr, vo = ens.step_traced(20)
    st, bk = ens.read_state(), ens.read_books()
    ens.close()
    rst, rbk = O.run(descs, 0xDEADBEEF12345, 11, ids=np.arange(10) * 7 + 3)
    rst, rbk, rpr, rvo = O.run(descs, 0xDEADBEEF12345, 20, ids=np.arange(10) * 7 + 3, states=rst,
                               book=rbk, trace=True)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)
    np.testing.assert_array_equal(_u32(pr), rpr)
    np.testing.assert_array_equal(_u32(vo), rvo.astype(np.uint32))


def test_naive_engine_splitmix():
    E = _engine()
    descs = W.uniform(40, 64, 200, 4, 9, n_noise=120, n_mom=40, h=2,
                      flags=O.model_flags(O.MODEL_MID, 1000, O.GEN_SPLITMIX))
    ens = E.Ensemble(descs, 99)
    ens.step_naive(7)
    ens.step(6)
    st, bk = ens.read_state(), ens.read_books()
    ens.close()
    rst, rbk = O.run(descs, 99, 13)
    _assert_books(descs, bk, rbk)
    _assert_states(st, rst)
