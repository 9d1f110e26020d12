"""CPU oracle for the call-auction ensemble -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  It wraps ``liboracle.so`` (plain C, see ``cae_oracle.c``) with ctypes and numpy.
Nothing here is shared with the GPU library.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

STATE_DTYPE = np.dtype([
    ("last", np.uint32), ("prev", np.uint32), ("steps_done", np.uint64),
    ("n_trade", np.uint64), ("sum_vol", np.uint64), ("sum_px", np.uint64),
    ("sum_spread", np.uint64), ("n_spread", np.uint64),
    ("sum_r", np.float64), ("sum_r2", np.float64), ("ref2", np.uint32), ("reserved", np.uint32),
])
MARKET_DTYPE = np.dtype([
    ("L", np.uint32), ("A", np.uint32), ("K", np.uint32), ("Q", np.uint32),
    ("n_noise", np.uint32), ("n_mom", np.uint32), ("h", np.uint32), ("flags", np.uint32),
])
BUY, SELL = 0, 1


def lib():
    global _lib
    if _lib is None:
        if _build.needs_build():
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        u32, u64, i32 = C.c_uint32, C.c_uint64, C.c_int
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_range.argtypes = [u32, u32]
        L.orc_range.restype = u32
        L.orc_initial_state.argtypes = [P, P]
        L.orc_agent_order.argtypes = [P, u32, u64, u32, u32, u32, u32, P, P, P]
        L.orc_clear.argtypes = [u32, P, P, P, P]
        L.orc_update_stats.argtypes = [u32, P, P, u32, u64, P, P]
        L.orc_market_run.argtypes = [P, u32, u64, u32, P, P, P]
        L.orc_market_run.restype = i32
        L.orc_run.argtypes = [P, P, P, u32, u64, u32, P, P, i32]
        L.orc_run.restype = i32
        L.orc_market_run_traced.argtypes = [P, u32, u64, u32, P, P, P, P, P]
        L.orc_market_run_traced.restype = i32
        L.orc_run_traced.argtypes = [P, P, P, u32, u64, u32, P, P, i32, P, P, u64]
        L.orc_run_traced.restype = i32
        L.orc_clear_batch.argtypes = [u32, u32, P, P, P]
        L.orc_philox_batch.argtypes = [u32, P, P, P]
        L.orc_orders.argtypes = [P, u32, u64, u32, u32, u32, P, P, P]
        L.orc_orders_mid.argtypes = [P, u32, u64, u32, u32, u32, P, P, P]
        L.orc_splitmix64_mix.argtypes = [u64]
        L.orc_splitmix64_mix.restype = u64
        L.orc_splitmix_batch.argtypes = [u32, P, P, u64, P]
        L.orc_state_size.restype = u32
        L.orc_market_size.restype = u32
        assert L.orc_state_size() == STATE_DTYPE.itemsize
        assert L.orc_market_size() == MARKET_DTYPE.itemsize
        if hasattr(L, "orm_forward"):
            from . import mlp as _mlp
            _mlp._bind(L)
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    """Philox4x32-10 of one counter (4 words) under one key (2 words)."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def philox_batch(ctrs, key):
    c = np.ascontiguousarray(ctrs, dtype=np.uint32).reshape(-1, 4)
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros_like(c)
    lib().orc_philox_batch(len(c), _p(c), _p(k), _p(out))
    return out


def urange(w, n):
    return int(lib().orc_range(int(w) & 0xFFFFFFFF, int(n)))


MODEL_LAST, MODEL_MID = 0, 1
GEN_PHILOX, GEN_SPLITMIX = 0, 1


def model_flags(model=MODEL_LAST, p_mkt16=0, gen=GEN_PHILOX):
    """Descriptor flags: agent model in bits 0-7, generator in bits 8-15, P_mkt (units of
    2^-16) in bits 16-31."""
    return (int(p_mkt16) << 16) | (int(gen) << 8) | int(model)


def splitmix64(x):
    """The SplitMix64 output function of one 64-bit input."""
    return int(lib().orc_splitmix64_mix(int(x) & (2**64 - 1)))


def splitmix_words(gid, steps, seed):
    """Words (n, 4) of the SplitMix64 reading for global agent ids gid[n] at steps[n]."""
    g = np.ascontiguousarray(gid, dtype=np.uint64)
    st = np.ascontiguousarray(steps, dtype=np.uint32)
    out = np.zeros((len(g), 4), np.uint32)
    lib().orc_splitmix_batch(len(g), _p(g), _p(st), int(seed) & (2**64 - 1), _p(out))
    return out


def market(L, A, K, Q, n_noise=None, n_mom=0, h=2, flags=0):
    d = np.zeros(1, MARKET_DTYPE)
    d["L"], d["A"], d["K"], d["Q"] = L, A, K, Q
    d["n_noise"] = A if n_noise is None else n_noise
    d["n_mom"], d["h"], d["flags"] = n_mom, h, flags
    return d


def initial_state(desc):
    st = np.zeros(1, STATE_DTYPE)
    lib().orc_initial_state(_p(desc), _p(st))
    return st


def orders(desc, m, seed, s, last, prev):
    A = int(desc["A"][0])
    side = np.zeros(A, np.uint32)
    tick = np.zeros(A, np.uint32)
    qty = np.zeros(A, np.uint32)
    lib().orc_orders(_p(desc), m, seed, s, last, prev, _p(side), _p(tick), _p(qty))
    return side, tick, qty


def orders_mid(desc, m, seed, s, mid2, mid2_prev):
    """Mid-price-model orders of every agent at step s, for mid = mid2 / 2 and previous mid
    mid2_prev / 2."""
    A = int(desc["A"][0])
    side = np.zeros(A, np.uint32)
    tick = np.zeros(A, np.uint32)
    qty = np.zeros(A, np.uint32)
    lib().orc_orders_mid(_p(desc), m, seed, s, mid2, mid2_prev, _p(side), _p(tick), _p(qty))
    return side, tick, qty


def clear(bid, ask):
    """Clear one book in place semantics; returns (p*, V*, residual bid, residual ask)."""
    b = np.array(bid, dtype=np.uint32)
    a = np.array(ask, dtype=np.uint32)
    assert b.shape == a.shape
    ps = np.zeros(1, np.uint32)
    vs = np.zeros(1, np.uint64)
    lib().orc_clear(len(b), _p(b), _p(a), _p(ps), _p(vs))
    return int(ps[0]), int(vs[0]), b, a


def clear_batch(books):
    """books: (n, 2, L) uint32 (bid, ask).  Returns p*, V* and the residual books."""
    bk = np.ascontiguousarray(books, dtype=np.uint32).copy()
    n, two, L = bk.shape
    assert two == 2
    ps = np.zeros(n, np.uint32)
    vs = np.zeros(n, np.uint64)
    lib().orc_clear_batch(L, n, _p(bk), _p(ps), _p(vs))
    return ps, vs, bk


def update_stats(bid, ask, pstar, vstar, lnp, state):
    b = np.ascontiguousarray(bid, dtype=np.uint32)
    a = np.ascontiguousarray(ask, dtype=np.uint32)
    lp = np.ascontiguousarray(lnp, dtype=np.float64)
    lib().orc_update_stats(len(b), _p(b), _p(a), pstar, vstar, _p(lp), _p(state))
    return state


def market_run(desc, m, seed, S, state=None, book=None, agent_order=None):
    """S steps of one market with index m.  Returns (state, book) with book = bid||ask."""
    L = int(desc["L"][0])
    st = initial_state(desc) if state is None else state.copy()
    bk = np.zeros(2 * L, np.uint32) if book is None else np.array(book, dtype=np.uint32)
    order = None
    if agent_order is not None:
        order = np.ascontiguousarray(agent_order, dtype=np.uint32)
    rc = lib().orc_market_run(_p(desc), m, seed, S, _p(st), _p(bk),
                              _p(order) if order is not None else None)
    if rc != 0:
        raise ValueError("oracle market_run failed (%d)" % rc)
    return st, bk


def book_offsets(descs):
    L = descs["L"].astype(np.uint64)
    off = np.zeros(len(descs), np.uint64)
    off[1:] = np.cumsum(2 * L)[:-1]
    return off, int(2 * L.sum())


def run(descs, seed, S, ids=None, states=None, book=None, nthreads=None, trace=False):
    """S steps of several markets.  descs[i] describes market ids[i] (default: i).

    Books are packed per market (bid[L] then ask[L]) in descs order.  With trace=True also
    returns the per-step series: price[i, t] = the last clearing tick after step t of this call,
    volume[i, t] = the volume executed in it (uint64)."""
    descs = np.ascontiguousarray(descs, dtype=MARKET_DTYPE)
    n = len(descs)
    ids = np.arange(n, dtype=np.uint32) if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
    off, words = book_offsets(descs)
    if states is None:
        states = np.zeros(n, STATE_DTYPE)
        for i in range(n):
            lib().orc_initial_state(_p(descs[i:i + 1]), _p(states[i:i + 1]))
    else:
        states = np.ascontiguousarray(states, dtype=STATE_DTYPE).copy()
    bk = np.zeros(words, np.uint32) if book is None else np.array(book, dtype=np.uint32)
    if nthreads is None:
        nthreads = min(os.cpu_count() or 1, 16)
    if trace:
        price = np.zeros((n, S), np.uint32)
        vol = np.zeros((n, S), np.uint64)
        rc = lib().orc_run_traced(_p(descs), _p(ids), _p(off), n, seed, S, _p(states), _p(bk),
                                  nthreads, _p(price), _p(vol), S)
    else:
        rc = lib().orc_run(_p(descs), _p(ids), _p(off), n, seed, S, _p(states), _p(bk), nthreads)
    if rc != 0:
        raise ValueError("oracle run failed (%d)" % rc)
    if trace:
        return states, bk, price, vol
    return states, bk


def log_prices(L):
    return np.log(np.arange(L, 2 * L, dtype=np.float64))


def pooled_stats(states, S_total):
    """Ensemble outputs pooled in market order: mean volume per step, mean spread,
    population variance of the per-step log return."""
    n = float(len(states) * S_total)
    vol = float(np.sum(states["sum_vol"].astype(np.float64))) / n
    ns = float(np.sum(states["n_spread"].astype(np.float64)))
    spread = float(np.sum(states["sum_spread"].astype(np.float64))) / ns if ns > 0 else float("nan")
    mr = float(np.sum(states["sum_r"])) / n
    var = float(np.sum(states["sum_r2"])) / n - mr * mr
    return spread, var, vol
