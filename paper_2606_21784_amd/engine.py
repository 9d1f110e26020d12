"""Python handle for a call-auction ensemble on one GPU.

PyTorch provides the device memory (tensors owned by the ``Ensemble``) and the stream; every
computation runs in libcae (HIP kernels for gfx950) through the C ABI.
"""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import Buffers, Market, Sizes, State, Tuning, check, lib

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
assert STATE_DTYPE.itemsize == C.sizeof(State) == 80
assert MARKET_DTYPE.itemsize == C.sizeof(Market) == 32


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def model_flags(model=_lib.MODEL_LAST, p_mkt=0.0, gen=_lib.GEN_PHILOX):
    """Descriptor flags for an agent model (MODEL_LAST / MODEL_MID), the generator
    (GEN_PHILOX / GEN_SPLITMIX) and, for the mid-price model, the marketable-order probability
    P_mkt (rounded to a multiple of 2^-16)."""
    p16 = int(round(float(p_mkt) * 65536))
    if not 0 <= p16 < 65536:
        raise ValueError("P_mkt must lie in [0, 1)")
    if p16 and model != _lib.MODEL_MID:
        raise ValueError("P_mkt needs the mid-price model")
    if gen not in (_lib.GEN_PHILOX, _lib.GEN_SPLITMIX):
        raise ValueError("unknown generator")
    return (p16 << _lib.PMKT_SHIFT) | (int(gen) << _lib.GEN_SHIFT) | int(model)


def markets(L, A, K, Q, M=1, n_noise=None, n_mom=0, h=2, flags=0):
    """M identical market descriptors (structured numpy array)."""
    d = np.zeros(M, MARKET_DTYPE)
    d["L"], d["A"], d["K"], d["Q"] = L, A, K, Q
    d["n_noise"] = A if n_noise is None else n_noise
    d["n_mom"], d["h"], d["flags"] = n_mom, h, flags
    return d


def sizes(descs):
    descs = np.ascontiguousarray(descs, dtype=MARKET_DTYPE)
    out = Sizes()
    check("cae_sizes", lib().cae_sizes(_p(descs), len(descs), C.byref(out)))
    return out


def tuning_struct(t=None):
    """A cae_tuning from a dict {waves_per_group, groups_per_cu, max_lds_bytes, flags,
    waves_per_market: {class: waves}, pipelined: {class: 1}, overlap: {class: k},
    class_cost_ns: {class: ns}, pack: {class: 2 or 4}} (or None)."""
    if t is None:
        return None
    if isinstance(t, Tuning):
        return t
    ts = Tuning()
    ts.waves_per_group = int(t.get("waves_per_group", 0))
    ts.groups_per_cu = int(t.get("groups_per_cu", 0))
    ts.max_lds_bytes = int(t.get("max_lds_bytes", 0))
    ts.flags = int(t.get("flags", 0))
    for c, w in dict(t.get("waves_per_market", {})).items():
        ts.waves_per_market[int(c)] = int(w)
    for c, v in dict(t.get("pipelined", {})).items():
        ts.pipelined[int(c)] = 1 if v else 0
    for c, v in dict(t.get("overlap", {})).items():
        ts.overlap[int(c)] = int(v)
    for c, v in dict(t.get("class_cost_ns", {})).items():
        ts.class_cost[int(c)] = float(v)
    for c, v in dict(t.get("pack", {})).items():
        ts.pack[int(c)] = int(v)
    return ts


def size_class(L, A):
    lc = 0
    while lc < 4 and (64 << lc) < L:
        lc += 1
    lg = int(A).bit_length() - 1
    return lc * 8 + min(max(lg, 6), 13) - 6


class Ensemble:
    """M independent markets stepped by the persistent engine.

    descs: structured array of MARKET_DTYPE (see ``markets``); seed: 64-bit generator key;
    market_ids: generator market index of each market (default 0..M-1), so a subset of a larger
    ensemble reproduces its markets; stream: a torch.cuda.Stream (default: the current stream);
    tuning: see ``tuning_struct``.
    """

    def __init__(self, descs, seed, stream=None, tuning=None, device=None, market_ids=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the call-auction engine needs a ROCm GPU")
        L_ = lib()
        self.descs = np.ascontiguousarray(descs, dtype=MARKET_DTYPE)
        self.M = len(self.descs)
        self.seed = int(seed)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.sz = sizes(self.descs)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream()
            # caller-owned device memory (the library never allocates)
            self.book = torch.empty(int(self.sz.book_words), dtype=torch.int32, device=self.device)
            self.state = torch.empty(int(self.sz.state_bytes), dtype=torch.uint8, device=self.device)
            self.workspace = torch.empty(int(self.sz.workspace_bytes), dtype=torch.uint8,
                                         device=self.device)
            bufs = Buffers(self.book.data_ptr(), self.state.data_ptr(), self.workspace.data_ptr())
            h = C.c_void_p()
            ts = tuning_struct(tuning)
            ids = None
            if market_ids is not None:
                ids = np.ascontiguousarray(market_ids, dtype=np.uint32)
                if ids.shape != (self.M,):
                    raise ValueError("market_ids must have one entry per market")
            self.market_ids = ids
            check("cae_create", L_.cae_create(_p(self.descs), self.M, self.seed & (2**64 - 1),
                                              _p(ids) if ids is not None else None,
                                              C.byref(bufs), C.c_void_p(self.stream.cuda_stream),
                                              C.byref(ts) if ts is not None else None,
                                              C.byref(h)))
        self._h = h
        self.steps = 0

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("ensemble destroyed")
        return self._h

    def step(self, S):
        """Advance every market by S steps (one persistent launch, asynchronous)."""
        check("cae_step", lib().cae_step(self.handle, int(S)))
        self.steps += int(S)

    def step_traced(self, S, price=True, volume=True, out=None, col=0):
        """S steps that also record every market's per-step series (asynchronous).

        Returns (price, volume): int32 device tensors of shape (M, S) holding the uint32 values
        (the tick `last` after each step; the volume executed in it), or None for a series not
        asked for.  out: optional (price, volume) tensors of shape (M, W) to fill at columns
        [col, col + S) instead (either may be None)."""
        import torch
        S = int(S)
        if out is None:
            mk = lambda want: (torch.empty((self.M, S), dtype=torch.int32, device=self.device)
                               if want else None)
            pr, vo, ld, off = mk(price), mk(volume), S, 0
        else:
            pr, vo = out
            ld = next(t.shape[1] for t in (pr, vo) if t is not None)
            off = int(col)
            for t in (pr, vo):
                if t is not None and (t.dtype != torch.int32 or not t.is_contiguous()
                                      or tuple(t.shape) != (self.M, ld) or t.device != self.device):
                    raise ValueError("trace tensors must be contiguous int32 (M, W) on the device")
            if off + S > ld:
                raise ValueError("columns [%d, %d) exceed the trace width %d" % (off, off + S, ld))
        ptr = lambda t: C.c_void_p(t.data_ptr() + 4 * off) if t is not None else None
        check("cae_step_traced", lib().cae_step_traced(self.handle, S, ptr(pr), ptr(vo), ld))
        self.steps += S
        return pr, vo

    def step_naive(self, S):
        """The same S steps with the naive one-thread-per-market engine (ablation)."""
        check("cae_step_naive", lib().cae_step_naive(self.handle, int(S)))
        self.steps += int(S)

    def last_step_ms(self):
        ms = C.c_float()
        check("cae_last_step_ms", lib().cae_last_step_ms(self.handle, C.byref(ms)))
        return float(ms.value)

    def read_books(self):
        out = np.zeros(int(self.sz.book_words), np.uint32)
        check("cae_read_books", lib().cae_read_books(self.handle, _p(out), out.size))
        return out

    def read_state(self):
        out = np.zeros(self.M, STATE_DTYPE)
        check("cae_read_state", lib().cae_read_state(self.handle, _p(out), self.M))
        return out

    def write_state(self, states, book):
        st = np.ascontiguousarray(states, dtype=STATE_DTYPE)
        bk = np.ascontiguousarray(book, dtype=np.uint32)
        check("cae_write_state", lib().cae_write_state(self.handle, _p(st), len(st), _p(bk), bk.size))

    def tuning(self):
        t = Tuning()
        check("cae_get_tuning", lib().cae_get_tuning(self.handle, C.byref(t)))
        return {"waves_per_group": t.waves_per_group, "groups_per_cu": t.groups_per_cu,
                "max_lds_bytes": t.max_lds_bytes, "flags": t.flags,
                "waves_per_market": {c: int(t.waves_per_market[c])
                                     for c in range(_lib.NUM_CLASSES) if t.waves_per_market[c]},
                "pipelined": {c: 1 for c in range(_lib.NUM_CLASSES) if t.pipelined[c]},
                "overlap": {c: int(t.overlap[c]) for c in range(_lib.NUM_CLASSES) if t.overlap[c]},
                "class_cost_ns": {c: float(t.class_cost[c])
                                  for c in range(_lib.NUM_CLASSES) if t.class_cost[c] > 0},
                "pack": {c: int(t.pack[c]) for c in range(_lib.NUM_CLASSES) if t.pack[c]}}

    def book_offsets(self):
        L = self.descs["L"].astype(np.uint64)
        off = np.zeros(self.M, np.uint64)
        off[1:] = np.cumsum(2 * L)[:-1]
        return off

    def close(self):
        if self._h is not None:
            lib().cae_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def clear_books(books_dev, L, M, stream=None):
    """One clearing pass over M books of L ticks held in a device int32 tensor (packed bid||ask
    per book), in place.  Returns device tensors (p*, V*)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    ps = torch.empty(M, dtype=torch.int32, device=books_dev.device)
    vs = torch.empty(M, dtype=torch.int32, device=books_dev.device)
    check("cae_clear", lib().cae_clear(int(L), int(M), books_dev.data_ptr(), ps.data_ptr(),
                                       vs.data_ptr(), C.c_void_p(s.cuda_stream)))
    return ps, vs


def device_info():
    ncu = C.c_uint32()
    ver = C.c_uint32()
    check("cae_device_info", lib().cae_device_info(C.byref(ncu), C.byref(ver)))
    return {"num_cu": ncu.value, "version": ver.value}
