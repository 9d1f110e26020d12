"""ctypes declarations for libcae.so (the C ABI in include/cae.h).

Argument marshalling only: every step of the engine runs in the HIP library.  Loading fails
loudly when the library has not been built; there is no fallback path.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcae.so")

CAE_OK, CAE_EINVAL, CAE_EOVERFLOW, CAE_ENOSPACE, CAE_EHIP, CAE_ESTATE = 0, -1, -2, -3, -4, -5
NUM_CLASSES = 40


class Market(C.Structure):
    _fields_ = [("L", C.c_uint32), ("A", C.c_uint32), ("K", C.c_uint32), ("Q", C.c_uint32),
                ("n_noise", C.c_uint32), ("n_mom", C.c_uint32),
                ("maker_half_spread", C.c_uint32), ("flags", C.c_uint32)]


class State(C.Structure):
    _fields_ = [("last", C.c_uint32), ("prev", C.c_uint32), ("steps_done", C.c_uint64),
                ("n_trade", C.c_uint64), ("sum_vol", C.c_uint64), ("sum_px", C.c_uint64),
                ("sum_spread", C.c_uint64), ("n_spread", C.c_uint64),
                ("sum_r", C.c_double), ("sum_r2", C.c_double),
                ("ref2", C.c_uint32), ("reserved", C.c_uint32)]


# Agent models (descriptor flags bits 0-7), generators (bits 8-15) and the position of P_mkt
# (bits 16-31).
MODEL_LAST, MODEL_MID, PMKT_SHIFT = 0, 1, 16
GEN_PHILOX, GEN_SPLITMIX, GEN_SHIFT = 0, 1, 8


class Sizes(C.Structure):
    _fields_ = [("book_words", C.c_uint64), ("book_bytes", C.c_uint64),
                ("state_bytes", C.c_uint64), ("workspace_bytes", C.c_uint64)]


class Buffers(C.Structure):
    _fields_ = [("book", C.c_void_p), ("state", C.c_void_p), ("workspace", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("waves_per_group", C.c_uint32), ("groups_per_cu", C.c_uint32),
                ("max_lds_bytes", C.c_uint32), ("flags", C.c_uint32),
                ("waves_per_market", C.c_uint8 * NUM_CLASSES),
                ("pipelined", C.c_uint8 * NUM_CLASSES),
                ("overlap", C.c_uint8 * NUM_CLASSES),
                ("class_cost", C.c_float * NUM_CLASSES),
                ("pack", C.c_uint8 * NUM_CLASSES)]


class Mlp(C.Structure):
    _fields_ = [("d_in", C.c_uint32), ("d_hidden", C.c_uint32), ("d_out", C.c_uint32),
                ("flags", C.c_uint32), ("params", C.c_void_p), ("weights", C.c_void_p)]


class MlpSizes(C.Structure):
    _fields_ = [("n_params", C.c_uint64), ("n_weights", C.c_uint64),
                ("workspace_bytes", C.c_uint64)]


class CaeError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__("%s failed (%d): %s" % (fn, code, msg))
        self.code = code


EXPORTS = ["cae_strerror", "cae_last_error", "cae_device_info", "cae_sizes", "cae_create",
           "cae_step", "cae_step_naive", "cae_step_traced", "cae_read_books", "cae_read_state", "cae_write_state", "cae_get_tuning",
           "cae_last_step_ms", "cae_destroy", "cae_clear", "cae_mlp_sizes",
           "cae_mlp_refresh_weights", "cae_mlp_forward", "cae_mlp_predict",
           "cae_mlp_backward",
           "cae_mlp_adam", "cae_mlp_train_step", "cae_mlp_train_step_noalloc",
           "cae_mlp_loss_grad"]

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcae.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_2606_21784_amd/build.py" % LIB_PATH)
    # torch ships its own HIP runtime.  Loaded first, it is the one libcae.so binds to, so the
    # library's calls see the same devices, memory and streams as torch's tensors; loading
    # libcae.so first would map the system runtime as a second copy that torch does not use.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
    L.cae_strerror.argtypes = [i32]
    L.cae_strerror.restype = C.c_char_p
    L.cae_last_error.restype = C.c_char_p
    L.cae_device_info.argtypes = [P, P]
    L.cae_sizes.argtypes = [P, u32, P]
    L.cae_create.argtypes = [P, u32, u64, P, P, P, P, P]
    L.cae_step.argtypes = [P, u32]
    L.cae_step_naive.argtypes = [P, u32]
    L.cae_step_traced.argtypes = [P, u32, P, P, u64]
    L.cae_read_books.argtypes = [P, P, u64]
    L.cae_read_state.argtypes = [P, P, u32]
    L.cae_write_state.argtypes = [P, P, u32, P, u64]
    L.cae_get_tuning.argtypes = [P, P]
    L.cae_last_step_ms.argtypes = [P, P]
    L.cae_destroy.argtypes = [P]
    L.cae_clear.argtypes = [u32, u32, P, P, P, P]
    f32 = C.c_float
    L.cae_mlp_sizes.argtypes = [u32, u32, u32, u32, P]
    L.cae_mlp_refresh_weights.argtypes = [P, P]
    L.cae_mlp_forward.argtypes = [P, P, P, u32, P, P]
    L.cae_mlp_predict.argtypes = [P, P, P, u32, P]
    L.cae_mlp_backward.argtypes = [P, P, P, P, u32, P, P]
    L.cae_mlp_adam.argtypes = [P, P, P, P, u32, f32, f32, f32, f32, P]
    L.cae_mlp_loss_grad.argtypes = [P, P, P, P, u32, i32, f32, P]
    L.cae_mlp_train_step.argtypes = [P, P, P, P, u32, P, P, u32, f32, f32, f32, f32, i32, f32, P, P, P, P]
    L.cae_mlp_train_step_noalloc.argtypes = [P, P, P, P, u32, P, P, u32, f32, f32, f32, f32, i32, f32, P, P, P]
    for name in EXPORTS:
        if name not in ("cae_strerror", "cae_last_error"):
            getattr(L, name).restype = i32
    _lib = L
    return L


def check(fn, code):
    if code != CAE_OK:
        msg = lib().cae_last_error().decode(errors="replace")
        raise CaeError(fn, code, msg)
    return code
