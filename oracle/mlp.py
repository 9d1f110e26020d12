"""ctypes wrappers of the surrogate network's CPU oracle (mlp_oracle.c) -- test infrastructure."""
import ctypes as C

import numpy as np

_L = None


def _bind(L):
    global _L
    P, u32, u64, i32, dbl = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int, C.c_double
    L.orm_bf16.argtypes = [dbl]
    L.orm_bf16.restype = dbl
    L.orm_param_count.argtypes = [u32, u32, u32]
    L.orm_param_count.restype = u64
    L.orm_forward.argtypes = [P, u32, u32, u32, P, u32, i32, P, P, P, P, P]
    L.orm_backward.argtypes = [P, u32, u32, u32, P, P, u32, i32, P]
    L.orm_adam.argtypes = [P, P, P, P, u64, u32, dbl, dbl, dbl, dbl]
    _L = L


def _lib():
    if _L is None:
        from . import lib
        lib()
    return _L


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def bf16(x):
    f = np.vectorize(lambda v: _lib().orm_bf16(float(v)))
    return f(np.asarray(x, dtype=np.float64)).astype(np.float64)


def param_count(d_in, H, d_out):
    return int(_lib().orm_param_count(d_in, H, d_out))


def forward(params, dims, x, round_bf16=True, keep=False):
    d_in, H, d_out = dims
    p = np.ascontiguousarray(params, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, d_in)
    N = len(xx)
    y = np.zeros((N, d_out))
    if keep:
        z1, h1, z2, h2 = (np.zeros((N, H)) for _ in range(4))
        _lib().orm_forward(_p(p), d_in, H, d_out, _p(xx), N, int(round_bf16), _p(y), _p(z1),
                           _p(h1), _p(z2), _p(h2))
        return y, (z1, h1, z2, h2)
    _lib().orm_forward(_p(p), d_in, H, d_out, _p(xx), N, int(round_bf16), _p(y), None, None,
                       None, None)
    return y


def backward(params, dims, x, dy, round_bf16=True):
    d_in, H, d_out = dims
    p = np.ascontiguousarray(params, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, d_in)
    g = np.ascontiguousarray(dy, dtype=np.float64).reshape(-1, d_out)
    out = np.zeros(len(p))
    _lib().orm_backward(_p(p), d_in, H, d_out, _p(xx), _p(g), len(xx), int(round_bf16), _p(out))
    return out


def adam(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    p = np.array(params, dtype=np.float64)
    mm = np.array(m, dtype=np.float64)
    vv = np.array(v, dtype=np.float64)
    g = np.ascontiguousarray(grads, dtype=np.float64)
    _lib().orm_adam(_p(p), _p(g), _p(mm), _p(vv), len(p), t, lr, beta1, beta2, eps)
    return p, mm, vv


def split(params, dims):
    d_in, H, d_out = dims
    sizes = [d_in * H, H, H * H, H, H * d_out, d_out]
    out, o = [], 0
    for s in sizes:
        out.append(np.asarray(params[o:o + s]))
        o += s
    W1, b1, W2, b2, W3, b3 = out
    return W1.reshape(d_in, H), b1, W2.reshape(H, H), b2, W3.reshape(H, d_out), b3
