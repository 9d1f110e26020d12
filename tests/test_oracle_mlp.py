"""Pins of the surrogate network's CPU oracle (f64 with bfloat16 rounding points).

* bfloat16 rounding: hand values (ties to even) and torch's float32 -> bfloat16 conversion;
* SiLU against torch.nn.functional.silu;
* forward indexing: one-hot weights that make the network compute a closed form;
* backward: central finite differences of sum(dy * y) with rounding off;
* Adam: the first step's closed form and torch.optim.Adam over several steps.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as M


@pytest.fixture(scope="module", autouse=True)
def _load():
    oracle.lib()


def test_bf16_hand_values():
    one = 1.0
    assert M.bf16(one) == one
    assert M.bf16(1 + 2**-8) == 1.0  # halfway, even neighbour 1.0
    assert M.bf16(1 + 3 * 2**-8) == 1 + 2**-6  # halfway, even neighbour 1 + 2^-6
    assert M.bf16(1 + 2**-8 + 2**-20) == 1 + 2**-7  # just above halfway
    assert M.bf16(-3.0) == -3.0
    assert M.bf16(0.0) == 0.0


def test_bf16_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-3, 1000), rng.normal(0, 1e4, 1000)])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), ref)


def test_silu_matches_torch_and_closed_form_network():
    import torch
    d_in, H, d_out = 4, 4, 3
    P = M.param_count(d_in, H, d_out)
    rng = np.random.default_rng(1)
    x = rng.normal(0, 1.5, (50, d_in))
    p = np.zeros(P)
    W1, b1, W2, b2, W3, b3 = M.split(p, (d_in, H, d_out))
    # y0 = silu(silu(x2)) + 0.5 ; y1 = -silu(silu(x0) ) ; y2 = 2 * silu(silu(x3) + 1) - 1
    W1[2, 0] = 1.0
    W1[0, 1] = 1.0
    W1[3, 2] = 1.0
    W2[0, 0] = 1.0
    W2[1, 1] = 1.0
    W2[2, 2] = 1.0
    b2[2] = 1.0
    W3[0, 0] = 1.0
    W3[1, 1] = -1.0
    W3[2, 2] = 2.0
    b3[:] = [0.5, 0.0, -1.0]
    y = M.forward(p, (d_in, H, d_out), x, round_bf16=False)
    s = lambda t: torch.nn.functional.silu(torch.tensor(t, dtype=torch.float64)).numpy()
    np.testing.assert_allclose(y[:, 0], s(s(x[:, 2])) + 0.5, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(y[:, 1], -s(s(x[:, 0])), rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(y[:, 2], 2 * s(s(x[:, 3]) + 1.0) - 1.0, rtol=1e-14, atol=1e-14)
    # with rounding the activations are the bfloat16 values of the same closed form
    yr = M.forward(p, (d_in, H, d_out), x, round_bf16=True)
    xr = M.bf16(x)
    np.testing.assert_allclose(yr[:, 0], M.bf16(s(M.bf16(s(xr[:, 2])))) + 0.5, rtol=1e-14)


def test_backward_finite_differences():
    dims = (4, 8, 3)
    P = M.param_count(*dims)
    rng = np.random.default_rng(2)
    p = rng.normal(0, 0.5, P)
    x = rng.normal(0, 1, (7, 4))
    dy = rng.normal(0, 1, (7, 3))
    g = M.backward(p, dims, x, dy, round_bf16=False)
    f = lambda q: float(np.sum(dy * M.forward(q, dims, x, round_bf16=False)))
    eps = 1e-6
    idx = list(range(P)) if P < 300 else rng.choice(P, 300, replace=False)
    for i in idx:
        e = np.zeros(P)
        e[i] = eps
        fd = (f(p + e) - f(p - e)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_backward_rounded_close_to_exact():
    dims = (4, 32, 3)
    P = M.param_count(*dims)
    rng = np.random.default_rng(3)
    p = rng.normal(0, 0.3, P)
    x = rng.normal(0, 1, (64, 4))
    dy = rng.normal(0, 1, (64, 3))
    g0 = M.backward(p, dims, x, dy, round_bf16=False)
    g1 = M.backward(p, dims, x, dy, round_bf16=True)
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 0.05


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p = rng.normal(0, 1, 100)
    g = rng.normal(0, 1, 100)
    lr, eps = 1e-2, 1e-8
    p1, m1, v1 = M.adam(p, g, np.zeros(100), np.zeros(100), 1, lr, eps=eps)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-12)


def test_adam_matches_torch_optim():
    import torch
    rng = np.random.default_rng(5)
    n = 257
    p = rng.normal(0, 1, n)
    grads = rng.normal(0, 1, (6, n))
    lr, b1, b2, eps = 3e-3, 0.9, 0.99, 1e-7
    t = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=lr, betas=(b1, b2), eps=eps)
    m = np.zeros(n)
    v = np.zeros(n)
    q = p.copy()
    for k in range(6):
        t.grad = torch.tensor(grads[k], dtype=torch.float64)
        opt.step()
        q, m, v = M.adam(q, grads[k], m, v, k + 1, lr, b1, b2, eps)
    np.testing.assert_allclose(q, t.detach().numpy(), rtol=1e-12, atol=1e-14)
