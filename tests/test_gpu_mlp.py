"""Surrogate network kernels (bfloat16 matrix cores, fp32 accumulation) against the f64 oracle
with bfloat16 rounding at the same points.  Through the C ABI."""
import numpy as np
import pytest

import oracle
from oracle import mlp as OM

pytestmark = pytest.mark.gpu


def _mlp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_21784_amd import mlp
    oracle.lib()
    return mlp


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


@pytest.mark.parametrize("dims,N", [((4, 256, 3), 300), ((7, 48, 5), 33), ((1, 16, 1), 1),
                                    ((4, 256, 3), 4096)])
def test_forward_matches_oracle(dims, N):
    import torch
    M = _mlp()
    net = M.MLP(*dims, max_batch=max(N, 16), seed=1)
    rng = np.random.default_rng(2)
    p = net.get_params().astype(np.float64)
    p[dims[0] * dims[1]:dims[0] * dims[1] + dims[1]] = rng.normal(0, 0.1, dims[1])  # nonzero b1
    net.set_params(p)
    x = rng.normal(0, 1, (N, dims[0])).astype(np.float32)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    yo = OM.forward(net.get_params().astype(np.float64), dims, x.astype(np.float64), round_bf16=True)
    assert _rel(y, yo) < 2e-3, _rel(y, yo)


@pytest.mark.parametrize("dims,N", [((4, 256, 3), 6553), ((7, 48, 5), 33), ((1, 16, 1), 1),
                                    ((4, 256, 3), 32), ((33, 496, 16), 65), ((4, 256, 3), 100000)])
def test_predict_equals_forward(dims, N):
    """The fused inference kernel gives cae_mlp_forward's outputs bit for bit (same tiles, order
    and rounding points), for ragged batches and any N, and so the oracle's within tolerance."""
    import torch
    M = _mlp()
    chunk = min(N, 8192)
    net = M.MLP(*dims, max_batch=chunk, seed=4)
    rng = np.random.default_rng(5)
    p = net.get_params().astype(np.float64)
    p[dims[0] * dims[1]:dims[0] * dims[1] + dims[1]] = rng.normal(0, 0.1, dims[1])
    net.set_params(p)
    x = torch.from_numpy(rng.normal(0, 1, (N, dims[0])).astype(np.float32)).cuda()
    yp = net.predict(x).cpu().numpy()
    yf = np.concatenate([net.forward(x[i:i + chunk].contiguous()).cpu().numpy()
                         for i in range(0, N, chunk)])
    np.testing.assert_array_equal(yp, yf)
    k = min(N, 300)
    yo = OM.forward(net.get_params().astype(np.float64), dims, x[:k].cpu().numpy().astype(np.float64),
                    round_bf16=True)
    assert _rel(yp[:k], yo) < 2e-3, _rel(yp[:k], yo)


def test_predict_rejects_wide_hidden_layer():
    import ctypes as C
    M = _mlp()
    from paper_2606_21784_amd import _lib
    import torch
    net = M.MLP(4, 512, 3, max_batch=16, seed=0)
    x = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    y = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    rc = _lib.lib().cae_mlp_predict(C.byref(net.net), x.data_ptr(), y.data_ptr(), 4, None)
    assert rc == _lib.CAE_EINVAL


# Batches above 256 samples split the weight gradients' batch dimension over workgroups (a
# fixed-order sum of partial products): 257 (a one-sample second part), 1000 (ragged last part),
# 1024 (the training batch, 4 parts), 4097 (17 parts).
@pytest.mark.parametrize("dims,N", [((4, 256, 3), 256), ((7, 48, 5), 37), ((4, 256, 3), 257),
                                    ((4, 256, 3), 1000), ((4, 256, 3), 1024), ((4, 256, 3), 4097),
                                    ((7, 48, 5), 600)])
def test_backward_matches_oracle(dims, N):
    import torch
    M = _mlp()
    net = M.MLP(*dims, max_batch=N, seed=3)
    rng = np.random.default_rng(4)
    x = rng.normal(0, 1, (N, dims[0])).astype(np.float32)
    dy = rng.normal(0, 1, (N, dims[2])).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    net.forward(xd)
    g = net.backward(xd, torch.from_numpy(dy).cuda()).cpu().numpy().astype(np.float64)
    go = OM.backward(net.get_params().astype(np.float64), dims, x.astype(np.float64),
                     dy.astype(np.float64), round_bf16=True)
    parts_g, parts_o = OM.split(g, dims), OM.split(go, dims)
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], parts_g, parts_o):
        assert _rel(a, b) < 5e-3, (name, _rel(a, b))
    # and close to the exact (unrounded) gradient
    ge = OM.backward(net.get_params().astype(np.float64), dims, x.astype(np.float64),
                     dy.astype(np.float64), round_bf16=False)
    assert np.linalg.norm(g - ge) / np.linalg.norm(ge) < 0.05


def test_adam_matches_oracle():
    import torch
    M = _mlp()
    dims = (4, 32, 3)
    net = M.MLP(*dims, max_batch=64, seed=5)
    rng = np.random.default_rng(6)
    p = net.get_params().astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 6):
        g = rng.normal(0, 1, p.size).astype(np.float32)
        net.grads.copy_(torch.from_numpy(g))
        net.adam(1e-3, 0.9, 0.999, 1e-8)
        p, m, v = OM.adam(p, g.astype(np.float64), m, v, t, 1e-3, 0.9, 0.999, 1e-8)
    np.testing.assert_allclose(net.get_params(), p, rtol=1e-5, atol=1e-6)
    # bf16 weight copies follow the parameters
    W = net.weights.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    Wf = W.view(np.float32)
    W1, b1, W2, b2, W3, b3 = OM.split(net.get_params(), dims)
    ref = np.concatenate([W1.ravel(), W2.ravel(), W3.ravel(), W2.T.ravel()])
    np.testing.assert_array_equal(Wf, OM.bf16(ref).astype(np.float32))


@pytest.mark.parametrize("delta", [None, 0.05, 0.7])
def test_loss_grad_matches_torch_autograd(delta):
    import torch
    M = _mlp()
    net = M.MLP(4, 16, 3, max_batch=16, seed=0)
    rng = np.random.default_rng(7)
    y = rng.normal(0, 1, (1000, 3)).astype(np.float32)
    t = rng.normal(0, 1, (1000, 3)).astype(np.float32)
    dy = net.loss_grad(torch.from_numpy(y).cuda(), torch.from_numpy(t).cuda(),
                       huber_delta=delta).cpu().numpy()
    yt = torch.tensor(y, dtype=torch.float64, requires_grad=True)
    tt = torch.tensor(t, dtype=torch.float64)
    if delta is None:
        loss = torch.nn.functional.mse_loss(yt, tt)
    else:
        loss = torch.nn.functional.huber_loss(yt, tt, delta=delta)
    loss.backward()
    np.testing.assert_allclose(dy, yt.grad.numpy(), rtol=1e-5, atol=1e-9)
    assert abs(float(net.loss.item()) - float(loss.item())) < 1e-5 * max(1.0, float(loss.item()))


@pytest.mark.parametrize("fused", [False, True])
def test_training_fits_smooth_function(fused):
    import torch
    M = _mlp()
    rng = np.random.default_rng(8)
    x = rng.uniform(-1, 1, (4096, 4)).astype(np.float32)
    t = np.stack([np.sin(2 * x[:, 0]) + x[:, 1] ** 2, x[:, 2] * x[:, 3], np.exp(0.5 * x[:, 0])],
                 axis=1).astype(np.float32)
    t = (t - t.mean(0)) / t.std(0)
    net = M.MLP(4, 256, 3, max_batch=512, seed=9)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    first = None
    for epoch in range(60):
        perm = torch.randperm(4096, device="cuda")
        pi = perm.to(torch.int32)
        for b in range(8):
            idx = perm[b * 512:(b + 1) * 512]
            if fused:
                loss = net.train_step_fused(xd, td, 2e-3, idx=pi[b * 512:(b + 1) * 512])
            else:
                loss = net.train_step(xd[idx].contiguous(), td[idx].contiguous(), 2e-3)
        if first is None:
            first = float(loss.item())
    y = net.forward(xd[:512].contiguous())
    final = float(((y - td[:512]) ** 2).mean().item())
    assert final < 0.02 and final < first / 10, (first, final)


def _huber_grad(y, t, delta, n):
    r = y - t
    if delta is None:
        return 2.0 * r / n, float(np.sum(r * r) / n)
    a = np.abs(r)
    loss = np.where(a <= delta, 0.5 * r * r, delta * (a - 0.5 * delta))
    return np.clip(r, -delta, delta) / n, float(loss.sum() / n)


# The fused step (two launches): gradients against the oracle's back-propagation of the loss
# gradient of the oracle's own forward pass (same bfloat16 rounding points), parameters against
# the oracle's Adam fed the GPU's gradient, on a gathered batch (rows idx of a larger sample set).
# Batches: the training batch (1024), ragged ones (1000, 37: padded to a multiple of 32 with rows
# that must contribute nothing), a large one (4097), and another shape.
@pytest.mark.parametrize("dims,N,delta", [((4, 256, 3), 1024, 0.05), ((4, 256, 3), 1000, None),
                                          ((4, 256, 3), 37, 0.05), ((4, 256, 3), 4097, 0.7),
                                          ((7, 64, 5), 600, 0.05), ((32, 32, 16), 33, None)])
def test_fused_train_step_matches_oracle(dims, N, delta):
    import torch
    M = _mlp()
    net = M.MLP(*dims, max_batch=N, seed=13)
    rng = np.random.default_rng(14)
    p0 = net.get_params().astype(np.float64)
    d_in, H, d_out = dims
    o = d_in * H
    p0[o:o + H] = rng.normal(0, 0.1, H)  # nonzero biases
    p0[o + H + H * H:o + 2 * H + H * H] = rng.normal(0, 0.1, H)
    net.set_params(p0)
    p0 = net.get_params().astype(np.float64)
    m0 = rng.normal(0, 1e-3, p0.size)
    v0 = rng.uniform(0, 1e-4, p0.size)
    net.m.copy_(torch.from_numpy(m0.astype(np.float32)))
    net.v.copy_(torch.from_numpy(v0.astype(np.float32)))
    net.step_count = 4  # the call makes step 5
    rows = N + 500
    X = rng.normal(0, 1, (rows, d_in)).astype(np.float32)
    T = rng.normal(0, 0.3, (rows, d_out)).astype(np.float32)
    idx = rng.permutation(rows)[:N].astype(np.int32)
    loss = net.train_step_fused(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), 1e-3,
                                idx=torch.from_numpy(idx).cuda(), huber_delta=delta, grads=True)
    g = net.grads.cpu().numpy().astype(np.float64)
    xb, tb = X[idx].astype(np.float64), T[idx].astype(np.float64)
    y = OM.forward(p0, dims, xb, round_bf16=True)
    dy, loss_ref = _huber_grad(y, tb, delta, N * d_out)
    go = OM.backward(p0, dims, xb, dy, round_bf16=True)
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], OM.split(g, dims), OM.split(go, dims)):
        assert _rel(a, b) < 5e-3, (name, _rel(a, b))
    assert abs(float(loss.item()) - loss_ref) <= 2e-3 * loss_ref
    p1, m1, v1 = OM.adam(p0, g, m0.astype(np.float32).astype(np.float64),
                         v0.astype(np.float32).astype(np.float64), 5, 1e-3)
    np.testing.assert_allclose(net.get_params(), p1, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(net.m.cpu().numpy(), m1, rtol=1e-5, atol=1e-9)
    # the kernels take 1 - beta2 in fp32: 1 - fp32(0.999) is 0.001 (1 + 1.3e-5), which the
    # second moment inherits where the squared gradient dominates it
    np.testing.assert_allclose(net.v.cpu().numpy(), v1, rtol=3e-5, atol=1e-12)
    W = (net.weights.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    W1, b1, W2, b2, W3, b3 = OM.split(net.get_params(), dims)
    ref = np.concatenate([W1.ravel(), W2.ravel(), W3.ravel(), W2.T.ravel()])
    np.testing.assert_array_equal(W, OM.bf16(ref).astype(np.float32))


def test_fused_train_step_equals_unfused_sequence():
    """The fused step and the four unfused calls give the same gradients (to fp32 summation
    order) on the same batch; without idx the batch is the first N rows."""
    import torch
    M = _mlp()
    dims, N = (4, 256, 3), 1024
    rng = np.random.default_rng(15)
    X = torch.from_numpy(rng.normal(0, 1, (N, 4)).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.normal(0, 0.3, (N, 3)).astype(np.float32)).cuda()
    a, b = M.MLP(*dims, max_batch=N, seed=16), M.MLP(*dims, max_batch=N, seed=16)
    a.train_step_fused(X, T, 1e-3, huber_delta=0.05, grads=True)
    b.train_step(X, T, 1e-3, huber_delta=0.05)
    ga, gb = a.grads.cpu().numpy(), b.grads.cpu().numpy()
    for name, u, w in zip(["W1", "b1", "W2", "b2", "W3", "b3"], OM.split(ga, dims), OM.split(gb, dims)):
        assert _rel(u, w) < 1e-3, (name, _rel(u, w))
    assert abs(float(a.loss.item()) - float(b.loss.item())) <= 1e-5 * float(b.loss.item())


def test_fused_train_step_rejects_bad_shapes():
    import ctypes as C
    import torch
    M = _mlp()
    from paper_2606_21784_amd import _lib
    for dims in ((4, 48, 3), (4, 512, 3), (40, 64, 3)):  # H not a multiple of 32, H > 256, d_in > 32
        net = M.MLP(*dims, max_batch=16, seed=0)
        x = torch.zeros((16, dims[0]), dtype=torch.float32, device="cuda")
        t = torch.zeros((16, dims[2]), dtype=torch.float32, device="cuda")
        with pytest.raises(_lib.CaeError):
            net.train_step_fused(x, t, 1e-3)
    net = M.MLP(4, 32, 3, max_batch=16, seed=0)
    rc = _lib.lib().cae_mlp_train_step(C.byref(net.net), None, None, None, 4, net.m.data_ptr(), net.v.data_ptr(), 1,
                                       1e-3, 0.9, 0.999, 1e-8, 0, 0.0, net.loss.data_ptr(), None,
                                       net.ws.data_ptr(), None)
    assert rc == _lib.CAE_EINVAL
