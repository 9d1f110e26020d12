"""cae_mlp_train_step_noalloc (the training step on the library's static scratch, for callers
that cannot allocate device memory) against cae_mlp_train_step with a caller workspace: the same
kernels, so parameters, Adam moments, bfloat16 weight copies, gradients and loss must agree bit
for bit, on two calls in a row (the second with a smaller, ragged batch that reuses the scratch
the first left behind).  Batches beyond the scratch are refused before any launch."""
import ctypes as C

import numpy as np
import pytest

from paper_2606_21784_amd import _lib

DIMS = (4, 256, 3)
SCRATCH_BYTES = 8 << 20


def _train_ws_bytes(d_in, H, N):
    """The fused step's workspace, as the library lays it out (256-byte aligned parts)."""
    al = lambda x: (x + 255) // 256 * 256
    Bp = (N + 31) // 32 * 32
    o = 0
    for part in (2 * d_in * Bp, 2 * H * Bp, 2 * H * Bp, 2 * 16 * Bp, 2 * H * Bp, 2 * H * Bp, 4 * (Bp // 16)):
        o = al(o + part)
    return o


def test_noalloc_rejects_batches_beyond_the_scratch():
    """Host-side refusal: no device pointer is dereferenced and nothing is launched."""
    L = _lib.lib()
    N = 1
    while _train_ws_bytes(DIMS[0], DIMS[1], N) <= SCRATCH_BYTES:
        N += 32
    fake = C.c_void_p(256)  # never dereferenced: the call fails on the host
    net = _lib.Mlp(DIMS[0], DIMS[1], DIMS[2], 0, fake, fake)
    rc = L.cae_mlp_train_step_noalloc(C.byref(net), fake, fake, None, N, fake, fake, 1, 1e-3, 0.9, 0.999, 1e-8,
                                      0, 0.0, fake, None, None)
    assert rc == _lib.CAE_EINVAL
    assert b"scratch" in L.cae_last_error()


def _state(net):
    return {"params": net.params.clone(), "m": net.m.clone(), "v": net.v.clone(),
            "weights": net.weights.clone(), "grads": net.grads.clone(), "loss": net.loss.clone()}


@pytest.mark.gpu
def test_noalloc_equals_workspace_entry_on_two_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_21784_amd import mlp
    rng = np.random.default_rng(31)
    rows = 5000
    X = torch.from_numpy(rng.normal(0, 1, (rows, DIMS[0])).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.normal(0, 0.3, (rows, DIMS[2])).astype(np.float32)).cuda()
    a = mlp.MLP(*DIMS, max_batch=4000, seed=32)  # caller workspace
    b = mlp.MLP(*DIMS, max_batch=16, seed=32)    # its own workspace is too small to be the one used
    assert torch.equal(a.params, b.params)
    # first call: a large batch chosen by an index list; second: a smaller ragged batch of the
    # first rows (the scratch still holds the first call's activations)
    batches = [(torch.from_numpy(rng.permutation(rows)[:3000].astype(np.int32)).cuda(), None, 0.05),
               (None, 300, None)]
    for k, (idx, n, delta) in enumerate(batches):
        for net, noalloc in ((a, False), (b, True)):
            net.train_step_fused(X, T, 1e-3, idx=idx, n=n, huber_delta=delta, grads=True, noalloc=noalloc)
        torch.cuda.synchronize()
        sa, sb = _state(a), _state(b)
        for key in sa:
            assert torch.equal(sa[key], sb[key]), (k, key)
        assert np.isfinite(float(sa["loss"].item()))
    # the refused batch leaves the network untouched
    before = _state(b)
    with pytest.raises(_lib.CaeError):
        b.train_step_fused(X, T, 1e-3, n=rows, noalloc=True)
    torch.cuda.synchronize()
    for key, val in _state(b).items():
        assert torch.equal(val, before[key]), key
