"""The calibration surrogate's network on the GPU: a d_in -> H -> H -> d_out SiLU perceptron
with bfloat16 weights trained by libcae's matrix-core kernels (forward, backward, Adam).

PyTorch only owns the device buffers and the stream; every step runs in libcae.
"""
import ctypes as C

import numpy as np

from ._lib import Mlp, MlpSizes, check, lib


class MLP:
    def __init__(self, d_in=4, d_hidden=256, d_out=3, max_batch=8192, seed=0, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the surrogate network needs a ROCm GPU")
        self.dims = (int(d_in), int(d_hidden), int(d_out))
        self.max_batch = int(max_batch)
        sz = MlpSizes()
        check("cae_mlp_sizes", lib().cae_mlp_sizes(d_in, d_hidden, d_out, self.max_batch, C.byref(sz)))
        self.n_params = int(sz.n_params)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        dev = self.device
        self.params = torch.zeros(self.n_params, dtype=torch.float32, device=dev)
        self.weights = torch.zeros(int(sz.n_weights), dtype=torch.int16, device=dev)
        self.grads = torch.zeros(self.n_params, dtype=torch.float32, device=dev)
        self.m = torch.zeros(self.n_params, dtype=torch.float32, device=dev)
        self.v = torch.zeros(self.n_params, dtype=torch.float32, device=dev)
        self.ws = torch.empty(int(sz.workspace_bytes), dtype=torch.uint8, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.net = Mlp(d_in, d_hidden, d_out, 0, self.params.data_ptr(), self.weights.data_ptr())
        self.step_count = 0
        self._last_n = None
        self.set_params(self.init_params(seed))

    @property
    def stream(self):
        import torch
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def init_params(self, seed):
        """Weights N(0, 1/fan_in), biases zero (host draw with a fixed seed)."""
        d_in, H, d_out = self.dims
        rng = np.random.Generator(np.random.PCG64(seed))
        parts = [rng.normal(0, 1 / np.sqrt(d_in), d_in * H), np.zeros(H),
                 rng.normal(0, 1 / np.sqrt(H), H * H), np.zeros(H),
                 rng.normal(0, 1 / np.sqrt(H), H * d_out), np.zeros(d_out)]
        return np.concatenate(parts).astype(np.float32)

    def set_params(self, p):
        import torch
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params
        self.params.copy_(torch.from_numpy(p))
        check("cae_mlp_refresh_weights", lib().cae_mlp_refresh_weights(C.byref(self.net), self.stream))
        self.m.zero_()
        self.v.zero_()
        self.step_count = 0

    def get_params(self):
        return self.params.detach().cpu().numpy().copy()

    def forward(self, x, y=None):
        """x: (N, d_in) float32 device tensor -> (N, d_out) float32 device tensor."""
        import torch
        n = int(x.shape[0])
        if n > self.max_batch:
            raise ValueError("batch %d exceeds max_batch %d" % (n, self.max_batch))
        assert x.dtype == torch.float32 and x.is_contiguous() and x.shape[1] == self.dims[0]
        if y is None:
            y = torch.empty((n, self.dims[2]), dtype=torch.float32, device=self.device)
        check("cae_mlp_forward", lib().cae_mlp_forward(C.byref(self.net), x.data_ptr(), y.data_ptr(),
                                                       n, self.ws.data_ptr(), self.stream))
        self._last_n = n
        return y

    def predict(self, x, y=None):
        """Inference only (one fused launch, any batch size): the same outputs as ``forward``,
        keeping nothing for ``backward``."""
        import torch
        n = int(x.shape[0])
        assert x.dtype == torch.float32 and x.is_contiguous() and x.shape[1] == self.dims[0]
        if y is None:
            y = torch.empty((n, self.dims[2]), dtype=torch.float32, device=self.device)
        check("cae_mlp_predict", lib().cae_mlp_predict(C.byref(self.net), x.data_ptr(), y.data_ptr(), n,
                                                       self.stream))
        return y

    def backward(self, x, dy):
        """Gradients (fp32, parameter layout) of sum(dy * y) for the last forward's batch."""
        n = int(dy.shape[0])
        assert n == self._last_n, "backward must follow a forward on the same batch"
        check("cae_mlp_backward", lib().cae_mlp_backward(C.byref(self.net), x.data_ptr(), dy.data_ptr(),
                                                         self.grads.data_ptr(), n, self.ws.data_ptr(),
                                                         self.stream))
        return self.grads

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        check("cae_mlp_adam", lib().cae_mlp_adam(C.byref(self.net), self.grads.data_ptr(), self.m.data_ptr(),
                                                 self.v.data_ptr(), self.step_count, lr, beta1, beta2, eps,
                                                 self.stream))

    def loss_grad(self, y, t, dy=None, huber_delta=None):
        """Mean squared error (huber_delta None) or mean Huber loss and its gradient."""
        import torch
        if dy is None:
            dy = torch.empty_like(y)
        kind, delta = (0, 0.0) if huber_delta is None else (1, float(huber_delta))
        check("cae_mlp_loss_grad", lib().cae_mlp_loss_grad(y.data_ptr(), t.data_ptr(), dy.data_ptr(),
                                                           self.loss.data_ptr(), y.numel(), kind, delta,
                                                           self.stream))
        return dy

    def train_step_fused(self, x, t, lr, idx=None, n=None, beta1=0.9, beta2=0.999, eps=1e-8, huber_delta=None,
                         grads=False, noalloc=False):
        """One training step in two launches (``cae_mlp_train_step``): the batch is rows idx of
        x / t (int32 device tensor, or None for the first n rows; x: (rows, d_in), t: (rows,
        d_out) float32 device tensors).  Returns the device tensor holding the batch's mean loss
        (and fills ``self.grads`` when grads is true).  noalloc: the same step through
        ``cae_mlp_train_step_noalloc``, on the library's static scratch instead of self.ws."""
        import torch
        assert x.dtype == torch.float32 and t.dtype == torch.float32 and x.is_contiguous() and t.is_contiguous()
        if idx is not None:
            assert idx.dtype == torch.int32 and idx.is_contiguous()
            n = int(idx.numel())
        n = int(x.shape[0]) if n is None else int(n)
        if n > self.max_batch and not noalloc:
            raise ValueError("batch %d exceeds max_batch %d" % (n, self.max_batch))
        self.step_count += 1
        kind, delta = (0, 0.0) if huber_delta is None else (1, float(huber_delta))
        common = (C.byref(self.net), x.data_ptr(), t.data_ptr(), idx.data_ptr() if idx is not None else None, n,
                  self.m.data_ptr(), self.v.data_ptr(), self.step_count, lr, beta1, beta2, eps, kind, delta,
                  self.loss.data_ptr(), self.grads.data_ptr() if grads else None)
        if noalloc:
            check("cae_mlp_train_step_noalloc", lib().cae_mlp_train_step_noalloc(*common, self.stream))
        else:
            check("cae_mlp_train_step", lib().cae_mlp_train_step(*common, self.ws.data_ptr(), self.stream))
        return self.loss

    def train_step(self, x, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, huber_delta=None):
        """The same step as ``train_step_fused`` by the unfused kernels (forward, loss gradient,
        backward, Adam: one call each)."""
        y = self.forward(x)
        dy = self.loss_grad(y, t, huber_delta=huber_delta)
        self.backward(x, dy)
        self.adam(lr, beta1, beta2, eps)
        return self.loss
