"""Python face of the calibration network kernels (abm_mlp_* in include/abm.h).

Parameters live on the GPU as an FP32 master copy and a BF16 copy used by the
matrix-core kernels; Adam runs in the library.  Nothing here computes the network.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


class MLP:
    """192 -> 256 -> 256 -> 16 network for batches up to ``max_batch``."""

    def __init__(self, max_batch: int, init: np.ndarray | None = None, seed: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the calibration network needs a ROCm GPU")
        self.torch = torch
        self.lib = L.lib()
        self.max_batch = int(max_batch)
        n = C.c_size_t(0)
        self._rc(self.lib.abm_mlp_workspace_size(self.max_batch, C.byref(n)))
        self.ws_bytes = int(n.value)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        if init is None:
            rng = np.random.default_rng(seed)
            init = he_uniform(rng)
        self.master = torch.from_numpy(np.asarray(init, np.float32).copy()).cuda()
        self.params = torch.empty(L.MLP_NPARAM, dtype=torch.bfloat16, device="cuda")
        self.m = torch.zeros(L.MLP_NPARAM, dtype=torch.float32, device="cuda")
        self.v = torch.zeros_like(self.m)
        self.grads = torch.zeros_like(self.m)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.step_count = 0
        # BF16 copy of the initial weights: an Adam step with zero rate and zero gradient
        self._adam(0.0, 0.9, 0.999, 1e-8, 1)
        self.m.zero_()
        self.v.zero_()

    def _rc(self, rc):
        if rc != 0:
            raise L.AbmError(rc, "calibration network call failed")

    def _p(self, t):
        return C.c_void_p(t.data_ptr())

    def forward(self, x):
        """x: float32 [B, 192] on the GPU -> y float32 [B, 16]."""
        x = x.contiguous()
        B = int(x.shape[0])
        assert x.shape[1] == L.MLP_IN and x.dtype == self.torch.float32 and B <= self.max_batch
        y = self.torch.empty((B, L.MLP_OUT), dtype=self.torch.float32, device="cuda")
        self._rc(self.lib.abm_mlp_forward(self._p(self.ws), self.ws_bytes, self._p(self.params),
                                          self._p(x), B, self._p(y), C.c_void_p(self.stream.cuda_stream)))
        return y

    def backward(self, target, n_out: int):
        """Gradient of the mean squared error on the first n_out outputs of the last
        forward; returns the loss (device tensor)."""
        target = target.contiguous()
        B = int(target.shape[0])
        self._rc(self.lib.abm_mlp_backward(self._p(self.ws), self.ws_bytes, self._p(self.params),
                                           self._p(target), B, int(n_out), self._p(self.grads),
                                           self._p(self.loss), C.c_void_p(self.stream.cuda_stream)))
        return self.loss

    def _adam(self, lr, b1, b2, eps, step):
        self._rc(self.lib.abm_mlp_adam(self._p(self.master), self._p(self.params), self._p(self.m),
                                       self._p(self.v), self._p(self.grads), float(lr), float(b1),
                                       float(b2), float(eps), int(step),
                                       C.c_void_p(self.stream.cuda_stream)))

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        self._adam(lr, b1, b2, eps, self.step_count)

    def train_step(self, x, target, n_out, lr=1e-3):
        self.forward(x)
        loss = self.backward(target, n_out)
        self.adam(lr)
        return loss

    def workspace_views(self, B: int):
        """(Xb, H1, H2, Y, dY, dH2, dH1) views of the workspace for a batch of B."""
        t = self.torch
        off = 256
        out = []
        for n, dt in ((B * 192, t.bfloat16), (B * 256, t.bfloat16), (B * 256, t.bfloat16),
                      (B * 16, t.float32), (B * 16, t.float32), (B * 256, t.float32),
                      (B * 256, t.float32)):
            size = n * (2 if dt == t.bfloat16 else 4)
            out.append(self.ws[off:off + size].view(dt))
            off = (off + size + 255) // 256 * 256
        return out


def he_uniform(rng):
    """He-uniform weights, zero biases, in the parameter blob layout."""
    parts = []
    for o, i in ((256, 192), (256, 256), (16, 256)):
        lim = np.sqrt(6.0 / i)
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)
