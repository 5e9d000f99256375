"""The allocation-free forward pass of the calibration network
(abm_mlp_forward_noalloc, scratch in the library's own per-GPU array) against the
workspace forward pass (abm_mlp_forward), both through the C ABI: equal bit for bit on
two calls in a row, the second with a smaller batch, and a batch beyond the scratch's
room is refused."""
import ctypes as C

import numpy as np
import pytest

from helpers import require_gpu

pytestmark = pytest.mark.gpu


def test_noalloc_forward_equals_workspace_forward():
    require_gpu()
    import torch
    from paper_2110_04421_amd import _lib as L
    from paper_2110_04421_amd.mlp import MLP
    lib = L.lib()
    net = MLP(L.MLP_NOALLOC_MAX_BATCH, seed=5)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(17)
    ptr = lambda t: C.c_void_p(t.data_ptr())
    for B in (L.MLP_NOALLOC_MAX_BATCH, 37):        # the second call is smaller
        x = torch.from_numpy(rng.normal(size=(B, L.MLP_IN)).astype(np.float32)).cuda()
        ref = net.forward(x)
        y = torch.full((B, L.MLP_OUT), float("nan"), dtype=torch.float32, device="cuda")
        assert lib.abm_mlp_forward_noalloc(ptr(net.params), ptr(x), B, ptr(y), stream) == 0
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        assert torch.equal(y, ref), f"batch {B}: {float((y - ref).abs().max())}"
    big = L.MLP_NOALLOC_MAX_BATCH + 1
    x = torch.zeros((big, L.MLP_IN), dtype=torch.float32, device="cuda")
    y = torch.zeros((big, L.MLP_OUT), dtype=torch.float32, device="cuda")
    assert lib.abm_mlp_forward_noalloc(ptr(net.params), ptr(x), big, ptr(y), stream) == -3
    assert lib.abm_mlp_forward_noalloc(ptr(net.params), ptr(x), 0, ptr(y), stream) == -1
