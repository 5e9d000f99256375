"""Pins of the FP64 calibration-network oracle: BF16 rounding against torch's own
conversion, backward against central differences (unquantised), the closed-form first
Adam step, and over-fitting a tiny set."""
import numpy as np
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -2.5e-39]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    blob = mlp.init_params(3) * 0.5
    x = rng.normal(size=(6, mlp.IN))
    t = rng.uniform(size=(6, mlp.OUT))
    loss, g, _ = mlp.loss_and_backward(blob, x, t, 10, quantize=False)
    idx = rng.choice(blob.size, 40, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, mlp.NPARAM - 20, 256 * 192 + 5]])
    for i in idx:
        h = 1e-6
        bp, bm = blob.copy(), blob.copy()
        bp[i] += h
        bm[i] -= h
        fd = (mlp.loss_and_backward(bp, x, t, 10, False)[0] - mlp.loss_and_backward(bm, x, t, 10, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_first_adam_step_moves_each_weight_by_lr():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    w, m, v = mlp.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1e-2, 0.9, 0.999, 1e-12, 1)
    assert np.allclose(w, [-1e-2, 1e-2, -1e-2, 0.0], rtol=1e-8, atol=0)


def test_overfits_a_tiny_set():
    rng = np.random.default_rng(2)
    blob = mlp.init_params(4)
    x = rng.normal(size=(16, mlp.IN))
    t = rng.uniform(size=(16, mlp.OUT))
    m = np.zeros_like(blob)
    v = np.zeros_like(blob)
    first = None
    for step in range(1, 301):
        loss, g, _ = mlp.loss_and_backward(blob, x, t, 10, quantize=False)
        first = loss if first is None else first
        blob, m, v = mlp.adam(blob, m, v, g, 1e-3, 0.9, 0.999, 1e-8, step)
    assert loss < 1e-3 * first
