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


def test_exact_operand_recipe_leaves_nothing_to_round():
    """The operands of the GPU's bit-exact network test (inputs in {-1, 0, 1}, weights
    and biases in {-1, 0, 1}/16, targets a quarter step from the output, B * n_out =
    1024): every layer computed with FP32 accumulation in two different orders equals
    the FP64 oracle exactly, so the test's claim of bit-exactness does not depend on the
    kernels' summation order."""
    for B, n_out in ((64, 16), (128, 8)):
        rng = np.random.default_rng(3)
        blob = mlp.pack({name: rng.integers(-1, 2, size=shp) / 16.0 for name, shp in mlp.SHAPES})
        x = rng.integers(-1, 2, size=(B, 192)).astype(np.float64)
        y, c = mlp.forward(blob, x)
        t = np.zeros((B, 16))
        t[:, :n_out] = y[:, :n_out] - rng.integers(-1, 2, size=(B, n_out)) / 4.0
        loss, g, _ = mlp.loss_and_backward(blob, x, t, n_out)

        def mm32(a, b, rev):
            a32, b32 = np.asarray(a, np.float32), np.asarray(b, np.float32)
            order = range(a32.shape[1] - 1, -1, -1) if rev else range(a32.shape[1])
            acc = np.zeros((a32.shape[0], b32.shape[1]), np.float32)
            for k in order:
                acc += np.outer(a32[:, k], b32[k, :])
            return acc.astype(np.float64)

        W = c["W"]
        for rev in (False, True):
            h1 = mlp.bf16_round(np.maximum(mm32(c["x"], W["W1"].T, rev) + W["b1"], 0))
            h2 = mlp.bf16_round(np.maximum(mm32(h1, W["W2"].T, rev) + W["b2"], 0))
            y32 = mm32(h2, W["W3"].T, rev) + W["b3"]
            assert np.array_equal(h1, c["h1"]) and np.array_equal(h2, c["h2"])
            assert np.array_equal(y32, y)
            dy = np.zeros_like(y)
            dy[:, :n_out] = 2.0 * (y32[:, :n_out] - t[:, :n_out]) / (B * n_out)
            dh2 = mm32(mlp.bf16_round(dy), W["W3"], rev) * (h2 > 0)
            dh1 = mm32(mlp.bf16_round(dh2), W["W2"], rev) * (h1 > 0)
            g32 = mlp.pack({"W3": mm32(mlp.bf16_round(dy).T, h2, rev), "b3": dy.sum(0),
                             "W2": mm32(mlp.bf16_round(dh2).T, h1, rev), "b2": dh2.sum(0),
                             "W1": mm32(mlp.bf16_round(dh1).T, c["x"], rev), "b1": dh1.sum(0)})
            assert np.array_equal(g32, g)
            assert np.array_equal(np.asarray(g32, np.float32).astype(np.float64), g32)
        assert float(np.float32(loss)) == loss
