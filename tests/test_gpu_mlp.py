"""BF16 matrix-core network kernels against the FP64 oracle on the same BF16 operands."""
import numpy as np
import pytest

from helpers import require_gpu
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _net(B, seed=0, scale=1.0):
    require_gpu()
    from paper_2110_04421_amd.mlp import MLP, he_uniform
    init = he_uniform(np.random.default_rng(seed)) * scale
    init[-16:] = np.linspace(-0.5, 0.5, 16)           # non-zero output biases
    return MLP(B, init=init), init


def _bf(t):
    return t.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("B", [1, 37, 256, 1000])
def test_forward_layers_match_fp64_on_bf16_operands(B):
    import torch
    net, init = _net(max(B, 64))
    x = np.random.default_rng(B).normal(size=(B, 192)).astype(np.float32)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    xb, h1, h2, *_ = net.workspace_views(B)
    P = omlp.unpack(omlp.bf16_round(init))
    xq = omlp.bf16_round(x)
    assert np.array_equal(_bf(xb).reshape(B, 192), xq)
    # layer 1 from the same BF16 operands: the GPU's BF16 store is within one rounding
    h1_ref = np.maximum(xq @ P["W1"].T + P["b1"], 0)
    g1 = _bf(h1).reshape(B, 256)
    assert np.all(np.abs(g1 - h1_ref) <= 2.0 ** -7 * np.abs(h1_ref) + 1e-4)
    g2 = _bf(h2).reshape(B, 256)
    h2_ref = np.maximum(g1 @ P["W2"].T + P["b2"], 0)
    assert np.all(np.abs(g2 - h2_ref) <= 2.0 ** -7 * np.abs(h2_ref) + 1e-4)
    # output layer (FP32 out): FP32 accumulation within 1e-3 of FP64
    y_ref = g2 @ P["W3"].T + P["b3"]
    assert np.all(np.abs(y - y_ref) <= 1e-3 * (np.abs(y_ref) + np.abs(y_ref).mean()))
    # end to end against the oracle's forward (its own BF16 activations)
    y_o, _ = omlp.forward(init, x)
    assert np.abs(y - y_o).max() <= 2e-2 * np.abs(y_o).max()


@pytest.mark.parametrize("B,n_out", [(64, 10), (300, 16)])
def test_backward_matches_oracle(B, n_out):
    import torch
    net, init = _net(B, seed=1)
    rng = np.random.default_rng(5)
    x = rng.normal(size=(B, 192)).astype(np.float32)
    t = rng.uniform(size=(B, 16)).astype(np.float32)
    net.forward(torch.from_numpy(x).cuda())
    loss = float(net.backward(torch.from_numpy(t).cuda(), n_out).cpu())
    g = net.grads.cpu().numpy().astype(np.float64)
    loss_o, g_o, _ = omlp.loss_and_backward(init, x, t, n_out)
    assert abs(loss - loss_o) <= 1e-2 * loss_o
    Po, Pg = omlp.unpack(g_o), omlp.unpack(g)
    for k in Po:
        num = np.linalg.norm(Pg[k] - Po[k])
        assert num <= 2e-2 * np.linalg.norm(Po[k]) + 1e-7, (k, num, np.linalg.norm(Po[k]))
    # the dW3 product itself, on the GPU's own BF16 operands, is exact to FP32 accumulation
    _, _, h2, _, dy, _, _ = net.workspace_views(B)
    ref = omlp.bf16_round(dy.cpu().numpy().reshape(B, 16)).T @ _bf(h2).reshape(B, 256)
    assert np.all(np.abs(Pg["W3"] - ref) <= 1e-3 * (np.abs(ref) + np.abs(ref).mean()))


def test_adam_step_matches_oracle():
    import torch
    net, init = _net(16, seed=2)
    g = np.random.default_rng(6).normal(size=omlp.NPARAM).astype(np.float32)
    net.grads.copy_(torch.from_numpy(g))
    m = np.zeros(omlp.NPARAM)
    v = np.zeros(omlp.NPARAM)
    w = init.astype(np.float64)
    for step in range(1, 4):
        net.adam(1e-3)
        w, m, v = omlp.adam(w, m, v, g.astype(np.float64), 1e-3, 0.9, 0.999, 1e-8, step)
    wg = net.master.cpu().numpy().astype(np.float64)
    assert np.abs(wg - w).max() <= 1e-6
    assert np.array_equal(net.params.float().cpu().numpy().astype(np.float64), omlp.bf16_round(wg))


def test_training_overfits_a_small_set():
    import torch
    net, _ = _net(64, seed=3)
    rng = np.random.default_rng(7)
    x = torch.from_numpy(rng.normal(size=(64, 192)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.uniform(size=(64, 16)).astype(np.float32)).cuda()
    first = float(net.train_step(x, t, 10).cpu())
    for _ in range(400):
        loss = net.train_step(x, t, 10, lr=1e-3)
    assert float(loss.cpu()) < 0.02 * first


def _exact_case(B, n_out, seed):
    """Operands whose every product and partial sum is exact in FP32 and whose hidden
    activations are exact in BF16 where the kernels store them (inputs in {-1, 0, 1},
    weights and biases in {-1, 0, 1}/16, targets a quarter step from the oracle's
    output, B * n_out = 1024): the FP32-accumulating matrix-core kernels then owe the
    FP64 oracle every bit, whatever their summation order."""
    rng = np.random.default_rng(seed)
    blob = omlp.pack({name: rng.integers(-1, 2, size=shp) / 16.0 for name, shp in omlp.SHAPES})
    x = rng.integers(-1, 2, size=(B, 192)).astype(np.float64)
    y_o, _ = omlp.forward(blob, x)
    t = np.zeros((B, 16))
    t[:, :n_out] = y_o[:, :n_out] - rng.integers(-1, 2, size=(B, n_out)) / 4.0
    return blob, x, t, y_o


@pytest.mark.parametrize("B,n_out", [(64, 16), (128, 8)])
def test_forward_and_backward_bit_exact_on_exact_operands(B, n_out):
    require_gpu()
    import torch
    from paper_2110_04421_amd.mlp import MLP
    blob, x, t, y_o = _exact_case(B, n_out, 3)
    net = MLP(B, init=blob.astype(np.float32))
    y = net.forward(torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    assert np.array_equal(y, y_o)
    loss = float(net.backward(torch.from_numpy(t.astype(np.float32)).cuda(), n_out).cpu())
    loss_o, g_o, _ = omlp.loss_and_backward(blob, x, t, n_out)
    assert loss == loss_o
    g = net.grads.cpu().numpy().astype(np.float64)
    for k, v in omlp.unpack(g_o).items():
        assert np.array_equal(omlp.unpack(g)[k], v), k
