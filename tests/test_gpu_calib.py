"""Learned calibration on the GPU: the BF16 network trained on simulator runs predicts
parameters whose re-simulation reproduces held-out curves better than the training
mean does and at least as well as grid search over R (the method without it), and it
does so without simulating per query."""
import json

import pytest

from helpers import require_gpu

pytestmark = pytest.mark.gpu


def test_mlp_calibration_gains_over_grid_search():
    require_gpu()
    from paper_2110_04421_amd import calib
    s = calib.run(n_train=2048, n_heldout=128, n_agents=10000, epochs=80, days=120, tol=0.5)
    print(json.dumps(s))
    e = s["resim_rel_l2"]
    assert e["mlp"] < 0.8 * e["training_mean_params"]
    assert e["mlp"] <= 1.1 * e["grid"]
    assert s["R_rmse"]["mlp"] < 1.0
    assert s["train_loss_last"] < 0.7 * s["train_loss_first"]
