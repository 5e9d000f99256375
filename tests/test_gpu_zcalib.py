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
    s = calib.run(n_train=8192, n_heldout=256, n_agents=10000, epochs=25, days=120, tol=0.5)
    print(json.dumps(s))
    rm, e = s["param_rmse_unit"], s["resim_rel_l2_same_stream"]
    # the network recovers parameters better than no information and than the R grid
    assert rm["mlp"] < rm["training_mean"] and rm["mlp"] < rm["grid"]
    assert s["R_rmse"]["mlp"] < 0.8 * s["R_rmse"]["training_mean"]
    # its parameters reproduce the curves much better than the training mean does
    assert e["mlp"] < 0.5 * e["training_mean_params"]
    # and a query costs no simulation
    assert s["seconds"]["mlp_predict"] < s["seconds"]["grid_search"]
