"""Learned calibration on the GPU against the methods without the network.

The BF16 network, trained on 8,192 runs the simulator generates, maps a held-out
incidence curve to (R, S_0..S_8).  R and the S_a enter eq. 1 only as products, and one
aggregate curve identifies little beyond their mean (the transmissibility), so the
judged quantities are the transmissibility and the plain simulator re-run at the
prediction.  Against grid search over R, over R x one shared susceptibility (231
runs), and over that grid with as many runs as the network's training set:

* the network's transmissibility is the closest (log RMSE), with no simulation per query
  (its training runs are spent once, like the grids' runs);
* its prediction re-simulated on an independent stream is the closest to the target;
* refined by 20 gradient steps through the adjoint on the target's own stream, it
  reproduces the curve on that stream better than the same refinement started without
  the network (from the prior mean), in mean and median; better than every grid in
  mean; and better than the R grid and the 231-run grid in median.  (The grid with the
  network's simulation budget is level with it in median; that is reported, not
  asserted.)"""
import json

import pytest

from helpers import require_gpu

pytestmark = pytest.mark.gpu


def test_mlp_calibration_gains_over_grid_search():
    require_gpu()
    from paper_2110_04421_amd import calib
    s = calib.run(n_train=8192, n_heldout=256, n_agents=10000, epochs=25, days=120, tol=0.5,
                  n_gd=128, gd_iters=20)
    print(json.dumps({k: v for k, v in s.items() if k != "gradient_descent"}))
    print(json.dumps(s["gradient_descent"]))
    grids = ("grid", "grid2d", "grid2d_matched")
    tr, ind = s["transmissibility_rmse_log"], s["resim_rel_l2_independent_stream"]
    assert s["simulations_per_method"]["grid2d_matched"] >= s["simulations_per_method"]["mlp"] - 64
    for g in grids:
        assert tr["mlp"] < 0.9 * tr[g], (g, tr)
        assert ind["mlp"] < ind[g], (g, ind)
    assert tr["mlp"] < 0.5 * tr["training_mean_params"]
    gd = s["gradient_descent"]
    mean, med = gd["resim_rel_l2_same_stream"], gd["resim_rel_l2_same_stream_median"]
    for m in (mean, med):
        assert m["gd_from_mlp"] < 0.9 * m["gd_from_mean"], m
    for g in grids:
        assert mean["gd_from_mlp"] < mean[g], (g, mean)
    for g in ("grid", "grid2d"):
        assert med["gd_from_mlp"] < med[g], (g, med)
