"""Pins of the relaxed (soft) oracle: as the Gumbel-softmax temperature goes to zero
it reproduces the hard oracle's incidence draw for draw (same uniforms); its
forward-mode tangents match central finite differences of its own forward."""
import numpy as np
import pytest

from oracle import step as ostep
from oracle.soft import SoftModel, gradient, sigmoid
from synthpop import workload


def test_zero_temperature_limit_equals_hard_step():
    p, pop = workload(4, n=4000, gumbel_tau=1e-7)
    T = 35
    c, _, _ = SoftModel(pop, p).run(T, tangents=False)
    hard = dict(p, mode=0)
    traj, _, _ = ostep.run(pop, hard, n_steps=T)
    assert np.array_equal(c[0], traj[:, 0, ostep.C_NEW].astype(np.float64))
    assert c[0].sum() > 50


@pytest.mark.parametrize("h", [1e-3, 1e-4])
def test_tangents_match_central_differences(h):
    p, pop = workload(4, n=2500)
    T = 30
    m = SoftModel(pop, p)
    c, cd, _ = m.run(T)
    dL = np.random.default_rng(3).normal(size=c.shape)
    g = gradient(cd, dL)
    th = np.concatenate([m.R[:, None], m.S], 1)
    for k in (0, 1, 5, 9):
        tp, tm = th.copy(), th.copy()
        tp[0, k] += h
        tm[0, k] -= h
        Lp = (dL * SoftModel(pop, p, R=tp[:, 0], S=tp[:, 1:]).run(T, tangents=False)[0]).sum()
        Lm = (dL * SoftModel(pop, p, R=tm[:, 0], S=tm[:, 1:]).run(T, tangents=False)[0]).sum()
        fd = (Lp - Lm) / (2 * h)
        assert abs(g[0, k] - fd) <= 1e-5 * max(abs(fd), np.abs(g).max())


def test_sigmoid_is_the_logistic_function():
    z = np.array([-800.0, -30.0, -1.0, 0.0, 2.0, 40.0, 800.0])
    ref = np.array([0.0, 9.357622968840175e-14, 0.2689414213699951, 0.5, 0.8807970779778823,
                    1.0, 1.0])
    assert np.allclose(sigmoid(z), ref, rtol=1e-12, atol=1e-300)


def test_straight_through_forward_is_the_hard_step_at_any_temperature():
    """The straight-through forward pass takes the relaxed sample's sign, which is the
    hard draw u < p, so its incidence is the hard oracle's at a finite temperature; its
    tangents are the relaxed sample's, so they differ from the relaxed run's only
    through the different trajectory (equal on day 0, where the state is the same)."""
    p, pop = workload(4, n=4000, gumbel_tau=0.5)
    T = 35
    c, cd, _ = SoftModel(pop, p, straight_through=True).run(T)
    traj, _, _ = ostep.run(pop, dict(p, mode=0), n_steps=T)
    assert np.array_equal(c[0], traj[:, 0, ostep.C_NEW].astype(np.float64))
    assert c[0].sum() > 50
    _, cd_soft, _ = SoftModel(pop, p).run(1)
    assert np.allclose(cd[:, 0], cd_soft[:, 0], rtol=1e-12, atol=0)
    assert np.abs(cd[:, 1:]).max() > 0
