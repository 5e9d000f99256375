"""Digital exposure notification and test turnaround (section 4) on the GPU against the
FP64 oracle, in lockstep; resuming mid-run rebuilds the last days' graphs and gives
the uninterrupted run; graph replay and eager launches agree."""
import numpy as np
import pytest

from helpers import require_gpu, lockstep
from oracle import step as ostep
from synthpop import workload
from synthpop.configs import TEST_TYPES
from test_gpu_parity import _lockstep

pytestmark = pytest.mark.gpu

DEN = dict(test_rate=0.05, app_adoption=0.5, den_compliance=0.8, den_window=7, **TEST_TYPES["rt_pcr"])


def _sim(p, pop, **kw):
    require_gpu()
    from paper_2110_04421_amd.sim import Simulator
    return Simulator(p, pop, **kw)


def test_notification_lockstep_with_interventions():
    p, pop = workload(1, n=20000, n_steps=45, vacc_trigger=0.002, **DEN)
    near, worst = _lockstep(p, pop, 45, check_csr_every=15)
    assert worst < 1e-5
    traj, _, _ = ostep.run(pop, p)
    assert traj[:, 0, ostep.C_NOTIFIED].sum() > 50


@pytest.mark.parametrize("two", [False, True])
def test_notification_batched_and_course_lockstep(two):
    """Two-tile leaves build the day's graph into the ring slot as one-tile leaves do."""
    p, pop = workload(3, n=30000, n_rep=4, n_steps=30, disease_model=1, **DEN)
    lockstep(lambda p_, pop_, **kw: _sim(p_, pop_, two_tile_leaves=two, **kw), p, pop, 30)


def test_resume_with_notification_equals_uninterrupted():
    p, pop = workload(1, n=15000, n_steps=30, **DEN)
    with _sim(p, pop) as s:
        full = s.run(30)
    with _sim(p, pop) as s:
        a = s.run(12)
        st, latch = s.state(), s.latch()
    with _sim(p, pop) as s:
        s.set_state(12, latch, st)
        b = s.run(18)
    assert full[:, 0, ostep.C_NOTIFIED].sum() > 0
    assert np.array_equal(np.concatenate([a, b]), full)


def test_notification_graph_and_eager_agree():
    p, pop = workload(1, n=15000, n_steps=25, **DEN)
    outs = []
    for graph in (True, False):
        with _sim(p, pop, graph=graph) as s:
            outs.append((s.run(25), s.state()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
