"""The two forms of the force of infection (eq. 1) agree bit for bit.

On a day with at most N/256 infectious agents the library sums only the rows that hold
an infectious source, found from the infectious agents' own rows (the daily graph is
symmetric); otherwise, or with ``dense_message``, every edge is streamed.  Populations
here are below 2^20 agents, so ``frontier_any_size`` turns the frontier path on.  An epidemic
that starts from a few seeds and grows past N/256 infectious agents crosses from one
form to the other; daily lambda, counts (infectious-edge counts included) and the final
state must be identical to the streaming-only run."""
import dataclasses

import numpy as np
import pytest

from helpers import require_gpu
from synthpop import workload

pytestmark = pytest.mark.gpu


def _days(p, pop, days, dense):
    from paper_2110_04421_amd.sim import Simulator
    out = []
    with Simulator(p, pop, dense_message=dense, frontier_any_size=not dense) as s:
        for _ in range(days):
            c = s.run(1)
            out.append((c.copy(), s.lam().view(np.uint32).copy()))
        st = s.state()
    return out, st


@pytest.mark.parametrize("case", ["plain", "batched-course-notification"])
def test_frontier_and_streaming_agree_bitwise(case):
    require_gpu()
    from paper_2110_04421_amd import _lib as L
    if case == "plain":
        p, pop = workload(1, n=30000, n_steps=70)
        pop = dataclasses.replace(pop, R=np.full(1, 9.0, np.float32))   # a faster outbreak
    else:
        from synthpop.configs import TEST_TYPES
        p, pop = workload(3, n=40000, n_rep=5, n_steps=70, disease_model=1, test_rate=0.05,
                          app_adoption=0.4, **TEST_TYPES["rt_pcr"])
    days = int(p["n_steps"])
    a, sa = _days(p, pop, days, dense=False)
    b, sb = _days(p, pop, days, dense=True)
    for t, ((ca, la), (cb, lb)) in enumerate(zip(a, b)):
        assert np.array_equal(ca, cb), f"counts differ on day {t}"
        assert np.array_equal(la, lb), f"lambda differs on day {t}"
    assert np.array_equal(sa, sb)
    # the run crosses the threshold: some days with few, some with many infectious agents
    counts = np.concatenate([c for c, _ in a])
    inf = (counts[:, :, L.C_E] + counts[:, :, L.C_I]).sum(axis=1)
    N = int(pop.n_agents)
    assert inf.min() * 256 <= N < inf.max() * 256, (inf.min(), inf.max(), N)
    assert counts[:, :, L.C_INF_EDGES].sum() > 0
