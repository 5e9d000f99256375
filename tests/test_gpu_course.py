"""The eleven-stage course on the GPU against the FP64 oracle, in lockstep: codes,
force of infection, every field of the agent state (course path and stage end day
included) and the daily counts, with testing, quarantine and vaccination on, in one
population and in a batch of replicates of different sizes."""
import numpy as np
import pytest

from helpers import require_gpu
from oracle import step as ostep
from synthpop import workload
from test_gpu_parity import _lockstep

pytestmark = pytest.mark.gpu

SEVERE = dict(disease_model=1, p_severe=[0.5] * 9, p_hosp=[0.8] * 9, p_icu=[0.5] * 9)


def test_course_lockstep_with_interventions():
    require_gpu()
    p, pop = workload(1, n=20000, n_steps=60, vacc_trigger=0.002, **SEVERE)
    near, worst = _lockstep(p, pop, 60, check_csr_every=30)
    assert worst < 1e-5


def test_asymptomatic_vaccine_immunity_lockstep():
    """Protected agents infected at the usual rate, on the asymptomatic course."""
    require_gpu()
    p, pop = workload(1, n=20000, n_steps=60, vacc_trigger=0.002, vacc_rate=0.03, eff1=0.9,
                      vacc_immunity=1, **SEVERE)
    near, worst = _lockstep(p, pop, 60)
    assert worst < 1e-5


def test_course_batched_replicates_lockstep():
    require_gpu()
    p, pop = workload(3, n=30000, n_rep=5, n_steps=30, vacc_trigger=0.002, **SEVERE)
    _lockstep(p, pop, 30)


def test_degenerate_course_equals_seirm_on_the_gpu():
    require_gpu()
    from paper_2110_04421_amd.sim import Simulator
    p, pop = workload(1, n=20000, n_steps=50, vacc_trigger=0.002)
    p0 = dict(p, p_death=[0.0] * 9)
    p1 = dict(p0, disease_model=1, p_asym=[0.0] * 9, p_severe=[0.0] * 9,
              dur_shift=[5, 1, 10, 1, 1, 1, 1, 1, 1], dur_extra=[0.0, 1.0, 0.0] + [1.0] * 6)
    outs = []
    for q in (p0, p1):
        with Simulator(q, pop) as s:
            outs.append((s.run(50), s.lam()))
    assert outs[0][0][:, :, ostep.C_NEW].sum() > 100
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1].view(np.uint32), outs[1][1].view(np.uint32))


def test_course_counts_hospital_and_intensive_care():
    require_gpu()
    from paper_2110_04421_amd.sim import Simulator
    p, pop = workload(1, n=50000, n_steps=120, **SEVERE)
    with Simulator(p, pop) as s:
        c = s.run(120)[:, 0, :]
    assert np.all(c[:, :5].sum(1) + c[:, ostep.C_HOSP] + c[:, ostep.C_ICU] == pop.n_agents)
    assert c[:, ostep.C_HOSP].max() > 0 and c[:, ostep.C_ICU].max() > 0 and c[-1, ostep.C_M] > 0
