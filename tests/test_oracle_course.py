"""The oracle's eleven-stage course (section 3, "Agent State Definition" and "Disease
Progression"), pinned three ways: with a degenerate course (no asymptomatic or severe
infections, fixed 5- and 10-day stages, nobody dying) it reproduces the SEIRM day step
count for count; its branch draws follow the age tables; its stage durations are
shift + Poisson(extra)."""
import numpy as np
from scipy import stats

from oracle import step as ostep
from oracle import tables as T
from synthpop import workload


def test_degenerate_course_reproduces_seirm_exactly():
    p, pop = workload(1, n=6000, n_steps=45, vacc_trigger=0.002, test_rate=0.1)
    p0 = dict(p, p_death=[0.0] * 9)
    p1 = dict(p0, disease_model=1, p_asym=[0.0] * 9, p_severe=[0.0] * 9,
              dur_shift=[5, 1, 10, 1, 1, 1, 1, 1, 1], dur_extra=[0.0, 1.0, 0.0] + [1.0] * 6)
    t0, s0, _ = ostep.run(pop, p0)
    t1, s1, _ = ostep.run(pop, p1)
    assert t0[:, :, ostep.C_NEW].sum() > 150 and t0[:, :, ostep.C_DOSE1].sum() > 0 and t0[:, :, ostep.C_POS].sum() > 0
    assert np.array_equal(t0, t1)
    assert np.all(t1[:, :, ostep.C_HOSP] == 0) and np.all(t1[:, :, ostep.C_ICU] == 0)


def test_course_branches_follow_the_age_tables():
    p, pop = workload(1, n=240000, n_steps=5)
    p = dict(p, disease_model=1)
    m = ostep.Model(pop, p)
    st = m.init_state()
    ids = np.arange(pop.n_agents)
    m.infect(st, ids, 7)
    c, s, age = st["course"], st["stage"], m.age
    kind = c & 3

    def check(mask, hit, prob):
        n = mask.sum()
        expect = prob[age[mask]].sum()
        var = (prob[age[mask]] * (1 - prob[age[mask]])).sum()
        z = (hit[mask].sum() - expect) / np.sqrt(var)
        assert abs(z) < 5, (n, z)

    f = {k: np.asarray(p[k], np.float32).astype(np.float64) for k in ("p_asym", "p_severe", "p_hosp", "p_icu")}
    check(np.ones(ids.size, bool), kind == 0, f["p_asym"])
    check(kind != 0, kind == 2, f["p_severe"])
    check(kind == 2, (c & 4) != 0, f["p_hosp"])
    check((c & 4) != 0, (c & 8) != 0, f["p_icu"])
    assert np.all(s[kind == 0] == T.STAGE_ASYM) and np.all(s[kind == 1] == T.STAGE_PRE_MILD)
    assert np.all(s[kind == 2] == T.STAGE_PRE_SEVERE)
    assert np.all((c & 8 == 0) | (c & 4 != 0))      # intensive care only after hospital


def test_stage_durations_are_shifted_poisson():
    p, pop = workload(1, n=100000, n_steps=5)
    p = dict(p, disease_model=1)
    m = ostep.Model(pop, p)
    ids = np.arange(pop.n_agents)
    for k, day in ((T.DUR_PRE, 3), (T.DUR_HOSP_R, 11)):
        d = m.duration(ids, day, k)
        shift, extra = p["dur_shift"][k], p["dur_extra"][k]
        assert d.min() >= shift
        obs = np.bincount(d - shift, minlength=40)[:40]
        pmf = stats.poisson.pmf(np.arange(40), extra) * ids.size
        keep = pmf > 5
        chi2 = ((obs[keep] - pmf[keep]) ** 2 / pmf[keep]).sum()
        assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3


def test_course_run_conserves_agents_and_deaths_come_from_intensive_care():
    p, pop = workload(1, n=20000, n_steps=80)
    p = dict(p, disease_model=1, p_severe=[0.5] * 9, p_hosp=[0.8] * 9, p_icu=[0.5] * 9)
    traj, st, _ = ostep.run(pop, p)
    c = traj[:, 0, :]
    N = pop.n_agents
    five = c[:, :5].sum(1) + c[:, ostep.C_HOSP] + c[:, ostep.C_ICU]
    assert np.all(five == N)
    assert c[:, ostep.C_HOSP].max() > 0 and c[:, ostep.C_ICU].max() > 0 and c[-1, ostep.C_M] > 0
    dead = st["stage"] == T.STAGE_M
    assert np.all(st["course"][dead] & 28 == 28)      # hospitalised, ICU, dies
    S = np.concatenate([[N - 10], c[:, ostep.C_S]])
    assert np.array_equal(-np.diff(S), c[:, ostep.C_NEW])


def test_asymptomatic_vaccine_immunity():
    """Section 5's second immunity: a protected agent is infected at the usual rate and
    its course is asymptomatic.  With no asymptomatic share in the tables and certain
    protection from dose_lag days after the first dose, an infection is asymptomatic
    exactly when it falls on a protected day; under sterilising immunity no infection
    falls on such a day."""
    base = dict(n=8000, n_steps=70, vacc_trigger=0.002, vacc_rate=0.03, eff1=1.0, eff2=1.0, dose_lag=3,
                disease_model=1, p_asym=[0.0] * 9)
    out = {}
    for imm in (0, 1):
        p, pop = workload(1, vacc_immunity=imm, **base)
        out[imm] = ostep.run(pop, p)
    for imm, (traj, st, _) in out.items():
        inf = st["t_exp"] >= 0
        prot = inf & (st["d1"] != ostep.NEVER) & (st["t_exp"] >= st["d1"].astype(np.int64) + 3)
        asym = inf & ((st["course"] & 3) == ostep.K_ASYM)
        if imm == 0:
            assert not prot.any() and not asym.any()
        else:
            assert prot.sum() > 5
            assert np.array_equal(asym, prot)
    assert out[1][0][:, :, ostep.C_NEW].sum() > out[0][0][:, :, ostep.C_NEW].sum()
