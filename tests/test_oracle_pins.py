"""Pins of five oracle branches against what the paper and probability fix, each on a
state built by hand so that the branch alone decides the outcome:

* SEIRM death at removal (section 3, "Disease Progression"): deaths among the agents
  removed on a day are Binomial(removed in age group a, p_death[a]) per group, taken
  from lane 1 of the agent's day block, and nobody dies at any other time.
* Quarantine dropout (section 4, "Self-quarantine"): a quarantine that may end on any
  day with probability d lasts k days with probability (1-d)^k d for k < 14, and the
  full 14 days with probability (1-d)^14.
* Vaccine allocation order (section 5, Table 1): with capacity for k doses, the dosed
  agents are the first k of the paper's Table 1 order over the six worked-example
  archetypes, ties by ascending agent id; dead, not-yet-due and fully dosed agents are
  never dosed.
* Intensive-care death (section 3): the death flag drawn on entering intensive care is
  Binomial(entrants in age group a, p_die[a]) per group.
* The course's per-class infectiousness factor A_s of eq. 1: lambda of a susceptible
  agent with asymptomatic, presymptomatic, symptomatic and hospitalised neighbours at
  distinct factors, against the Gamma integral written with scipy's incomplete gamma.
"""
import math
import os

import numpy as np
import pytest
from scipy import special, stats

from conftest import GOLDEN
from oracle import philox
from oracle import step as ostep
from oracle import tables as T
from synthpop import workload
from synthpop.population import Population


def _flat_pop(ages, delay=21):
    """One replicate of singleton households with the given age groups, no workplaces,
    no seeds."""
    N = len(ages)
    return Population(np.array([0, N], np.int64), np.asarray(ages, np.uint8),
                      np.arange(N + 1, dtype=np.int32), np.zeros(N, np.uint8),
                      np.zeros(1, np.int32), np.zeros(0, np.int32), np.array([0, 0], np.int64),
                      np.zeros(0, np.int32), np.array([5.18], np.float32),
                      np.linspace(0.35, 1.47, 9, dtype=np.float32)[None, :],
                      np.array([delay], np.int32))


def _per_group_binomial(age, hit, prob, z_max=5.0):
    """Every age group's hit count is within z_max standard deviations of
    Binomial(n_a, prob[a]); a group with prob 0 or 1 must be exact."""
    for a in range(9):
        sel = age == a
        n = int(sel.sum())
        k = int(hit[sel].sum())
        p = float(prob[a])
        if p in (0.0, 1.0):
            assert k == round(n * p), (a, n, k, p)
            continue
        z = (k - n * p) / math.sqrt(n * p * (1 - p))
        assert abs(z) < z_max, (a, n, k, p, z)


def _f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def test_seirm_death_at_removal_is_binomial_per_age_group():
    N = 180_000
    rng = np.random.default_rng(11)
    ages = rng.integers(0, 9, N)
    pop = _flat_pop(ages)
    p_death = [0.0, 0.02, 0.05, 0.11, 0.2, 0.33, 0.5, 0.71, 0.9]
    params = dict(workload(0)[0], mu_random=[0.0] * 9, p_death=p_death)
    m = ostep.Model(pop, params)
    st = m.init_state()
    # everyone infected; tau on day 3 spreads over 1..20, so a fifteenth of them
    # reach the removal day tau = e_days + i_days = 15 today
    tau = rng.integers(1, 21, N)
    t = 3
    st["t_exp"][:] = t - tau
    st["stage"][:] = np.where(tau <= 5, T.STAGE_E, T.STAGE_I)
    new, _ = m.step(st, t, np.zeros((1, ostep.NC), np.int64))
    removed = (st["stage"] == T.STAGE_I) & (tau == 15)
    dead = new["stage"] == T.STAGE_M
    assert np.array_equal(dead | (new["stage"] == T.STAGE_R), removed)     # removal day only
    assert removed.sum() > 8000
    _per_group_binomial(ages[removed], dead[removed], _f32(p_death))
    # the draw is lane 1 of the agent's AGENT block of the day, compared with u < p
    w = philox.draw_words(0, np.arange(N), t, 0, philox.PURPOSE_AGENT, 0)
    u1 = philox.uniform(w[1])
    assert np.array_equal(dead, removed & (u1 < _f32(p_death)[ages]))


def test_quarantine_dropout_stays_follow_the_truncated_geometric_law():
    N, d, qd = 60_000, 0.12, 14
    pop = _flat_pop(np.zeros(N, np.int64))
    params = dict(workload(0)[0], mu_random=[0.0] * 9, quarantine_days=qd, test_rate=0.0,
                  quarantine_dropout=d, test_delay=2, test_delay_max=2)
    m = ostep.Model(pop, params)
    st = m.init_state()
    st["stage"][:] = T.STAGE_R
    # every agent's positive result arrives on day 0: quarantined from day 0
    st["pending"][:] = True
    st["positive"][:] = True
    st["test_day"][:] = -2
    quarantined = np.zeros(N, np.int64)
    prev = np.zeros((1, ostep.NC), np.int64)
    for t in range(qd + 3):
        st, out = m.step(st, t, prev)
        quarantined += t < st["q_until"]          # quarantined on day t (after its pre-pass)
        prev = out["counts"]
    obs = np.bincount(quarantined, minlength=qd + 1)
    assert obs.size == qd + 1                     # never longer than 14 days
    f = _f32(d)
    law = np.array([(1 - f) ** k * f for k in range(qd)] + [(1 - f) ** qd])
    assert abs(law.sum() - 1.0) < 1e-12
    e = law * N
    chi2 = ((obs - e) ** 2 / e).sum()
    assert stats.chi2.sf(chi2, qd) > 1e-3
    # a dropped-out quarantine ends on its dropout day: q_until is that day
    assert np.all(st["q_until"] == quarantined)


def _table1():
    people, strat = {}, {}
    for line in open(os.path.join(GOLDEN, "table1_priority.txt")):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "person":
            people[f[1]] = (int(f[2]), int(f[3]))
        else:
            strat[int(f[1])] = f[2:]
    return people, strat


@pytest.mark.parametrize("strategy", [0, 1, 2])
def test_vaccine_allocation_follows_table1_then_agent_id(strategy):
    people, strat = _table1()
    names = list(people)
    group = lambda years: min(8, max(0, (years - 1) // 10))     # decade groups 0-10 .. 80+
    copies, t, delay = 40, 60, 21
    rng = np.random.default_rng(100 + strategy)
    # 6 archetypes x 40 copies, shuffled over the ids, plus agents that may never be
    # dosed: dead, second dose not yet due, both doses given
    kind = np.concatenate([np.repeat(np.arange(6), copies), np.full(30, 6)])
    rng.shuffle(kind)
    N = kind.size
    ages = np.array([group(people[names[k]][1]) if k < 6 else rng.integers(0, 9) for k in kind])
    pop = _flat_pop(ages, delay=delay)
    order = {nm: i for i, nm in enumerate(strat[strategy])}
    rank_of_kind = np.array([order[nm] for nm in names])
    for cap in (1, 37, 119, 200, 240, 260):
        params = dict(workload(1)[0], strategy=strategy, vacc_rate=(cap + 0.5) / N, vacc_trigger=0.0)
        m = ostep.Model(pop, params)
        st = m.init_state()
        st["latch"][:] = True
        dose2 = np.array([k < 6 and people[names[k]][0] == 2 for k in kind])
        st["vacc"][dose2] = 1
        st["d1"][dose2] = t - delay - rng.integers(0, 5, dose2.sum())
        bad = np.flatnonzero(kind == 6)
        third = len(bad) // 3
        st["stage"][bad[:third]] = T.STAGE_M                             # dead
        st["vacc"][bad[third:2 * third]] = 1
        st["d1"][bad[third:2 * third]] = t - delay + 1                   # due tomorrow
        st["vacc"][bad[2 * third:]] = 2                                  # fully dosed
        st["d1"][bad[2 * third:]] = t - 50
        st["d2"][bad[2 * third:]] = t - 20
        before = {k: v.copy() for k, v in st.items()}
        d1n, d2n = m.vaccinate(st, t, np.zeros((1, ostep.NC), np.int64))
        good = np.flatnonzero(kind < 6)
        expect = good[np.lexsort((good, rank_of_kind[kind[good]]))][:cap]
        dosed = np.flatnonzero(st["vacc"] != before["vacc"])
        assert np.array_equal(np.sort(dosed), np.sort(expect)), (strategy, cap)
        assert np.all(st["vacc"][dosed] == before["vacc"][dosed] + 1)
        assert d1n[0] + d2n[0] == min(cap, good.size)
        got1 = dosed[before["vacc"][dosed] == 0]
        assert np.all(st["d1"][got1] == t) and np.all(st["d2"][dosed[before["vacc"][dosed] == 1]] == t)


def test_intensive_care_death_is_binomial_per_age_group():
    N = 150_000
    rng = np.random.default_rng(21)
    ages = rng.integers(0, 9, N)
    pop = _flat_pop(ages)
    p_die = [0.0, 0.04, 0.13, 0.22, 0.35, 0.47, 0.61, 0.79, 1.0]
    params = dict(workload(1)[0], disease_model=1, p_die=p_die, p_icu=[0.3] * 9)
    m = ostep.Model(pop, params)
    st = m.init_state()
    t = 9
    # every agent is hospitalised with an intensive-care course, and the hospital
    # stage ends today: all enter intensive care and draw whether they die there
    st["stage"][:] = T.STAGE_HOSP
    st["course"][:] = ostep.K_SEVERE | ostep.B_HOSP | ostep.B_ICU
    st["t_exp"][:] = t - 12
    st["t_next"][:] = t
    new = {k: v.copy() for k, v in st.items()}
    m.progress(st, new, t)
    assert np.all(new["stage"] == T.STAGE_ICU)
    dies = (new["course"] & ostep.B_DIE) != 0
    _per_group_binomial(ages, dies, _f32(p_die))
    # the stay's length is drawn from the duration that matches the outcome
    dur = new["t_next"] - t
    w = philox.draw_words(0, np.arange(N), t, 0, philox.PURPOSE_COURSE, 1)
    k_die = T.poisson_count(w[0], T.poisson_thresholds(float(params["dur_extra"][T.DUR_ICU_DIE])))
    k_rec = T.poisson_count(w[0], T.poisson_thresholds(float(params["dur_extra"][T.DUR_ICU_R])))
    assert np.array_equal(dur, np.where(dies, params["dur_shift"][T.DUR_ICU_DIE] + k_die,
                                        params["dur_shift"][T.DUR_ICU_R] + k_rec))
    # the outcome is independent of the stay's own draw: the day's lane-0 count has the
    # same law among those who die and those who recover (mixed-probability groups)
    mixed = (ages >= 1) & (ages <= 7)
    res = stats.mannwhitneyu(k_die[mixed & dies], k_die[mixed & ~dies])
    assert res.pvalue > 1e-4
    # and it is lane 1 of the course's block 1 of the day
    assert np.array_equal(dies, philox.uniform(w[1]) < _f32(p_die)[ages])


def _phi(tau, shape=2.5, scale=2.0):
    """Gamma(shape, scale) mass of day [tau - 1, tau], from scipy's regularised
    incomplete gamma."""
    return float(special.gammainc(shape, tau / scale) - special.gammainc(shape, (tau - 1) / scale))


def test_course_infectiousness_factors_per_class():
    # destination 0 (age group 4, susceptible) has one edge from each source:
    #   1 asymptomatic, tau 3     2 presymptomatic (mild), tau 2
    #   3 symptomatic (severe), tau 8     4 hospitalised, tau 10
    #   5 symptomatic, tau 6, quarantined today
    A_asym, A_pre, A_sym = 0.3, 0.7, 1.1
    ages = [4, 0, 1, 2, 3, 5]
    pop = _flat_pop(ages)
    params = dict(workload(1)[0], disease_model=1, A_asym=A_asym, A_stage=[0.0, A_pre, A_sym, 0.0, 0.0],
                  kappa=1.0 / 11.0)
    m = ostep.Model(pop, params)
    st = m.init_state()
    t = 20
    stage = [T.STAGE_S, T.STAGE_ASYM, T.STAGE_PRE_MILD, T.STAGE_SEVERE, T.STAGE_HOSP, T.STAGE_MILD]
    tau = [0, 3, 2, 8, 10, 6]
    st["stage"][:] = stage
    st["t_exp"][1:] = t - np.array(tau[1:])
    st["q_until"][5] = t + 3
    code = m.codes(st, t)
    w = [1.0, 0.2, 0.2, 0.2, 0.2]          # household-weight edge from the asymptomatic one
    rp = np.array([0, 5, 5, 5, 5, 5, 5])
    col = np.array([1, 2, 3, 4, 5])
    lam, _ = m.force_of_infection(code, (rp, col, np.array(w), None))
    R, kappa, S4 = _f32(5.18), _f32(1.0 / 11.0), _f32(np.linspace(0.35, 1.47, 9))[4]
    hand = R * kappa * S4 * (1.0 * A_asym * _phi(3) + 0.2 * A_pre * _phi(2) + 0.2 * A_sym * _phi(8))
    assert abs(lam[0] - hand) < 1e-13 * hand
    assert np.all(lam[1:] == 0.0)
    # each class alone
    for src, A, tt, ww in ((1, A_asym, 3, 1.0), (2, A_pre, 2, 0.2), (3, A_sym, 8, 0.2)):
        only = np.where(np.arange(6) == src, code, 0)
        lam1, _ = m.force_of_infection(only, (rp, col, np.array(w), None))
        assert abs(lam1[0] - R * kappa * S4 * ww * A * _phi(tt)) < 1e-13 * lam1[0]


def test_seirm_stage_factors_apply_by_days_since_exposure():
    """SEIRM with A_E != A_I: a source counts with A_E on days 1..5 since exposure
    and with A_I on days 6..15 (eq. 1's A_{s_i} per stage)."""
    A_E, A_I = 0.6, 1.3
    pop = _flat_pop([4, 0, 0, 0])
    params = dict(workload(0)[0], A_stage=[0.0, A_E, A_I, 0.0, 0.0], kappa=1.0)
    m = ostep.Model(pop, params)
    st = m.init_state()
    t = 30
    st["stage"][1:] = [T.STAGE_E, T.STAGE_I, T.STAGE_I]
    st["t_exp"][1:] = t - np.array([5, 6, 15])
    code = m.codes(st, t)
    rp = np.array([0, 3, 3, 3, 3])
    col = np.array([1, 2, 3])
    lam, _ = m.force_of_infection(code, (rp, col, np.array([0.2, 0.2, 1.0]), None))
    R, S4 = _f32(5.18), _f32(np.linspace(0.35, 1.47, 9))[4]
    hand = R * S4 * (0.2 * A_E * _phi(5) + 0.2 * A_I * _phi(6) + 1.0 * A_I * _phi(15))
    assert abs(lam[0] - hand) < 1e-13 * hand
