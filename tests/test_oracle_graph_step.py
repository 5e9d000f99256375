"""Pins of the oracle's contact graph and daily step: an independent scalar reading of
the graph, structural invariants, a hand-computed force of infection, an exact
enumeration of infection outcomes, an exact closed-form expectation of the first
day's offspring, conservation and the fixed-duration identities, Table 1."""
import math
import os

import numpy as np
import pytest
from scipy import stats

from conftest import GOLDEN
from oracle import graph as og
from oracle import step as ostep
from oracle.tables import phi
from synthpop import workload, make_population
from synthpop.population import Population


@pytest.mark.parametrize("k,n,nrep", [(0, None, None), (1, 2500, None), (3, 4000, 5)])
def test_graph_vectorised_equals_scalar_reading(k, n, nrep):
    p, pop = workload(k, n=n, n_rep=nrep)
    for t in (0, 7):
        rp, col, w, _ = og.build_graph(pop, p, t)
        rp2, col2, w2 = og.build_graph_naive(pop, p, t)
        assert np.array_equal(rp, rp2) and np.array_equal(col, col2) and np.array_equal(w, w2)


def test_graph_structure_invariants():
    p, pop = workload(1, n=20000)
    rp, col, w, blk = og.build_graph(pop, p, 5)
    N = pop.n_agents
    rows = np.repeat(np.arange(N), np.diff(rp))
    assert not np.any(rows == col)                          # no self-contacts
    fwd = np.sort(rows * N * 8 + col * 8 + np.round(w * 5).astype(np.int64))
    bwd = np.sort(col * N * 8 + rows * 8 + np.round(w * 5).astype(np.int64))
    assert np.array_equal(fwd, bwd)                         # symmetric with weights
    # household block: exactly the other members, ascending
    maps = og.static_maps(pop)
    hh = blk == og.BLK_HH
    assert np.array_equal(np.bincount(rows[hh], minlength=N), maps["hh_hi"] - maps["hh_lo"] - 1)
    # occupation contacts stay inside the workplace
    occ = (blk == og.BLK_OCC_OWN) | (blk == og.BLK_OCC_RECV)
    assert np.array_equal(maps["wp_of"][rows[occ]], maps["wp_of"][col[occ]])
    # mean in-degree: household + mu_occ + mu_rand within 6 sigma
    E = col.size
    contacts = (blk == og.BLK_OCC_OWN).sum() + (blk == og.BLK_RAND_OWN).sum()
    mu_c = N * (2.0 + 2.42)
    assert abs(contacts - mu_c) < 6 * math.sqrt(mu_c)
    assert E == hh.sum() + 2 * contacts


def _tiny_pop(age, hh_start):
    N = len(age)
    return Population(np.array([0, N], np.int64), np.array(age, np.uint8),
                      np.array(hh_start, np.int32), np.zeros(N, np.uint8),
                      np.zeros(1, np.int32), np.zeros(0, np.int32), np.array([0, 0], np.int64),
                      np.zeros(0, np.int32), np.array([5.18], np.float32),
                      np.linspace(0.35, 1.47, 9, dtype=np.float32)[None, :],
                      np.array([21], np.int32))


def test_force_of_infection_hand_computed():
    # A (id 0) exposed with tau=1; C (id 1, age group 4) susceptible, same household;
    # B (id 2) infected with tau=7; D (id 3, age group 0) susceptible.
    # contacts: household A-C (w 1.0); random C-B, D-B twice, D-A (w 0.2).
    pop = _tiny_pop([0, 4, 0, 0], [0, 2, 3, 4])
    params = dict(workload(0)[0], kappa=1.0)
    m = ostep.Model(pop, params)
    st = m.init_state()
    st["stage"][[0, 2]] = [1, 2]
    st["t_exp"][[0, 2]] = [-1, -7]
    code = m.codes(st, 0)
    assert list(code) == [1, 0, 7, 0]
    edges = {1: [(0, 1.0), (2, 0.2)], 3: [(2, 0.2), (2, 0.2), (0, 0.2)],
             0: [(1, 1.0), (3, 0.2)], 2: [(1, 0.2), (3, 0.2), (3, 0.2)]}
    rp = [0]
    col, w = [], []
    for j in range(4):
        col += [c for c, _ in edges[j]]
        w += [x for _, x in edges[j]]
        rp.append(len(col))
    lam, _ = m.force_of_infection(code, (np.array(rp), np.array(col), np.array(w), None))
    R, S = float(np.float32(5.18)), np.linspace(0.35, 1.47, 9).astype(np.float32).astype(float)
    f1, f7 = phi(1, 2.5, 2.0), phi(7, 2.5, 2.0)
    lam_c = R * S[4] * (1.0 * f1 + 0.2 * f7)
    lam_d = R * S[0] * (0.2 * f7 + 0.2 * f7 + 0.2 * f1)
    assert abs(lam[1] - lam_c) < 1e-15 and abs(lam[3] - lam_d) < 1e-15
    assert lam[0] == 0.0 and lam[2] == 0.0
    # same numbers with R = 5.18 exactly, as written out by hand: 0.2571375..., 0.0756352...
    assert abs(5.18 * 0.91 * (f1 + 0.2 * f7) - 0.257137548879784) < 1e-14
    assert abs(5.18 * 0.35 * (0.4 * f7 + 0.2 * f1) - 0.0756352589381372) < 1e-14


def test_infection_outcomes_exact_enumeration():
    """Households of 8: two infectors (tau = 1 and 8) and six susceptibles of distinct
    ages; no other contacts.  The outcome pattern of the six is drawn with the exact
    product law prod p^y (1-p)^(1-y), p_j = 1 - exp(-lambda_j) (eq. 2)."""
    nrep = 6000
    pop = make_population([8] * nrep, workplaces=False, n_seeds=0, pop_seed=77)
    pop.hh_start = (np.arange(nrep + 1) * 8).astype(np.int32)
    ages = np.array([0, 0, 1, 3, 4, 6, 7, 8], np.uint8)
    pop.age = np.tile(ages, nrep)
    params = dict(workload(0)[0], mu_random=[0.0] * 9, kappa=1.0)
    m = ostep.Model(pop, params)
    st = m.init_state()
    base = np.arange(nrep) * 8
    st["stage"][base] = 1
    st["t_exp"][base] = -1
    st["stage"][base + 1] = 2
    st["t_exp"][base + 1] = -8          # tau 8 (day 0): infected stage
    new, out = m.step(st, 0, np.zeros((nrep, ostep.NC), np.int64))
    inf = (new["stage"].reshape(nrep, 8)[:, 2:] == 1)
    pat = (inf * (1 << np.arange(6))).sum(1)
    obs = np.bincount(pat, minlength=64)
    R = float(np.float32(5.18))
    S = np.linspace(0.35, 1.47, 9).astype(np.float32).astype(float)
    lam = R * S[ages[2:]] * (phi(1, 2.5, 2.0) + phi(8, 2.5, 2.0))
    p = 1 - np.exp(-lam)
    probs = np.array([np.prod([p[i] if (y >> i) & 1 else 1 - p[i] for i in range(6)])
                      for y in range(64)])
    e = probs * nrep
    keep = e >= 5
    chi2 = ((obs[keep] - e[keep]) ** 2 / e[keep]).sum() + \
        (obs[~keep].sum() - e[~keep].sum()) ** 2 / max(e[~keep].sum(), 1e-9)
    assert stats.chi2.sf(chi2, keep.sum()) > 1e-3


def test_first_day_offspring_closed_form():
    """One infector per replicate of n agents, random contacts only, mean in-degree mu.
    The number of contacts between the infector and any other agent is exactly
    Poisson(mu / (n-1)) (thinned Poisson draws from both ends), so the expected
    number infected on day 0 is (n-1)(1 - exp(-(mu/(n-1))(1 - exp(-R kappa w Phi(tau)))))."""
    nrep, n, mu = 1500, 200, 10.0
    pop = make_population([n] * nrep, workplaces=False, n_seeds=1, pop_seed=88)
    pop.hh_start = np.arange(nrep * n + 1, dtype=np.int32)           # singletons
    pop.susceptibility[:] = 1.0
    params = dict(workload(0)[0], mu_random=[mu] * 9, kappa=1.0)
    m = ostep.Model(pop, params)
    st = m.init_state()
    seeds = np.asarray(pop.initial_infected, np.int64)
    taus = 1 + np.arange(nrep) % 8
    st["t_exp"][seeds] = -taus
    st["stage"][seeds] = np.where(taus <= 5, 1, 2)
    new, out = m.step(st, 0, np.zeros((nrep, ostep.NC), np.int64))
    got = out["counts"][:, ostep.C_NEW]
    R = float(np.float32(5.18))
    wr = float(np.float32(0.2))
    c = np.array([R * wr * phi(int(t), 2.5, 2.0) for t in taus])
    expect = (n - 1) * (1 - np.exp(-(mu / (n - 1)) * (1 - np.exp(-c))))
    # Var of a sum of (dependent only through the infector) Bernoullis: bound by mean
    z = (got.sum() - expect.sum()) / math.sqrt(expect.sum() * 1.5)
    assert abs(z) < 4.5


def test_conservation_and_fixed_durations():
    p, pop = workload(0)
    traj, st, _ = ostep.run(pop, p)
    c = traj[:, 0, :]
    N = pop.n_agents
    assert np.all(c[:, :5].sum(1) == N)
    S = np.concatenate([[N - 10], c[:, 0]])
    assert np.all(np.diff(S) <= 0) and np.array_equal(-np.diff(S), c[:, ostep.C_NEW])
    inc = {-1: 10}
    for t in range(c.shape[0]):
        inc[t] = int(c[t, ostep.C_NEW])
    for t in range(c.shape[0]):
        # state(t+1): E = exposed on days t-4..t, I = exposed on days t-14..t-5
        assert c[t, ostep.C_E] == sum(inc.get(d, 0) for d in range(t - 4, t + 1))
        assert c[t, ostep.C_I] == sum(inc.get(d, 0) for d in range(t - 14, t - 4))
    assert c[-1, ostep.C_R] + c[-1, ostep.C_M] == sum(inc.get(d, 0) for d in range(-1, c.shape[0] - 15))


def test_table1_priority_orders():
    people, strat = {}, {}
    for line in open(os.path.join(GOLDEN, "table1_priority.txt")):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "person":
            people[f[1]] = (int(f[2]), int(f[3]))
        else:
            strat[int(f[1])] = f[2:]
    group = lambda years: min(8, max(0, (years - 1) // 10))     # 0-10, 11-20, ..., 80+
    assert group(78) == 7 and group(68) == 6 and group(40) == 3 and group(85) == 8
    names = list(people)
    for s, expected in strat.items():
        keys = [int(ostep.vaccination_priority(s, people[nm][0], group(people[nm][1])))
                for nm in names]
        order = [nm for _, nm in sorted(zip(keys, names))]
        assert order == expected
        assert len(set(keys)) == len(keys)


def test_intervention_marginals():
    p, pop = workload(1, n=30000, vacc_trigger=0.0, n_steps=40)
    m = ostep.Model(pop, p)
    st = m.init_state()
    prev = np.zeros((1, ostep.NC), np.int64)
    m.put_counts(prev, st)
    hist = []
    cap = math.floor(0.005 * 30000)
    for t in range(40):
        old = st
        st, out = m.step(st, t, prev)
        c = out["counts"][0]
        prev = out["counts"]
        hist.append((old, st, c))
        # capacity-limited doses, standard order: second doses before any first dose
        assert c[ostep.C_DOSE1] + c[ostep.C_DOSE2] == cap
        # tests: binomial share of the eligible
        elig = ((old["stage"] != 4) & (t >= st["q_until"]) & ~(old["pending"] & (t != old["test_day"] + 2))).sum()
        assert abs(c[ostep.C_TESTS] - 0.05 * elig) < 5 * math.sqrt(0.05 * 0.95 * elig)
        # a positive result due today starts exactly 14 days of quarantine
        due = old["pending"] & (old["test_day"] + 2 == t) & old["positive"]
        assert np.all(st["q_until"][due] == t + 14)
        assert c[ostep.C_POS] == due.sum()
    # second doses: exactly those with first dose >= 21 days ago, oldest first
    assert (st["vacc"] == 2).sum() > 0
    assert np.all(st["d2"][st["vacc"] == 2] - st["d1"][st["vacc"] == 2] >= 21)
    # immunity share among first-dose recipients 12+ days ago ~ eff1
    imm = m.immune(st, 40)
    sel = (st["vacc"] == 1) & (st["d1"] <= 40 - 12)
    share = imm[sel].mean()
    assert abs(share - 0.52) < 5 * math.sqrt(0.25 / sel.sum())
    sel2 = (st["vacc"] == 2) & (st["d2"] <= 40 - 12)
    if sel2.sum() > 100:
        assert abs(imm[sel2].mean() - 0.95) < 5 * math.sqrt(0.05 / sel2.sum())
