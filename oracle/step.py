"""One simulated day of DeepABM-COVID in FP64 (plain, hard-threshold method).

Follows section 3 (transmission eqs. 1-2, disease progression), section 4
(self-quarantine, testing) and section 5 (two-dose vaccination, priority orders of
Table 1, sterilising immunity), with the model instance of the workloads: SEIRM
stages with fixed durations, Gamma(2.5, 2) infectiousness.

Synchronous update: every decision of day t reads the state at the start of day t
and writes the state of day t+1.  Order inside a day:
  1. pre: due test results -> quarantine; quarantine dropout; infectiousness codes.
  2. vaccination (once the prevalence latch is set).
  3. the day's contact graph.
  4. force of infection lambda_j (eq. 1 summed over j's contacts).
  5. infection with probability 1 - exp(-lambda dt) (eq. 2 over the day's
     contacts), stage timers, death draw.
  6. testing; daily counts.

Float parameters that the library receives as FP32 (R, susceptibility, kappa, dt,
network weights, death / test / efficacy / dropout probabilities) are taken at their
FP32 value (``f32``); the table parameters (Gamma shape and scale, stage factors,
contact means) and the vaccination rate and trigger are FP64.  All arithmetic is FP64.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox
from .graph import build_graph, static_maps
from .tables import STAGE_S, STAGE_E, STAGE_I, STAGE_R, STAGE_M, infectiousness_table

NEVER = -32768
NC = 13
(C_S, C_E, C_I, C_R, C_M, C_NEW, C_TESTS, C_POS, C_DOSE1, C_DOSE2, C_EDGES, C_NEAR,
 C_INF_EDGES) = range(NC)
NEAR_EPS = 1e-6


def f32(x):
    return float(np.float32(x))


def f32v(x):
    return np.asarray(x, np.float32).astype(np.float64)


def vaccination_priority(strategy: int, dose: int, age_group):
    """Priority rank (lower = earlier) of a (dose, age group) class; section 5, Table 1.

    standard (0): second doses due first, then first doses; oldest first in each.
    delayed second dose (1): first doses first, then second doses; oldest first.
    delayed except 65+ (2): age groups 61-70 and older (the "above 65" of Table 1 on
    decade groups) by age, first dose before second within an age group; then the
    younger ones' first doses, then their second doses, oldest first."""
    a = np.asarray(age_group, np.int64)
    if strategy == 0:
        return (0 if dose == 2 else 9) + (8 - a)
    if strategy == 1:
        return (0 if dose == 1 else 9) + (8 - a)
    if strategy == 2:
        old = 2 * (8 - a) + (0 if dose == 1 else 1)
        young = 6 + (0 if dose == 1 else 6) + (5 - a)
        return np.where(a >= 6, old, young)
    raise ValueError("unknown strategy")


class Model:
    """Static data of a run: population, maps, tables, per-replicate parameters."""

    def __init__(self, pop, params):
        self.pop = pop
        self.p = dict(params)
        self.maps = static_maps(pop)
        self.N = int(pop.agent_offset[-1])
        self.rep = self.maps["rep"]
        self.loc = self.maps["local"]
        self.word = self.maps["stream"]          # Philox stream word of each agent's replicate
        self.nrep = int(pop.agent_offset.size - 1)
        self.sizes = np.diff(np.asarray(pop.agent_offset))
        p = self.p
        self.Atab = np.array(infectiousness_table(float(p["gamma_shape"]), float(p["gamma_scale"]),
                                                  int(p["e_days"]), int(p["i_days"]),
                                                  [float(a) for a in p["A_stage"]]))
        self.age = np.asarray(pop.age, np.int64)
        R = f32v(pop.R)
        S = f32v(pop.susceptibility)
        kappa = f32(p["kappa"])
        # coef_j = R * kappa * S[age_j]  (eq. 1 prefactor of the susceptible j)
        self.coef = R[self.rep] * kappa * S[self.rep, self.age]
        self.R = R
        self.S = S
        self.kappa = kappa
        self.p_death = f32v(p["p_death"])
        self.delay = np.asarray(pop.dose2_delay, np.int64)

    def init_state(self):
        N = self.N
        st = dict(stage=np.zeros(N, np.int64), t_exp=np.full(N, NEVER, np.int64),
                  q_until=np.full(N, NEVER, np.int64), test_day=np.full(N, NEVER, np.int64),
                  pending=np.zeros(N, bool), positive=np.zeros(N, bool),
                  vacc=np.zeros(N, np.int64), d1=np.full(N, NEVER, np.int64),
                  d2=np.full(N, NEVER, np.int64), latch=np.zeros(self.nrep, bool))
        seeds = np.asarray(self.pop.initial_infected, np.int64)
        st["stage"][seeds] = STAGE_E
        st["t_exp"][seeds] = -1        # exposed the day before day 0: infectious from day 0
        return st

    def counts_of(self, st):
        c = np.zeros((self.nrep, 5), np.int64)
        for s in range(5):
            c[:, s] = np.bincount(self.rep[st["stage"] == s], minlength=self.nrep)
        return c

    # --- step pieces -------------------------------------------------------------
    def uniforms(self, t, purpose, ids=None, day=None):
        ids = np.arange(self.N) if ids is None else ids
        d = t if day is None else day
        w = philox.draw_words(int(self.p["seed"]), self.loc[ids], d, self.word[ids], purpose, 0)
        return [philox.uniform(x) for x in w]

    def codes(self, st, t):
        """Days since exposure for infectious (E, I), non-quarantined agents, else 0."""
        tau = t - st["t_exp"]
        inf = ((st["stage"] == STAGE_E) | (st["stage"] == STAGE_I)) & (t >= st["q_until"])
        return np.where(inf, tau, 0)

    def immune(self, st, t):
        """Sterilising vaccine immunity on day t (section 5): one uniform per agent,
        keyed on the first-dose day, immune once lag days have passed after dose 1 if
        u < eff1, or after dose 2 if u < eff2."""
        p = self.p
        has1 = st["d1"] != NEVER
        out = np.zeros(self.N, bool)
        if not has1.any():
            return out
        ids = np.flatnonzero(has1)
        w = philox.draw_words(int(p["seed"]), self.loc[ids], st["d1"][ids], self.word[ids],
                              philox.PURPOSE_VACC, 0)
        u = philox.uniform(w[0])
        lag = int(p["dose_lag"])
        i1 = (t >= st["d1"][ids] + lag) & (u < f32(p["eff1"]))
        has2 = st["d2"][ids] != NEVER
        i2 = has2 & (t >= st["d2"][ids] + lag) & (u < f32(p["eff2"]))
        out[ids] = i1 | i2
        return out

    def vaccinate(self, st, t, prev_counts):
        """Capacity-limited, priority-ordered doses of day t (section 5)."""
        p = self.p
        d1n = np.zeros(self.nrep, np.int64)
        d2n = np.zeros(self.nrep, np.int64)
        rate = float(p["vacc_rate"])
        if rate <= 0.0:
            return d1n, d2n
        trig = float(p["vacc_trigger"])
        for r in range(self.nrep):
            n = int(self.sizes[r])
            if not st["latch"][r]:
                if float(prev_counts[r, C_E] + prev_counts[r, C_I]) >= trig * float(n):
                    st["latch"][r] = True
            if not st["latch"][r]:
                continue
            cap = int(math.floor(rate * float(n)))
            lo = int(self.pop.agent_offset[r])
            sl = slice(lo, lo + n)
            alive = st["stage"][sl] != STAGE_M
            e1 = alive & (st["vacc"][sl] == 0)
            e2 = alive & (st["vacc"][sl] == 1) & (t >= st["d1"][sl] + int(self.delay[r]))
            a = self.age[sl]
            rank = np.full(n, 1 << 30, np.int64)
            rank[e1] = vaccination_priority(int(p["strategy"]), 1, a[e1])
            rank[e2] = vaccination_priority(int(p["strategy"]), 2, a[e2])
            elig = np.flatnonzero(e1 | e2)
            order = elig[np.lexsort((elig, rank[elig]))]    # by rank, ties by agent id
            chosen = order[:cap] + lo
            c1 = chosen[st["vacc"][chosen] == 0]
            c2 = chosen[st["vacc"][chosen] == 1]
            st["vacc"][c1] = 1
            st["d1"][c1] = t
            st["vacc"][c2] = 2
            st["d2"][c2] = t
            d1n[r], d2n[r] = c1.size, c2.size
        return d1n, d2n

    def force_of_infection(self, code, graph):
        """lambda_j = R kappa S[a_j] * sum_{e in row j} B_{n(e)} * A Phi(tau_src(e))
        (eq. 1 summed over the day's contacts; non-infectious sources contribute 0)."""
        row_ptr, col, w, _ = graph
        rows = np.repeat(np.arange(self.N), np.diff(row_ptr))
        terms = w * self.Atab[code[col]]
        sigma = np.bincount(rows, weights=terms, minlength=self.N)
        return self.coef * sigma, sigma

    def step(self, st, t, prev_counts, graph=None):
        """Advance state(t) -> state(t+1).  Returns (new_state, out) with out holding
        lambda, p, the infection uniforms, counts[R, NC]."""
        p = self.p
        new = {k: v.copy() for k, v in st.items()}
        counts = np.zeros((self.nrep, NC), np.int64)
        # 1. pre: test results due today
        qd = int(p["quarantine_days"])
        due = st["pending"] & (t == st["test_day"] + int(p["test_delay"]))
        pos_due = due & st["positive"]
        counts[:, C_POS] = np.bincount(self.rep[pos_due], minlength=self.nrep)
        if qd > 0:
            new["q_until"][pos_due] = t + qd
        new["pending"][due] = False
        new["positive"][due] = False
        drop = f32(p["quarantine_dropout"])
        if drop > 0.0:
            inq = np.flatnonzero(t < new["q_until"])
            if inq.size:
                u = self.uniforms(t, philox.PURPOSE_AGENT2, inq)[0]
                new["q_until"][inq[u < drop]] = t
        code = self.codes({**st, "q_until": new["q_until"]}, t)
        # 2. vaccination
        d1n, d2n = self.vaccinate(new, t, prev_counts)
        counts[:, C_DOSE1], counts[:, C_DOSE2] = d1n, d2n
        immune = self.immune(new, t)
        # 3. graph, 4. lambda
        if graph is None:
            graph = build_graph(self.pop, p, t, self.maps)
        lam, sigma = self.force_of_infection(code, graph)
        counts[:, C_EDGES] = np.bincount(self.rep, weights=np.diff(graph[0]),
                                         minlength=self.nrep).astype(np.int64)
        rows = np.repeat(np.arange(self.N), np.diff(graph[0]))
        counts[:, C_INF_EDGES] = np.bincount(self.rep[rows[code[graph[1]] != 0]],
                                             minlength=self.nrep)
        # 5. infection and progression
        u0, u1, u2, u3 = self.uniforms(t, philox.PURPOSE_AGENT)
        prob = -np.expm1(-lam * f32(p["dt"]))
        stage, tau = st["stage"], t - st["t_exp"]
        sus = (stage == STAGE_S) & ~immune
        inf = sus & (u0 < prob)
        counts[:, C_NEAR] = np.bincount(self.rep[sus & (np.abs(u0 - prob) <= NEAR_EPS)],
                                        minlength=self.nrep)
        new["stage"][inf] = STAGE_E
        new["t_exp"][inf] = t
        counts[:, C_NEW] = np.bincount(self.rep[inf], minlength=self.nrep)
        ed, idays = int(p["e_days"]), int(p["i_days"])
        new["stage"][(stage == STAGE_E) & (tau == ed)] = STAGE_I
        rem = (stage == STAGE_I) & (tau == ed + idays)
        dies = rem & (u1 < self.p_death[self.age])
        new["stage"][rem & ~dies] = STAGE_R
        new["stage"][dies] = STAGE_M
        # 6. testing of eligible agents (alive, not quarantined, no result pending)
        rate = f32(p["test_rate"])
        if rate > 0.0:
            elig = (stage != STAGE_M) & (t >= new["q_until"]) & ~new["pending"]
            tested = elig & (u2 < rate)
            result = tested & ((stage == STAGE_E) | (stage == STAGE_I)) & (u3 < f32(p["test_sensitivity"]))
            new["pending"][tested] = True
            new["positive"][tested] = result[tested]
            new["test_day"][tested] = t
            counts[:, C_TESTS] = np.bincount(self.rep[tested], minlength=self.nrep)
        counts[:, :5] = self.counts_of(new)
        return new, dict(lam=lam, sigma=sigma, prob=prob, u0=u0, code=code, immune=immune,
                         counts=counts, graph=graph)


def run(pop, params, n_steps=None, keep=False):
    """Whole run: counts[T, R, NC] (and per-day outputs if ``keep``)."""
    m = Model(pop, params)
    st = m.init_state()
    T = int(params["n_steps"] if n_steps is None else n_steps)
    prev = np.zeros((m.nrep, NC), np.int64)
    prev[:, :5] = m.counts_of(st)
    traj = np.zeros((T, m.nrep, NC), np.int64)
    kept = []
    for t in range(T):
        st, out = m.step(st, t, prev)
        traj[t] = out["counts"]
        prev = out["counts"]
        if keep:
            kept.append(out)
    return traj, st, kept
