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
from .tables import (STAGE_S, STAGE_E, STAGE_I, STAGE_R, STAGE_M, STAGE_ASYM, STAGE_PRE_MILD,
                     STAGE_PRE_SEVERE, STAGE_MILD, STAGE_SEVERE, STAGE_HOSP, STAGE_ICU,
                     DUR_PRE, DUR_ASYM, DUR_MILD, DUR_SEV_HOSP, DUR_SEV_R, DUR_HOSP_ICU,
                     DUR_HOSP_R, DUR_ICU_DIE, DUR_ICU_R, N_DUR, CLASS_ASYM, CLASS_PRE,
                     CLASS_SYM, infectiousness_table, course_infectiousness_table,
                     poisson_thresholds, poisson_count)

NEVER = -32768
NC = 16
(C_S, C_E, C_I, C_R, C_M, C_NEW, C_TESTS, C_POS, C_DOSE1, C_DOSE2, C_EDGES, C_NEAR,
 C_INF_EDGES, C_HOSP, C_ICU, C_NOTIFIED) = range(NC)
# course path bits: 0-1 kind (0 asymptomatic, 1 mild, 2 severe), 2 hospitalised,
# 3 intensive care, 4 dies
K_ASYM, K_MILD, K_SEVERE = 0, 1, 2
B_HOSP, B_ICU, B_DIE = 4, 8, 16
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


def lambda_rows(coef, atab, code, row_ptr, col, w, lo, hi):
    """(lambda_j, sigma_j) for the destinations lo <= j < hi: sigma_j sums B_{n(e)} *
    Atab[code of e's source] over row j of the day's graph and lambda_j = coef_j *
    sigma_j (eq. 1 summed over the day's contacts of j).  Rows are independent, so a
    range of them can be computed apart from the rest."""
    e0, e1 = int(row_ptr[lo]), int(row_ptr[hi])
    rows = np.repeat(np.arange(hi - lo), np.diff(np.asarray(row_ptr[lo:hi + 1])))
    terms = np.asarray(w[e0:e1]) * atab[np.asarray(code)[np.asarray(col[e0:e1])]]
    sigma = np.bincount(rows, weights=terms, minlength=hi - lo)
    return np.asarray(coef[lo:hi]) * sigma, sigma


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
        self.eleven = int(p.get("disease_model", 0)) == 1
        if self.eleven:
            A = [float(a) for a in p["A_stage"]]
            self.Atab = np.array(course_infectiousness_table(
                float(p["gamma_shape"]), float(p["gamma_scale"]), float(p["A_asym"]),
                A[STAGE_E], A[STAGE_I]))
            self.ptab = {k: f32v(p[k]) for k in ("p_asym", "p_severe", "p_hosp", "p_icu", "p_die")}
            self.dshift = np.asarray(p["dur_shift"], np.int64)
            self.dthr = [poisson_thresholds(float(x)) for x in p["dur_extra"]]
        else:
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
        # testing and digital exposure notification (section 4)
        self.dmin = int(p["test_delay"])
        self.dmax = int(p.get("test_delay_max", self.dmin))
        self.den = f32(p.get("app_adoption", 0.0)) > 0.0
        self.window = int(p.get("den_window", 7))
        # section 5's second immunity: protected agents are infected at the usual rate and
        # their infections are asymptomatic (course model only)
        self.immune_asym = int(p.get("vacc_immunity", 0)) == 1
        if self.immune_asym and not self.eleven:
            raise ValueError("asymptomatic vaccine immunity needs the eleven-stage course")
        self.history = {}
        if self.den:
            w = philox.draw_words(int(p["seed"]), self.loc, 0, self.word, philox.PURPOSE_APP, 0)
            self.app = philox.uniform(w[0]) < f32(p["app_adoption"])
        self.delay = np.asarray(pop.dose2_delay, np.int64)

    def init_state(self):
        N = self.N
        st = dict(stage=np.zeros(N, np.int64), t_exp=np.full(N, NEVER, np.int64),
                  q_until=np.full(N, NEVER, np.int64), test_day=np.full(N, NEVER, np.int64),
                  pending=np.zeros(N, bool), positive=np.zeros(N, bool),
                  vacc=np.zeros(N, np.int64), d1=np.full(N, NEVER, np.int64),
                  d2=np.full(N, NEVER, np.int64), latch=np.zeros(self.nrep, bool),
                  course=np.zeros(N, np.int64), t_next=np.full(N, NEVER, np.int64),
                  notified=np.zeros(N, bool))
        seeds = np.asarray(self.pop.initial_infected, np.int64)
        st["t_exp"][seeds] = -1        # exposed the day before day 0: infectious from day 0
        if self.eleven:
            self.infect(st, seeds, -1)
        else:
            st["stage"][seeds] = STAGE_E
        return st

    # --- testing and exposure notification (section 4) ------------------------------
    def result_delay(self, ids, test_day):
        """Days from a test to its result: test_delay, or uniform over test_delay ..
        test_delay_max from lane 1 of AGENT2 on the test day, k = floor(x * n / 2^32)."""
        n = self.dmax - self.dmin + 1
        if n <= 1:
            return np.full(ids.size, self.dmin, np.int64)
        w = philox.draw_words(int(self.p["seed"]), self.loc[ids], test_day, self.word[ids],
                              philox.PURPOSE_AGENT2, 0)
        return self.dmin + ((w[1].astype(np.uint64) * np.uint64(n)) >> np.uint64(32)).astype(np.int64)

    def graph_of(self, d):
        if d not in self.history:
            rp, col, _, _ = build_graph(self.pop, self.p, d, self.maps)
            self.history[d] = (rp, col)
        return self.history[d]

    def notify(self, st, index, t):
        """Digital exposure notification: every contact, over the last ``window`` days'
        graphs, of an app user whose positive result arrives today, when the contact
        also uses the app and is not in quarantine (``st`` carries today's quarantine)."""
        out = np.zeros(self.N, bool)
        idx = np.flatnonzero(index)
        if idx.size == 0:
            return out
        for k in range(1, self.window + 1):
            d = t - k
            if d < 0:
                break
            rp, col = self.graph_of(d)
            lo, hi = rp[idx], rp[idx + 1]
            n = hi - lo
            if n.sum() == 0:
                continue
            pos = np.repeat(lo - np.concatenate([[0], np.cumsum(n)[:-1]]), n) + np.arange(n.sum())
            out[col[pos]] = True
        return out & self.app & (t >= st["q_until"])

    # --- eleven-stage course (section 3, "Disease Progression") ------------------
    def duration(self, ids, t, which):
        """shift + Poisson(extra) days, from lane 0 of the course's block 1 on day t."""
        w = philox.draw_words(int(self.p["seed"]), self.loc[ids], t, self.word[ids],
                              philox.PURPOSE_COURSE, 1)
        which = np.broadcast_to(np.asarray(which, np.int64), ids.shape)
        out = np.zeros(ids.size, np.int64)
        for k in range(N_DUR):
            sel = which == k
            if sel.any():
                out[sel] = self.dshift[k] + poisson_count(w[0][sel], self.dthr[k])
        return out

    def infect(self, st, ids, t, protected=None):
        """The course of agents infected on day t: asymptomatic with p_asym[a], else
        severe with p_severe[a] (mild otherwise); a severe course is hospitalised with
        p_hosp[a], and a hospitalised one reaches intensive care with p_icu[a].  Lanes
        0..3 of the course's block 0 on day t; the first stage's duration from block 1.
        ``protected`` (per id): vaccine-protected agents under asymptomatic immunity,
        whose course is asymptomatic whatever the draw (section 5)."""
        if ids.size == 0:
            return
        a = self.age[ids]
        w = philox.draw_words(int(self.p["seed"]), self.loc[ids], t, self.word[ids],
                              philox.PURPOSE_COURSE, 0)
        u = [philox.uniform(x) for x in w]
        asym = u[0] < self.ptab["p_asym"][a]
        if protected is not None:
            asym = asym | protected
        severe = ~asym & (u[1] < self.ptab["p_severe"][a])
        hosp = severe & (u[2] < self.ptab["p_hosp"][a])
        icu = hosp & (u[3] < self.ptab["p_icu"][a])
        kind = np.where(asym, K_ASYM, np.where(severe, K_SEVERE, K_MILD))
        st["course"][ids] = kind | np.where(hosp, B_HOSP, 0) | np.where(icu, B_ICU, 0)
        st["stage"][ids] = np.where(asym, STAGE_ASYM, np.where(severe, STAGE_PRE_SEVERE, STAGE_PRE_MILD))
        st["t_next"][ids] = t + self.duration(ids, t, np.where(asym, DUR_ASYM, DUR_PRE))

    def progress(self, st, new, t):
        """Transitions of day t (agents whose current stage ends today), read from st,
        written to new."""
        due = np.flatnonzero(st["t_next"] == t)
        if due.size == 0:
            return
        s, c = st["stage"][due], st["course"][due]
        to_r = (s == STAGE_ASYM) | (s == STAGE_MILD) | ((s == STAGE_SEVERE) & (c & B_HOSP == 0)) | \
            ((s == STAGE_HOSP) & (c & B_ICU == 0)) | ((s == STAGE_ICU) & (c & B_DIE == 0))
        to_m = (s == STAGE_ICU) & (c & B_DIE != 0)
        new["stage"][due[to_r]] = STAGE_R
        new["stage"][due[to_m]] = STAGE_M
        new["t_next"][due[to_r | to_m]] = NEVER
        nxt = np.full(due.size, -1, np.int64)
        stage2 = np.full(due.size, -1, np.int64)
        m = s == STAGE_PRE_MILD
        stage2[m], nxt[m] = STAGE_MILD, DUR_MILD
        m = s == STAGE_PRE_SEVERE
        stage2[m], nxt[m] = STAGE_SEVERE, np.where(c[m] & B_HOSP != 0, DUR_SEV_HOSP, DUR_SEV_R)
        m = (s == STAGE_SEVERE) & (c & B_HOSP != 0)
        stage2[m], nxt[m] = STAGE_HOSP, np.where(c[m] & B_ICU != 0, DUR_HOSP_ICU, DUR_HOSP_R)
        m = (s == STAGE_HOSP) & (c & B_ICU != 0)
        if m.any():
            # whether the stay in intensive care ends in death: lane 1 of block 1 today
            ids = due[m]
            w = philox.draw_words(int(self.p["seed"]), self.loc[ids], t, self.word[ids],
                                  philox.PURPOSE_COURSE, 1)
            die = philox.uniform(w[1]) < self.ptab["p_die"][self.age[ids]]
            new["course"][ids] = c[m] | np.where(die, B_DIE, 0)
            stage2[m], nxt[m] = STAGE_ICU, np.where(die, DUR_ICU_DIE, DUR_ICU_R)
        go = stage2 >= 0
        if go.any():
            ids = due[go]
            new["stage"][ids] = stage2[go]
            new["t_next"][ids] = t + self.duration(ids, t, nxt[go])

    def counts_of(self, st):
        """S, E, I, R, M, hospitalised, ICU per replicate.  In the eleven-stage course E
        counts the infected without symptoms (asymptomatic, presymptomatic) and I the
        symptomatic ones outside hospital."""
        g = st["stage"].copy()
        g[(g == STAGE_ASYM) | (g == STAGE_PRE_MILD) | (g == STAGE_PRE_SEVERE)] = STAGE_E
        g[(g == STAGE_MILD) | (g == STAGE_SEVERE)] = STAGE_I
        c = np.zeros((self.nrep, 7), np.int64)
        for k, s in enumerate((STAGE_S, STAGE_E, STAGE_I, STAGE_R, STAGE_M, STAGE_HOSP, STAGE_ICU)):
            c[:, k] = np.bincount(self.rep[g == s], minlength=self.nrep)
        return c

    def put_counts(self, counts, st):
        c = self.counts_of(st)
        counts[:, :5] = c[:, :5]
        counts[:, C_HOSP], counts[:, C_ICU] = c[:, 5], c[:, 6]

    # --- step pieces -------------------------------------------------------------
    def uniforms(self, t, purpose, ids=None, day=None):
        ids = np.arange(self.N) if ids is None else ids
        d = t if day is None else day
        w = philox.draw_words(int(self.p["seed"]), self.loc[ids], d, self.word[ids], purpose, 0)
        return [philox.uniform(x) for x in w]

    def codes(self, st, t):
        """Days since exposure for infectious (E, I), non-quarantined agents, else 0.
        Eleven-stage course: 16 * class + days since exposure (1..15) for asymptomatic,
        presymptomatic and symptomatic agents outside hospital, else 0."""
        tau = t - st["t_exp"]
        if self.eleven:
            s = st["stage"]
            cls = np.where(s == STAGE_ASYM, CLASS_ASYM,
                           np.where((s == STAGE_PRE_MILD) | (s == STAGE_PRE_SEVERE), CLASS_PRE,
                                    np.where((s == STAGE_MILD) | (s == STAGE_SEVERE), CLASS_SYM, 0)))
            inf = (cls > 0) & (tau >= 1) & (tau <= 15) & (t >= st["q_until"])
            return np.where(inf, 16 * cls + tau, 0)
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
                infected = prev_counts[r, C_E] + prev_counts[r, C_I] + prev_counts[r, C_HOSP] + prev_counts[r, C_ICU]
                if float(infected) >= trig * float(n):
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
        return lambda_rows(self.coef, self.Atab, code, row_ptr, col, w, 0, self.N)

    def step(self, st, t, prev_counts, graph=None):
        """Advance state(t) -> state(t+1).  Returns (new_state, out) with out holding
        lambda, p, the infection uniforms, counts[R, NC]."""
        p = self.p
        new = {k: v.copy() for k, v in st.items()}
        counts = np.zeros((self.nrep, NC), np.int64)
        # 1. pre: test results due today
        qd = int(p["quarantine_days"])
        due = np.zeros(self.N, bool)
        pend = np.flatnonzero(st["pending"])
        due[pend] = t == st["test_day"][pend] + self.result_delay(pend, st["test_day"][pend])
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
        # contacts of today's positive app users are told to test tomorrow (if they use
        # the app and, after today's results, are not in quarantine)
        new["notified"] = (self.notify({**st, "q_until": new["q_until"]}, pos_due & self.app, t)
                           if self.den else np.zeros(self.N, bool))
        counts[:, C_NOTIFIED] = np.bincount(self.rep[new["notified"]], minlength=self.nrep)
        code = self.codes({**st, "q_until": new["q_until"]}, t)
        # 2. vaccination
        d1n, d2n = self.vaccinate(new, t, prev_counts)
        counts[:, C_DOSE1], counts[:, C_DOSE2] = d1n, d2n
        immune = self.immune(new, t)
        # 3. graph, 4. lambda
        if graph is None:
            graph = build_graph(self.pop, p, t, self.maps)
        if self.den:
            self.history[t] = (graph[0], graph[1])
            for d in [d for d in self.history if d < t - self.window]:
                del self.history[d]
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
        sus = (stage == STAGE_S) & (~immune | self.immune_asym)
        inf = sus & (u0 < prob)
        counts[:, C_NEAR] = np.bincount(self.rep[sus & (np.abs(u0 - prob) <= NEAR_EPS)],
                                        minlength=self.nrep)
        new["t_exp"][inf] = t
        counts[:, C_NEW] = np.bincount(self.rep[inf], minlength=self.nrep)
        if self.eleven:
            self.progress(st, new, t)
            ids = np.flatnonzero(inf)
            self.infect(new, ids, t, immune[ids] & self.immune_asym)
        else:
            new["stage"][inf] = STAGE_E
            ed, idays = int(p["e_days"]), int(p["i_days"])
            new["stage"][(stage == STAGE_E) & (tau == ed)] = STAGE_I
            rem = (stage == STAGE_I) & (tau == ed + idays)
            dies = rem & (u1 < self.p_death[self.age])
            new["stage"][rem & ~dies] = STAGE_R
            new["stage"][dies] = STAGE_M
        # 6. testing of eligible agents (alive, not quarantined, no result pending)
        rate = f32(p["test_rate"])
        if rate > 0.0 or self.den:
            elig = (stage != STAGE_M) & (t >= new["q_until"]) & ~new["pending"]
            tested = elig & (u2 < rate)
            if self.den:
                # notified yesterday: tested today with the compliance probability
                cand = np.flatnonzero(elig & st["notified"])
                if cand.size:
                    uc = self.uniforms(t, philox.PURPOSE_AGENT2, cand)[2]
                    tested[cand[uc < f32(p["den_compliance"])]] = True
            infected = (stage != STAGE_S) & (stage != STAGE_R) & (stage != STAGE_M)
            result = tested & infected & (u3 < f32(p["test_sensitivity"]))
            new["pending"][tested] = True
            new["positive"][tested] = result[tested]
            new["test_day"][tested] = t
            counts[:, C_TESTS] = np.bincount(self.rep[tested], minlength=self.nrep)
        self.put_counts(counts, new)
        return new, dict(lam=lam, sigma=sigma, prob=prob, u0=u0, code=code, immune=immune,
                         counts=counts, graph=graph)


def run(pop, params, n_steps=None, keep=False):
    """Whole run: counts[T, R, NC] (and per-day outputs if ``keep``)."""
    m = Model(pop, params)
    st = m.init_state()
    T = int(params["n_steps"] if n_steps is None else n_steps)
    prev = np.zeros((m.nrep, NC), np.int64)
    m.put_counts(prev, st)
    traj = np.zeros((T, m.nrep, NC), np.int64)
    kept = []
    for t in range(T):
        st, out = m.step(st, t, prev)
        traj[t] = out["counts"]
        prev = out["counts"]
        if keep:
            kept.append(out)
    return traj, st, kept
