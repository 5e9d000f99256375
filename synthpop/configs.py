"""Parameter sets of the five workloads (plain small, plain at paper scale, plain at
50M agents, batched ensemble, differentiable calibration).

Every value is a model parameter, not code: the oracle and the GPU library each take
this flat dict and compute on their own.  Readings of the paper that fix a value are
noted beside it (section 3, eqs. 1-2; section 4; section 5).
"""
from __future__ import annotations

import copy

import numpy as np

from .population import make_population, replicate_population, N_AGE, N_OCC

MODE_HARD, MODE_SOFT = 0, 1
STRAT_STANDARD, STRAT_DELAYED, STRAT_DELAYED_EXCEPT_65 = 0, 1, 2

BASE = dict(
    seed=0,                     # Philox key = (seed & 0xffffffff, seed >> 32)
    dt=1.0,                     # one step is one day
    kappa=1.0 / 11.0,           # 1 / I-bar of eq. 1 (nominal mean daily in-degree)
    gamma_shape=2.5, gamma_scale=2.0,    # infectiousness profile (mean 5 d, var 10 d^2)
    A_stage=[0.0, 1.0, 1.0, 0.0, 0.0],   # per-stage factor for S, E, I, R, M infectors
    w_household=1.0, w_occupation=0.2, w_random=0.2,   # network factor B_n
    mu_random=[4.84] * N_AGE,            # mean daily random in-degree per age group
    mu_occupation=[4.0] * N_OCC,         # mean daily workplace in-degree per occupation
    p_death=[0.05 * a / 8.0 for a in range(N_AGE)],
    e_days=5, i_days=10,
    quarantine_days=0, test_delay=2, quarantine_dropout=0.0,
    test_rate=0.0, test_sensitivity=0.95,
    test_delay_max=2,                    # result after test_delay .. test_delay_max days (uniform)
    app_adoption=0.0,                    # digital exposure notification: app users' share (0 = off)
    den_compliance=0.8,                  # notified app users who test the next day
    den_window=7,                        # days of contacts a positive result notifies
    vacc_immunity=0,                     # 0 sterilising, 1 asymptomatic infections (course)
    vacc_rate=0.0, vacc_trigger=0.01, eff1=0.52, eff2=0.95, dose_lag=12,
    strategy=STRAT_STANDARD,
    mode=MODE_HARD, gumbel_tau=0.5, checkpoint_every=10,
    # eleven-stage course (disease_model 1; section 3 names the stages, the values are
    # readings): per age group 0-10 .. 80+, the share of infections that stay
    # asymptomatic, of symptomatic ones that turn severe, of severe ones hospitalised,
    # of hospitalised ones in intensive care, and of those in intensive care who die
    disease_model=0,
    p_asym=[0.45, 0.45, 0.40, 0.35, 0.30, 0.25, 0.20, 0.20, 0.20],
    p_severe=[0.01, 0.02, 0.05, 0.08, 0.12, 0.18, 0.28, 0.40, 0.50],
    p_hosp=[0.30, 0.30, 0.35, 0.40, 0.45, 0.50, 0.60, 0.70, 0.80],
    p_icu=[0.05, 0.05, 0.08, 0.10, 0.15, 0.20, 0.25, 0.30, 0.30],
    p_die=[0.10, 0.10, 0.15, 0.20, 0.30, 0.40, 0.50, 0.60, 0.70],
    A_asym=0.5,                          # asymptomatic infectiousness (A_E, A_I as above)
    # stage durations = shift + Poisson(extra) days (means 5, 10, 8, 6, 12, 3, 10, 8, 12):
    # presymptomatic, asymptomatic, mild, severe -> hospital, severe -> recovered,
    # hospital -> ICU, hospital -> recovered, ICU -> death, ICU -> recovered
    dur_shift=[1] * 9,
    dur_extra=[4.0, 9.0, 7.0, 5.0, 11.0, 2.0, 9.0, 7.0, 11.0],
    n_steps=180,
    edge_capacity=0,
)

# the three test types of section 4 (accuracy read as sensitivity; turnaround in days)
TEST_TYPES = {"rt_pcr": dict(test_sensitivity=0.95, test_delay=3, test_delay_max=5),
              "antigen": dict(test_sensitivity=0.65, test_delay=2, test_delay_max=2),
              "point_of_care": dict(test_sensitivity=0.85, test_delay=1, test_delay_max=1)}

INTERVENTIONS = dict(quarantine_days=14, test_delay=2, test_rate=0.05, test_sensitivity=0.95,
                     vacc_rate=0.005, vacc_trigger=0.01, eff1=0.52, eff2=0.95, dose_lag=12)

WORKLOADS = {
    0: dict(name="plain-1k", n=1000, workplaces=False, n_seeds=10, T=30,
            params=dict(kappa=1.0 / 12.16, mu_random=[10.0] * N_AGE,
                        mu_occupation=[0.0] * N_OCC, w_occupation=0.0)),
    1: dict(name="plain-100k", n=100_000, workplaces=True, n_seeds=10, T=180,
            params=dict(INTERVENTIONS, kappa=1.0 / 11.0)),
    2: dict(name="plain-50M", n=50_000_000, workplaces=True, n_seeds=5000, T=180,
            params=dict(INTERVENTIONS, kappa=1.0 / 20.0, mu_random=[13.84] * N_AGE)),
    3: dict(name="batched-256", n=None, workplaces=True, n_seeds=10, T=180,
            params=dict(INTERVENTIONS, kappa=1.0 / 11.0)),
    4: dict(name="calib-100k", n=100_000, workplaces=True, n_seeds=10, T=180,
            params=dict(kappa=1.0 / 11.0, mode=MODE_SOFT, gumbel_tau=0.5,
                        checkpoint_every=10)),
}


def params_for(k: int, **overrides) -> dict:
    p = copy.deepcopy(BASE)
    p.update(copy.deepcopy(WORKLOADS[k]["params"]))
    p["n_steps"] = WORKLOADS[k]["T"]
    p.update(overrides)
    return p


def ensemble_draws(n_rep: int = 256, seed: int = 3000):
    """Per-replicate sizes (log-uniform 1e4..5e5), R ~ U[3,7], dose-2 delay in
    {21, 42, 84} for the batched ensemble."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 3])))
    sizes = np.rint(np.exp(rng.uniform(np.log(1e4), np.log(5e5), size=n_rep))).astype(np.int64)
    R = rng.uniform(3.0, 7.0, size=n_rep).astype(np.float32)
    delay = rng.choice(np.array([21, 42, 84], np.int32), size=n_rep)
    return sizes, R, delay


def workload(k: int, n: int | None = None, n_rep: int | None = None, pop_seed: int | None = None,
             **overrides):
    """(params, population) of workload ``k``; ``n`` shrinks the population (tests)."""
    w = WORKLOADS[k]
    p = params_for(k, **overrides)
    ps = 1000 + k if pop_seed is None else pop_seed
    if k == 3:
        nr = 256 if n_rep is None else n_rep
        sizes, R, delay = ensemble_draws(nr)
        if n is not None:      # shrink every replicate proportionally (tests)
            sizes = np.maximum(64, (sizes * (n / sizes.sum())).astype(np.int64))
        pop = make_population(sizes, workplaces=True, n_seeds=w["n_seeds"], pop_seed=ps,
                              seed_seed=2000 + k, R=R, dose2_delay=delay)
        return p, pop
    N = w["n"] if n is None else n
    pop = make_population([N], workplaces=w["workplaces"], n_seeds=w["n_seeds"],
                          pop_seed=ps, seed_seed=2000 + k)
    if n_rep:
        pop = replicate_population(pop, n_rep)
    return p, pop
