"""An exact distributional pin of the day step: a homogeneous random network.

No households or workplaces, every S_a = 1, no interventions.  Each agent draws
Poisson(mu/2) partners uniform over the others and every draw gives both directed edges,
so the number of edges between two agents on a day is Poisson(mu/(N-1)), independently
over pairs (Poisson splitting).  An infector at tau days since exposure contributes
coef * w * Atab[tau] per edge to a susceptible's force of infection (eq. 1), and a
susceptible is infected with probability 1 - exp(-lambda) (eq. 2).  Averaging over the
day's edges, each susceptible is therefore infected independently with probability

    p(t) = 1 - exp(-G(t) / (N - 1)),   G(t) = sum over infectors of mu (1 - exp(-coef w Atab[tau])),

so the day's incidence given the epidemic's history is exactly Binomial(S(t), p(t)).
The infectors by tau follow from the incidence history itself (every exposed agent is
infectious for tau = 1..15 and seeds have tau = t + 1), so a run's own trajectory fixes
every p(t), and the standardised residuals must be standard normal.  The oracle is held
to this on the CPU at 20,000 agents, the GPU at 2 million agents by 16 replicates."""
import dataclasses

import numpy as np
import pytest

from helpers import require_gpu
from oracle import step as ostep
from oracle.tables import infectiousness_table
from synthpop import make_population, replicate_population
from synthpop.configs import params_for
from synthpop.population import N_AGE, N_OCC

MU, W, R0 = 10.0, 0.2, 5.18


def _setup(N, reps, seeds, T):
    p = params_for(0, n_steps=T, kappa=1.0, mu_random=[MU] * N_AGE, mu_occupation=[0.0] * N_OCC,
                   w_occupation=0.0, w_random=W)
    base = make_population([N], workplaces=False, n_seeds=seeds, R=R0, susceptibility=np.ones(N_AGE))
    base = dataclasses.replace(base, hh_start=np.arange(N + 1, dtype=np.int32))   # single-agent households
    return p, replicate_population(base, reps)          # independent Philox streams


def _offspring(p):
    """g(tau) = mu (1 - exp(-coef w Atab[tau])): expected daily infections caused by one
    infector at tau days since exposure in a fully susceptible population."""
    coef = float(np.float32(np.float32(R0 * 1.0) * np.float32(1.0)))
    atab = np.array(infectiousness_table(p["gamma_shape"], p["gamma_scale"], p["e_days"],
                                         p["i_days"], p["A_stage"]), np.float64)
    return MU * (1.0 - np.exp(-coef * W * atab))


def _residuals(inc, S_end, N, seeds, p, min_var):
    """Standardised residuals of the incidence [T, reps] against Binomial(S(t), p(t))."""
    T, reps = inc.shape
    S_start = np.vstack([np.full((1, reps), N - seeds, np.float64), S_end[:-1]])
    g = _offspring(p)
    assert g[0] == 0.0 and np.all(g[16:] == 0.0) and np.all(g[1:16] > 0.0)
    G = np.zeros((T, reps))
    for t in range(T):
        G[t] += seeds * g[t + 1]
        for tau in range(1, min(t, 15) + 1):
            G[t] += inc[t - tau] * g[tau]
    prob = -np.expm1(-G / (N - 1))
    mean, var = S_start * prob, S_start * prob * (1.0 - prob)
    z_all = (inc - mean).sum() / np.sqrt(var.sum())
    z_rep = (inc - mean).sum(0) / np.sqrt(var.sum(0))
    days = var.sum(1) >= min_var          # the normal approximation needs some variance
    z_day = (inc - mean)[days].sum(1) / np.sqrt(var[days].sum(1))
    cell = var >= min_var
    chi2 = (((inc - mean) ** 2)[cell] / var[cell]).sum()
    print(f"z overall {z_all:.2f}; max |z| over {days.sum()} days {np.abs(z_day).max():.2f}, "
          f"over replicates {np.abs(z_rep).max():.2f}; chi-square {chi2:.1f} over {cell.sum()} cells")
    return z_all, z_rep, z_day, chi2, int(cell.sum())


def _assert_binomial(res, min_days, min_cells):
    z_all, z_rep, z_day, chi2, dof = res
    assert z_day.size >= min_days and dof >= min_cells
    assert abs(z_all) < 5.0
    assert np.abs(z_day).max() < 5.0
    assert np.abs(z_rep).max() < 5.0
    assert abs(chi2 - dof) < 6.0 * np.sqrt(2.0 * dof), (chi2, dof)   # binomial dispersion


def test_oracle_homogeneous_incidence_is_binomial_given_history():
    N, REPS, SEEDS, T = 20_000, 4, 20, 30
    p, pop = _setup(N, REPS, SEEDS, T)
    traj, _, _ = ostep.run(pop, p)
    inc = traj[:, :, ostep.C_NEW].astype(np.float64)
    assert inc.sum(0).min() > 0.9 * N
    _assert_binomial(_residuals(inc, traj[:, :, ostep.C_S].astype(np.float64), N, SEEDS, p, 5.0),
                     min_days=15, min_cells=40)


@pytest.mark.gpu
def test_gpu_homogeneous_incidence_is_binomial_given_history():
    require_gpu()
    from paper_2110_04421_amd.sim import Simulator
    from paper_2110_04421_amd import _lib as L
    N, REPS, SEEDS, T = 2_000_000, 16, 200, 32
    p, pop = _setup(N, REPS, SEEDS, T)
    with Simulator(p, pop) as s:
        counts = s.run(T)                       # [T, REPS, NC]
    inc = counts[:, :, L.C_NEW].astype(np.float64)
    # the epidemic must take off and deplete, so the pin covers growth and saturation
    assert inc.sum(0).min() > 0.9 * N and inc[0].mean() > 20
    _assert_binomial(_residuals(inc, counts[:, :, L.C_S].astype(np.float64), N, SEEDS, p, 10.0),
                     min_days=25, min_cells=300)
    # early growth rate: r = ln rho, rho the root of sum_tau g(tau) rho^-tau = 1 (discrete
    # Euler-Lotka for the renewal J(t) = sum_tau g(tau) J(t - tau)); the slope of the
    # log mean incidence over days 2..7, while under about 1 % of N is infected, is r
    g = _offspring(p)
    lo, hi = 1.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if (g[1:16] * mid ** -np.arange(1.0, 16.0)).sum() > 1.0 else (lo, mid)
    r = np.log(lo)
    days = np.arange(2, 8)
    assert inc[:8].sum(0).max() < 0.012 * N
    slope = np.polyfit(days, np.log(inc[days].mean(1)), 1)[0]
    print(f"growth rate {slope:.4f}/day against r = {r:.4f}")
    assert abs(slope / r - 1.0) < 0.03
