"""Per-run tables of the oracle, in FP64 (Python floats).

* ``gamma_p``  -- regularised lower incomplete gamma P(a, x) by its power series.
* ``phi``      -- the daily infectiousness integral of eq. 1 (section 3, "Infection
  Transmission"): the Gamma density integrated over the day [tau-1, tau] since
  infection, with shape/scale from the workload (2.5, 2).
* ``infectiousness_table`` -- A(stage(tau)) * Phi(tau) per day since exposure.
* ``poisson_thresholds``   -- integer thresholds turning one 32-bit word into a
  Poisson count (inverse-CDF sampling).
"""
from __future__ import annotations

import math

STAGE_S, STAGE_E, STAGE_I, STAGE_R, STAGE_M = 0, 1, 2, 3, 4
# eleven-stage course (section 3, "Agent State Definition"): the paper's susceptible,
# recovered and dead are S, R, M above; its "vaccinated" is a susceptible agent with
# vaccine immunity
(STAGE_ASYM, STAGE_PRE_MILD, STAGE_PRE_SEVERE, STAGE_MILD, STAGE_SEVERE, STAGE_HOSP,
 STAGE_ICU) = 5, 6, 7, 8, 9, 10, 11
# stage durations of the course, in this order: presymptomatic, asymptomatic -> R,
# mild -> R, severe -> hospital, severe -> R, hospital -> ICU, hospital -> R,
# ICU -> death, ICU -> R
(DUR_PRE, DUR_ASYM, DUR_MILD, DUR_SEV_HOSP, DUR_SEV_R, DUR_HOSP_ICU, DUR_HOSP_R,
 DUR_ICU_DIE, DUR_ICU_R) = range(9)
N_DUR = 9
# infectiousness classes of the course: code = 16 * class + days since exposure
CLASS_ASYM, CLASS_PRE, CLASS_SYM = 1, 2, 3


def gamma_p(a: float, x: float) -> float:
    """P(a, x) = x^a e^-x sum_{n>=0} x^n / Gamma(a + n + 1)  (series definition)."""
    if x <= 0.0:
        return 0.0
    # term_n = x^(a+n) e^-x / Gamma(a+n+1), summed until negligible
    log_t = a * math.log(x) - x - math.lgamma(a + 1.0)
    t = math.exp(log_t)
    s = t
    n = 0
    while True:
        n += 1
        t *= x / (a + n)
        s += t
        if t < 1e-18 * s and n > x:
            break
        if n > 10000:
            raise RuntimeError("gamma_p series did not converge")
    return min(s, 1.0)


def phi(tau: int, shape: float, scale: float) -> float:
    """Integral of the Gamma(shape, scale) density over [tau-1, tau] (eq. 1 with t the
    time since infection, in days).  Phi(0) = 0: no transmission on the day of exposure."""
    if tau <= 0:
        return 0.0
    return gamma_p(shape, tau / scale) - gamma_p(shape, (tau - 1) / scale)


def infectiousness_table(shape: float, scale: float, e_days: int, i_days: int,
                         A_stage, size: int = 64):
    """Atab[tau] = A_{stage(tau)} * Phi(tau): stage E for 1 <= tau <= e_days, I for
    e_days < tau <= e_days + i_days, not infectious otherwise (eq. 1's A_{s_i} factor
    applied per stage; removal at tau = e_days + i_days)."""
    tab = [0.0] * size
    for tau in range(1, e_days + i_days + 1):
        st = STAGE_E if tau <= e_days else STAGE_I
        tab[tau] = float(A_stage[st]) * phi(tau, shape, scale)
    return tab


def course_infectiousness_table(shape: float, scale: float, A_asym: float, A_pre: float,
                                A_sym: float, size: int = 64):
    """Eleven-stage course: Atab[16 c + tau] = A_c * Phi(tau) for the infectious classes
    c (asymptomatic, presymptomatic, symptomatic) and 1 <= tau <= 15 (eq. 1's A_{s_i}
    per stage class); hospitalised and ICU agents are isolated and infect nobody."""
    tab = [0.0] * size
    for c, A in ((CLASS_ASYM, A_asym), (CLASS_PRE, A_pre), (CLASS_SYM, A_sym)):
        for tau in range(1, 16):
            tab[16 * c + tau] = float(A) * phi(tau, shape, scale)
    return tab


def poisson_thresholds(mu_half: float, n: int = 64):
    """T_k = min(floor(F_k * 2^32), 2^32 - 1), F_k the Poisson(mu_half) CDF summed left
    to right from pmf_0 = exp(-m), pmf_k = pmf_{k-1} * m / k.  A word x maps to the
    count k = #{k < n-1 : T_k <= x} (inverse-CDF sampling, capped at n-1)."""
    pmf = math.exp(-mu_half)
    F = pmf
    out = []
    for k in range(n):
        if k:
            pmf = pmf * mu_half / k
            F = F + pmf
        out.append(min(int(math.floor(F * 4294967296.0)), 4294967295))
    return out


def poisson_count(word, thresholds):
    """Count for a uint32 word (vectorised): number of thresholds T_0..T_{n-2} <= x."""
    import numpy as np
    T = np.asarray(thresholds[:-1], np.uint64)
    x = np.asarray(word, np.uint64)
    return (x[..., None] >= T).sum(axis=-1).astype(np.int64)
