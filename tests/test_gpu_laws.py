"""Distribution-level pins of the GPU day step, independent of the oracle.

Households of 8 with no other contacts: an infector at tau = 1 (a seed), one at tau = 8
and six susceptibles of distinct age groups.  Each susceptible's force of infection is
fixed, lambda_j = coef[a_j] (Atab[1] + Atab[8]) (eq. 1), and the six are infected
independently with p_j = 1 - exp(-lambda_j) (eq. 2), so the 64 outcome patterns of a
household follow the product law exactly.  A million households exercise the
infection draw of eight million agents against that law."""
import dataclasses

import numpy as np
import pytest
from scipy import stats

from helpers import require_gpu
from oracle.tables import phi
from synthpop import workload, make_population

pytestmark = pytest.mark.gpu


def test_infection_outcome_patterns_follow_the_product_law():
    require_gpu()
    from paper_2110_04421_amd.sim import Simulator
    from paper_2110_04421_amd import _lib as L
    H = 1_000_000
    ages = np.array([0, 0, 1, 3, 4, 6, 7, 8], np.uint8)
    pop = make_population([8 * H], workplaces=False, n_seeds=0, pop_seed=77)
    base = np.arange(H, dtype=np.int64) * 8
    pop = dataclasses.replace(pop, hh_start=(np.arange(H + 1) * 8).astype(np.int32),
                              age=np.tile(ages, H), initial_infected=base.astype(np.int32),
                              init_offset=np.array([0, H], np.int64))
    params = dict(workload(0)[0], mu_random=[0.0] * 9, kappa=1.0, n_steps=2)
    with Simulator(params, pop) as s:
        rec = s.state()
        assert np.all(rec["stage"][base] == 1) and np.all(rec["t_exp"][base] == -1)
        rec["stage"][base + 1] = 2                  # infectious stage, tau 8 on day 0
        rec["t_exp"][base + 1] = -8
        s.set_state(0, s.latch(), rec)
        counts = s.run(1)
        after = s.state()
    inf = after["stage"].reshape(H, 8)[:, 2:] == 1
    assert np.all(after["t_exp"].reshape(H, 8)[:, 2:][inf] == 0)
    assert counts[0, 0, L.C_NEW] == inf.sum()
    pat = (inf * (1 << np.arange(6))).sum(1)
    obs = np.bincount(pat, minlength=64)
    R = float(np.float32(5.18))
    S = np.linspace(0.35, 1.47, 9).astype(np.float32).astype(float)
    lam = R * S[ages[2:]] * (phi(1, 2.5, 2.0) + phi(8, 2.5, 2.0))
    p = -np.expm1(-lam)
    # marginals first: each member's infection rate within 5 sigma of p_j
    z = (inf.sum(0) - H * p) / np.sqrt(H * p * (1 - p))
    assert np.all(np.abs(z) < 5.0), z
    probs = np.array([np.prod([p[i] if (y >> i) & 1 else 1 - p[i] for i in range(6)])
                      for y in range(64)])
    e = probs * H
    assert e.min() > 50
    chi2 = ((obs - e) ** 2 / e).sum()
    pv = stats.chi2.sf(chi2, 63)
    print(f"chi-square {chi2:.1f} on 63 dof (p = {pv:.3g}); marginal z {np.round(z, 2)}")
    assert pv > 1e-3
