"""Pins of the oracle's random numbers and tables against things other than itself:
published known-answer vectors, numpy's own Philox, closed forms, scipy."""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special, stats

from conftest import GOLDEN
from oracle import philox
from oracle.tables import gamma_p, phi, infectiousness_table, poisson_thresholds, poisson_count


def _kat():
    rows = []
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[:4], w[4:6], w[6:10]))
    return rows


def test_philox4x32_known_answers_generic_and_vectorised():
    for ctr, key, out in _kat():
        assert list(philox.philox4_generic(ctr, key, 32, philox.M4x32, philox.W4x32)) == out
        seed = key[0] | (key[1] << 32)
        v = philox.philox4x32(*ctr, seed)
        assert [int(x) for x in v] == out


def test_generic_round_matches_numpy_philox4x64():
    # numpy's Philox is 4x64-10 and increments its counter before each block
    bg = np.random.Philox(key=np.array([7, 9], np.uint64), counter=np.zeros(4, np.uint64))
    raw = [int(x) for x in bg.random_raw(12)]
    mine = []
    for c in (1, 2, 3):
        mine += list(philox.philox4_generic((c, 0, 0, 0), (7, 9), 64, philox.M4x64, philox.W4x64))
    assert mine == raw


def test_vectorised_equals_generic_on_random_counters():
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2**32, size=(4, 200), dtype=np.uint64)
    seed = 0x1234567890ABCDEF
    v = philox.philox4x32(*ctr, seed)
    for j in range(200):
        g = philox.philox4_generic([int(c[j]) for c in ctr], (seed & 0xFFFFFFFF, seed >> 32),
                                   32, philox.M4x32, philox.W4x32)
        assert tuple(int(x[j]) for x in v) == g


def test_uniform_mapping_exact_and_open_interval():
    x = np.array([0, 1, 511, 512, 2**31, 2**32 - 1], np.uint64)
    u = philox.uniform(x)
    assert u.min() > 0 and u.max() < 1
    assert np.all(u.astype(np.float32).astype(np.float64) == u)     # exact in FP32
    assert u[0] == 2.0 ** -24 and u[-1] == 1 - 2.0 ** -24
    k = u * 2**24
    assert np.all(k == np.floor(k)) and np.all(k % 2 == 1)


def test_lanes_uniform_chi2():
    n = 200_000
    for lane in range(4):
        w = philox.draw_words(0, np.arange(n), 3, 1, philox.PURPOSE_AGENT, 0)[lane]
        h = np.bincount((philox.uniform(w) * 64).astype(np.int64), minlength=64)
        chi2 = ((h - n / 64) ** 2 / (n / 64)).sum()
        assert stats.chi2.sf(chi2, 63) > 1e-4


def _p25_closed(x):
    # P(5/2, x) = erf(sqrt x) - (2/sqrt(pi)) e^-x (sqrt x + (2/3) x^(3/2))
    return math.erf(math.sqrt(x)) - 2 / math.sqrt(math.pi) * math.exp(-x) * (
        math.sqrt(x) + 2.0 / 3.0 * x ** 1.5)


def test_gamma_p_closed_form_scipy_and_quadrature():
    for x in [0.1, 0.5, 1.0, 2.5, 4.0, 7.5, 12.0]:
        assert abs(gamma_p(2.5, x) - _p25_closed(x)) < 1e-14
        assert abs(gamma_p(2.5, x) - special.gammainc(2.5, x)) < 1e-14
    for a in (1.0, 2.0, 3.7):
        for x in (0.3, 2.0, 9.0):
            assert abs(gamma_p(a, x) - special.gammainc(a, x)) < 1e-13
    # shape 1 is the exponential law: P(1, x) = 1 - e^-x
    assert abs(gamma_p(1.0, 0.7) - (1 - math.exp(-0.7))) < 1e-15


def test_phi_daily_integral():
    pdf = lambda u: stats.gamma.pdf(u, 2.5, scale=2.0)
    vals = [phi(t, 2.5, 2.0) for t in range(16)]
    assert vals[0] == 0.0
    for t in range(1, 16):
        q = integrate.quad(pdf, t - 1, t, epsabs=1e-14, epsrel=1e-13)[0]
        assert abs(vals[t] - q) < 1e-11
        assert abs(vals[t] - (_p25_closed(t / 2) - _p25_closed((t - 1) / 2))) < 1e-14
    # mass over the 15 infectious days = P(2.5, 7.5); peak on day 4 (mean 5, mode 3)
    assert abs(sum(vals) - _p25_closed(7.5)) < 1e-14
    assert int(np.argmax(vals)) == 4
    assert abs(vals[1] - 0.0374342267527037) < 1e-15


def test_infectiousness_table_stage_factors():
    A = [0.0, 0.5, 1.0, 0.0, 0.0]
    tab = infectiousness_table(2.5, 2.0, 5, 10, A)
    assert tab[0] == 0.0 and all(v == 0.0 for v in tab[16:])
    for t in range(1, 6):
        assert tab[t] == 0.5 * phi(t, 2.5, 2.0)
    for t in range(6, 16):
        assert tab[t] == phi(t, 2.5, 2.0)


@pytest.mark.parametrize("mu", [0.0, 0.5, 2.0, 2.42, 5.0, 6.92])
def test_poisson_thresholds_match_scipy_cdf(mu):
    T = poisson_thresholds(mu)
    cdf = stats.poisson.cdf(np.arange(64), mu)
    ref = np.minimum(np.floor(cdf * 2.0**32), 2.0**32 - 1)
    assert np.all(np.abs(np.array(T, np.float64) - ref) <= 2)
    assert all(T[i] <= T[i + 1] for i in range(63))


def test_poisson_sampling_chi2():
    mu = 2.42
    T = poisson_thresholds(mu)
    w = philox.draw_words(0, np.arange(400_000), 1, 0, philox.PURPOSE_RAND, 0)[0]
    k = poisson_count(w, T)
    h = np.bincount(k, minlength=12)[:12].astype(np.float64)
    h[11] += (k >= 12).sum()
    p = stats.poisson.pmf(np.arange(12), mu)
    p[11] = stats.poisson.sf(10, mu)
    e = p * k.size
    assert stats.chi2.sf(((h - e) ** 2 / e).sum(), 11) > 1e-4
    assert abs(k.mean() - mu) < 5 * math.sqrt(mu / k.size)
