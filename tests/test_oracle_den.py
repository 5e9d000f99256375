"""The oracle's digital exposure notification and test turnaround (section 4), pinned:
the notified set of each day equals the one found from the drawn contact lists and the
households directly (not from the day graphs the oracle keeps); app access and result
delays follow their laws."""
import numpy as np
from scipy import stats

from oracle import graph as og
from oracle import step as ostep
from synthpop import workload


def _den_params(**kw):
    p, pop = workload(1, n=4000, n_steps=30, test_rate=0.08, app_adoption=0.6, den_compliance=0.9,
                      den_window=5, test_delay=1, test_delay_max=3, **kw)
    return p, pop


def test_notified_sets_match_contacts_from_the_draw_lists():
    p, pop = _den_params()
    m = ostep.Model(pop, p)
    st = m.init_state()
    prev = np.zeros((m.nrep, ostep.NC), np.int64)
    m.put_counts(prev, st)
    maps = og.static_maps(pop)
    contacts = {}                              # day -> set of undirected pairs
    total = 0
    for t in range(26):
        dr = og.daily_draws(pop, p, t, maps)
        pairs = set()
        for net in ("occ", "rand"):
            for i, j in zip(dr[net]["init"].tolist(), dr[net]["partner"].tolist()):
                pairs.add((i, j))
                pairs.add((j, i))
        contacts[t] = pairs
        # index cases of day t: positive results that arrive today, app users
        pend = np.flatnonzero(st["pending"])
        due = np.zeros(m.N, bool)
        due[pend] = t == st["test_day"][pend] + m.result_delay(pend, st["test_day"][pend])
        index = set(np.flatnonzero(due & st["positive"] & m.app).tolist())
        expect = np.zeros(m.N, bool)
        for d in range(max(0, t - 5), t):
            for i, j in contacts[d]:
                if i in index:
                    expect[j] = True
        if t > 0:                              # household members: contacts every day
            for i in index:
                for k in range(int(maps["hh_lo"][i]), int(maps["hh_hi"][i])):
                    if k != i:
                        expect[k] = True
        new, out = m.step(st, t, prev)
        expect &= m.app & (t >= new["q_until"])
        assert np.array_equal(new["notified"], expect), (t, np.flatnonzero(new["notified"] ^ expect)[:10])
        assert out["counts"][0, ostep.C_NOTIFIED] == expect.sum()
        total += int(expect.sum())
        st, prev = new, out["counts"]
    assert total > 20


def test_app_access_and_result_delays_follow_their_laws():
    p, pop = workload(1, n=200000, n_steps=5, app_adoption=0.3, test_delay=3, test_delay_max=5)
    m = ostep.Model(pop, p)
    n = m.app.sum()
    z = (n - 0.3 * m.N) / np.sqrt(m.N * 0.3 * 0.7)
    assert abs(z) < 5
    d = m.result_delay(np.arange(m.N), 11)
    obs = np.bincount(d - 3, minlength=3)
    assert d.min() == 3 and d.max() == 5
    assert stats.chisquare(obs).pvalue > 1e-3


def test_notification_leads_to_tests_the_next_day():
    p, pop = workload(1, n=20000, n_steps=40, test_rate=0.05, app_adoption=1.0, den_compliance=1.0,
                      den_window=7)
    traj, st, _ = ostep.run(pop, p)
    c = traj[:, 0, :]
    assert c[:, ostep.C_NOTIFIED].sum() > 100
    p0 = dict(p, app_adoption=0.0)
    traj0, _, _ = ostep.run(pop, p0)
    # with every contact told to test, more tests are taken than without notification
    assert traj[:, 0, ostep.C_TESTS].sum() > traj0[:, 0, ostep.C_TESTS].sum()
    assert np.all(traj0[:, 0, ostep.C_NOTIFIED] == 0)
