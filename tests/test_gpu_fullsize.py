"""Full-size check at 50 million agents in the configuration the benchmark times
(partitioned builder, autotuned tiling): sampled rows of day 0's contact graph and
their force of infection, computed one by one by the oracle, against the GPU, plus
properties that hold at any size."""
import numpy as np
import pytest

from helpers import require_gpu, lam_close
from oracle import graph as og
from oracle import step as ostep
from synthpop import workload

pytestmark = pytest.mark.gpu


def _oracle_rows(pop, p, t, sample, maps):
    """Canonical rows of the sampled destinations: household members, own draws, and
    the draws of every initiator whose partner is a sampled agent (scanned in chunks)."""
    N = pop.n_agents
    want = np.zeros(N, bool)
    want[sample] = True
    own = og.daily_draws(pop, p, t, maps, agents=sample)
    recv = {"occ": [], "rand": []}
    step = 4_000_000
    for a0 in range(0, N, step):
        dr = og.daily_draws(pop, p, t, maps, agents=np.arange(a0, min(N, a0 + step)))
        for net in ("occ", "rand"):
            hit = want[dr[net]["partner"]]
            recv[net].append(np.stack([dr[net]["partner"][hit], dr[net]["init"][hit],
                                       dr[net]["draw"][hit]], 1))
    recv = {k: np.concatenate(v) for k, v in recv.items()}
    rows = {}
    for j in sample:
        row = [m for m in range(int(maps["hh_lo"][j]), int(maps["hh_hi"][j])) if m != j]
        w = [p["w_household"]] * len(row)
        for net, wn in (("occ", p["w_occupation"]), ("rand", p["w_random"])):
            o = own[net]
            sel = o["init"] == j
            mine = o["partner"][sel][np.argsort(o["draw"][sel], kind="stable")]
            r = recv[net]
            r = r[r[:, 0] == j]
            r = r[np.lexsort((r[:, 2], r[:, 1]))][:, 1]
            row += list(mine) + list(r)
            w += [wn] * (len(mine) + len(r))
        rows[int(j)] = (np.array(row, np.int64), np.array(w, np.float64))
    return rows


def test_fifty_million_agents_sampled_rows_and_lambda():
    require_gpu()
    from paper_2110_04421_amd.sim import Simulator
    p, pop = workload(2, n_steps=2)
    maps = og.static_maps(pop)
    rng = np.random.default_rng(99)
    seeds = np.asarray(pop.initial_infected, np.int64)
    # rows next to an initial infection (nonzero force of infection) plus random rows
    near = np.unique(np.concatenate([np.arange(maps["hh_lo"][s], maps["hh_hi"][s]) for s in seeds[:300]]))
    sample = np.unique(np.concatenate([near[:600], rng.choice(pop.n_agents, 600, replace=False)]))
    with Simulator(p, pop, autotune=True) as s:
        counts = s.run(1)
        rp, col, w = s.csr()
        lam = s.lam()
    N = pop.n_agents
    E = int(rp[-1])
    # any-size properties: degrees consistent, edge total near its mean
    assert counts[0, 0, ostep.C_EDGES] == E
    hh = np.diff(np.asarray(pop.hh_start, np.int64))
    e_hh = int((hh * (hh - 1)).sum())
    assert (E - e_hh) % 2 == 0
    mean_c = N * (4.0 + 13.84) / 2
    assert abs((E - e_hh) / 2 - mean_c) < 6 * np.sqrt(mean_c)
    assert col.min() >= 0 and col.max() < N
    # sampled rows, exactly
    rows = _oracle_rows(pop, p, 0, sample, maps)
    for j, (rc, rw) in rows.items():
        g = col[rp[j]:rp[j + 1]].astype(np.int64)
        assert np.array_equal(g, rc), j
        assert np.array_equal(w[rp[j]:rp[j + 1]], rw.astype(np.float32)), j
    # force of infection of the sampled rows (eq. 1) from the oracle's day-0 state
    m = ostep.Model(pop, p)
    code = m.codes(m.init_state(), 0)
    lam_o = np.array([m.coef[j] * (rows[j][1] * m.Atab[code[rows[j][0]]]).sum() for j in sample])
    ok, err = lam_close(lam[sample], lam_o)
    assert ok, err
    assert (lam_o > 0).sum() > 100
