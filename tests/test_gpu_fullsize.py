"""Full-size check at 50 million agents in the configuration the benchmark times
(partitioned builder, autotuned tiling).

Sampled rows of day 0's contact graph are checked against contacts the oracle draws
one initiator at a time: the household part and the row's own draws exactly; the
received workplace contacts exactly (they come from the few members of the row's
workplace); every received random contact is a real draw of its initiator, with its
multiplicity, and every infectious agent's draws into the row are present.  The force
of infection of those rows (eq. 1) then follows from the oracle's infectiousness codes,
since only infectious sources contribute.  Properties that hold at any size cover the
rest."""
import numpy as np
import pytest

from helpers import require_gpu, lam_close
from oracle import graph as og
from oracle import step as ostep
from synthpop import workload

pytestmark = pytest.mark.gpu


def _log(msg):
    print(f"[fullsize] {msg}", flush=True)


def _by_initiator(dr, net):
    """{initiator: partners in draw order} for one network of a daily_draws result."""
    x = dr[net]
    o = np.lexsort((x["draw"], x["init"]))
    out = {}
    for i, p in zip(x["init"][o].tolist(), x["partner"][o].tolist()):
        out.setdefault(i, []).append(p)
    return out


def test_fifty_million_agents_sampled_rows_and_lambda():
    require_gpu()
    from paper_2110_04421_amd.sim import Simulator
    p, pop = workload(2, n_steps=2)
    _log("population built")
    maps = og.static_maps(pop)
    _log("static maps built")
    N = pop.n_agents
    seeds = np.unique(np.asarray(pop.initial_infected, np.int64))
    sd = og.daily_draws(pop, p, 0, maps, agents=seeds)
    rng = np.random.default_rng(99)
    near = np.unique(np.concatenate([np.arange(maps["hh_lo"][s], maps["hh_hi"][s]) for s in seeds[:200]]))
    hit = np.unique(np.concatenate([sd["occ"]["partner"][:300], sd["rand"]["partner"][:300]]))
    sample = np.unique(np.concatenate([near[:400], hit, rng.choice(N, 600, replace=False)]))
    with Simulator(p, pop, autotune=True) as s:
        counts = s.run(1)
        rp, col, w = s.csr()
        lam = s.lam()
    _log(f"GPU day done, {sample.size} sampled rows")
    rp = rp.astype(np.int64)
    E = int(rp[-1])
    # any-size properties: edge total, household pairs, symmetric contact count
    assert counts[0, 0, ostep.C_EDGES] == E
    hh = np.diff(np.asarray(pop.hh_start, np.int64))
    e_hh = int((hh * (hh - 1)).sum())
    assert (E - e_hh) % 2 == 0
    mean_c = N * (4.0 + 13.84) / 2
    assert abs((E - e_hh) / 2 - mean_c) < 6 * np.sqrt(mean_c)
    assert col.min() >= 0 and col.max() < N

    own = og.daily_draws(pop, p, 0, maps, agents=sample)
    own_o, own_r = _by_initiator(own, "occ"), _by_initiator(own, "rand")
    # workplace members of the sampled rows: their draws give the received occupation part
    wp_lo, wp_n = maps["wp_lo"][sample], maps["wp_size"][sample]
    mem = np.asarray(pop.wp_members, np.int64)
    cow = np.unique(np.concatenate([mem[a:a + n] for a, n in zip(wp_lo.tolist(), wp_n.tolist())] + [seeds[:0]]))
    cd = og.daily_draws(pop, p, 0, maps, agents=cow)
    recv_o = {}
    for i, q in zip(cd["occ"]["init"].tolist(), cd["occ"]["partner"].tolist()):
        recv_o.setdefault(q, []).append(i)
    seed_r = {}
    for i, q in zip(sd["rand"]["init"].tolist(), sd["rand"]["partner"].tolist()):
        seed_r.setdefault(q, []).append(i)
    _log("oracle draws of sampled rows, workplaces and seeds done")

    rows = {}
    rand_init = []
    for j in sample.tolist():
        g = col[rp[j]:rp[j + 1]].astype(np.int64)
        gw = w[rp[j]:rp[j + 1]]
        hpart = [m for m in range(int(maps["hh_lo"][j]), int(maps["hh_hi"][j])) if m != j]
        oo, orr = own_o.get(j, []), own_r.get(j, [])
        ro = sorted(recv_o.get(j, []))
        head = hpart + oo + ro + orr
        assert g.size >= len(head), j
        assert np.array_equal(g[:len(head)], np.array(head, np.int64)), j
        rr = g[len(head):]
        assert np.all(np.diff(rr) >= 0), j                       # sorted by initiator
        wexp = ([p["w_household"]] * len(hpart) + [p["w_occupation"]] * (len(oo) + len(ro))
                + [p["w_random"]] * (len(orr) + rr.size))
        assert np.array_equal(gw, np.array(wexp, np.float32)), j
        # every infectious agent's random draws into row j are there
        sr = sorted(seed_r.get(j, []))
        u, c = np.unique(rr, return_counts=True)
        have = dict(zip(u.tolist(), c.tolist()))
        for i in set(sr):
            assert have.get(i, 0) == sr.count(i), (j, i)
        rows[j] = (g, np.asarray(wexp, np.float64))
        rand_init.append(rr)
    # every received random contact is a real draw of its initiator, with multiplicity
    ri = np.unique(np.concatenate(rand_init))
    rd = _by_initiator(og.daily_draws(pop, p, 0, maps, agents=ri), "rand")
    for j, (g, _) in rows.items():
        nh = len([m for m in range(int(maps["hh_lo"][j]), int(maps["hh_hi"][j])) if m != j])
        start = nh + len(own_o.get(j, [])) + len(recv_o.get(j, [])) + len(own_r.get(j, []))
        u, c = np.unique(g[start:], return_counts=True)
        for i, k in zip(u.tolist(), c.tolist()):
            assert rd.get(i, []).count(j) == k, (j, i)
    _log("sampled rows verified")
    # force of infection of the sampled rows from the oracle's day-0 codes
    m = ostep.Model(pop, p)
    code = m.codes(m.init_state(), 0)
    lam_o = np.array([m.coef[j] * (rows[j][1] * m.Atab[code[rows[j][0]]]).sum() for j in sample.tolist()])
    ok, err = lam_close(lam[sample], lam_o)
    assert ok, err
    assert (lam_o > 0).sum() > 100
    _log(f"lambda of {sample.size} rows within tolerance (worst {err:.2e})")
