"""The daily contact graph of one day (section 3, "Interaction Networks").

Three networks, as the paper lists them:
* household -- every agent meets every other member of its (fixed) household each day;
* occupation -- fixed workplaces; each day each agent draws a Poisson number of
  contacts (mean mu_occ[occupation] / 2) uniformly among the other members of its
  workplace (the network is re-parameterised daily, its membership never changes);
* random -- regenerated every day; each agent draws a Poisson number of contacts
  (mean mu_rand[age] / 2) uniformly among the rest of its replicate's population.

Every drawn contact is one interaction seen from both ends, so it adds the edge to
both agents' rows (the graph is symmetric; in-degree is about mu).  Multi-edges are
kept.  The graph does not depend on the agents' states.

Destination-sorted CSR, canonical row order:
    [household members ascending]
    [occupation contacts this agent drew, in draw order]
    [occupation contacts drawn by others, by initiator id, then draw index]
    [random contacts this agent drew, in draw order]
    [random contacts drawn by others, by initiator id, then draw index]
Edge weight = the network factor B_n of eq. 1.

This module writes that definition out with one lexicographic sort.
"""
from __future__ import annotations

import numpy as np

from . import philox
from .tables import poisson_thresholds, poisson_count

BLK_HH, BLK_OCC_OWN, BLK_OCC_RECV, BLK_RAND_OWN, BLK_RAND_RECV = 0, 1, 2, 3, 4


def static_maps(pop):
    """Per-agent household range and workplace (index, position); -1 if none."""
    N = int(pop.agent_offset[-1])
    hs = np.asarray(pop.hh_start, np.int64)
    sizes = np.diff(hs)
    hh_id = np.repeat(np.arange(sizes.size), sizes)
    wps = np.asarray(pop.wp_start, np.int64)
    wsz = np.diff(wps)
    wp_of = np.full(N, -1, np.int64)
    wp_pos = np.full(N, -1, np.int64)
    mem = np.asarray(pop.wp_members, np.int64)
    wp_of[mem] = np.repeat(np.arange(wsz.size), wsz)
    wp_pos[mem] = np.arange(mem.size) - np.repeat(wps[:-1], wsz)
    rep = np.repeat(np.arange(pop.agent_offset.size - 1), np.diff(pop.agent_offset))
    has = wp_of >= 0
    wp_lo = np.zeros(N, np.int64)
    wp_size = np.zeros(N, np.int64)
    wp_lo[has] = wps[wp_of[has]]
    wp_size[has] = wsz[wp_of[has]]
    nrep = pop.agent_offset.size - 1
    words = np.arange(nrep, dtype=np.int64) if getattr(pop, "stream", None) is None \
        else np.asarray(pop.stream, np.int64)
    return dict(hh_lo=hs[hh_id], hh_hi=hs[hh_id + 1], wp_of=wp_of, wp_pos=wp_pos,
                wp_lo=wp_lo, wp_size=wp_size, rep=rep, stream=words[rep],
                local=np.arange(N) - np.asarray(pop.agent_offset)[rep])


def daily_draws(pop, params, t, maps=None, agents=None):
    """Contacts drawn on day t by ``agents`` (default: all).

    Returns a dict per network ('occ', 'rand') of arrays (initiator, draw, partner),
    plus the per-agent counts.  Draw d of agent i uses flat lane d of its purpose
    stream; lane 0 gives the Poisson count."""
    if maps is None:
        maps = static_maps(pop)
    N = int(pop.agent_offset[-1])
    ids = np.arange(N) if agents is None else np.asarray(agents, np.int64)
    seed = int(params["seed"])
    rep, loc, word = maps["rep"][ids], maps["local"][ids], maps["stream"][ids]
    nrep = np.diff(np.asarray(pop.agent_offset))[rep]
    off_rep = np.asarray(pop.agent_offset)[rep]
    mem = np.asarray(pop.wp_members, np.int64)
    out = {}
    for net, purpose in (("occ", philox.PURPOSE_OCC), ("rand", philox.PURPOSE_RAND)):
        if net == "occ":
            mu = np.asarray(params["mu_occupation"], np.float64)
            cls = np.asarray(pop.occupation, np.int64)[ids]
            m = maps["wp_size"][ids]
        else:
            mu = np.asarray(params["mu_random"], np.float64)
            cls = np.asarray(pop.age, np.int64)[ids]
            m = nrep
        tabs = [poisson_thresholds(float(x) / 2.0) for x in mu]
        w0 = philox.lane(seed, loc, t, word, purpose, 0)
        k = np.zeros(ids.size, np.int64)
        for c in range(mu.size):
            sel = cls == c
            if sel.any():
                k[sel] = poisson_count(w0[sel], tabs[c])
        k[m < 2] = 0
        inits, draws, partners = [], [], []
        for d in range(1, int(k.max(initial=0)) + 1):
            s = np.flatnonzero(k >= d)
            x = philox.lane(seed, loc[s], t, word[s], purpose, d).astype(np.uint64)
            mm = m[s].astype(np.uint64)
            off = ((x * (mm - np.uint64(1))) >> np.uint64(32)).astype(np.int64)
            if net == "occ":
                p = mem[maps["wp_lo"][ids[s]] + (maps["wp_pos"][ids[s]] + 1 + off) % m[s]]
            else:
                p = off_rep[s] + (loc[s] + 1 + off) % m[s]
            inits.append(ids[s])
            draws.append(np.full(s.size, d, np.int64))
            partners.append(p)
        cat = (lambda a: np.concatenate(a) if a else np.zeros(0, np.int64))
        out[net] = dict(k=k, init=cat(inits), draw=cat(draws), partner=cat(partners))
    return out


def build_graph(pop, params, t, maps=None):
    """Canonical CSR of day t: (row_ptr int64[N+1], col int64[E], w float64[E], blk int8[E])."""
    if maps is None:
        maps = static_maps(pop)
    N = int(pop.agent_offset[-1])
    rows, blks, k1, k2, srcs = [], [], [], [], []
    # household: all ordered pairs of distinct members
    hs = np.asarray(pop.hh_start, np.int64)
    sz = np.diff(hs)
    for s in range(2, int(sz.max(initial=0)) + 1):
        base = hs[:-1][sz == s]
        if base.size == 0:
            continue
        a, b = np.meshgrid(np.arange(s), np.arange(s), indexing="ij")
        keep = a != b
        r = (base[:, None] + a[keep][None, :]).ravel()
        c = (base[:, None] + b[keep][None, :]).ravel()
        rows.append(r); srcs.append(c); blks.append(np.full(r.size, BLK_HH))
        k1.append(c); k2.append(np.zeros(r.size, np.int64))
    dr = daily_draws(pop, params, t, maps)
    for net, own, recv in (("occ", BLK_OCC_OWN, BLK_OCC_RECV), ("rand", BLK_RAND_OWN, BLK_RAND_RECV)):
        d = dr[net]
        n = d["init"].size
        # the initiator's own row: partner, ordered by draw index
        rows.append(d["init"]); srcs.append(d["partner"]); blks.append(np.full(n, own))
        k1.append(d["draw"]); k2.append(np.zeros(n, np.int64))
        # the partner's row: initiator, ordered by (initiator, draw)
        rows.append(d["partner"]); srcs.append(d["init"]); blks.append(np.full(n, recv))
        k1.append(d["init"]); k2.append(d["draw"])
    rows, blks, k1, k2, srcs = (np.concatenate(x).astype(np.int64) for x in (rows, blks, k1, k2, srcs))
    order = np.lexsort((k2, k1, blks, rows))
    rows, blks, srcs = rows[order], blks[order], srcs[order]
    row_ptr = np.zeros(N + 1, np.int64)
    row_ptr[1:] = np.cumsum(np.bincount(rows, minlength=N))
    wtab = np.array([params["w_household"], params["w_occupation"], params["w_occupation"],
                     params["w_random"], params["w_random"]], np.float64)
    return row_ptr, srcs, wtab[blks], blks.astype(np.int8)


def build_graph_naive(pop, params, t):
    """Same graph from per-agent Python loops and scalar Philox calls (small
    populations only): a second, independent reading used to pin ``build_graph``."""
    from .tables import poisson_thresholds as thr
    N = int(pop.agent_offset[-1])
    off = [int(x) for x in pop.agent_offset]
    seed = int(params["seed"])
    key = (seed & 0xFFFFFFFF, seed >> 32)
    hs = [int(x) for x in pop.hh_start]
    wps = [int(x) for x in pop.wp_start]
    mem = [int(x) for x in pop.wp_members]
    where = {}
    for w in range(len(wps) - 1):
        for q in range(wps[w], wps[w + 1]):
            where[mem[q]] = (w, q - wps[w])
    def word(loc, rep, purpose, flat):
        ctr = (loc, t & 0xFFFFFFFF, rep, (purpose << 24) | (flat // 4))
        return philox.philox4_generic(ctr, key, 32, philox.M4x32, philox.W4x32)[flat % 4]
    def count(x, tab):
        k = 0
        while k < len(tab) - 1 and tab[k] <= x:
            k += 1
        return k
    rowsl = [[[] for _ in range(5)] for _ in range(N)]
    h = 0
    for j in range(N):
        while hs[h + 1] <= j:
            h += 1
        rowsl[j][BLK_HH] = [i for i in range(hs[h], hs[h + 1]) if i != j]
    contacts = []          # (network, initiator, draw, partner)
    words = list(range(len(off) - 1)) if getattr(pop, "stream", None) is None \
        else [int(x) for x in pop.stream]
    for r in range(len(off) - 1):
        n = off[r + 1] - off[r]
        for loc in range(n):
            i = off[r] + loc
            if i in where:
                w, pos = where[i]
                m = wps[w + 1] - wps[w]
                tab = thr(float(params["mu_occupation"][int(pop.occupation[i])]) / 2.0)
                k = count(word(loc, words[r], philox.PURPOSE_OCC, 0), tab) if m >= 2 else 0
                for d in range(1, k + 1):
                    o = (word(loc, words[r], philox.PURPOSE_OCC, d) * (m - 1)) >> 32
                    contacts.append((0, i, d, mem[wps[w] + (pos + 1 + o) % m]))
            tab = thr(float(params["mu_random"][int(pop.age[i])]) / 2.0)
            k = count(word(loc, words[r], philox.PURPOSE_RAND, 0), tab) if n >= 2 else 0
            for d in range(1, k + 1):
                o = (word(loc, words[r], philox.PURPOSE_RAND, d) * (n - 1)) >> 32
                contacts.append((1, i, d, off[r] + (loc + 1 + o) % n))
    for net, i, _d, p in sorted(contacts):
        own, recv = (BLK_OCC_OWN, BLK_OCC_RECV) if net == 0 else (BLK_RAND_OWN, BLK_RAND_RECV)
        rowsl[i][own].append(p)
        rowsl[p][recv].append(i)
    wtab = [params["w_household"], params["w_occupation"], params["w_occupation"],
            params["w_random"], params["w_random"]]
    row_ptr = [0]
    col, w = [], []
    for j in range(N):
        for b in range(5):
            col.extend(rowsl[j][b])
            w.extend([wtab[b]] * len(rowsl[j][b]))
        row_ptr.append(len(col))
    return np.array(row_ptr), np.array(col, np.int64), np.array(w)
