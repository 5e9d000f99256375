"""Synthetic populations with the structure of DeepABM-COVID's agents (section 3, "Agent
State Definition" and "Interaction Networks"): static age group, household, occupation
and workplace membership.  The paper initialises these from King County census data,
which is not available; the recipe below stands in for it.

Recipe (per replicate, numpy ``Generator(PCG64(SeedSequence([pop_seed, r])))``):

1. household sizes drawn from a categorical law over 1..6 with probabilities
   (0.28, 0.35, 0.15, 0.13, 0.06, 0.03) until the population is filled; the last
   household is truncated.  Agent ids are household-contiguous.
2. ages uniform over the 9 age groups (0-10, ..., 80+).
3. occupation type uniform over the 23 occupations.
4. each occupation's agents are shuffled and cut into fixed workplaces of size
   U{5..30}; a remainder under 5 joins the previous workplace.
5. initial infections: ``n_seeds`` distinct agents drawn with
   ``Generator(PCG64(SeedSequence([seed_seed, r]))).choice``.

All ids in the arrays are global (replicates are concatenated); households and
workplaces never cross a replicate boundary.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

HOUSEHOLD_P = (0.28, 0.35, 0.15, 0.13, 0.06, 0.03)
N_AGE = 9
N_OCC = 23
WP_MIN, WP_MAX = 5, 30


@dataclass
class Population:
    agent_offset: np.ndarray          # int64 [R+1]
    age: np.ndarray                   # uint8 [N]
    hh_start: np.ndarray              # int32 [H+1], global agent ids
    occupation: np.ndarray            # uint8 [N]
    wp_start: np.ndarray              # int32 [W+1]
    wp_members: np.ndarray            # int32 [wp_start[-1]], global agent ids
    init_offset: np.ndarray           # int64 [R+1]
    initial_infected: np.ndarray      # int32 [init_offset[-1]], global agent ids
    R: np.ndarray                     # float32 [R]
    susceptibility: np.ndarray        # float32 [R, 9]
    dose2_delay: np.ndarray           # int32 [R]
    meta: dict = field(default_factory=dict)
    stream: np.ndarray | None = None  # uint32 [R] Philox stream word per replicate (None: r)

    @property
    def n_agents(self) -> int:
        return int(self.agent_offset[-1])

    @property
    def n_replicates(self) -> int:
        return int(self.agent_offset.size - 1)

    def sizes(self) -> np.ndarray:
        return np.diff(self.agent_offset)


def _households(rng: np.random.Generator, n: int) -> np.ndarray:
    """Household sizes (int64) summing exactly to n."""
    mean = float(np.dot(np.arange(1, 7), HOUSEHOLD_P))
    out = []
    total = 0
    while total < n:
        m = int((n - total) / mean * 1.1) + 16
        s = rng.choice(np.arange(1, 7), size=m, p=HOUSEHOLD_P)
        out.append(s)
        total += int(s.sum())
    sizes = np.concatenate(out)
    cs = np.cumsum(sizes)
    last = int(np.searchsorted(cs, n))       # first index with cs >= n
    sizes = sizes[: last + 1].copy()
    sizes[-1] -= int(cs[last] - n)
    assert sizes.sum() == n and sizes.min() >= 1
    return sizes


def _workplaces(rng: np.random.Generator, occ: np.ndarray, base: int):
    """Fixed workplaces per occupation type: returns (sizes list, members list)."""
    sizes_all, members_all = [], []
    for o in range(N_OCC):
        agents = np.flatnonzero(occ == o)
        m = agents.size
        if m == 0:
            continue
        agents = agents[rng.permutation(m)] + base
        s = rng.integers(WP_MIN, WP_MAX + 1, size=m // WP_MIN + 2)
        cs = np.cumsum(s)
        last = int(np.searchsorted(cs, m))
        s = s[: last + 1].copy()
        s[-1] -= int(cs[last] - m)
        if s[-1] < WP_MIN and s.size > 1:
            s[-2] += s[-1]
            s = s[:-1]
        assert s.sum() == m
        sizes_all.append(s)
        members_all.append(agents)
    return sizes_all, members_all


def make_population(sizes, *, workplaces: bool = True, n_seeds=10, pop_seed: int = 1000,
                    seed_seed: int = 2000, R=5.18, susceptibility=None, dose2_delay=21,
                    occupations: bool | None = None) -> Population:
    """Concatenate one synthetic population per entry of ``sizes``.

    ``R``, ``susceptibility`` (9 values or [R,9]), ``dose2_delay`` and ``n_seeds`` may be
    scalars or per-replicate sequences.
    """
    sizes = [int(s) for s in np.atleast_1d(sizes)]
    nrep = len(sizes)
    if occupations is None:
        occupations = workplaces
    off = np.zeros(nrep + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    N = int(off[-1])
    age = np.empty(N, np.uint8)
    occ = np.zeros(N, np.uint8)
    hh_parts = []
    wp_sizes, wp_members = [], []
    init_parts = []
    seeds = np.broadcast_to(np.asarray(n_seeds, np.int64), (nrep,))
    for r, n in enumerate(sizes):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([pop_seed, r])))
        b = int(off[r])
        hs = _households(rng, n)
        hh_parts.append(hs)
        age[b:b + n] = rng.integers(0, N_AGE, size=n, dtype=np.uint8)
        if occupations:
            occ[b:b + n] = rng.integers(0, N_OCC, size=n, dtype=np.uint8)
        if workplaces:
            s, m = _workplaces(rng, occ[b:b + n], b)
            wp_sizes.extend(s)
            wp_members.extend(m)
        srng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed_seed, r])))
        k = int(min(seeds[r], n))
        init_parts.append(np.sort(srng.choice(n, size=k, replace=False)).astype(np.int64) + b)
    hh = np.concatenate(hh_parts)
    hh_start = np.zeros(hh.size + 1, np.int64)
    hh_start[1:] = np.cumsum(hh)
    if wp_sizes:
        ws = np.concatenate(wp_sizes)
        wp_start = np.zeros(ws.size + 1, np.int64)
        wp_start[1:] = np.cumsum(ws)
        wpm = np.concatenate(wp_members)
    else:
        wp_start = np.zeros(1, np.int64)
        wpm = np.zeros(0, np.int64)
    init_off = np.zeros(nrep + 1, np.int64)
    init_off[1:] = np.cumsum([p.size for p in init_parts])
    Rv = np.broadcast_to(np.asarray(R, np.float32), (nrep,)).copy()
    if susceptibility is None:
        susceptibility = np.linspace(0.35, 1.47, N_AGE)
    sus = np.broadcast_to(np.asarray(susceptibility, np.float32), (nrep, N_AGE)).copy()
    dd = np.broadcast_to(np.asarray(dose2_delay, np.int32), (nrep,)).copy()
    if N >= 2**31:
        raise ValueError("population too large for int32 agent ids")
    return Population(off, age, hh_start.astype(np.int32), occ, wp_start.astype(np.int32),
                      wpm.astype(np.int32), init_off,
                      np.concatenate(init_parts).astype(np.int32), Rv, sus, dd,
                      meta=dict(pop_seed=pop_seed, seed_seed=seed_seed, sizes=sizes,
                                workplaces=workplaces))


def replicate_population(pop: Population, n: int, R=None, susceptibility=None,
                         dose2_delay=None) -> Population:
    """``n`` copies of a single-replicate population (same agents), optionally with
    per-copy parameters.  Used for ensembles that vary parameters, not agents."""
    assert pop.n_replicates == 1
    N = pop.n_agents
    off = np.arange(n + 1, dtype=np.int64) * N
    H = pop.hh_start.size - 1
    hh = np.concatenate([pop.hh_start[:-1] + r * N for r in range(n)] + [np.array([n * N])])
    W = pop.wp_start.size - 1
    nm = int(pop.wp_start[-1])
    wps = np.concatenate([pop.wp_start[:-1] + r * nm for r in range(n)] + [np.array([n * nm])])
    wpm = np.concatenate([pop.wp_members.astype(np.int64) + r * N for r in range(n)])
    ni = pop.initial_infected.size
    ioff = np.arange(n + 1, dtype=np.int64) * ni
    init = np.concatenate([pop.initial_infected.astype(np.int64) + r * N for r in range(n)])
    Rv = np.broadcast_to(np.asarray(pop.R[0] if R is None else R, np.float32), (n,)).copy()
    sus = pop.susceptibility[0] if susceptibility is None else susceptibility
    sus = np.broadcast_to(np.asarray(sus, np.float32), (n, N_AGE)).copy()
    dd = pop.dose2_delay[0] if dose2_delay is None else dose2_delay
    dd = np.broadcast_to(np.asarray(dd, np.int32), (n,)).copy()
    assert hh.size == n * H + 1 and wps.size == n * W + 1
    if n * N >= 2**31:
        raise ValueError("population too large for int32 agent ids")
    return Population(off, np.tile(pop.age, n), hh.astype(np.int32), np.tile(pop.occupation, n),
                      wps.astype(np.int32), wpm.astype(np.int32), ioff, init.astype(np.int32),
                      Rv, sus, dd, meta=dict(pop.meta, replicated=n))


def extract_replicate(pop: Population, r: int) -> Population:
    """Replicate r of a batch as a stand-alone population that keeps its Philox stream
    word (so that a run of it alone reproduces its part of the batched run)."""
    lo, hi = int(pop.agent_offset[r]), int(pop.agent_offset[r + 1])
    hs = np.asarray(pop.hh_start, np.int64)
    h0, h1 = int(np.searchsorted(hs, lo)), int(np.searchsorted(hs, hi))
    wps = np.asarray(pop.wp_start, np.int64)
    mem = np.asarray(pop.wp_members, np.int64)
    sizes = np.diff(wps)
    if sizes.size:
        first = mem[np.minimum(wps[:-1], max(mem.size - 1, 0))]
        keep = (sizes > 0) & (first >= lo) & (first < hi)
        ks = sizes[keep]
        wp_start = np.concatenate([[0], np.cumsum(ks)])
        wpm = mem[np.repeat(keep, sizes)] - lo
    else:
        wp_start, wpm = np.zeros(1, np.int64), np.zeros(0, np.int64)
    i0, i1 = int(pop.init_offset[r]), int(pop.init_offset[r + 1])
    words = np.arange(pop.n_replicates) if pop.stream is None else np.asarray(pop.stream)
    return Population(np.array([0, hi - lo], np.int64), pop.age[lo:hi].copy(),
                      (hs[h0:h1 + 1] - lo).astype(np.int32), pop.occupation[lo:hi].copy(),
                      wp_start.astype(np.int32), wpm.astype(np.int32),
                      np.array([0, i1 - i0], np.int64),
                      (np.asarray(pop.initial_infected[i0:i1], np.int64) - lo).astype(np.int32),
                      pop.R[r:r + 1].copy(), pop.susceptibility[r:r + 1].copy(),
                      pop.dose2_delay[r:r + 1].copy(), meta=dict(pop.meta, extracted=r),
                      stream=np.array([words[r]], np.uint32))


def split_replicates(pop: Population):
    """All replicates of a batch as stand-alone populations (``extract_replicate`` for
    every r, computed in one pass)."""
    off = np.asarray(pop.agent_offset, np.int64)
    hs = np.asarray(pop.hh_start, np.int64)
    wps = np.asarray(pop.wp_start, np.int64)
    mem = np.asarray(pop.wp_members, np.int64)
    sizes = np.diff(wps)
    wrep = np.searchsorted(off, mem[wps[:-1]], side="right") - 1 if sizes.size else np.zeros(0, np.int64)
    order = np.argsort(wrep, kind="stable")
    sizes_o = sizes[order]
    mem_o = np.concatenate([mem[wps[w]:wps[w + 1]] for w in order]) if order.size else mem
    wstart_o = np.concatenate([[0], np.cumsum(sizes_o)])
    wr_bounds = np.searchsorted(wrep[order], np.arange(off.size))
    words = np.arange(pop.n_replicates) if pop.stream is None else np.asarray(pop.stream)
    out = []
    for r in range(pop.n_replicates):
        lo, hi = int(off[r]), int(off[r + 1])
        h0, h1 = int(np.searchsorted(hs, lo)), int(np.searchsorted(hs, hi))
        w0, w1 = int(wr_bounds[r]), int(wr_bounds[r + 1])
        ws = wstart_o[w0:w1 + 1] - wstart_o[w0]
        wm = mem_o[wstart_o[w0]:wstart_o[w1]] - lo
        i0, i1 = int(pop.init_offset[r]), int(pop.init_offset[r + 1])
        out.append(Population(
            np.array([0, hi - lo], np.int64), pop.age[lo:hi].copy(),
            (hs[h0:h1 + 1] - lo).astype(np.int32), pop.occupation[lo:hi].copy(),
            ws.astype(np.int32), wm.astype(np.int32), np.array([0, i1 - i0], np.int64),
            (np.asarray(pop.initial_infected[i0:i1], np.int64) - lo).astype(np.int32),
            pop.R[r:r + 1].copy(), pop.susceptibility[r:r + 1].copy(),
            pop.dose2_delay[r:r + 1].copy(), meta=dict(pop.meta, extracted=r),
            stream=np.array([words[r]], np.uint32)))
    return out
