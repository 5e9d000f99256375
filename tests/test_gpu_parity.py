"""GPU (libabm through the C ABI) against the FP64 oracle, element by element.

Bars: integer state, stage timers, CSR and tables bit-exact; lambda within 1e-5
relative (exact zero where the oracle has zero); an agent's state may differ only where
its infection draw lay within 1e-6 of the oracle's threshold, and those draws are
counted (zero on the 1,000-agent workload).
"""
import numpy as np
import pytest

from helpers import require_gpu, lockstep, from_records, state_mismatch
from oracle import graph as og
from oracle import philox as oph
from oracle import step as ostep
from oracle.tables import infectiousness_table, poisson_thresholds
from synthpop import workload, extract_replicate

pytestmark = pytest.mark.gpu


def _sim(params, pop, **kw):
    require_gpu()
    from paper_2110_04421_amd.sim import Simulator
    return Simulator(params, pop, **kw)


def test_philox_matches_oracle_bitwise():
    require_gpu()
    from paper_2110_04421_amd.sim import philox
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 2**32, size=(5000, 4), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    ctr[1] = 0xFFFFFFFF
    for seed in (0, 0x299F31D0A4093822, 2**64 - 1):
        g = philox(seed, ctr)
        o = np.stack(oph.philox4x32(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], seed), 1)
        assert np.array_equal(g, o)


def test_tables_match_oracle():
    p, pop = workload(1, n=3000)
    p["mu_occupation"] = [0.5 + 0.3 * k for k in range(23)]
    p["mu_random"] = [1.0 + 1.7 * a for a in range(9)]
    p["A_stage"] = [0.0, 0.37, 1.0, 0.0, 0.0]
    with _sim(p, pop) as s:
        at = s.atab()
        ref = np.array(infectiousness_table(2.5, 2.0, 5, 10, p["A_stage"]), np.float32)
        assert np.array_equal(at, ref)
        pt = s.poisson_tables()
        for k in range(23):
            assert list(pt[k]) == poisson_thresholds(p["mu_occupation"][k] / 2.0)
        for a in range(9):
            assert list(pt[23 + a]) == poisson_thresholds(p["mu_random"][a] / 2.0)


@pytest.mark.parametrize("two", [False, True])
@pytest.mark.parametrize("k,n,nrep", [(0, None, None), (1, 20000, None), (3, 30000, 7)])
def test_csr_bit_exact(k, n, nrep, two):
    """Leaves of one tile (below 2^25 agents) and of two (beyond; forced here): two
    tiles of a leaf may belong to different replicates and one may be ragged."""
    p, pop = workload(k, n=n, n_rep=nrep, n_steps=8)
    with _sim(p, pop, two_tile_leaves=two) as s:
        for t in range(3):
            s.run(1)
            rp, col, w = s.csr()
            rp_o, col_o, w_o, _ = og.build_graph(pop, p, t)
            assert np.array_equal(rp.astype(np.int64), rp_o)
            assert np.array_equal(col.astype(np.int64), col_o)
            assert np.array_equal(w, w_o.astype(np.float32))


@pytest.mark.parametrize("mu", [15.0, 40.0])
@pytest.mark.parametrize("two", [False, True])
def test_csr_bit_exact_at_high_contact_means(mu, two):
    """At mean 15 a batch's draws pass the level-1 scatter's and the row pass's LDS
    and register room (their direct and re-read paths run); at the validator's largest
    mean, 40 per network, the claim builder takes over.  Either way the graph is the
    oracle's."""
    p, pop = workload(1, n=3000, n_steps=4, mu_random=[mu] * 9, mu_occupation=[mu] * 23)
    with _sim(p, pop, two_tile_leaves=two) as s:
        for t in range(2):
            s.run(1)
            rp, col, w = s.csr()
            rp_o, col_o, w_o, _ = og.build_graph(pop, p, t)
            assert np.array_equal(rp.astype(np.int64), rp_o)
            assert np.array_equal(col.astype(np.int64), col_o)
            assert np.array_equal(w, w_o.astype(np.float32))


def _lockstep(p, pop, T, graph=True, allow_near=True, check_csr_every=0):
    """Step GPU and oracle together (helpers.lockstep); (near draws, worst lambda err)."""
    near, worst, _ = lockstep(_sim, p, pop, T, graph=graph, allow_near=allow_near,
                              check_csr_every=check_csr_every)
    return near, worst


def test_trajectory_plain_1k_bit_exact():
    p, pop = workload(0)
    near, worst = _lockstep(p, pop, 30, allow_near=False, check_csr_every=7)
    assert near == 0
    assert worst < 1e-5


def test_full_run_plain_1k_counts_equal_oracle():
    p, pop = workload(0)
    traj_o, st_o, _ = ostep.run(pop, p)
    with _sim(p, pop) as s:
        traj_g = s.run(30)
        keep = [c for c in range(ostep.NC) if c != ostep.C_NEAR]
        assert np.array_equal(traj_g[..., keep], traj_o[..., keep])
        gst = from_records(s.state(), s.latch())
        assert state_mismatch(gst, st_o).size == 0


def test_lockstep_interventions_20k():
    p, pop = workload(1, n=20000, vacc_trigger=0.0015, n_steps=60)
    near, worst = _lockstep(p, pop, 60, check_csr_every=20)
    assert worst < 1e-5


def test_lockstep_strategies_and_dropout():
    for strat in (1, 2):
        p, pop = workload(1, n=8000, vacc_trigger=0.0, vacc_rate=0.02, strategy=strat,
                          quarantine_dropout=0.1, test_rate=0.2, n_steps=40)
        p["dose_lag"] = 3
        _lockstep(p, pop, 40, graph=False)


def test_lockstep_segmented_vaccination_plan():
    """The plan the path takes above 2048 tiles a replicate (forced here): replicates of
    several 256-tile segments, one ragged, with the capacity running out inside a
    priority class on most days."""
    p, pop = workload(3, n=150000, n_rep=2, n_steps=15, vacc_trigger=0.0, vacc_rate=0.02,
                      strategy=1)
    p["dose_lag"] = 3
    nt = np.diff(np.asarray(pop.agent_offset)) // 256
    assert nt.max() > 256
    _, _, doses = lockstep(lambda p_, pop_, **kw: _sim(p_, pop_, segment_vplan=True, **kw),
                           p, pop, 15)
    assert (doses[..., 0] > 0).all()


@pytest.mark.parametrize("strat", [0, 1, 2])
def test_segmented_vaccination_plan_equals_one_workgroup(strat):
    p, pop = workload(3, n=400000, n_rep=3, n_steps=20, vacc_trigger=0.001, vacc_rate=0.01,
                      strategy=strat)
    out = []
    for seg in (False, True):
        with _sim(p, pop, segment_vplan=seg) as s:
            out.append((s.run(20), s.state(), s.latch()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])
    assert out[0][0][..., ostep.C_DOSE1].sum() > 0


def test_batched_equals_sequential():
    p, pop = workload(3, n=60000, n_rep=6, n_steps=40, vacc_trigger=0.002)
    with _sim(p, pop) as s:
        tb = s.run(40)
        sb = s.state()
    for r in range(pop.n_replicates):
        sub = extract_replicate(pop, r)
        with _sim(p, sub) as s:
            ts = s.run(40)
            ss = s.state()
        assert np.array_equal(tb[:, r, :], ts[:, 0, :])
        lo, hi = pop.agent_offset[r], pop.agent_offset[r + 1]
        assert np.array_equal(sb[lo:hi], ss)


def test_runs_are_deterministic_graph_and_eager():
    p, pop = workload(1, n=30000, n_steps=25, vacc_trigger=0.001)
    outs = []
    for graph in (True, True, False):
        with _sim(p, pop, graph=graph) as s:
            outs.append((s.run(25), s.state(), s.lam()))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0])
        assert np.array_equal(o[1], outs[0][1])
        assert np.array_equal(o[2].view(np.uint32), outs[0][2].view(np.uint32))


def test_capacity_overflow_is_reported():
    from paper_2110_04421_amd._lib import AbmError
    p, pop = workload(0, edge_capacity=1000)
    with _sim(p, pop) as s:
        with pytest.raises(AbmError) as e:
            s.run(1)
        assert e.value.code == -4


def test_resume_equals_uninterrupted():
    p, pop = workload(1, n=10000, n_steps=30, vacc_trigger=0.001)
    with _sim(p, pop) as s:
        full = s.run(30)
    with _sim(p, pop) as s:
        a = s.run(12)
        st, latch = s.state(), s.latch()
    with _sim(p, pop) as s:
        s.set_state(12, latch, st)
        b = s.run(18)
    assert np.array_equal(np.concatenate([a, b]), full)


def test_claim_builder_builds_the_same_graph():
    p, pop = workload(3, n=40000, n_rep=5, n_steps=4)
    outs = []
    for claim in (False, True):
        with _sim(p, pop, claim_builder=claim) as s:
            c = s.run(3)
            outs.append((c, s.csr(), s.state()))
    assert np.array_equal(outs[0][0], outs[1][0])
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b)
    assert np.array_equal(outs[0][2], outs[1][2])


@pytest.mark.parametrize("two", [False, True])
def test_csr_bit_exact_several_level1_buckets(two):
    # 600k agents: the partitioned builder splits destinations over 10 level-1 buckets
    # of 65,536 slots (5 of 131,072 with two-tile leaves)
    p, pop = workload(1, n=600_000, n_steps=2)
    with _sim(p, pop, two_tile_leaves=two) as s:
        s.run(1)
        rp, col, w = s.csr()
    rp_o, col_o, w_o, _ = og.build_graph(pop, p, 0)
    assert np.array_equal(rp.astype(np.int64), rp_o)
    assert np.array_equal(col.astype(np.int64), col_o)
    assert np.array_equal(w, w_o.astype(np.float32))


@pytest.mark.parametrize("two", [False, True])
def test_builder_small_lds_room_builds_the_same_graph(two):
    # batches scattered and leaves laid out by direct writes, received entries re-read
    p, pop = workload(3, n=60000, n_rep=5, n_steps=4)
    outs = []
    for small in (False, True):
        with _sim(p, pop, min_lds_room=small, two_tile_leaves=two) as s:
            c = s.run(3)
            outs.append((c, s.csr(), s.state()))
    assert np.array_equal(outs[0][0], outs[1][0])
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b)
    assert np.array_equal(outs[0][2], outs[1][2])
    rp_o, col_o, w_o, _ = og.build_graph(pop, p, 2)
    assert np.array_equal(outs[1][1][1].astype(np.int64), col_o)


def test_autotuned_tiling_gives_identical_results():
    p, pop = workload(3, n=50000, n_rep=6, n_steps=12, vacc_trigger=0.001)
    outs = []
    for tune in (False, True):
        with _sim(p, pop, autotune=tune) as s:
            outs.append((s.run(12), s.state(), s.lam(), s.tuning()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][2].view(np.uint32), outs[1][2].view(np.uint32))
    t = outs[1][3]
    assert t["message_chunk"] in (256, 512, 1024, 2048, 4096) and 1 <= t["message_grid"]
    assert t["message_shape"] in (0, 1, 2, 3)
