"""Degenerate and ragged inputs on the GPU against the FP64 oracle: replicates of 1 to
1,000 agents that straddle tile boundaries (single-agent replicates and workplaces
draw no partners), households of the largest size (255 members: tiles far beyond the
row pass's LDS room), and no initial infections."""
import dataclasses

import numpy as np
import pytest

from helpers import require_gpu, lam_close, lockstep
from oracle import graph as og
from oracle import step as ostep
from synthpop import make_population
from synthpop.configs import params_for
from test_gpu_parity import _sim

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("two", [False, True])
def test_ragged_replicates_with_interventions_in_lockstep(two):
    """With two-tile leaves, most leaves hold the ragged tiles of two replicates."""
    require_gpu()
    sizes = [1, 2, 3, 63, 64, 65, 255, 256, 257, 1000]
    pop = make_population(sizes, workplaces=True, n_seeds=[min(2, n) for n in sizes], pop_seed=5)
    p = params_for(1, n_steps=12, vacc_trigger=0.0, vacc_rate=0.05)
    near, worst, _ = lockstep(lambda p_, pop_, **kw: _sim(p_, pop_, two_tile_leaves=two, **kw), p, pop, 12,
                              check_csr_every=1)
    assert worst < 1e-5


@pytest.mark.parametrize("two", [False, True])
def test_largest_households_overflow_a_tile_room(two):
    require_gpu()
    from paper_2110_04421_amd.sim import Simulator
    from paper_2110_04421_amd._lib import AbmError
    base = make_population([20000], workplaces=True, n_seeds=10, pop_seed=6)
    hs = np.asarray(base.hh_start, np.int64)
    big = 5000 + 255 * np.arange(13)                  # twelve households of the largest size
    hs = np.union1d(hs[(hs <= big[0]) | (hs >= big[-1])], big)
    pop = dataclasses.replace(base, hh_start=hs.astype(np.int32))
    p = params_for(1, n_steps=3)
    with Simulator(p, pop, two_tile_leaves=two) as s:
        s.run(1)
        rp, col, w = s.csr()
        lam = s.lam()
    rp_o, col_o, w_o, _ = og.build_graph(pop, p, 0)
    tile = rp_o[5120 + 256] - rp_o[5120]               # a tile inside them: about 65,000 entries
    assert tile > 256 * 254
    assert np.array_equal(rp.astype(np.int64), rp_o)
    assert np.array_equal(col.astype(np.int64), col_o)
    assert np.array_equal(w, w_o.astype(np.float32))
    m = ostep.Model(pop, p)
    _, out = m.step(m.init_state(), 0, np.zeros((1, ostep.NC), np.int64))
    ok, err = lam_close(lam, out["lam"])
    assert ok, err
    # one member more than a household may have is an argument error
    hs2 = np.union1d(hs[(hs <= 5000) | (hs >= 5256)], [5000, 5256])
    with pytest.raises(AbmError) as e:
        Simulator(p, dataclasses.replace(base, hh_start=hs2.astype(np.int32)))
    assert e.value.code == -1


def test_no_initial_infections_stay_uninfected():
    require_gpu()
    from paper_2110_04421_amd.sim import Simulator
    pop = make_population([5000, 7000], workplaces=True, n_seeds=0, pop_seed=7)
    p = params_for(1, n_steps=10)
    with Simulator(p, pop) as s:
        c = s.run(10)
        lam = s.lam()
        rp, col, w = s.csr()
    assert np.all(c[:, :, ostep.C_S] == np.array([5000, 7000]))
    assert np.all(c[:, :, ostep.C_NEW] == 0) and np.all(lam == 0)
    rp_o, col_o, _, _ = og.build_graph(pop, p, 9)
    assert np.array_equal(col.astype(np.int64), col_o)
