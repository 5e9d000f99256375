#!/usr/bin/env python
"""Throughput of the DeepABM-COVID daily step on one MI355X.

One step = one simulated day of the whole hot path (graph build, force of infection,
fused infection/progression, testing, quarantine, vaccination) over the workload.
Default workload: 50M agents, 20 contacts per agent per day (about 1e9 directed edges
per day), interventions on.  W warm-up days, then K timed days (W + K = 180 by default:
one full run).  value = edge-interactions per second over the timed days, where an
edge-interaction is one directed edge of a day's contact graph.

Extras on the same JSON line: the 100k-agent, 180-day run (the paper's 200M-interaction
workload) with the paper's figure for context; the 256-replicate ensemble in one launch
vs the same replicates run one by one; the per-kernel roofline of the dominant kernel;
and the FP64 CPU oracle timed on a bounded sample of the 100k-agent workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edge-interactions/s at 100k & 50M agents (HBM GB/s); batched replicates/s vs plain"
HBM_PEAK_GBS = 8000.0
PAPER_C1_RATE = 200e6 / 90.0      # 200M interactions in about 90 s (abstract, section 1)


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def household_edges(pop) -> int:
    s = np.diff(np.asarray(pop.hh_start, np.int64))
    return int((s * (s - 1)).sum())


def level1_buckets(N: int) -> int:
    """Level-1 buckets of the partitioned builder (same rule as the library, one
    replicate): destinations are numbered by tile slot, leaves are one or two tiles."""
    slots = -(-N // 256) * 256
    nb1 = lambda l2: -(-slots // (1 << (l2 + 8)))
    return nb1(9) if nb1(8) > 512 else nb1(8)


def kernel_bytes(name: str, N: int, E: float, C: float, vacc: bool, Einf: float = None) -> float:
    """Algorithmic HBM bytes of one launch (one day) of a step.  E = directed edges of
    the day, Einf = those with an infectious source, C = contacts drawn (each gives two
    edges), N = agents."""
    Einf = E if Einf is None else Einf
    nbt, nb1 = -(-N // 1024), level1_buckets(N)
    table = {
        # force of infection: col (source and network) + 1 mask bit per edge, a code
        # byte per infectious edge; row_ptr, age, lambda per row
        "message": 4.125 * E + 1.0 * Einf + 9.0 * N,
        # partitioned builder
        # draws: static record in; counts, own list and histograms out
        "pb_gen": 18.0 * N + 4.0 * C + 4.0 * nbt * nb1,
        "pb_scan1": 12.0 * nbt * nb1,              # histograms read twice, offsets written
        "pb_scatter1": 2.0 * N + 10.0 * C,         # counts and own list in, 6-byte entries out
        "pb_hist2": 2.0 * C,                       # the 16-bit destination parts
        "pb_scatter2": 14.0 * C,                   # 6-byte entries in, 8-byte leaf entries out
        "pb_leaves": 16.0 * nbt * 4,               # per tile: degree and leaf bounds in, start out
        # leaf entries, own list, counts and static records in; col and row_ptr out
        "pb_rows": 4.0 * E + 12.0 * C + 22.0 * N,
        # claim-based builder
        "count": 18.0 * N + 8.0 * C, "scan": 26.0 * N, "fill": 4.0 * E + 8.0 * C + 24.0 * N,
        "canon": 11.0 * N + 8.0 * C, "clear": 4.0 * N,
        # agent kernels
        "pre": (18.0 if vacc else 17.0) * N,       # state in, code out (age in with vaccination)
        "mask": 1.125 * N,
        "fused": 37.0 * N,                         # state in/out, lambda, age
    }
    return table.get(name, 0.0)


KERNEL_SOURCES = {"message": "k_step.hip", "fused": "k_step.hip", "pre": "k_step.hip",
                  "mask": "k_step.hip", "pb_rows": "k_build.hip", "pb_leaves": "k_build.hip",
                  "pb_gen": "k_build.hip", "pb_scatter1": "k_build.hip",
                  "pb_hist2": "k_build.hip", "pb_scatter2": "k_build.hip",
                  "pb_scan1": "k_build.hip"}


def source_sha(kernel: str):
    import hashlib
    f = KERNEL_SOURCES.get(kernel)
    if not f:
        return None
    path = os.path.join(ROOT, "paper_2110_04421_amd", "csrc", f)
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 PMC summary (FETCH_SIZE +
    WRITE_SIZE, scaled by the same counters on a copy kernel of known size), or None
    when the summary is missing or the kernel's source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh).get(kernel)
    if not t or t.get("source_sha256") != source_sha(kernel):
        return None
    return t["bytes_per_launch"]


def copy_probe(nbytes: int = 1 << 30):
    """A plain device copy of known size, for scaling the PMC byte counters."""
    import torch
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()


def copy_bandwidth(nbytes: int = 2 << 30, reps: int = 5) -> float:
    """Achieved bandwidth of a plain device-to-device copy (read + write bytes over the
    best of ``reps`` timed copies), the practical ceiling for a streaming kernel."""
    import torch
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del x, y
    return 2.0 * nbytes / best / 1e9


def time_days(sim, W: int, K: int):
    import torch
    if W:
        sim.run(W)
    sim.profile_reset() if sim_profiled(sim) else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    counts = sim.run(K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return counts, t1 - t0


def streaming_run(p, pop, warmup: int, steps: int):
    """The same days with every edge streamed through the force-of-infection kernel
    every day (dense_message): the day time and that kernel's, for comparison with the
    frontier path, which must give the same counts."""
    from paper_2110_04421_amd.sim import Simulator
    with Simulator(p, pop, autotune=True, dense_message=True) as sim:
        counts, wall = time_days(sim, warmup, steps)
    with Simulator(p, pop, profile=True, autotune=True, dense_message=True) as sim:
        time_days(sim, warmup, steps)
        prof = sim.profile()
    ms, n = prof["message"]
    return counts, wall, ms / max(n, 1)


def sim_profiled(sim) -> bool:
    return bool(sim._p.flags & 1)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---- the oracle's force-of-infection pass split over destination ranges ------------
# (worker processes are spawned: they import numpy and the oracle only, never the GPU)
_LAM = {}


def _lam_init(folder):
    for k in ("coef", "atab", "code", "row_ptr", "col", "w"):
        _LAM[k] = np.load(os.path.join(folder, k + ".npy"), mmap_mode="r")


def _lam_part(rng):
    from oracle import step as ostep
    lo, hi = rng
    return ostep.lambda_rows(_LAM["coef"], np.asarray(_LAM["atab"]), _LAM["code"], _LAM["row_ptr"],
                             _LAM["col"], _LAM["w"], lo, hi)[0]


def lambda_pass_split(n: int = 1_000_000, max_procs: int = 16):
    """The oracle's lambda pass (eq. 1 over one day's graph) on a population of ``n``
    agents with the 50M-agent workload's contact structure (20 contacts per agent per
    day), infectious codes on a seeded 2 % of agents: one process, then the rows split
    into equal-edge destination ranges over min(cpu_count, max_procs) spawned worker
    processes.  The two results must be bitwise equal (each row is summed in the same
    order)."""
    import multiprocessing as mp
    import shutil
    import tempfile
    from synthpop import workload
    from oracle import graph as og
    from oracle import step as ostep
    p, pop = workload(2, n=n)
    N = pop.n_agents
    rp, col, w, _ = og.build_graph(pop, p, 0)
    m = ostep.Model(pop, p)
    rng = np.random.default_rng(5)
    code = np.where(rng.random(N) < 0.02, rng.integers(1, 16, N), 0).astype(np.int64)
    E = int(rp[-1])
    t0 = time.perf_counter()
    lam1, _ = ostep.lambda_rows(m.coef, m.Atab, code, rp, col, w, 0, N)
    t_one = time.perf_counter() - t0
    P = max(1, min(os.cpu_count() or 1, max_procs))
    cuts = np.searchsorted(rp, np.linspace(0, E, P + 1)).clip(0, N)
    cuts[0], cuts[-1] = 0, N
    ranges = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    shm = "/dev/shm" if os.path.isdir("/dev/shm") else None
    folder = tempfile.mkdtemp(prefix="abm_lam_", dir=shm)
    try:
        for k, v in (("coef", m.coef), ("atab", m.Atab), ("code", code), ("row_ptr", rp), ("col", col), ("w", w)):
            np.save(os.path.join(folder, k + ".npy"), np.ascontiguousarray(v))
        with mp.get_context("spawn").Pool(P, initializer=_lam_init, initargs=(folder,)) as pool:
            pool.map(_lam_part, ranges)                  # warm-up: imports, page-in
            t0 = time.perf_counter()
            parts = pool.map(_lam_part, ranges)
            t_multi = time.perf_counter() - t0
    finally:
        shutil.rmtree(folder, ignore_errors=True)
    lamP = np.concatenate(parts)
    return {"agents": N, "edges": E, "single_process_s": t_one, "processes": P,
            "multi_process_s": t_multi, "single_process_edges_per_s": E / t_one,
            "multi_process_edges_per_s": E / t_multi,
            "bitwise_equal": bool(np.array_equal(lamP.view(np.uint64), lam1.view(np.uint64))),
            "sample": f"one day's graph of a {N}-agent population with the plain-50M contact "
                      f"structure; FP64 numpy oracle lambda pass"}


def cpu_baseline(budget_s: float = 15.0):
    """The FP64 oracle, as it stands, on the first days of the 100k-agent workload."""
    from synthpop import workload
    from oracle import step as ostep
    p, pop = workload(1)
    m = ostep.Model(pop, p)
    st = m.init_state()
    prev = np.zeros((1, ostep.NC), np.int64)
    m.put_counts(prev, st)
    edges, days = 0, 0
    t0 = time.perf_counter()
    while days < 2 or (time.perf_counter() - t0 < budget_s and days < 180):
        st, out = m.step(st, days, prev)
        prev = out["counts"]
        edges += int(out["counts"][0, ostep.C_EDGES])
        days += 1
    wall = time.perf_counter() - t0
    return {"value": edges / wall, "unit": "edge-interactions/s", "cores": 1, "kind": "oracle",
            "sample": f"plain-100k (100,000 agents), days 0..{days - 1} of 180, FP64 numpy oracle, "
                      f"one process (one core); {edges} edge-interactions in {wall:.1f} s",
            "host_cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
            "lambda_pass": lambda_pass_split()}


def course_run(days: int = 40, warmup: int = 5):
    """The 50M-agent day with the eleven-stage course instead of SEIRM (HIP-graph day
    loop), and the per-kernel time of its fused step from a profiled pass."""
    import torch
    from paper_2110_04421_amd.sim import Simulator
    from synthpop import workload
    p, pop = workload(2, n_steps=days + warmup, disease_model=1)
    with Simulator(p, pop, autotune=True) as s:
        s.run(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = s.run(days)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    with Simulator(p, pop, profile=True, autotune=True) as s:
        s.run(warmup)
        s.profile_reset()
        s.run(10)
        prof = s.profile()
    fused_ms = prof["fused"][0] / max(prof["fused"][1], 1)
    return {"workload": "plain-50M, eleven-stage course", "agents": int(pop.n_agents), "days_timed": days,
            "ms_per_day": wall / days * 1e3, "fused_ms": fused_ms,
            "hospitalised_peak": int(c[:, 0, 13].max()), "icu_peak": int(c[:, 0, 14].max())}


def den_run(days: int = 30, warmup: int = 10):
    """The 50M-agent day with exposure notification on (app adoption 0.3, RT-PCR
    testing): each day's graph is built into its slot of the 7-day ring, and the
    pre-pass reads a positive app user's rows of the last seven days."""
    import torch
    from paper_2110_04421_amd.sim import Simulator
    from synthpop import workload
    from synthpop.configs import TEST_TYPES
    p, pop = workload(2, n_steps=days + warmup, app_adoption=0.3, den_compliance=0.8,
                      **TEST_TYPES["rt_pcr"])
    with Simulator(p, pop, autotune=True) as s:
        s.run(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = s.run(days)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    with Simulator(p, pop, profile=True, autotune=True) as s:
        s.run(warmup)
        s.profile_reset()
        s.run(5)
        prof = s.profile()
    pre = prof["pre"]
    return {"workload": "plain-50M, exposure notification", "agents": int(pop.n_agents), "days_timed": days,
            "ms_per_day": wall / days * 1e3, "pre_ms": pre[0] / max(pre[1], 1),
            "notified_per_day": float(c[:, 0, 15].mean())}


def c1_run(reps: int = 3):
    """Full 180-day runs of the 100k-agent workload (HIP-graph day loop)."""
    import torch
    from paper_2110_04421_amd.sim import Simulator
    from synthpop import workload
    p, pop = workload(1)
    walls, edges = [], 0
    with Simulator(p, pop) as s:
        init, latch = s.state(), np.zeros(1, np.uint8)
        s.run(180)                                  # warm-up run
        for _ in range(reps):
            s.set_state(0, latch, init)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c = s.run(180)
            walls.append(time.perf_counter() - t0)
            edges = int(c[:, 0, 10].sum())
    wall = statistics.median(walls)
    return {"workload": "plain-100k", "agents": 100_000, "days": 180,
            "edge_interactions": edges, "seconds_per_run": wall,
            "value": edges / wall, "unit": "edge-interactions/s",
            "paper_context": {"value": PAPER_C1_RATE, "note": "200M interactions in about 90 s on an "
                              "unnamed GPU (abstract, section 1); not the same hardware"},
            "ratio_vs_paper_context": (edges / wall) / PAPER_C1_RATE}


def batched_vs_plain(n_rep: int = 256):
    """256 replicates (10k-500k agents each) in one launch vs one by one."""
    import torch
    from paper_2110_04421_amd.sim import Simulator
    from synthpop import workload, split_replicates
    p, pop = workload(3, n_rep=n_rep)
    with Simulator(p, pop, autotune=True) as s:
        s.run(1)
        s.set_state(0, np.zeros(n_rep, np.uint8), _initial(s, pop))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cb = s.run(180)
        tb = time.perf_counter() - t0
    subs = split_replicates(pop)
    ts, equal = 0.0, True
    for r, sub in enumerate(subs):
        with Simulator(p, sub) as s:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cs = s.run(180)
            ts += time.perf_counter() - t0
        equal &= bool(np.array_equal(cs[:, 0, :], cb[:, r, :]))
    return {"workload": "batched-256", "replicates": n_rep, "agents": int(pop.n_agents),
            "batched_seconds": tb, "sequential_seconds": ts,
            "batched_replicates_per_s": n_rep / tb, "sequential_replicates_per_s": n_rep / ts,
            "speedup": ts / tb, "per_replicate_bit_equal": equal}


def adjoint_cost(days: int = 180):
    """Relaxed forward + hand-written adjoint vs the relaxed and the plain forward, at
    100,000 agents (checkpoints every 10 days)."""
    import torch
    from paper_2110_04421_amd.sim import Simulator
    from synthpop import workload
    p, pop = workload(4, n_steps=days)
    dL = np.ones((1, days), np.float32)
    with Simulator(p, pop) as s:
        s.run(days)                                  # warm-up
    with Simulator(p, pop) as s:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(days)
        t_fwd = time.perf_counter() - t0
        t0 = time.perf_counter()
        g = s.grad(dL)
        t_bwd = time.perf_counter() - t0
    with Simulator(dict(p, mode=0), pop) as s:
        s.run(days)
    with Simulator(dict(p, mode=0), pop) as s:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(days)
        t_hard = time.perf_counter() - t0
    return {"workload": "calib-100k", "days": days, "soft_forward_s": t_fwd, "adjoint_s": t_bwd,
            "plain_forward_s": t_hard, "cost_vs_soft_forward": (t_fwd + t_bwd) / t_fwd,
            "cost_vs_plain_forward": (t_fwd + t_bwd) / t_hard,
            "dL_dR_of_total_incidence": float(g[0, 0])}


def mlp_throughput(reps: int = 50):
    """Achieved TFLOP/s of the calibration network's BF16 matrix-core kernels: the
    forward pass at a batch of 1024 and a training step (forward, backward, Adam) at
    a batch of 256, timed with HIP events on the stream the kernels run on."""
    import torch
    from paper_2110_04421_amd.mlp import MLP
    from paper_2110_04421_amd import _lib as L
    net = MLP(1024, seed=1)
    fwd_flop = 2.0 * (L.MLP_IN * L.MLP_H + L.MLP_H * L.MLP_H + L.MLP_H * L.MLP_OUT)
    x = torch.randn(1024, L.MLP_IN, device="cuda")
    xt, yt = x[:256].contiguous(), torch.zeros(256, L.MLP_OUT, device="cuda")
    out = {"workload": "calibration network 192-256-256-16, BF16 operands, FP32 accumulation",
           "peak_TFLOP_per_s": 2500.0}
    for name, fn, flop in (("forward_batch_1024", lambda: net.forward(x), 1024 * fwd_flop),
                           # backward: two products per layer (weights and inputs; the
                           # first layer's input gradient is not formed)
                           ("train_step_batch_256", lambda: net.train_step(xt, yt, 10, lr=0.0),
                            256 * fwd_flop * (3.0 - (L.MLP_IN * L.MLP_H) / (fwd_flop / 2.0)))):
        for _ in range(5):
            fn()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        e1.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        out[name] = {"us_per_call": sec * 1e6, "TFLOP_per_s": flop / sec / 1e12,
                     "frac_of_peak": flop / sec / 1e12 / 2500.0}
    return out


def calibration_leg(n_train: int = 4096, n_heldout: int = 256, agents: int = 10_000, days: int = 120):
    """Learned calibration against grid search, re-simulation error and wall time of
    each (the network, the 41-point R grid, the 231-point R x shared-susceptibility
    grid, and that grid at the network's simulation budget)."""
    from paper_2110_04421_amd import calib
    s = calib.run(n_train=n_train, n_heldout=n_heldout, n_agents=agents, epochs=20, days=days,
                  n_gd=64, gd_iters=20)
    keys = ("resim_rel_l2_same_stream", "resim_rel_l2_same_stream_median",
            "resim_rel_l2_independent_stream", "transmissibility_rmse_log", "simulations_per_method",
            "seconds")
    out = {"workload": f"calib-{agents // 1000}k: {agents} agents, {days} days, {n_train} training runs, "
                       f"{n_heldout} held-out curves; gradient refinement on the first 64"}
    out.update({k: s[k] for k in keys})
    gd = s["gradient_descent"]
    out["gradient_refinement"] = {k: gd[k] for k in ("resim_rel_l2_same_stream",
                                                     "resim_rel_l2_same_stream_median", "seconds")}
    return out


def _initial(sim, pop):
    rec = np.zeros(sim.N, sim.state().dtype)
    rec["t_exp"] = rec["q_until"] = rec["test_day"] = rec["d1"] = rec["d2"] = -32768
    seeds = np.asarray(pop.initial_infected, np.int64)
    rec["stage"][seeds] = 1
    rec["t_exp"][seeds] = -1
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=175, help="timed days")
    ap.add_argument("--warmup", type=int, default=5, help="untimed days before the timed ones")
    ap.add_argument("--workload", default="plain-50M", choices=["plain-50M", "plain-100k"])
    ap.add_argument("--n", type=int, default=None, help="override the agent count (testing)")
    ap.add_argument("--no-extras", action="store_true", help="skip the 100k, batched and CPU legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dense-message", action="store_true",
                    help="time the streaming force of infection every day (no frontier days)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB device copy (PMC counter scale)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(replicates and agent ranges would shard across GPUs; see the design notes).",
              file=sys.stderr)
        sys.exit(2)
    if args.warmup + args.steps > 180:
        sys.exit("warmup + steps must be <= 180 (one run)")
    import torch
    from paper_2110_04421_amd.sim import Simulator
    from synthpop import workload
    k = 2 if args.workload == "plain-50M" else 1
    log(f"generating {args.workload}")
    p, pop = workload(k, n=args.n)
    N = pop.n_agents
    log(f"{N} agents; creating the simulation")
    ehh = household_edges(pop)
    # the throughput is timed on the production path (each day one HIP graph launch);
    # the same days are then run again with HIP events around every kernel for the
    # per-kernel durations (eager launches, so slightly slower as a whole)
    dense = args.dense_message
    with Simulator(p, pop, autotune=True, dense_message=dense) as sim:
        tuning = sim.tuning()
        log(f"warm-up {args.warmup} days, timing {args.steps} days (tiling {tuning})")
        counts, wall = time_days(sim, args.warmup, args.steps)
    log(f"timed {args.steps} days in {wall:.3f} s; again with per-kernel events")
    with Simulator(p, pop, profile=True, autotune=True, dense_message=dense) as sim:
        counts_p, wall_p = time_days(sim, args.warmup, args.steps)
        prof = sim.profile()
    assert np.array_equal(counts, counts_p)
    log(f"profiled {args.steps} days in {wall_p:.3f} s")
    E_days = counts[:, :, 10].sum(axis=1).astype(np.float64)
    E_tot = float(E_days.sum())
    E_mean = float(E_days.mean())
    Einf_mean = float(counts[:, :, 12].sum(axis=1).astype(np.float64).mean())
    C_mean = (E_mean - ehh) / 2.0
    vacc = p["vacc_rate"] > 0
    # infectious agents a day (exposed or infectious, an upper bound of the agents whose
    # code is nonzero): at most N/256 on a day, and its force of infection takes the
    # frontier path, whose bytes depend on which rows hold infectious sources
    n_inf_max = int((counts[:, :, 1] + counts[:, :, 2]).sum(axis=1).max())
    frontier = n_inf_max * 256 <= N and N >= 1 << 20 and not dense
    kernels = {}
    for name, (ms, n) in prof.items():
        if n == 0:
            continue
        avg = ms / n
        b = None if (name == "message" and frontier) else kernel_bytes(name, N, E_mean, C_mean, vacc, Einf_mean)
        kernels[name] = {"ms_per_launch": avg, "launches": n,
                         "algorithmic_GB": None if b is None else b / 1e9,
                         "GB_per_s": (b / 1e9) / (avg / 1e3) if b and avg > 0 else None}
    if frontier:
        kernels["message"]["path"] = "frontier (rows holding an infectious source)"
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_launch"])
    dk = kernels[dom]
    achieved = dk["GB_per_s"] or 0.0
    # (not in counter runs, where the 1 GiB --copy-probe copy must be the only large one)
    copy_gbs = None if args.copy_probe else copy_bandwidth()
    step_bytes = sum((v["algorithmic_GB"] or 0.0) * 1e9 for v in kernels.values())
    step_ms = sum(v["ms_per_launch"] for v in kernels.values())
    line = {
        "metric": METRIC,
        "value": E_tot / wall,
        "unit": "edge-interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "profiled_ms_per_step": wall_p / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "agents": N, "days_timed": args.steps,
                   "edges_per_day": E_mean, "contacts_per_agent_day": E_mean / N,
                   "infectious_source_edges_per_day": Einf_mean, "autotuned_tiling": tuning,
                   "exposed_or_infectious_max": n_inf_max,
                   "force_of_infection": "frontier" if frontier else "streaming",
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom),
                     "algorithmic_bytes_per_launch": dk["algorithmic_GB"] * 1e9,
                     "step_kernels_GB_per_s": (step_bytes / 1e9) / (step_ms / 1e3),
                     "step_kernels_frac": (step_bytes / 1e9) / (step_ms / 1e3) / HBM_PEAK_GBS,
                     "copy_GB_per_s": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs if copy_gbs else None,
                     "step_kernels_frac_of_copy": (step_bytes / 1e9) / (step_ms / 1e3) / copy_gbs
                     if copy_gbs else None},
        "kernels": kernels,
    }
    if not args.no_extras and not dense:
        log("the same days with every edge streamed through the force of infection")
        counts_s, wall_s, msg_ms = streaming_run(p, pop, args.warmup, args.steps)
        assert np.array_equal(counts, counts_s)
        b = kernel_bytes("message", N, E_mean, C_mean, vacc, Einf_mean)
        line["streaming_message"] = {"ms_per_step": wall_s / args.steps * 1e3, "message_ms": msg_ms,
                                     "message_GB_per_s": b / 1e9 / (msg_ms / 1e3),
                                     "message_algorithmic_GB": b / 1e9, "counts_equal": True}
    if args.copy_probe:
        copy_probe()
    if not args.no_extras:
        log("100k-agent runs")
        line["c1"] = c1_run()
        log("batched ensemble vs one by one")
        line["batched"] = batched_vs_plain()
        log("adjoint cost")
        line["adjoint"] = adjoint_cost()
        log("calibration network throughput")
        line["mlp"] = mlp_throughput()
        log("learned calibration against grid search")
        line["calibration"] = calibration_leg()
        log("eleven-stage course at 50M agents")
        line["course"] = course_run()
        log("exposure notification at 50M agents")
        line["notification"] = den_run()
    if not args.no_extras and not args.no_cpu_baseline:
        log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
