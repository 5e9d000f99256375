"""Shared test helpers: state conversion between the oracle and the library, skips."""
import numpy as np
import pytest

from oracle import step as ostep


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def require_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def to_records(st, dtype):
    """Oracle state dict -> array of the library's 16-byte agent records."""
    N = st["stage"].size
    rec = np.zeros(N, dtype)
    rec["stage"] = st["stage"]
    rec["flags"] = (st["pending"].astype(np.uint8) | (st["positive"].astype(np.uint8) << 1)
                    | (st["notified"].astype(np.uint8) << 2))
    rec["vacc"] = st["vacc"]
    for k in ("t_exp", "q_until", "test_day", "d1", "d2"):
        rec[k] = st[k]
    rec["course"] = st["course"]
    rec["t_next"] = st["t_next"]
    return rec


def from_records(rec, latch):
    """Library records -> oracle state dict."""
    st = dict(stage=rec["stage"].astype(np.int64), t_exp=rec["t_exp"].astype(np.int64),
              q_until=rec["q_until"].astype(np.int64), test_day=rec["test_day"].astype(np.int64),
              pending=(rec["flags"] & 1).astype(bool), positive=(rec["flags"] & 2).astype(bool),
              vacc=rec["vacc"].astype(np.int64), d1=rec["d1"].astype(np.int64),
              d2=rec["d2"].astype(np.int64), latch=np.asarray(latch, bool).copy(),
              course=rec["course"].astype(np.int64), t_next=rec["t_next"].astype(np.int64),
              notified=(rec["flags"] & 4).astype(bool))
    return st


FIELDS = ("stage", "t_exp", "q_until", "test_day", "pending", "positive", "vacc", "d1", "d2",
          "course", "t_next", "notified")


def state_mismatch(a, b):
    """Agents whose state differs between two oracle-format states."""
    bad = np.zeros(a["stage"].size, bool)
    for k in FIELDS:
        bad |= a[k] != b[k]
    return np.flatnonzero(bad)


def lam_close(lam_gpu, lam_ora, rtol=1e-5):
    lam_gpu = lam_gpu.astype(np.float64)
    zero = lam_ora == 0
    ok_zero = np.all(lam_gpu[zero] == 0)
    err = np.abs(lam_gpu - lam_ora) / np.maximum(np.abs(lam_ora), 1e-300)
    return ok_zero and bool(np.all(err[~zero] <= rtol)), float(err[~zero].max(initial=0.0))


def lockstep(make_sim, p, pop, T, graph=True, allow_near=True, check_csr_every=0):
    """Step GPU and oracle together; resync the GPU from the oracle after a counted
    near-threshold disagreement.  ``make_sim(p, pop, graph=...)`` opens the GPU
    simulator.  Returns (near draws seen, worst lambda rel err, doses [T, R, 2]: first
    and second doses given per day and replicate)."""
    m = ostep.Model(pop, p)
    st = m.init_state()
    prev = np.zeros((m.nrep, ostep.NC), np.int64)
    m.put_counts(prev, st)
    near_total, worst = 0, 0.0
    doses = np.zeros((T, m.nrep, 2), np.int64)
    with make_sim(p, pop, graph=graph) as s:
        for t in range(T):
            cg = s.run(1)[0]
            doses[t] = cg[:, [ostep.C_DOSE1, ostep.C_DOSE2]]
            new, out = m.step(st, t, prev)
            assert np.array_equal(s.code().astype(np.int64), out["code"]), f"codes differ on day {t}"
            ok, err = lam_close(s.lam(), out["lam"])
            worst = max(worst, err)
            assert ok, f"lambda rel err {err} on day {t}"
            if check_csr_every and t % check_csr_every == 0:
                rp, col, w = s.csr()
                assert np.array_equal(col.astype(np.int64), out["graph"][1])
            gst = from_records(s.state(), s.latch())
            bad = state_mismatch(gst, new)
            near = (st["stage"] == 0) & ~out["immune"] & (np.abs(out["u0"] - out["prob"]) <= 1e-6)
            near_total += int(near.sum())
            assert set(bad.tolist()) <= set(np.flatnonzero(near).tolist()), \
                f"day {t}: {bad.size} agents differ outside the near-threshold window"
            assert np.array_equal(gst["latch"], new["latch"])
            if bad.size:
                assert allow_near
                s.set_state(t + 1, new["latch"].astype(np.uint8), to_records(new, s.state().dtype))
            else:
                keep = [c for c in range(ostep.NC) if c != ostep.C_NEAR]
                assert np.array_equal(cg[:, keep], out["counts"][:, keep]), f"counts differ on day {t}"
            st, prev = new, out["counts"]
    return near_total, worst, doses
