"""Philox counter-based random numbers (Salmon, Moraes, Dror, Shaw, "Parallel Random
Numbers: As Easy as 1, 2, 3", SC'11) and the draws the simulator takes from them.

Every random decision of a day is a pure function of (seed, replicate, day, agent,
purpose, lane): the step is therefore a deterministic function of its inputs, and the
oracle can reproduce each draw independently.

Counter layout used by the model (one Philox4x32-10 call = one block of 4 lanes):
    key     = (seed & 0xffffffff, seed >> 32)
    counter = (agent_local_id, day, replicate, (purpose << 24) | block)
Purposes: AGENT (infection / death / test selection / test result in lanes 0..3),
AGENT2 (quarantine dropout, lane 0), VACC (vaccine immunity, lane 0, keyed with the
day of the first dose), OCC and RAND (flat lane 4*block+lane: lane 0 = Poisson
count, lanes 1..k = partners).
"""
from __future__ import annotations

import numpy as np

PURPOSE_AGENT, PURPOSE_AGENT2, PURPOSE_VACC, PURPOSE_OCC, PURPOSE_RAND = 0, 1, 2, 3, 4
PURPOSE_COURSE = 5     # eleven-stage course: block 0 = path at infection, block 1 = durations
PURPOSE_APP = 6        # exposure-notification app access, drawn once (day 0)

# Philox-4x32 multipliers and Weyl key increments (Salmon et al. 2011, table of constants)
M4x32 = (0xD2511F53, 0xCD9E8D57)
W4x32 = (0x9E3779B9, 0xBB67AE85)
# Philox-4x64 constants, used only to pin the generic round against numpy's Philox
M4x64 = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
W4x64 = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def philox4_generic(ctr, key, width, mult, weyl, rounds=10):
    """Plain-integer Philox-4xW: ``rounds`` S-P rounds, the key bumped by the Weyl
    constants between rounds.  One round multiplies words 0 and 2 by the two
    multipliers (full double-width product) and permutes:
        (c0,c1,c2,c3) -> (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)).
    Pure Python; for pins and tiny cases."""
    mask = (1 << width) - 1
    c = [int(x) & mask for x in ctr]
    k = [int(x) & mask for x in key]
    for r in range(rounds):
        if r:
            k = [(k[0] + weyl[0]) & mask, (k[1] + weyl[1]) & mask]
        p0 = mult[0] * c[0]
        p1 = mult[1] * c[2]
        hi0, lo0 = p0 >> width, p0 & mask
        hi1, lo1 = p1 >> width, p1 & mask
        c = [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]
    return tuple(c)


def philox4x32(c0, c1, c2, c3, seed: int):
    """Vectorised Philox4x32-10 over broadcastable uint32 counter words.
    Returns four uint32 arrays.  uint64 arithmetic holds the 32x32-bit products
    exactly."""
    m32 = np.uint64(0xFFFFFFFF)
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64((seed >> 32) & 0xFFFFFFFF)
    c0, c1, c2, c3 = np.broadcast_arrays(*(np.asarray(c, dtype=np.uint64) & m32
                                          for c in (c0, c1, c2, c3)))
    c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
    M0, M1 = np.uint64(M4x32[0]), np.uint64(M4x32[1])
    W0, W1 = np.uint64(W4x32[0]), np.uint64(W4x32[1])
    s32 = np.uint64(32)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & m32
            k1 = (k1 + W1) & m32
        p0 = M0 * c0
        p1 = M1 * c2
        n0 = (p1 >> s32) ^ c1 ^ k0
        n1 = p1 & m32
        n2 = (p0 >> s32) ^ c3 ^ k1
        n3 = p0 & m32
        c0, c1, c2, c3 = n0, n1, n2, n3
    return (c0.astype(np.uint32), c1.astype(np.uint32), c2.astype(np.uint32),
            c3.astype(np.uint32))


def draw_words(seed, agent_local, day, replicate, purpose, block):
    """The 4 lanes of block ``block`` of a purpose (counter layout in the module doc)."""
    word3 = (np.asarray(purpose, np.uint64) << np.uint64(24)) | np.asarray(block, np.uint64)
    return philox4x32(np.asarray(agent_local, np.int64).astype(np.uint64),
                      np.asarray(day, np.int64).astype(np.uint64) & np.uint64(0xFFFFFFFF),
                      np.asarray(replicate, np.uint64), word3, seed)


def lane(seed, agent_local, day, replicate, purpose, flat_lane):
    """uint32 word at flat lane index ``4*block + lane``."""
    flat_lane = np.asarray(flat_lane, np.int64)
    w = draw_words(seed, agent_local, day, replicate, purpose, flat_lane // 4)
    sel = flat_lane % 4
    stacked = np.stack(np.broadcast_arrays(*w), axis=0)
    return np.take_along_axis(stacked, np.broadcast_to(sel, stacked.shape[1:])[None], 0)[0]


def uniform(x):
    """Map a 32-bit word to (0, 1): u = (floor(x / 2^9) + 1/2) * 2^-23.
    Odd multiples of 2^-24, exactly representable in FP32 and FP64."""
    x = np.asarray(x, np.uint64)
    return ((x >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23
