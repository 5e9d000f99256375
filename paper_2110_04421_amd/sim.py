"""Python face of libabm: a ``Simulator`` over the C ABI.

PyTorch supplies the device workspace and the stream; every step of the simulation
runs in the library's HIP kernels.  Nothing here computes the model.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libabm needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


class Simulator:
    """One simulation (possibly many concatenated replicates) on the current GPU.

    ``params``: flat parameter dict (see synthpop.configs); ``pop``: population object with
    the arrays of abm_population.  ``profile`` times every kernel with HIP events;
    ``graph=False`` launches the day's kernels eagerly instead of replaying a HIP graph;
    ``claim_builder`` selects the per-edge atomic-claim graph builder; ``autotune`` times
    the force-of-infection kernel's tilings at create and keeps the fastest;
    ``min_lds_room`` (a test aid) gives the graph builder's level-1 scatter and row pass
    their smallest LDS and register room, which exercises their direct-write and re-read
    paths;
    ``dense_message`` streams every edge through the force-of-infection kernel every day
    (by default, with 2^20 agents or more, a day with at most N/256 infectious agents sums
    only the rows that hold an infectious source; the result is bitwise the same);
    ``frontier_any_size`` (a test aid) allows that path at any population size;
    ``straight_through`` (relaxed mode) takes the hard infection draw forward and the
    relaxed sample's derivative in the adjoint; ``two_tile_leaves`` (a test aid) gives
    the graph builder the two-tile leaves it takes by itself beyond 2^25 agents;
    ``segment_vplan`` (a test aid) plans the vaccination doses by segments of 256 tiles,
    as is done by itself above 2^19 agents a replicate.
    """

    def __init__(self, params: dict, pop, *, profile: bool = False, graph: bool = True,
                 claim_builder: bool = False, autotune: bool = False, min_lds_room: bool = False,
                 dense_message: bool = False, frontier_any_size: bool = False,
                 straight_through: bool = False, two_tile_leaves: bool = False,
                 segment_vplan: bool = False, stream=None):
        torch = _torch()
        self._lib = L.lib()
        flags = ((L.FLAG_PROFILE if profile else 0) | (0 if graph else L.FLAG_NO_GRAPH)
                 | (L.FLAG_CLAIM_BUILDER if claim_builder else 0)
                 | (L.FLAG_AUTOTUNE if autotune else 0)
                 | (L.FLAG_MIN_LDS_ROOM if min_lds_room else 0)
                 | (L.FLAG_DENSE_MESSAGE if dense_message else 0)
                 | (L.FLAG_FRONTIER_ANY_SIZE if frontier_any_size else 0)
                 | (L.FLAG_STRAIGHT_THROUGH if straight_through else 0)
                 | (L.FLAG_TWO_TILE_LEAVES if two_tile_leaves else 0)
                 | (L.FLAG_SEGMENT_VPLAN if segment_vplan else 0))
        self.params = dict(params)
        self._p = L.make_params(params, flags)
        self._pop, self._keep = L.make_population(pop)
        self.N = int(np.asarray(pop.agent_offset)[-1])
        self.R = int(np.asarray(pop.agent_offset).size - 1)
        self.T = int(params["n_steps"])
        nbytes = C.c_size_t(0)
        self._check(self._lib.abm_workspace_size(C.byref(self._p), C.byref(self._pop), C.byref(nbytes)))
        self.ws_bytes = int(nbytes.value)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = self._lib.abm_create(C.byref(self._p), C.byref(self._pop), C.c_void_p(self.ws.data_ptr()),
                                  self.ws_bytes, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._h = h
        if rc != 0:
            msg = self._lib.abm_last_error(h).decode() if h.value else ""
            self.close()
            raise L.AbmError(rc, msg)
        self._keep = None          # host arrays were copied at create

    # -- plumbing -------------------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            msg = ""
            if getattr(self, "_h", None) is not None and self._h.value:
                msg = self._lib.abm_last_error(self._h).decode()
            raise L.AbmError(rc, msg)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.abm_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- running --------------------------------------------------------------------
    def step(self, n_days: int = 1):
        """Enqueue n_days (asynchronous)."""
        self._check(self._lib.abm_step(self._h, int(n_days)))

    def run(self, n_days: int):
        """Run n_days; hard mode returns counts [n_days, R, NC] (int64), soft mode the
        relaxed daily incidence [R, n_days] (float32)."""
        if int(self.params.get("mode", 0)) == L.SOFT:
            out = np.zeros((self.R, n_days), np.float32)
            self._check(self._lib.abm_run(self._h, int(n_days), None, out.ctypes.data))
            return out
        out = np.zeros((n_days, self.R, L.NC), np.int64)
        self._check(self._lib.abm_run(self._h, int(n_days), out.ctypes.data, None))
        return out

    def grad(self, dL):
        """Soft mode: d loss / d(R, S_0..S_8) per replicate, given dL/d incidence [R, T]."""
        dL = np.ascontiguousarray(dL, np.float32)
        out = np.zeros((self.R, L.N_THETA), np.float32)
        self._check(self._lib.abm_grad(self._h, dL.ctypes.data, out.ctypes.data))
        return out

    def set_theta(self, theta):
        """Soft mode: new (R, S_0..S_8) per replicate [R, 10] and a rewind to day 0, so
        that the next run starts over at these parameters."""
        th = np.ascontiguousarray(theta, np.float32)
        if th.shape != (self.R, L.N_THETA):
            raise ValueError(f"theta must be [{self.R}, {L.N_THETA}], got {th.shape}")
        self._check(self._lib.abm_set_theta(self._h, th.ctypes.data))

    def sync(self):
        self._check(self._lib.abm_sync(self._h))

    # -- inspection -----------------------------------------------------------------
    def _get(self, what, dtype, n):
        out = np.empty(n, dtype)
        self._check(self._lib.abm_get(self._h, what, out.ctypes.data, out.nbytes))
        return out

    def day(self) -> int:
        return int(self._get(L.GET_DAY, np.int32, 1)[0])

    def state(self) -> np.ndarray:
        return self._get(L.GET_STATE, L.STATE_DTYPE, self.N)

    def lam(self) -> np.ndarray:
        return self._get(L.GET_LAMBDA, np.float32, self.N)

    def code(self) -> np.ndarray:
        return self._get(L.GET_CODE, np.uint8, self.N)

    def csr(self):
        rp = self._get(L.GET_ROWPTR, np.int32, self.N + 1)
        E = int(rp[-1])
        return rp, self._get(L.GET_COL, np.int32, E), self._get(L.GET_W, np.float32, E)

    def atab(self) -> np.ndarray:
        return self._get(L.GET_ATAB, np.float32, 64)

    def poisson_tables(self) -> np.ndarray:
        return self._get(L.GET_POISSON, np.uint32, 32 * 64).reshape(32, 64)

    def latch(self) -> np.ndarray:
        return self._get(L.GET_LATCH, np.uint8, self.R)

    def coef(self) -> np.ndarray:
        return self._get(L.GET_COEF, np.float32, self.R * 9).reshape(self.R, 9)

    def tuning(self) -> dict:
        v = self._get(L.GET_TUNING, np.int32, 3)
        return {"message_chunk": int(v[0]), "message_grid": int(v[1]), "message_shape": int(v[2])}

    def soft_s(self) -> np.ndarray:
        return self._get(L.GET_SOFT_S, np.float32, self.N)

    def set_state(self, day: int, latch, state: np.ndarray):
        latch = np.ascontiguousarray(latch, np.uint8)
        state = np.ascontiguousarray(state, L.STATE_DTYPE)
        self._check(self._lib.abm_set_state(self._h, int(day), latch.ctypes.data,
                                            state.ctypes.data, state.size))

    def profile(self):
        """{kernel name: (total ms, launches)} since create/reset (profile mode)."""
        K = self._lib.abm_profile_kernels(self._h)
        ms = np.zeros(K, np.float64)
        n = np.zeros(K, np.int64)
        self._check(self._lib.abm_profile_get(self._h, ms.ctypes.data, n.ctypes.data))
        return {self._lib.abm_profile_name(self._h, k).decode(): (float(ms[k]), int(n[k]))
                for k in range(K)}

    def profile_reset(self):
        self._check(self._lib.abm_profile_reset(self._h))


def philox(seed: int, ctr: np.ndarray) -> np.ndarray:
    """Philox4x32-10 of counters ctr [n, 4] (uint32) computed on the GPU."""
    torch = _torch()
    lib = L.lib()
    c = torch.from_numpy(np.ascontiguousarray(ctr, np.uint32).view(np.int32)).cuda()
    out = torch.empty_like(c)
    st = torch.cuda.current_stream()
    rc = lib.abm_philox(int(seed), C.c_void_p(c.data_ptr()), int(c.shape[0]),
                        C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream))
    if rc != 0:
        raise L.AbmError(rc)
    st.synchronize()
    return out.cpu().numpy().view(np.uint32)
