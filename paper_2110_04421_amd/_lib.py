"""ctypes view of libabm.so (include/abm.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libabm.so")

ABI_VERSION = 4
HARD, SOFT = 0, 1
SEIRM, COURSE = 0, 1
NC = 16
N_AGE, N_OCC, N_THETA, N_DUR = 9, 23, 10, 9
NEVER = -32768
FLAG_PROFILE, FLAG_NO_GRAPH, FLAG_CLAIM_BUILDER, FLAG_AUTOTUNE, FLAG_MIN_LDS_ROOM = 1, 2, 4, 8, 16
FLAG_DENSE_MESSAGE, FLAG_FRONTIER_ANY_SIZE, FLAG_STRAIGHT_THROUGH, FLAG_TWO_TILE_LEAVES = 32, 64, 128, 256
FLAG_SEGMENT_VPLAN = 512
(C_S, C_E, C_I, C_R, C_M, C_NEW, C_TESTS, C_POS, C_DOSE1, C_DOSE2, C_EDGES, C_NEAR,
 C_INF_EDGES, C_HOSP, C_ICU, C_NOTIFIED) = range(NC)
(GET_STATE, GET_LAMBDA, GET_CODE, GET_ROWPTR, GET_COL, GET_W, GET_ATAB, GET_POISSON, GET_DAY,
 GET_LATCH, GET_SOFT_S, GET_COEF, GET_TUNING) = range(13)
MLP_IN, MLP_H, MLP_OUT = 192, 256, 16
MLP_NPARAM = 256 * 192 + 256 + 256 * 256 + 256 + 16 * 256 + 16
MLP_NOALLOC_MAX_BATCH = 1024

ERRORS = {0: "ok", -1: "invalid argument", -2: "ABI mismatch", -3: "workspace too small",
          -4: "edge capacity exceeded", -5: "HIP runtime error", -6: "call out of order"}

STATE_DTYPE = np.dtype([("stage", "u1"), ("flags", "u1"), ("vacc", "u1"), ("course", "u1"),
                        ("t_exp", "<i2"), ("q_until", "<i2"), ("test_day", "<i2"),
                        ("d1", "<i2"), ("d2", "<i2"), ("t_next", "<i2")])
assert STATE_DTYPE.itemsize == 16


class AbmParams(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("abi_version", C.c_uint32),
        ("n_steps", C.c_int32), ("mode", C.c_int32), ("seed", C.c_uint64),
        ("dt", C.c_float), ("kappa", C.c_float),
        ("gamma_shape", C.c_double), ("gamma_scale", C.c_double),
        ("A_stage", C.c_double * 5),
        ("w_household", C.c_float), ("w_occupation", C.c_float), ("w_random", C.c_float),
        ("mu_random", C.c_double * N_AGE), ("mu_occupation", C.c_double * N_OCC),
        ("p_death", C.c_float * N_AGE),
        ("e_days", C.c_int32), ("i_days", C.c_int32),
        ("quarantine_days", C.c_int32), ("test_delay", C.c_int32),
        ("quarantine_dropout", C.c_float), ("test_rate", C.c_float), ("test_sensitivity", C.c_float),
        ("vacc_rate", C.c_double), ("vacc_trigger", C.c_double),
        ("eff1", C.c_float), ("eff2", C.c_float),
        ("dose_lag", C.c_int32), ("strategy", C.c_int32),
        ("gumbel_tau", C.c_float), ("checkpoint_every", C.c_int32),
        ("edge_capacity", C.c_int64), ("flags", C.c_int32), ("disease_model", C.c_int32),
        ("p_asym", C.c_float * N_AGE), ("p_severe", C.c_float * N_AGE), ("p_hosp", C.c_float * N_AGE),
        ("p_icu", C.c_float * N_AGE), ("p_die", C.c_float * N_AGE),
        ("A_asym", C.c_double),
        ("dur_shift", C.c_int32 * N_DUR), ("pad_", C.c_int32),
        ("dur_extra", C.c_double * N_DUR),
        ("test_delay_max", C.c_int32), ("app_adoption", C.c_float), ("den_compliance", C.c_float),
        ("den_window", C.c_int32),
        ("vacc_immunity", C.c_int32),
    ]


class AbmPopulation(C.Structure):
    _fields_ = [
        ("n_replicates", C.c_int32), ("n_households", C.c_int32), ("n_workplaces", C.c_int32),
        ("reserved", C.c_int32),
        ("agent_offset", C.c_void_p), ("age", C.c_void_p), ("hh_start", C.c_void_p),
        ("occupation", C.c_void_p), ("wp_start", C.c_void_p), ("wp_members", C.c_void_p),
        ("R", C.c_void_p), ("susceptibility", C.c_void_p), ("dose2_delay", C.c_void_p),
        ("init_offset", C.c_void_p), ("initial_infected", C.c_void_p), ("stream", C.c_void_p),
    ]


_lib = None


def lib():
    """Load libabm.so; raise if it was not built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2110_04421_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, f32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_float, C.c_size_t
    sig = {
        "abm_workspace_size": (C.c_int, [vp, vp, C.POINTER(sz)]),
        "abm_create": (C.c_int, [vp, vp, vp, sz, vp, C.POINTER(vp)]),
        "abm_step": (C.c_int, [vp, i32]),
        "abm_run": (C.c_int, [vp, i32, vp, vp]),
        "abm_grad": (C.c_int, [vp, vp, vp]),
        "abm_set_theta": (C.c_int, [vp, vp]),
        "abm_get": (C.c_int, [vp, i32, vp, sz]),
        "abm_set_state": (C.c_int, [vp, i32, vp, vp, sz]),
        "abm_sync": (C.c_int, [vp]),
        "abm_destroy": (None, [vp]),
        "abm_error_string": (C.c_char_p, [C.c_int]),
        "abm_last_error": (C.c_char_p, [vp]),
        "abm_profile_kernels": (C.c_int, [vp]),
        "abm_profile_name": (C.c_char_p, [vp, i32]),
        "abm_profile_get": (C.c_int, [vp, vp, vp]),
        "abm_profile_reset": (C.c_int, [vp]),
        "abm_philox": (C.c_int, [u64, vp, i64, vp, vp]),
        "abm_mlp_workspace_size": (C.c_int, [i32, C.POINTER(sz)]),
        "abm_mlp_forward": (C.c_int, [vp, sz, vp, vp, i32, vp, vp]),
        "abm_mlp_forward_noalloc": (C.c_int, [vp, vp, i32, vp, vp]),
        "abm_mlp_backward": (C.c_int, [vp, sz, vp, vp, i32, i32, vp, vp, vp]),
        "abm_mlp_adam": (C.c_int, [vp, vp, vp, vp, vp, f32, f32, f32, f32, i32, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def exported_symbols():
    """Names the header declares (checked against the shared library by the tests)."""
    return ["abm_workspace_size", "abm_create", "abm_step", "abm_run", "abm_grad", "abm_set_theta", "abm_get",
            "abm_set_state", "abm_sync", "abm_destroy", "abm_error_string", "abm_last_error",
            "abm_profile_kernels", "abm_profile_name", "abm_profile_get", "abm_profile_reset",
            "abm_philox", "abm_mlp_workspace_size", "abm_mlp_forward", "abm_mlp_forward_noalloc",
            "abm_mlp_backward", "abm_mlp_adam"]


class AbmError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{ERRORS.get(code, code)} ({code}): {msg}")
        self.code = code


def make_params(cfg: dict, flags: int = 0) -> AbmParams:
    p = AbmParams()
    p.struct_size = C.sizeof(AbmParams)
    p.abi_version = ABI_VERSION
    p.n_steps = int(cfg["n_steps"])
    p.mode = int(cfg.get("mode", HARD))
    p.seed = int(cfg["seed"])
    p.dt = float(cfg["dt"])
    p.kappa = float(cfg["kappa"])
    p.gamma_shape = float(cfg["gamma_shape"])
    p.gamma_scale = float(cfg["gamma_scale"])
    for k in range(5):
        p.A_stage[k] = float(cfg["A_stage"][k])
    p.w_household = float(cfg["w_household"])
    p.w_occupation = float(cfg["w_occupation"])
    p.w_random = float(cfg["w_random"])
    for k in range(N_AGE):
        p.mu_random[k] = float(cfg["mu_random"][k])
        p.p_death[k] = float(cfg["p_death"][k])
    for k in range(N_OCC):
        p.mu_occupation[k] = float(cfg["mu_occupation"][k])
    p.e_days = int(cfg["e_days"])
    p.i_days = int(cfg["i_days"])
    p.quarantine_days = int(cfg["quarantine_days"])
    p.test_delay = int(cfg["test_delay"])
    p.quarantine_dropout = float(cfg["quarantine_dropout"])
    p.test_rate = float(cfg["test_rate"])
    p.test_sensitivity = float(cfg["test_sensitivity"])
    p.vacc_rate = float(cfg["vacc_rate"])
    p.vacc_trigger = float(cfg["vacc_trigger"])
    p.eff1 = float(cfg["eff1"])
    p.eff2 = float(cfg["eff2"])
    p.dose_lag = int(cfg["dose_lag"])
    p.strategy = int(cfg["strategy"])
    p.gumbel_tau = float(cfg.get("gumbel_tau", 0.5))
    p.checkpoint_every = int(cfg.get("checkpoint_every", 10))
    p.edge_capacity = int(cfg.get("edge_capacity", 0))
    p.flags = int(flags)
    p.disease_model = int(cfg.get("disease_model", SEIRM))
    for name in ("p_asym", "p_severe", "p_hosp", "p_icu", "p_die"):
        v = cfg.get(name, [0.0] * N_AGE)
        for k in range(N_AGE):
            getattr(p, name)[k] = float(v[k])
    p.A_asym = float(cfg.get("A_asym", 0.0))
    shift, extra = cfg.get("dur_shift", [1] * N_DUR), cfg.get("dur_extra", [0.0] * N_DUR)
    for k in range(N_DUR):
        p.dur_shift[k] = int(shift[k])
        p.dur_extra[k] = float(extra[k])
    p.test_delay_max = int(cfg.get("test_delay_max", cfg["test_delay"]))
    p.app_adoption = float(cfg.get("app_adoption", 0.0))
    p.den_compliance = float(cfg.get("den_compliance", 0.0))
    p.den_window = int(cfg.get("den_window", 7))
    p.vacc_immunity = int(cfg.get("vacc_immunity", 0))
    return p


def make_population(pop):
    """(AbmPopulation, keep-alive list) from a synthpop.Population-like object."""
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(np.asarray(x, dtype=dt))
        keep.append(a)
        return a.ctypes.data if a.size else None

    P = AbmPopulation()
    P.n_replicates = int(np.asarray(pop.agent_offset).size - 1)
    P.n_households = int(np.asarray(pop.hh_start).size - 1)
    P.n_workplaces = int(np.asarray(pop.wp_start).size - 1)
    P.agent_offset = arr(pop.agent_offset, np.int64)
    P.age = arr(pop.age, np.uint8)
    P.hh_start = arr(pop.hh_start, np.int32)
    P.occupation = arr(pop.occupation, np.uint8)
    P.wp_start = arr(pop.wp_start, np.int32)
    P.wp_members = arr(pop.wp_members, np.int32) if np.asarray(pop.wp_members).size else None
    P.R = arr(pop.R, np.float32)
    P.susceptibility = arr(np.asarray(pop.susceptibility, np.float32).reshape(-1), np.float32)
    P.dose2_delay = arr(pop.dose2_delay, np.int32)
    P.init_offset = arr(pop.init_offset, np.int64)
    P.initial_infected = arr(pop.initial_infected, np.int32) if np.asarray(pop.initial_infected).size else None
    stream = getattr(pop, "stream", None)
    P.stream = arr(stream, np.uint32) if stream is not None else None
    return P, keep
