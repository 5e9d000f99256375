"""Host-side checks of the C ABI that need no GPU: the library loads and exports every
function include/abm.h declares, the ctypes structs have the C layout, and parameter,
ABI and workspace errors are reported before any device work."""
import ctypes as C
import dataclasses
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2110_04421_amd import _lib as L
from synthpop import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "abm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(abm_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = L.lib()
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(L.exported_symbols()) == declared


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "abm.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(abm_params),'
                   ' offsetof(abm_params, mu_random), offsetof(abm_params, vacc_rate),'
                   ' offsetof(abm_params, edge_capacity), sizeof(abm_population));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals == [C.sizeof(L.AbmParams), L.AbmParams.mu_random.offset, L.AbmParams.vacc_rate.offset,
                    L.AbmParams.edge_capacity.offset, C.sizeof(L.AbmPopulation)]


def _ws(p, pop, flags=0):
    lib = L.lib()
    P = L.make_params(p, flags)
    Q, keep = L.make_population(pop)
    n = C.c_size_t(0)
    rc = lib.abm_workspace_size(C.byref(P), C.byref(Q), C.byref(n))
    return rc, n.value, P, Q, keep


def test_workspace_size_and_errors():
    p, pop = workload(0)
    rc, n, *_ = _ws(p, pop)
    assert rc == 0 and n > 1000 * 61
    rc, *_ = _ws(dict(p, e_days=40, i_days=30), pop)
    assert rc == -1
    rc, *_ = _ws(dict(p, mu_random=[100.0] * 9), pop)
    assert rc == -1
    rc, *_ = _ws(dict(p, test_rate=0.1, test_delay=0), pop)
    assert rc == -1
    bad = workload(0)[1]
    bad.hh_start = bad.hh_start.copy()
    bad.hh_start[-1] -= 1
    rc, *_ = _ws(p, bad)
    assert rc == -1
    rc, *_ = _ws(dict(p, edge_capacity=2**31), pop)
    assert rc == -4
    rc, *_ = _ws(dict(p, vacc_immunity=1), pop)                     # needs the course model
    assert rc == -1
    rc, *_ = _ws(dict(p, vacc_immunity=1, disease_model=1), pop)
    assert rc == 0
    rc, *_ = _ws(dict(p, vacc_immunity=2, disease_model=1), pop)
    assert rc == -1
    # replicates are separate populations: a workplace may not span two of them
    p3, pop3 = workload(3, n=3000, n_rep=2)
    assert _ws(p3, pop3)[0] == 0
    cross = dataclasses.replace(pop3, wp_members=pop3.wp_members.copy())
    first = int(pop3.wp_start[0])
    cross.wp_members[first] = int(pop3.agent_offset[1]) + 5 if pop3.wp_members[first] < pop3.agent_offset[1] else 5
    assert _ws(p3, cross)[0] == -1


def test_high_contact_means_take_the_claim_builder():
    """At the validator's largest contact means a batch's draws exceed the generation
    pass's LDS room, so the layout is the claim builder's (no partition buffers)."""
    p, pop = workload(1, n=5000)
    hi = dict(p, mu_random=[40.0] * 9, mu_occupation=[40.0] * 23)
    rc, n_hi, *_ = _ws(hi, pop)
    rc2, n_claim, *_ = _ws(hi, pop, L.FLAG_CLAIM_BUILDER)
    assert rc == 0 and rc2 == 0 and n_hi == n_claim
    rc, n_lo, *_ = _ws(p, pop)
    rc2, n_lo_claim, *_ = _ws(p, pop, L.FLAG_CLAIM_BUILDER)
    assert n_lo > n_lo_claim                  # the default means partition


def test_int16_day_fields_stay_in_range():
    p, pop = workload(0)
    assert _ws(dict(p, n_steps=30000, quarantine_days=2767), pop)[0] == 0
    assert _ws(dict(p, n_steps=30000, quarantine_days=2768), pop)[0] == -1


def test_abi_mismatch_and_small_workspace_fail_before_device_work():
    lib = L.lib()
    p, pop = workload(0)
    rc, n, P, Q, keep = _ws(p, pop)
    P.struct_size = P.struct_size - 8
    h = C.c_void_p()
    assert lib.abm_workspace_size(C.byref(P), C.byref(Q), C.byref(C.c_size_t())) == -2
    assert lib.abm_create(C.byref(P), C.byref(Q), C.c_void_p(16), n, None, C.byref(h)) == -2
    assert b"mismatch" in lib.abm_last_error(h)
    lib.abm_destroy(h)
    P.struct_size = C.sizeof(L.AbmParams)
    h = C.c_void_p()
    assert lib.abm_create(C.byref(P), C.byref(Q), C.c_void_p(16), n - 1, None, C.byref(h)) == -3
    assert lib.abm_step(h, 1) == -3          # sticky
    lib.abm_destroy(h)


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        L.lib()


def test_relaxed_incidence_rejects_a_wrong_parameter_shape():
    import torch
    from paper_2110_04421_amd.autograd import relaxed_incidence
    from synthpop import workload
    p, pop = workload(4, n=1000, n_steps=5)
    with pytest.raises(ValueError):
        relaxed_incidence(torch.zeros(1, 9, dtype=torch.float64), p, pop, 5)


def test_header_constants_match_the_binding(tmp_path):
    """The flags, count slots, abm_get items and the ABI version the binding uses are
    the header's."""
    names = {"ABM_ABI_VERSION": L.ABI_VERSION, "ABM_NC": L.NC, "ABM_C_INF_EDGES": L.C_INF_EDGES,
             "ABM_C_HOSP": L.C_HOSP, "ABM_C_ICU": L.C_ICU, "ABM_C_NOTIFIED": L.C_NOTIFIED,
             "ABM_GET_COL": L.GET_COL, "ABM_GET_W": L.GET_W, "ABM_GET_DAY": L.GET_DAY,
             "ABM_FLAG_PROFILE": L.FLAG_PROFILE, "ABM_FLAG_NO_GRAPH": L.FLAG_NO_GRAPH,
             "ABM_FLAG_CLAIM_BUILDER": L.FLAG_CLAIM_BUILDER, "ABM_FLAG_AUTOTUNE": L.FLAG_AUTOTUNE,
             "ABM_FLAG_MIN_LDS_ROOM": L.FLAG_MIN_LDS_ROOM, "ABM_FLAG_DENSE_MESSAGE": L.FLAG_DENSE_MESSAGE,
             "ABM_FLAG_FRONTIER_ANY_SIZE": L.FLAG_FRONTIER_ANY_SIZE,
             "ABM_FLAG_TWO_TILE_LEAVES": L.FLAG_TWO_TILE_LEAVES,
             "ABM_FLAG_SEGMENT_VPLAN": L.FLAG_SEGMENT_VPLAN, "ABM_DISEASE_COURSE": L.COURSE,
             "ABM_IMMUNITY_ASYMPTOMATIC": 1}
    src = tmp_path / "k.c"
    body = "".join(f'printf("%ld\\n", (long)({n}));' for n in names)
    src.write_text('#include "abm.h"\n#include <stdio.h>\nint main(void){' + body + 'return 0;}\n')
    exe = tmp_path / "k"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert dict(zip(names, vals)) == names
