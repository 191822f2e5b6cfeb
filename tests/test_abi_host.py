"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol of include/qw.h, applies the Table II legality gates and emits the
refusal record of the EVAL-7 example."""
import json
import os
import re

import pytest

from paper_2609_23664_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def test_header_symbols_exported():
    hdr = open(os.path.join(ROOT, "include", "qw.h")).read()
    declared = set(re.findall(r"^(?:int|uint64_t|const char \*)\s*(qw_[a-z0-9_]+)\s*\(", hdr, re.M))
    assert len(declared) >= 20
    L = B.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(B.EXPORTED)
    assert B.lib().qw_version().decode().startswith("libqw")


_KIND = {"STATEVECTOR_BOUNDARY_STATE": B.QW_KIND_STATEVECTOR, "TABLEAU_BOUNDARY_STATE": B.QW_KIND_TABLEAU}
_BACK = {"SV": B.QW_BACKEND_SV, "STAB": B.QW_BACKEND_STAB_ONLY, "UNKNOWN": B.QW_BACKEND_UNKNOWN}
_EXACT = {"EXACT": B.QW_EXACT, "APPROX": B.QW_APPROX, "UNKNOWN": B.QW_EXACTNESS_UNKNOWN}


def test_table2_truth_table():
    rows = json.load(open(os.path.join(GOLDEN, "table2_legality.json")))["rows"]
    for r in rows:
        rc, js = B.legality_check(_KIND[r["source_kind"]], _EXACT[r["exactness"]],
                                  _BACK[r["source_backend"]], 10, _KIND[r["target_kind"]],
                                  _BACK[r["target_backend"]])
        if r["outcome"] == "EXACT":
            assert rc == B.QW_OK, (r["case"], js)
        else:
            assert rc == B.QW_E_REFUSED, r["case"]
            rec = json.loads(js)
            for f in ("reason", "detail", "source_kind", "target_kind", "source_backend", "target_backend"):
                assert f in rec


def test_eval7_refusal_record():
    g = json.load(open(os.path.join(GOLDEN, "refusal_eval7.json")))
    rc, js = B.legality_check(B.QW_KIND_STATEVECTOR, B.QW_EXACT, B.QW_BACKEND_STAB_ONLY, 4,
                              B.QW_KIND_STATEVECTOR, B.QW_BACKEND_STAB_ONLY)
    assert rc == B.QW_E_REFUSED
    rec = json.loads(js)
    assert list(rec.keys())[:6] == g["fields"]
    assert rec["reason"] == g["reason"]
    assert rec["source_kind"] == g["source_kind"] and rec["target_kind"] == g["target_kind"]
    assert rec["detail"] == "SV on stabilizer-only backend not supported."


def test_exactness_gate_runs_first():
    rc, js = B.legality_check(B.QW_KIND_STATEVECTOR, B.QW_APPROX, B.QW_BACKEND_UNKNOWN, 4,
                              B.QW_KIND_TABLEAU, B.QW_BACKEND_UNKNOWN)
    assert rc == B.QW_E_REFUSED and json.loads(js)["reason"] == "NON_EXACT_ARTIFACT"
    rc, js = B.legality_check(B.QW_KIND_STATEVECTOR, B.QW_EXACT, B.QW_BACKEND_UNKNOWN, 4,
                              B.QW_KIND_TABLEAU, B.QW_BACKEND_SV)
    assert json.loads(js)["reason"] == "UNKNOWN_BACKEND"


def test_bad_gates_rejected_by_planner():
    with pytest.raises(B.QwError):
        B.plan_describe(5, [("RY", (5,), 0.1)])
    with pytest.raises(B.QwError):
        B.plan_describe(5, [("CNOT", (2, 2), 0.0)])
    with pytest.raises(B.QwError):
        B.plan_describe(5, [("RY", (1,), float("nan"))])


def test_task_records_marshalled_field_by_field():
    """The qw_task records of a call: gate pointer and count, slot, a zero
    reserved word and the 32 provenance bytes (shorter ones zero-padded,
    longer ones refused), for explicit provenances and for none."""
    import ctypes

    g = [("RY", (0,), 0.25), ("CNOT", (0, 1), 0.0)]
    arrs_in = [B.GateArray(g), B.GateArray(g[:1]), B.GateArray([])]
    provs = [bytes(range(32)), b"\x07" * 5, bytes(32)]
    arrs, tasks = B._task_array(arrs_in, [4, 0, 9], None, provs)
    raw = bytes(tasks)
    size = ctypes.sizeof(B.QwTask)
    for k, (a, p) in enumerate(zip(arrs_in, provs)):
        t = tasks[k]
        assert ctypes.cast(t.gates, ctypes.c_void_p).value == ctypes.cast(a.ptr, ctypes.c_void_p).value
        assert t.n_gates == len(a) and t.reserved == 0
        assert t.dst_slot == [4, 0, 9][k]
        off = k * size + B.QwTask.expect_prov.offset
        assert raw[off:off + 32] == p.ljust(32, b"\0")
    _, none = B._task_array(arrs_in[:1], [1], None, None)
    assert bytes(none[0].expect_prov) == bytes(32)
    with pytest.raises(ValueError):
        B._task_array(arrs_in[:1], [0], None, [bytes(33)])
