"""ctypes binding of libqw (include/qw.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels. PyTorch provides device memory (state buffers are torch tensors)
and the HIP stream (torch's current stream). The binding raises if the
built library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
# QW_LIB: another build of the library to load (e.g. the sanitizer build)
LIB_PATH = os.environ.get("QW_LIB") or os.path.join(HERE, "libqw.so")

QW_OK = 0
QW_E_INVALID_ARG = 1
QW_E_OOM = 2
QW_E_HIP = 3
QW_E_REFUSED = 4
QW_E_UNSUPPORTED = 5
QW_E_ABANDONED = 6

GATE_KIND = {
    "X": 0x01, "Y": 0x02, "Z": 0x03, "H": 0x04, "S": 0x05, "SDG": 0x06,
    "T": 0x07, "TDG": 0x08, "RX": 0x21, "RY": 0x22, "RZ": 0x23, "P": 0x24,
    "CNOT": 0x41, "CZ": 0x42, "RENORM": 0x81, "MEASURE": 0x82, "RESET": 0x83,
    "PROJ0": 0x84, "PROJ1": 0x85,
}

QW_KIND_STATEVECTOR = 1
QW_KIND_TABLEAU = 2
QW_EXACTNESS_UNKNOWN = 0
QW_EXACT = 1
QW_APPROX = 2
QW_BACKEND_UNKNOWN = 0
QW_BACKEND_SV = 1
QW_BACKEND_STAB_ONLY = 2
QW_SNAP_COPY = 0
QW_SNAP_FREEZE = 1

QW_OPT_TILE_BITS = 1
QW_OPT_PROFILE = 2
QW_OPT_XCD_REMAP = 4
QW_OPT_JIT = 5
QW_OPT_RELABEL = 6
QW_OPT_SECOND_BUFFER_CAP = 7
QW_OPT_FUSED_EPILOGUE = 8
QW_OPT_TILE_ORDER = 9
QW_OPT_STREAM_LOADS = 10
QW_OPT_DEVICE_MEM_CAP = 11
QW_OPT_LAYOUT = 12
QW_OPT_PERSISTENT = 13
QW_OPT_SPIN_LIMIT = 14
QW_OPT_PERSIST_CHUNK = 15

EXPORTED = (
    "qw_ctx_create", "qw_ctx_destroy", "qw_last_error", "qw_ctx_sync",
    "qw_ctx_set_option", "qw_ctx_kernel_stats", "qw_state_alloc", "qw_state_free",
    "qw_state_reset", "qw_state_slot_ptr", "qw_apply_prefix", "qw_snapshot",
    "qw_snapshot_free", "qw_snapshot_info", "qw_run_suffix_batch",
    "qw_expect_pauli", "qw_sample", "qw_legality_check", "qw_plan_describe",
    "qw_mlp_workspace_floats", "qw_mlp_forward", "qw_mlp_backward", "qw_mlp_adam",
    "qw_plan_cost", "qw_jit_precompile", "qw_jit_precompile_terms", "qw_jit_precompile_suffix",
    "qw_jit_stats", "qw_version", "qw_outcomes", "qw_tableau_create", "qw_tableau_free",
    "qw_tableau_apply", "qw_tableau_rows", "qw_tableau_artifact", "qw_tableau_export",
    "qw_graph_begin", "qw_graph_end", "qw_graph_launch", "qw_graph_nodes", "qw_graph_free",
    "qw_graph_update_gates", "qw_sample_noalloc", "qw_mlp_backward_rows", "qw_mlp_loss",
    "qw_graph_outcomes", "qw_run_tree", "qw_ctx_abandon", "qw_persist_schedule",
)


class QwGate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("q0", ctypes.c_uint32), ("q1", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("param", ctypes.c_double)]


def _gate_dtype():
    import numpy as np
    return np.dtype([("kind", "<u4"), ("q0", "<u4"), ("q1", "<u4"), ("reserved", "<u4"),
                     ("param", "<f8")])





class QwArtifact(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("exactness", ctypes.c_uint32),
                ("backend", ctypes.c_uint32), ("n_qubits", ctypes.c_uint32),
                ("bytes", ctypes.c_uint64), ("provenance", ctypes.c_uint8 * 32)]


class QwTask(ctypes.Structure):
    _fields_ = [("gates", ctypes.POINTER(QwGate)), ("n_gates", ctypes.c_uint64),
                ("dst_slot", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("expect_prov", ctypes.c_uint8 * 32)]


class QwReduce(ctypes.Structure):
    _fields_ = [("x_mask", ctypes.POINTER(ctypes.c_uint64)),
                ("z_mask", ctypes.POINTER(ctypes.c_uint64)),
                ("coeff", ctypes.POINTER(ctypes.c_double)),
                ("n_terms", ctypes.c_uint32), ("out_is_host", ctypes.c_int32),
                ("out", ctypes.POINTER(ctypes.c_double))]


assert ctypes.sizeof(QwGate) == 24


class QwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libqw error {code}: {msg}")
        self.code = code
        self.msg = msg


class QwRefused(QwError):
    """A continuation failed a legality gate; ``record`` is the refusal JSON."""

    @property
    def record(self) -> dict:
        import json
        return json.loads(self.msg)


_lib = None


def lib() -> ctypes.CDLL:
    """Load libqw.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libqw.so not built at {LIB_PATH}: run "
                          "`python -m paper_2609_23664_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "qw_ctx_create": ([i32, vp, pp], i32),
        "qw_ctx_destroy": ([vp], i32),
        "qw_last_error": ([vp], ctypes.c_char_p),
        "qw_ctx_sync": ([vp], i32),
        "qw_ctx_set_option": ([vp, i32, ctypes.c_int64], i32),
        "qw_ctx_kernel_stats": ([vp, i32, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), i32], i32),
        "qw_state_alloc": ([vp, u32, u32, vp, u64, pp], i32),
        "qw_state_free": ([vp], i32),
        "qw_state_reset": ([vp, u32, u32], i32),
        "qw_state_slot_ptr": ([vp, u32, pp], i32),
        "qw_apply_prefix": ([vp, u32, ctypes.POINTER(QwGate), u64], i32),
        "qw_snapshot": ([vp, u32, ctypes.POINTER(ctypes.c_uint8), i32, vp, vp, u64, pp], i32),
        "qw_snapshot_free": ([vp], i32),
        "qw_snapshot_info": ([vp, ctypes.POINTER(QwArtifact)], i32),
        "qw_run_suffix_batch": ([vp, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(QwTask), u32,
                                 vp, ctypes.POINTER(QwReduce)], i32),
        "qw_expect_pauli": ([vp, u32, u32, ctypes.POINTER(u64), ctypes.POINTER(u64),
                             ctypes.POINTER(ctypes.c_double), u32, vp, i32], i32),
        "qw_sample": ([vp, u32, u32, u64, u64, u32, vp, i32], i32),
        "qw_sample_noalloc": ([vp, u32, u32, u64, u64, u32, vp, i32], i32),
        "qw_legality_check": ([ctypes.POINTER(QwArtifact), u32, u32, ctypes.c_char_p, u64], i32),
        "qw_plan_describe": ([u32, ctypes.POINTER(QwGate), u64, u32, ctypes.c_char_p, u64], i32),
        "qw_mlp_workspace_floats": ([u32], u64),
        "qw_mlp_forward": ([vp, vp, vp, u32, vp, vp], i32),
        "qw_mlp_backward": ([vp, vp, vp, vp, u32, vp, vp], i32),
        "qw_mlp_backward_rows": ([vp, vp, vp, vp, u32, vp, u32, vp, vp], i32),
        "qw_mlp_loss": ([vp, vp, vp, vp, u32, vp, vp], i32),
        "qw_mlp_adam": ([vp, vp, vp, vp, vp, u32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                         ctypes.c_float], i32),
        "qw_plan_cost": ([u32, ctypes.POINTER(QwGate), u64, u32, ctypes.POINTER(u64),
                          ctypes.POINTER(ctypes.c_double)], i32),
        "qw_jit_precompile": ([u32, ctypes.POINTER(QwGate), u64, u32, ctypes.c_char_p, u64], i32),
        "qw_jit_precompile_terms": ([u32, ctypes.POINTER(u64), ctypes.POINTER(u64), u32, u32,
                                     ctypes.c_char_p, u64], i32),
        "qw_jit_precompile_suffix": ([u32, ctypes.POINTER(QwGate), u64, ctypes.POINTER(u64),
                                      ctypes.POINTER(u64), u32, u32, ctypes.c_char_p, u64], i32),
        "qw_tableau_create": ([u32, ctypes.POINTER(ctypes.c_void_p)], i32),
        "qw_tableau_free": ([ctypes.c_void_p], i32),
        "qw_tableau_apply": ([ctypes.c_void_p, ctypes.POINTER(QwGate), u64], i32),
        "qw_tableau_rows": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], i32),
        "qw_tableau_artifact": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(QwArtifact)], i32),
        "qw_tableau_export": ([ctypes.c_void_p, ctypes.c_void_p, u32], i32),
        "qw_outcomes": ([ctypes.c_void_p, ctypes.c_void_p, u64, ctypes.POINTER(u64)], i32),
        "qw_jit_stats": ([ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double)],
                         i32),
        "qw_version": ([], ctypes.c_char_p),
        "qw_graph_begin": ([vp], i32),
        "qw_graph_end": ([vp, ctypes.POINTER(ctypes.c_void_p)], i32),
        "qw_graph_launch": ([vp], i32),
        "qw_graph_nodes": ([vp, ctypes.POINTER(u64)], i32),
        "qw_graph_free": ([vp], i32),
        "qw_graph_outcomes": ([vp, vp, u64, ctypes.POINTER(u64)], i32),
        "qw_run_tree": ([vp, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(QwTask),
                         ctypes.POINTER(ctypes.c_int32), vp, u32, vp], i32),
        "qw_ctx_abandon": ([vp], i32),
        "qw_persist_schedule": ([u32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(u32), ctypes.POINTER(u32),
                                 ctypes.POINTER(u32), u32, u32, ctypes.c_char_p, u64], i32),
        "qw_graph_update_gates": ([vp, u32, u32, ctypes.POINTER(QwGate), u64], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


class GateArray:
    """Gate records marshalled once into a qw_gate array (reusable across
    calls; `set_params` rewrites the angles in place). Accepted wherever a
    gate list is."""

    def __init__(self, gates: Sequence[Tuple[str, Tuple[int, ...], float]]):
        import numpy as np
        n = len(gates)
        rec = np.zeros(max(1, n), dtype=_gate_dtype())
        if n:
            rec["kind"][:n] = [GATE_KIND[g[0]] for g in gates]
            rec["q0"][:n] = [g[1][0] if len(g[1]) > 0 else 0 for g in gates]
            rec["q1"][:n] = [g[1][1] if len(g[1]) > 1 else 0 for g in gates]
            rec["param"][:n] = [float(g[2]) for g in gates]
        self.rec = rec
        self.n = n
        self.ptr = rec.ctypes.data_as(ctypes.POINTER(QwGate))

    def set_params(self, params) -> None:
        self.rec["param"][:self.n] = params

    def __len__(self):
        return self.n


def gate_array(gates):
    """A qw_gate array for `gates` ((name, qubits, param) records, or a
    GateArray, returned as is)."""
    if isinstance(gates, GateArray):
        return gates
    return GateArray(gates)


def _u64_array(vals):
    a = (ctypes.c_uint64 * max(1, len(vals)))()
    for i, v in enumerate(vals):
        a[i] = int(v)
    return a


def _f64_array(vals):
    a = (ctypes.c_double * max(1, len(vals)))()
    for i, v in enumerate(vals):
        a[i] = float(v)
    return a


def _prov(b: bytes):
    assert len(b) == 32
    return (ctypes.c_uint8 * 32)(*b)


def legality_check(kind: int, exactness: int, backend: int, n_qubits: int,
                   target_kind: int, target_backend: int) -> Tuple[int, str]:
    """Host-only legality gates; returns (status, refusal JSON or '')."""
    art = QwArtifact(kind, exactness, backend, n_qubits, 0, (ctypes.c_uint8 * 32)())
    buf = ctypes.create_string_buffer(1024)
    rc = lib().qw_legality_check(ctypes.byref(art), target_kind, target_backend, buf, 1024)
    return rc, buf.value.decode()


def plan_describe(n: int, gates, tile_bits: int = 14) -> dict:
    """Host-only: the pass plan for `gates` as a dict."""
    import json
    arr = gate_array(gates)
    cap = 1 << 16
    while True:
        buf = ctypes.create_string_buffer(cap)
        rc = lib().qw_plan_describe(n, arr.ptr, len(arr), tile_bits, buf, cap)
        if rc == QW_OK:
            return json.loads(buf.value.decode())
        if buf.value.startswith(b'{"error"'):
            raise QwError(rc, json.loads(buf.value.decode())["error"])
        cap *= 4
        if cap > (1 << 30):
            raise QwError(rc, "plan too large")


def plan_cost(n: int, gates, tile_bits: int = 14) -> Tuple[int, float]:
    """Host-only: (tile passes, HBM bytes) of `gates` on n qubits."""
    arr = gate_array(gates)
    npass, by = ctypes.c_uint64(), ctypes.c_double()
    rc = lib().qw_plan_cost(n, arr.ptr, len(arr), tile_bits, ctypes.byref(npass), ctypes.byref(by))
    if rc != QW_OK:
        raise QwError(rc, "plan_cost: invalid gates")
    return npass.value, by.value


def jit_precompile(n: int, gates, tile_bits: int = 14) -> None:
    """Host-only: compile the generated pass kernels of `gates` into the
    process and disk caches (no GPU needed)."""
    arr = gate_array(gates)
    cap = 1 << 20
    buf = ctypes.create_string_buffer(cap)
    rc = lib().qw_jit_precompile(n, arr.ptr, len(arr), tile_bits, buf, cap)
    if rc != QW_OK:
        raise QwError(rc, buf.value.decode(errors="replace"))


def jit_precompile_terms(n: int, terms, tile_bits: int = 14) -> None:
    """Host-only: compile the generated expectation reducers of the Pauli
    terms [(coeff, x_mask, z_mask), ...] into the caches (no GPU needed)."""
    nt = len(terms)
    xs = (ctypes.c_uint64 * max(1, nt))(*[int(t[1]) for t in terms])
    zs = (ctypes.c_uint64 * max(1, nt))(*[int(t[2]) for t in terms])
    cap = 1 << 20
    buf = ctypes.create_string_buffer(cap)
    rc = lib().qw_jit_precompile_terms(n, xs, zs, nt, tile_bits, buf, cap)
    if rc != QW_OK:
        raise QwError(rc, buf.value.decode(errors="replace"))


def jit_precompile_suffix(n: int, gates, terms, tile_bits: int = 14) -> None:
    """Host-only: compile the generated kernels of a suffix batch with an
    expectation epilogue (passes, fused last pass, remaining reducers)."""
    ga = gate_array(gates)
    nt = len(terms)
    xs = (ctypes.c_uint64 * max(1, nt))(*[int(t[1]) for t in terms])
    zs = (ctypes.c_uint64 * max(1, nt))(*[int(t[2]) for t in terms])
    cap = 1 << 20
    buf = ctypes.create_string_buffer(cap)
    rc = lib().qw_jit_precompile_suffix(n, ga.ptr, len(ga), xs, zs, nt, tile_bits, buf, cap)
    if rc != QW_OK:
        raise QwError(rc, buf.value.decode(errors="replace"))


def jit_stats() -> dict:
    """Generated-kernel counters of this process."""
    c, h, s = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_double()
    lib().qw_jit_stats(ctypes.byref(c), ctypes.byref(h), ctypes.byref(s))
    return {"compiled": c.value, "disk_hits": h.value, "compile_s": s.value}


def outcomes(ctx) -> "np.ndarray":
    """qw_outcomes: measurement outcomes (uint8, task order then gate order)
    of the context's last qw_apply_prefix / qw_run_suffix_batch."""
    import numpy as np
    cnt = ctypes.c_uint64()
    ctx.check(lib().qw_outcomes(ctx.h, None, 0, ctypes.byref(cnt)))
    out = np.zeros(cnt.value, dtype=np.uint8)
    if cnt.value:
        ctx.check(lib().qw_outcomes(ctx.h, ctypes.c_void_p(out.ctypes.data), cnt.value, ctypes.byref(cnt)))
    return out


class Tableau:
    """qw_tableau: stabilizer tableau of a Clifford circuit (host memory)."""

    def __init__(self, n: int):
        h = ctypes.c_void_p()
        rc = lib().qw_tableau_create(n, ctypes.byref(h))
        if rc:
            raise QwError(rc, "qw_tableau_create")
        self.h, self.n = h, n

    def apply(self, gates):
        arr = gate_array(gates)
        rc = lib().qw_tableau_apply(self.h, arr.ptr, len(arr))
        if rc:
            raise QwError(rc, "qw_tableau_apply: non-Clifford or bad gate")

    def rows(self):
        """(x, z, r) arrays of the 2n rows (stabilizer generators last)."""
        import numpy as np
        x = np.zeros(2 * self.n, dtype=np.uint64)
        z = np.zeros(2 * self.n, dtype=np.uint64)
        r = np.zeros(2 * self.n, dtype=np.uint8)
        rc = lib().qw_tableau_rows(self.h, ctypes.c_void_p(x.ctypes.data), ctypes.c_void_p(z.ctypes.data),
                                   ctypes.c_void_p(r.ctypes.data))
        if rc:
            raise QwError(rc, "qw_tableau_rows")
        return x, z, r

    def artifact(self, provenance: bytes) -> dict:
        a = QwArtifact()
        rc = lib().qw_tableau_artifact(self.h, _prov(provenance), ctypes.byref(a))
        if rc:
            raise QwError(rc, "qw_tableau_artifact")
        return {"kind": a.kind, "exactness": a.exactness, "backend": a.backend,
                "n_qubits": a.n_qubits, "bytes": a.bytes, "provenance": bytes(a.provenance)}

    def export(self, st: "State", slot: int):
        """qw_tableau_export into slot `slot` of `st`."""
        st.ctx.check(lib().qw_tableau_export(self.h, st.h, slot))

    def free(self):
        if self.h:
            lib().qw_tableau_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Ctx:
    """A libqw context on torch's current HIP stream of `device`."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = lib().qw_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != QW_OK:
            raise QwError(rc, "qw_ctx_create failed")
        self.h = h

    def check(self, rc: int):
        if rc == QW_OK:
            return
        msg = lib().qw_last_error(self.h).decode()
        if rc == QW_E_REFUSED:
            raise QwRefused(rc, msg)
        raise QwError(rc, msg)

    def set_option(self, key: int, value: int):
        self.check(lib().qw_ctx_set_option(self.h, key, int(value)))

    def sync(self):
        self.check(lib().qw_ctx_sync(self.h))

    def abandon(self):
        """qw_ctx_abandon: waits of persistent launches give up."""
        self.check(lib().qw_ctx_abandon(self.h))

    def kernel_stats(self, kernel: int, reset: bool = True):
        n = ctypes.c_uint64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        self.check(lib().qw_ctx_kernel_stats(self.h, kernel, ctypes.byref(n), ctypes.byref(ms),
                                             ctypes.byref(by), 1 if reset else 0))
        return int(n.value), float(ms.value), float(by.value)

    def begin_graph(self):
        """qw_graph_begin: the following calls' device work is recorded."""
        self.check(lib().qw_graph_begin(self.h))

    def end_graph(self) -> "Graph":
        """qw_graph_end: the recorded work as a replayable Graph."""
        g = ctypes.c_void_p()
        self.check(lib().qw_graph_end(self.h, ctypes.byref(g)))
        return Graph(self, g)

    def close(self):
        if self.h:
            lib().qw_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class State:
    """n-qubit state with `slots` slots; memory is a torch complex64 tensor."""

    def __init__(self, ctx: Ctx, n: int, slots: int):
        torch = ctx.torch
        self.ctx, self.n, self.slots = ctx, n, slots
        self.buf = torch.empty((slots, 1 << n), dtype=torch.complex64, device=f"cuda:{ctx.device}")
        h = ctypes.c_void_p()
        ctx.check(lib().qw_state_alloc(ctx.h, n, slots, ctypes.c_void_p(self.buf.data_ptr()),
                                       self.buf.numel() * 8, ctypes.byref(h)))
        self.h = h

    def reset(self, first: int = 0, count: Optional[int] = None):
        count = self.slots - first if count is None else count
        self.ctx.check(lib().qw_state_reset(self.h, first, count))

    def apply(self, slot: int, gates):
        arr = gate_array(gates)
        self.ctx.check(lib().qw_apply_prefix(self.h, slot, arr.ptr, len(arr)))

    def snapshot(self, slot: int, provenance: bytes, mode: int = QW_SNAP_FREEZE,
                 parent: "Optional[Snapshot]" = None) -> "Snapshot":
        return Snapshot(self, slot, provenance, mode, parent)

    def expect(self, first: int, count: int, terms, out_dev=None) -> Optional[List[float]]:
        """qw_expect_pauli. With `out_dev` (a float64 device tensor of
        `count` elements) the values go there and nothing is returned."""
        x = _u64_array([t[1] for t in terms])
        z = _u64_array([t[2] for t in terms])
        c = _f64_array([t[0] for t in terms])
        if out_dev is not None:
            _check_dev(out_dev, self.ctx.torch.float64, count)
            self.ctx.check(lib().qw_expect_pauli(self.h, first, count, x, z, c, len(terms),
                                                 ctypes.c_void_p(out_dev.data_ptr()), 0))
            return None
        out = (ctypes.c_double * max(1, count))()
        self.ctx.check(lib().qw_expect_pauli(self.h, first, count, x, z, c, len(terms),
                                             ctypes.cast(out, ctypes.c_void_p), 1))
        return [out[i] for i in range(count)]

    def sample(self, first: int, count: int, seed: int, task_base: int, shots: int, out_dev=None):
        """qw_sample. With `out_dev` (an int32 device tensor of count * shots
        elements, read as uint32) the indices go there and nothing is returned."""
        import numpy as np
        if out_dev is not None:
            _check_dev(out_dev, self.ctx.torch.int32, count * shots)
            self.ctx.check(lib().qw_sample(self.h, first, count, seed, task_base, shots,
                                           ctypes.c_void_p(out_dev.data_ptr()), 0))
            return None
        out = np.empty(count * shots, dtype=np.uint32)
        self.ctx.check(lib().qw_sample(self.h, first, count, seed, task_base, shots,
                                       ctypes.c_void_p(out.ctypes.data), 1))
        return out.reshape(count, shots)

    def sample_noalloc(self, first: int, count: int, seed: int, task_base: int, shots: int,
                       out_dev=None):
        """qw_sample_noalloc: qw_sample through the library's fixed device
        scratch (no allocation). Same arguments and results as sample()."""
        import numpy as np
        if out_dev is not None:
            _check_dev(out_dev, self.ctx.torch.int32, count * shots)
            self.ctx.check(lib().qw_sample_noalloc(self.h, first, count, seed, task_base, shots,
                                                   ctypes.c_void_p(out_dev.data_ptr()), 0))
            return None
        out = np.empty(count * shots, dtype=np.uint32)
        self.ctx.check(lib().qw_sample_noalloc(self.h, first, count, seed, task_base, shots,
                                               ctypes.c_void_p(out.ctypes.data), 1))
        return out.reshape(count, shots)

    def host(self, slot: int):
        """Copy of slot `slot` as a numpy complex64 array (synchronises)."""
        self.ctx.sync()
        return self.buf[slot].cpu().numpy()

    def free(self):
        if self.h:
            rc = lib().qw_state_free(self.h)
            self.h = None
            self.ctx.check(rc)

    def __del__(self):
        try:
            if self.h:
                lib().qw_state_free(self.h)
                self.h = None
        except Exception:
            pass


class Snapshot:
    """Typed boundary artifact (ArtifactRecord) of one state slot."""

    def __init__(self, state: State, slot: int, provenance: bytes, mode: int, parent=None):
        self.state = state
        self.provenance = bytes(provenance)
        self.copy_buf = None
        h = ctypes.c_void_p()
        copy_ptr, copy_bytes = None, 0
        if mode == QW_SNAP_COPY:
            torch = state.ctx.torch
            self.copy_buf = torch.empty(1 << state.n, dtype=torch.complex64,
                                        device=f"cuda:{state.ctx.device}")
            copy_ptr, copy_bytes = ctypes.c_void_p(self.copy_buf.data_ptr()), 8 << state.n
        state.ctx.check(lib().qw_snapshot(state.h, slot, _prov(self.provenance), mode,
                                          parent.h if parent is not None else None,
                                          copy_ptr, copy_bytes, ctypes.byref(h)))
        self.h = h

    def info(self) -> dict:
        a = QwArtifact()
        self.state.ctx.check(lib().qw_snapshot_info(self.h, ctypes.byref(a)))
        return {"kind": a.kind, "exactness": a.exactness, "backend": a.backend,
                "n_qubits": a.n_qubits, "bytes": a.bytes, "provenance": bytes(a.provenance)}

    def free(self):
        if self.h:
            lib().qw_snapshot_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _check_dev(t, dtype, numel):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() < numel:
        raise ValueError(f"expected a contiguous {dtype} device tensor of >= {numel} elements")


class Graph:
    """A recorded workload (qw_graph_*): replay() enqueues it once."""

    def __init__(self, ctx: Ctx, h):
        self.ctx, self.h = ctx, h
        self.keep = []  # objects the recorded calls reference (states, outputs)

    def replay(self):
        self.ctx.check(lib().qw_graph_launch(self.h))

    def update_gates(self, call: int, task: int, gates) -> None:
        """qw_graph_update_gates: new gates (same structure) for a recorded task."""
        arr = gate_array(gates)
        self.ctx.check(lib().qw_graph_update_gates(self.h, call, task, arr.ptr, len(arr)))

    def nodes(self) -> int:
        n = ctypes.c_uint64()
        self.ctx.check(lib().qw_graph_nodes(self.h, ctypes.byref(n)))
        return int(n.value)

    def outcomes(self) -> "np.ndarray":
        """qw_graph_outcomes: outcomes (uint8) of the recorded measured calls,
        as written by the most recent replay (synchronises)."""
        import numpy as np
        cnt = ctypes.c_uint64()
        self.ctx.check(lib().qw_graph_outcomes(self.h, None, 0, ctypes.byref(cnt)))
        out = np.zeros(cnt.value, dtype=np.uint8)
        if cnt.value:
            self.ctx.check(lib().qw_graph_outcomes(self.h, ctypes.c_void_p(out.ctypes.data), cnt.value,
                                                   ctypes.byref(cnt)))
        return out

    def free(self):
        if self.h:
            rc = lib().qw_graph_free(self.h)
            self.h = None
            self.ctx.check(rc)
        self.keep = []

    def __del__(self):
        try:
            if self.h:
                lib().qw_graph_free(self.h)
                self.h = None
        except Exception:
            pass


def _task_array(suffixes, dst_slots, srcs, expect_provs):
    """The qw_task records of a call (the gate arrays returned with them must
    outlive the call). A provenance is copied as 32 bytes in one move."""
    nt = len(suffixes)
    arrs = [gate_array(s) for s in suffixes]
    tasks = (QwTask * max(1, nt))()
    off = QwTask.expect_prov.offset
    base = ctypes.addressof(tasks)
    size = ctypes.sizeof(QwTask)
    zero = bytes(32)
    for k in range(nt):
        t = tasks[k]
        t.gates = arrs[k].ptr
        t.n_gates = len(arrs[k])
        t.dst_slot = int(dst_slots[k])
        prov = expect_provs[k] if expect_provs is not None else (
            srcs[k].provenance if srcs and srcs[k] is not None else zero)
        prov = bytes(prov)
        if len(prov) > 32:
            raise ValueError(f"task {k}: provenance longer than 32 bytes")
        ctypes.memmove(base + k * size + off, prov.ljust(32, b"\0"), 32)
    return arrs, tasks


def run_suffix_batch(ctx: Ctx, srcs: Sequence[Optional[Snapshot]], suffixes, dst: State,
                     dst_slots: Sequence[int], expect_provs: Sequence[bytes] = None,
                     terms=None, out_dev=None):
    """qw_run_suffix_batch; returns the per-task expectations if `terms`
    (or writes them to `out_dev`, a float64 device tensor, and returns None)."""
    nt = len(suffixes)
    arrs, tasks = _task_array(suffixes, dst_slots, srcs, expect_provs)
    src_arr = None
    if srcs is not None:
        src_arr = (ctypes.c_void_p * max(1, nt))()
        for k in range(nt):
            src_arr[k] = srcs[k].h.value if srcs[k] is not None else None
    red = None
    out = None
    keep = []
    if terms is not None:
        x = _u64_array([t[1] for t in terms])
        z = _u64_array([t[2] for t in terms])
        c = _f64_array([t[0] for t in terms])
        keep += [x, z, c]
        if out_dev is not None:
            _check_dev(out_dev, ctx.torch.float64, nt)
            red = QwReduce(ctypes.cast(x, ctypes.POINTER(ctypes.c_uint64)),
                           ctypes.cast(z, ctypes.POINTER(ctypes.c_uint64)),
                           ctypes.cast(c, ctypes.POINTER(ctypes.c_double)),
                           len(terms), 0, ctypes.cast(ctypes.c_void_p(out_dev.data_ptr()),
                                                      ctypes.POINTER(ctypes.c_double)))
        else:
            out = (ctypes.c_double * max(1, nt))()
            red = QwReduce(ctypes.cast(x, ctypes.POINTER(ctypes.c_uint64)),
                           ctypes.cast(z, ctypes.POINTER(ctypes.c_uint64)),
                           ctypes.cast(c, ctypes.POINTER(ctypes.c_double)),
                           len(terms), 1, ctypes.cast(out, ctypes.POINTER(ctypes.c_double)))
    rc = lib().qw_run_suffix_batch(ctx.h, src_arr, tasks, nt, dst.h,
                                   ctypes.byref(red) if red is not None else None)
    ctx.check(rc)
    if out is not None:
        return [out[i] for i in range(nt)]
    return None


def run_tree(ctx: Ctx, srcs: Optional[Sequence[Optional[Snapshot]]], suffixes, parents: Sequence[int],
             dst: State, dst_slots: Sequence[int], expect_provs: Sequence[bytes] = None,
             out_provs: Sequence[bytes] = None):
    """qw_run_tree: task k starts from task parents[k]'s final state (if >= 0),
    else from srcs[k] (if given), else from its destination slot."""
    nt = len(suffixes)
    arrs, tasks = _task_array(suffixes, dst_slots, srcs, expect_provs)
    src_arr = None
    if srcs is not None:
        src_arr = (ctypes.c_void_p * max(1, nt))()
        for k in range(nt):
            src_arr[k] = srcs[k].h.value if srcs[k] is not None else None
    par = (ctypes.c_int32 * max(1, nt))(*[int(p) for p in parents])
    outp = None
    if out_provs is not None:
        outp = (ctypes.c_uint8 * (32 * max(1, nt)))(*b"".join(bytes(o) for o in out_provs))
    rc = lib().qw_run_tree(ctx.h, src_arr, tasks, par, outp, nt, dst.h)
    ctx.check(rc)


def persist_schedule(parents: Sequence[int], passes: Sequence[int], kinds: Sequence[int],
                     units: Sequence[int], chunk_max: int = 8, grid: int = 256) -> dict:
    """Host-only qw_persist_schedule: the claim schedule of a persistent
    launch over a task tree (kinds and units per (task, pass), task-major)."""
    import json
    nt = len(parents)
    nd = len(kinds)
    par = (ctypes.c_int32 * max(1, nt))(*[int(p) for p in parents])
    npa = (ctypes.c_uint32 * max(1, nt))(*[int(p) for p in passes])
    kd = (ctypes.c_uint32 * max(1, nd))(*[int(k) for k in kinds])
    un = (ctypes.c_uint32 * max(1, nd))(*[int(u) for u in units])
    cap = 1 << 24
    buf = ctypes.create_string_buffer(cap)
    rc = lib().qw_persist_schedule(nt, par, npa, kd, un, chunk_max, grid, buf, cap)
    if rc != QW_OK:
        raise QwError(rc, buf.value.decode(errors="replace"))
    return json.loads(buf.value.decode())
