"""Oracle -- TEST INFRASTRUCTURE ONLY.

A plain CPU complex128 implementation of what the hot path computes. Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it. It shares no code with the product package
``paper_2609_23664_amd`` and never imports it; the only shared module is the
seeded input generator package ``workloads``.

Contents
  * ``simulate / apply_gates``   gate-by-gate statevector (C, ``qwo.c``)
  * ``simulate_measured``        the same with mid-circuit Z measurements and
                                 resets (Born rule, collapse, renormalise)
  * ``expect / expect_terms``    Pauli-sum expectation, plain definition
  * ``sample / uniform``         inverse-CDF Z-basis sampling, SplitMix64 hash
  * ``brute``                    numpy dense-unitary brute force (<= 8 qubits)
  * ``planner_ref``              Eq. (2) reuse rule and the Table II legality
                                 table, written out
  * ``mlp_ref``                  numpy float64 MLP forward/backward and a
                                 bf16-rounding mirror

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QWO_LIB: another build of the simulator to load (e.g. the sanitizer build)
_LIB_PATH = os.environ.get("QWO_LIB") or os.path.join(HERE, "_qwo.so")

# gate name -> code of qwo.c
_CODES = {
    "X": 1, "Y": 2, "Z": 3, "H": 4, "S": 5, "SDG": 6, "T": 7, "TDG": 8,
    "RX": 9, "RY": 10, "RZ": 11, "P": 12, "CNOT": 13, "CZ": 14, "RENORM": 15,
}

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    c_p = ctypes.c_void_p
    lib.qwo_init_zero.argtypes = [c_p, ctypes.c_int]
    lib.qwo_apply_gates.argtypes = [c_p, ctypes.c_int, ctypes.c_int64, c_p, c_p, c_p, c_p]
    lib.qwo_apply_gates.restype = ctypes.c_int
    lib.qwo_expect_pauli.argtypes = [c_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    lib.qwo_expect_pauli.restype = ctypes.c_double
    lib.qwo_norm2.argtypes = [c_p, ctypes.c_int]
    lib.qwo_norm2.restype = ctypes.c_double
    lib.qwo_splitmix64.argtypes = [ctypes.c_uint64]
    lib.qwo_splitmix64.restype = ctypes.c_uint64
    lib.qwo_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.qwo_uniform.restype = ctypes.c_double
    lib.qwo_sample.argtypes = [c_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                               ctypes.c_uint32, c_p]
    lib.qwo_sample.restype = ctypes.c_int
    _lib = lib
    return lib


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def _encode(gates: Sequence[Tuple[str, Tuple[int, ...], float]]):
    ng = len(gates)
    code = np.empty(ng, dtype=np.int32)
    q0 = np.full(ng, -1, dtype=np.int32)
    q1 = np.full(ng, -1, dtype=np.int32)
    par = np.zeros(ng, dtype=np.float64)
    for k, (name, qs, p) in enumerate(gates):
        code[k] = _CODES[name]
        if len(qs) > 0:
            q0[k] = qs[0]
        if len(qs) > 1:
            q1[k] = qs[1]
        par[k] = p
    return code, q0, q1, par


def _measure(psi: np.ndarray, n: int, q: int, u: float, reset: bool) -> int:
    """Projective Z measurement of qubit q in place (the measurement barrier
    that Sec. III-A's segmenter cuts at; the update is the textbook
    projective-measurement rule). With S = ||psi||^2 and S1 the probability
    mass on bit q = 1, the outcome is 1 iff u < S1 / S; the state becomes
    the projection onto that outcome divided by its norm. RESET then applies
    X on q when the outcome was 1."""
    idx = np.arange(1 << n, dtype=np.int64)
    one = ((idx >> q) & 1).astype(bool)
    w = psi.real ** 2 + psi.imag ** 2
    S = float(np.sum(w))
    S1 = float(np.sum(w[one]))
    b = 1 if u < S1 / S else 0
    keep = one if b else ~one
    psi[~keep] = 0.0
    psi /= np.sqrt(S1 if b else S - S1)
    if reset and b:
        psi[:] = psi[idx ^ (1 << q)]
    return b


def simulate_measured(n: int, gates):
    """(psi, outcomes) of ``gates`` from |0...0>, where ``MEASURE`` and
    ``RESET`` (qubit q, param u) measure as in ``_measure`` and every other
    gate is applied as in ``apply_gates``."""
    psi = zero_state(n)
    outs = []
    seg = []
    for g in gates:
        if g[0] in ("MEASURE", "RESET"):
            apply_gates(psi, n, seg)
            seg = []
            outs.append(_measure(psi, n, int(g[1][0]), float(g[2]), g[0] == "RESET"))
        else:
            seg.append(g)
    apply_gates(psi, n, seg)
    return psi, outs


def apply_gates(psi: np.ndarray, n: int, gates) -> np.ndarray:
    """Apply ``gates`` to ``psi`` in place, one at a time, in order
    (measurements: ``simulate_measured``)."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == (1 << n)
    if len(gates) == 0:
        return psi
    if any(g[0] in ("MEASURE", "RESET") for g in gates):
        raise ValueError("oracle: measurements go through simulate_measured")
    lib = _load()
    code, q0, q1, par = _encode(gates)
    rc = lib.qwo_apply_gates(psi.ctypes.data, n, len(gates), code.ctypes.data,
                             q0.ctypes.data, q1.ctypes.data, par.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle: bad gate at index {-1 - rc}: {gates[-1 - rc]}")
    return psi


def simulate(n: int, gates) -> np.ndarray:
    """psi = U(gates) |0...0>."""
    return apply_gates(zero_state(n), n, gates)


def norm2(psi: np.ndarray) -> float:
    n = int(psi.size).bit_length() - 1
    return float(_load().qwo_norm2(np.ascontiguousarray(psi).ctypes.data, n))


def expect_terms(psi: np.ndarray, n: int, terms) -> np.ndarray:
    """<P_j> for every term (coefficient not applied)."""
    lib = _load()
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    return np.array([lib.qwo_expect_pauli(psi.ctypes.data, n, int(x), int(z))
                     for (_, x, z) in terms], dtype=np.float64)


def expect(psi: np.ndarray, n: int, terms) -> float:
    """E = sum_j c_j <P_j>."""
    vals = expect_terms(psi, n, terms)
    return float(sum(float(c) * v for (c, _, _), v in zip(terms, vals)))


def splitmix64(v: int) -> int:
    return int(_load().qwo_splitmix64(ctypes.c_uint64(v & ((1 << 64) - 1))))


def uniform(seed: int, t: int, s: int) -> float:
    return float(_load().qwo_uniform(seed, t, s))


def sample(psi: np.ndarray, n: int, seed: int, task: int, shots: int) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty(shots, dtype=np.uint32)
    rc = _load().qwo_sample(psi.ctypes.data, n, seed, task, shots, out.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle sample")
    return out


def fidelity(a: np.ndarray, b: np.ndarray) -> float:
    """|<a|b>|^2 / (<a|a><b|b>), in float64."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    ov = np.vdot(a, b)
    return float((ov.real ** 2 + ov.imag ** 2) / (np.vdot(a, a).real * np.vdot(b, b).real))


def run_workload_reuse(w) -> List[np.ndarray]:
    """Final state of every task of a shared-prefix workload: the prefix is
    applied once and each suffix continues from a copy of that state (the
    reuse rewrite); gate order per task is unchanged."""
    base = simulate(w.n, w.prefix)
    return [apply_gates(base.copy(), w.n, s) for s in w.suffixes]


def run_task_direct(w, t: int) -> np.ndarray:
    """Task t from |0...0> through prefix then suffix (no reuse)."""
    return simulate(w.n, list(w.prefix) + list(w.suffixes[t]))
