"""Workload planner (host side): Eq. (1) fingerprints, prefix detection,
Table II legality, the Eq. (2) reuse rule with an analytic byte-count cost
model, and the EXPLAIN / CostRecord / ExecutionResult records (Sec. III-A,
Sec. IV). Execution goes through the C ABI (``binding``); the plan changes
timing only, never results.
"""
from __future__ import annotations

import hashlib
import struct
from typing import List, Sequence, Tuple

from .binding import GATE_KIND

Gate = Tuple[str, Tuple[int, ...], float]


def gate_bytes(g: Gate) -> bytes:
    """Byte record of one gate for Eq. (1): u8 kind, u32 q0, u32 q1, f64
    parameter, little-endian (absent qubits are 0xFFFFFFFF)."""
    name, qs, p = g
    q0 = qs[0] if len(qs) > 0 else 0xFFFFFFFF
    q1 = qs[1] if len(qs) > 1 else 0xFFFFFFFF
    return struct.pack("<BIId", GATE_KIND[name], q0, q1, float(p))


def layout_bytes(n: int) -> bytes:
    """Layout record for Eq. (1): u32 qubit count, then the u32 map from
    logical to physical qubits (the identity here)."""
    return struct.pack("<I", n) + struct.pack(f"<{n}I", *range(n))


def fingerprint(n: int, gates: Sequence[Gate]) -> bytes:
    """Eq. (1): SHA256(layout || g_1 || ... || g_l)."""
    h = hashlib.sha256()
    h.update(layout_bytes(n))
    for g in gates:
        h.update(gate_bytes(g))
    return h.digest()
