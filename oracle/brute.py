"""Dense-unitary brute force (TEST INFRASTRUCTURE ONLY, n <= 8).

Every gate becomes a full 2^n x 2^n matrix built from Kronecker products of
2x2 operators (qubit q = bit q of the basis index, so qubit n-1 is the
leftmost Kronecker factor); two-qubit gates are written with projectors
(CNOT = |0><0|_c (x) 1 + |1><1|_c (x) X_t, CZ = 1 - 2 |11><11|). The circuit
unitary is the ordered matrix product. This is a different construction from
the index loops of ``qwo.c`` and pins them.
"""
from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def one_qubit_matrix(name: str, theta: float) -> np.ndarray:
    if name == "X":
        return X
    if name == "Y":
        return Y
    if name == "Z":
        return Z
    if name == "H":
        return H
    if name == "S":
        return np.diag([1, 1j]).astype(np.complex128)
    if name == "SDG":
        return np.diag([1, -1j]).astype(np.complex128)
    if name == "T":
        return np.diag([1, np.exp(1j * np.pi / 4)])
    if name == "TDG":
        return np.diag([1, np.exp(-1j * np.pi / 4)])
    if name == "RX":   # exp(-i theta X / 2)
        return np.cos(theta / 2) * I2 - 1j * np.sin(theta / 2) * X
    if name == "RY":   # exp(-i theta Y / 2)
        return np.cos(theta / 2) * I2 - 1j * np.sin(theta / 2) * Y
    if name == "RZ":   # exp(-i theta Z / 2)
        return np.cos(theta / 2) * I2 - 1j * np.sin(theta / 2) * Z
    if name == "P":
        return np.diag([1, np.exp(1j * theta)])
    raise ValueError(name)


def embed(n: int, ops: dict) -> np.ndarray:
    """Kronecker product over qubits n-1 .. 0 of ops.get(q, identity)."""
    m = np.array([[1.0 + 0j]])
    for q in range(n - 1, -1, -1):
        m = np.kron(m, ops.get(q, I2))
    return m


def gate_matrix(n: int, gate) -> np.ndarray:
    name, qs, theta = gate
    if name == "CNOT":
        c, t = qs
        return embed(n, {c: P0}) + embed(n, {c: P1, t: X})
    if name == "CZ":
        a, b = qs
        return embed(n, {}) - 2.0 * embed(n, {a: P1, b: P1})
    return embed(n, {qs[0]: one_qubit_matrix(name, theta)})


def circuit_unitary(n: int, gates) -> np.ndarray:
    assert n <= 8
    u = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        if g[0] == "RENORM":
            continue
        u = gate_matrix(n, g) @ u
    return u


def pauli_matrix(n: int, x: int, z: int) -> np.ndarray:
    ops = {}
    for q in range(n):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        if xb and zb:
            ops[q] = Y
        elif xb:
            ops[q] = X
        elif zb:
            ops[q] = Z
    return embed(n, ops)
