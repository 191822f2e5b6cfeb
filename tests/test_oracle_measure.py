"""Pins of the oracle's mid-circuit Z measurement and reset
(``oracle.simulate_measured``): the Born-rule threshold, collapse and
renormalisation on states whose outcome probabilities and post-measurement
states are known in closed form, a repetition-code syndrome round whose
outcomes are fixed by the code, and a dense-projector brute force on random
small circuits."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute


def _ghz(n):
    return [("RY", (0,), math.pi / 2)] + [("CNOT", (q, q + 1), 0.0) for q in range(n - 1)]


@pytest.mark.parametrize("u,b", [(0.49, 1), (0.51, 0), (0.0, 1), (0.999, 0)])
def test_plus_state_threshold(u, b):
    psi, outs = oracle.simulate_measured(1, [("H", (0,), 0.0), ("MEASURE", (0,), u)])
    assert outs == [b]
    ref = np.zeros(2, dtype=complex)
    ref[b] = 1.0
    assert np.allclose(psi, ref, atol=1e-15)


@pytest.mark.parametrize("theta", [0.3, 1.1, 2.5])
def test_ry_probability_is_sin_squared(theta):
    p1 = math.sin(theta / 2) ** 2
    for u, b in ((p1 - 1e-9, 1), (p1 + 1e-9, 0)):
        psi, outs = oracle.simulate_measured(3, [("RY", (1,), theta), ("MEASURE", (1,), u)])
        assert outs == [b]
        assert abs(abs(psi[2 if b else 0]) - 1.0) <= 1e-14
        assert abs(np.vdot(psi, psi) - 1.0) <= 1e-14


@pytest.mark.parametrize("q", [0, 2, 4])
def test_ghz_collapse_and_reset(q):
    n = 5
    full = (1 << n) - 1
    for u, b in ((0.2, 1), (0.8, 0)):
        psi, outs = oracle.simulate_measured(n, _ghz(n) + [("MEASURE", (q,), u)])
        assert outs == [b]
        assert abs(abs(psi[full if b else 0]) - 1.0) <= 1e-14
        psi, outs = oracle.simulate_measured(n, _ghz(n) + [("RESET", (q,), u)])
        assert outs == [b]
        # the other qubits stay collapsed onto the outcome, q is back to 0
        idx = (full ^ (1 << q)) if b else 0
        assert abs(abs(psi[idx]) - 1.0) <= 1e-14


def _rep3(theta, error_on=None):
    """Three data qubits (0, 1, 2) in cos|000> + sin|111> and two ancillas
    (3, 4) measuring the parities Z0 Z1 and Z1 Z2."""
    g = [("RY", (0,), theta), ("CNOT", (0, 1), 0.0), ("CNOT", (1, 2), 0.0)]
    if error_on is not None:
        g.append(("X", (error_on,), 0.0))
    g += [("CNOT", (0, 3), 0.0), ("CNOT", (1, 3), 0.0), ("MEASURE", (3,), 0.5),
          ("CNOT", (1, 4), 0.0), ("CNOT", (2, 4), 0.0), ("MEASURE", (4,), 0.5)]
    return g


@pytest.mark.parametrize("err,syn", [(None, [0, 0]), (0, [1, 0]), (1, [1, 1]), (2, [0, 1])])
def test_repetition_code_syndromes(err, syn):
    theta = 1.3
    psi, outs = oracle.simulate_measured(5, _rep3(theta, err))
    assert outs == syn
    # the data keep their superposition; the ancillas hold the syndrome
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    flip = 0 if err is None else 1 << err
    anc = (syn[0] << 3) | (syn[1] << 4)
    ref = np.zeros(32, dtype=complex)
    ref[anc | (0 ^ flip)] = c
    ref[anc | (7 ^ flip)] = s
    assert np.max(np.abs(psi - ref)) <= 1e-14


def test_dense_projector_brute_force():
    g = np.random.default_rng(9090)
    names = ["RX", "RY", "RZ", "H", "S", "T"]
    for trial in range(12):
        n = int(g.integers(2, 6))
        gates = []
        for _ in range(int(g.integers(4, 12))):
            if g.random() < 0.3 and n > 1:
                a, b = (int(v) for v in g.choice(n, 2, replace=False))
                gates.append(("CNOT", (a, b), 0.0))
            else:
                gates.append((names[int(g.integers(len(names)))], (int(g.integers(n)),),
                              float(g.uniform(0, 2 * math.pi))))
        q, u = int(g.integers(n)), float(g.random())
        psi, outs = oracle.simulate_measured(n, gates + [("MEASURE", (q,), u)])
        before = brute.circuit_unitary(n, gates)[:, 0]
        # dense projector onto bit q = 1 from Kronecker factors
        P1 = brute.embed(n, {q: brute.P1})
        p1 = float(np.real(np.vdot(before, P1 @ before)))
        b = 1 if u < p1 else 0
        P = P1 if b else np.eye(1 << n) - P1
        ref = P @ before
        ref /= np.linalg.norm(ref)
        assert outs == [b], (trial, u, p1)
        assert np.max(np.abs(psi - ref)) <= 1e-12, trial
