"""Pins of the CPU oracle against facts fixed by the mathematics (CPU only).

Each test checks the oracle against something other than itself: closed-form
amplitudes (Bell, GHZ, one hardware-efficient layer, the 1-D cluster state),
closed-form expectations (single rotations, product states, GHZ), a dense
Kronecker-product brute force at <= 8 qubits, norm preservation, the
prefix-XOR form of the CNOT ladder, and the reuse rewrite of Sec. I / Fig. 1
(prefix once, suffix from the boundary state) being exactly the direct run.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from workloads import gen


def test_bell_state():
    psi = oracle.simulate(2, [("H", (0,), 0.0), ("CNOT", (0, 1), 0.0)])
    r = 1 / math.sqrt(2)
    assert np.allclose(psi, [r, 0, 0, r], atol=1e-15)


@pytest.mark.parametrize("n", [2, 3, 8, 16, 20])
def test_ghz_from_ry_and_ladder(n):
    # RY(pi/2) on q0 (all other angles 0) then the CNOT ladder gives GHZ.
    angles = [0.0] * (2 * n)
    angles[0] = math.pi / 2
    psi = oracle.simulate(n, gen.hea_layer(n, angles))
    r = 1 / math.sqrt(2)
    assert abs(psi[0] - r) < 1e-14
    assert abs(psi[(1 << n) - 1] - r) < 1e-14
    mask = np.ones(psi.size, dtype=bool)
    mask[[0, (1 << n) - 1]] = False
    assert np.max(np.abs(psi[mask])) < 1e-15


def test_cnot_ladder_is_prefix_xor_permutation():
    n = 9
    g = np.random.default_rng(1)
    psi = g.standard_normal(1 << n) + 1j * g.standard_normal(1 << n)
    psi /= np.linalg.norm(psi)
    ladder = [("CNOT", (q, q + 1), 0.0) for q in range(n - 1)]
    out = oracle.apply_gates(psi.copy(), n, ladder)
    j = np.arange(1 << n)
    src = j ^ ((j << 1) & ((1 << n) - 1))
    assert np.array_equal(out, psi[src])


@pytest.mark.parametrize("n", [5, 12, 20])
def test_one_hea_layer_closed_form(n):
    # psi[j] = prod_q a_q[j_q xor j_{q-1}] with j_{-1} = 0,
    # a_q[0] = e^{-i phi/2} cos(theta/2), a_q[1] = e^{+i phi/2} sin(theta/2).
    g = np.random.default_rng(n)
    ang = g.uniform(0, 2 * math.pi, 2 * n)
    psi = oracle.simulate(n, gen.hea_layer(n, ang))
    th, ph = ang[0::2], ang[1::2]
    a0 = np.exp(-0.5j * ph) * np.cos(th / 2)
    a1 = np.exp(0.5j * ph) * np.sin(th / 2)
    js = np.arange(1 << n) if n <= 12 else g.integers(0, 1 << n, 10000)
    for j in js:
        v = 1.0 + 0j
        prev = 0
        for q in range(n):
            b = (int(j) >> q) & 1
            v *= a1[q] if (b ^ prev) else a0[q]
            prev = b
        assert abs(psi[j] - v) < 1e-13


def test_cz_ladder_cluster_state():
    n = 10
    psi = oracle.simulate(n, gen.cz_layer(n, [math.pi / 2] * n))
    j = np.arange(1 << n)
    s = np.zeros_like(j)
    for q in range(n - 1):
        s += ((j >> q) & 1) * ((j >> (q + 1)) & 1)
    expect = (2.0 ** (-n / 2)) * np.where(s % 2 == 1, -1.0, 1.0)
    assert np.allclose(psi, expect, atol=1e-14)
    # theta = 0: the CZ ladder acts on e_0, every Z_i and Z_i Z_{i+1} is +1
    psi0 = oracle.simulate(n, gen.cz_layer(n, [0.0] * n))
    assert psi0[0] == 1.0
    terms = [(1.0, 0, 1 << i) for i in range(n)] + [(1.0, 0, 3 << i) for i in range(n - 1)]
    assert np.allclose(oracle.expect_terms(psi0, n, terms), 1.0, atol=0)


@pytest.mark.parametrize("q", [0, 3, 6])
def test_single_rotation_expectations(q):
    n = 7
    g = np.random.default_rng(q)
    for _ in range(5):
        th, ph = g.uniform(0, 2 * math.pi, 2)
        psi = oracle.simulate(n, [("RY", (q,), th), ("RZ", (q,), ph)])
        ex, ey, ez = oracle.expect_terms(psi, n, [(1, 1 << q, 0), (1, 1 << q, 1 << q), (1, 0, 1 << q)])
        assert abs(ex - math.sin(th) * math.cos(ph)) < 1e-14
        assert abs(ey - math.sin(th) * math.sin(ph)) < 1e-14
        assert abs(ez - math.cos(th)) < 1e-14


def _bloch(th, ph):
    return {"X": math.sin(th) * math.cos(ph), "Y": math.sin(th) * math.sin(ph), "Z": math.cos(th), "I": 1.0}


@pytest.mark.parametrize("n", [6, 14])
def test_product_state_expectations(n):
    # layer without the ladder: <P> factorises into single-qubit Bloch values
    g = np.random.default_rng(100 + n)
    ang = g.uniform(0, 2 * math.pi, 2 * n)
    gates = [gg for gg in gen.hea_layer(n, ang) if gg[0] != "CNOT"]
    psi = oracle.simulate(n, gates)
    terms = gen.random_pauli_terms(gen.rng(7, n), n, 40)
    vals = oracle.expect_terms(psi, n, terms)
    for t, v in zip(terms, vals):
        s = gen.pauli_string(t, n)
        e = 1.0
        for q, ch in enumerate(s):
            e *= _bloch(ang[2 * q], ang[2 * q + 1])[ch]
        assert abs(v - e) < 1e-13


def test_ghz_expectations():
    n = 12
    ang = [0.0] * (2 * n)
    ang[0] = math.pi / 2
    psi = oracle.simulate(n, gen.hea_layer(n, ang))
    full = (1 << n) - 1
    terms = [(1, 0, (1 << 2) | (1 << 9)), (1, full, 0), (1, 0, 1 << 5)]
    zz, xs, z5 = oracle.expect_terms(psi, n, terms)
    assert abs(zz - 1) < 1e-14 and abs(xs - 1) < 1e-14 and abs(z5) < 1e-14


def _random_circuit(n, g, count):
    names1 = ["X", "Y", "Z", "H", "S", "SDG", "T", "TDG", "RX", "RY", "RZ", "P"]
    gates = []
    for _ in range(count):
        r = g.random()
        if r < 0.7:
            gates.append((names1[g.integers(len(names1))], (int(g.integers(n)),),
                          float(g.uniform(0, 2 * math.pi))))
        else:
            a, b = g.choice(n, 2, replace=False)
            gates.append((("CNOT", "CZ")[int(g.integers(2))], (int(a), int(b)), 0.0))
    return gates


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_dense_unitary_brute_force(n):
    g = np.random.default_rng(200 + n)
    gates = _random_circuit(n, g, 60) if n >= 2 else [
        (nm, (0,), 0.7) for nm in ["H", "RX", "RY", "RZ", "S", "T", "X", "Y", "Z", "P", "SDG", "TDG"]]
    psi = oracle.simulate(n, gates)
    u = brute.circuit_unitary(n, gates)
    assert np.max(np.abs(psi - u[:, 0])) < 1e-12
    terms = gen.random_pauli_terms(gen.rng(9, n), n, min(12, 4 ** n - 1), max_weight=min(4, n))
    vals = oracle.expect_terms(psi, n, terms)
    for (c, x, z), v in zip(terms, vals):
        ref = np.vdot(psi, brute.pauli_matrix(n, x, z) @ psi)
        assert abs(ref.imag) < 1e-12
        assert abs(v - ref.real) < 1e-12


def test_norm_preserved():
    n = 12
    w = gen.small_vqe(n, 6, 2, 1, 1, seed=5)
    psi = oracle.simulate(n, w.task_gates(0))
    assert abs(oracle.norm2(psi) - 1.0) < 1e-12


def test_reuse_rewrite_is_bitwise_direct():
    w = gen.small_vqe(11, 4, 2, 5, 6, seed=17)
    reused = oracle.run_workload_reuse(w)
    for t in range(w.n_tasks):
        assert np.array_equal(reused[t], oracle.run_task_direct(w, t))


def test_renorm_marker():
    n = 5
    psi = oracle.zero_state(n) * 3.0
    oracle.apply_gates(psi, n, [("RENORM", (), 0.0)])
    assert abs(oracle.norm2(psi) - 1.0) < 1e-15
