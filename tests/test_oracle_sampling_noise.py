"""Pins of the oracle's sampler, counter hash, noise inputs and planner rules."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import planner_ref
from workloads import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    d = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))
    for s, o in zip(d["states"], d["outputs"]):
        assert oracle.splitmix64(int(s, 16)) == int(o, 16)


def test_uniform_range_and_mean():
    us = np.array([oracle.uniform(12345, t, s) for t in range(4) for s in range(4000)])
    assert us.min() >= 0.0 and us.max() < 1.0
    # mean of 16000 U(0,1): sd = 1/sqrt(12*16000)
    assert abs(us.mean() - 0.5) < 4 / math.sqrt(12 * 16000)
    assert len(set(us.tolist())) == us.size


def test_sample_two_outcome_tie_break():
    # p0 = 1/4, p1 = 3/4: outcome 0 iff u * total < CDF_0 = 1/4
    psi = np.array([0.5, math.sqrt(3) / 2], dtype=np.complex128)
    out = oracle.sample(psi, 1, 7, 3, 2000)
    for s, o in enumerate(out):
        u = oracle.uniform(7, 3, s)
        assert o == (0 if u < 0.25 else 1)
    frac1 = out.mean()
    assert abs(frac1 - 0.75) < 4 * math.sqrt(0.75 * 0.25 / 2000)


def test_sample_basis_state():
    n = 10
    psi = oracle.simulate(n, [("X", (3,), 0.0), ("X", (7,), 0.0)])
    out = oracle.sample(psi, n, 1, 0, 300)
    assert np.all(out == (1 << 3) | (1 << 7))


def test_sample_ghz():
    n = 14
    ang = [0.0] * (2 * n)
    ang[0] = math.pi / 2
    psi = oracle.simulate(n, gen.hea_layer(n, ang))
    out = oracle.sample(psi, n, 99, 5, 4096)
    assert set(np.unique(out).tolist()) <= {0, (1 << n) - 1}
    k = int(np.sum(out == 0))
    assert abs(k - 2048) < 4 * math.sqrt(4096 * 0.25)


def test_sample_product_state_marginals():
    n = 8
    g = np.random.default_rng(3)
    th = g.uniform(0.3, 2.8, n)
    psi = oracle.simulate(n, [("RY", (q,), float(th[q])) for q in range(n)])
    shots = 8000
    out = oracle.sample(psi, n, 2024, 11, shots)
    for q in range(n):
        p1 = math.sin(th[q] / 2) ** 2
        f = np.mean((out >> q) & 1)
        assert abs(f - p1) < 4 * math.sqrt(p1 * (1 - p1) / shots)


def test_noise_p_zero_is_noiseless():
    w0 = gen.small_noisy(8, 2, 2, 6, 0.0, seed=4, shots=0)
    for traj in w0.trajectories:
        assert traj == w0.suffix
    base = oracle.simulate(8, w0.prefix)
    ref = oracle.apply_gates(base.copy(), 8, w0.suffix)
    for traj in w0.trajectories:
        assert np.array_equal(oracle.apply_gates(base.copy(), 8, traj), ref)


def test_forced_x_flips_z():
    n = 9
    w = gen.small_vqe(n, 2, 1, 1, 1, seed=8)
    psi = oracle.simulate(n, w.task_gates(0))
    z3 = oracle.expect_terms(psi, n, [(1, 0, 1 << 3)])[0]
    oracle.apply_gates(psi, n, [("X", (3,), 0.0), ("RENORM", (), 0.0)])
    z3b = oracle.expect_terms(psi, n, [(1, 0, 1 << 3)])[0]
    assert abs(z3 + z3b) < 1e-13


def test_config4_jump_count_is_binomial():
    w = gen.config4()
    slots = sum(len(gg[1]) for gg in w.suffix)
    assert slots == 344
    jumps = sum(sum(1 for gg in t if gg[0] in ("X", "Y", "Z")) for t in w.trajectories)
    mean = 256 * slots * w.p
    sd = math.sqrt(256 * slots * w.p * (1 - w.p))
    assert abs(jumps - mean) < 4 * sd
    assert all(t[: len(t)] for t in w.trajectories)


def test_generator_deterministic():
    a, b = gen.small_vqe(12, 3, 2, 4, 9, seed=55), gen.small_vqe(12, 3, 2, 4, 9, seed=55)
    assert a.prefix == b.prefix and a.suffixes == b.suffixes and a.terms == b.terms
    c = gen.small_vqe(12, 3, 2, 4, 9, seed=56)
    assert c.prefix != a.prefix


def test_config_shapes():
    w1 = gen.config1()
    assert w1.n == 10 and len(w1.prefix) == 57 and w1.n_tasks == 16
    assert all(len(s) == 19 for s in w1.suffixes) and len(w1.terms) == 10
    w2 = gen.config2()
    assert w2.n == 24 and len(w2.prefix) == 426 and w2.n_tasks == 64
    assert all(len(s) == 142 for s in w2.suffixes) and len(w2.terms) == 50
    assert len({(x, z) for _, x, z in w2.terms}) == 50
    assert all(1 <= bin(x | z).count("1") <= 4 for _, x, z in w2.terms)
    w3 = gen.config3()
    assert len(w3.levels) == 2 and len(w3.levels[0]) == 8 and len(w3.levels[1]) == 64
    assert len(w3.leaves) == 512
    layers = [len(g) // 59 for _, g in w3.leaves]
    assert min(layers) >= 3 and max(layers) <= 14


def test_eq2_hand_values():
    # (N-1) C_p > C_m + N (C_r + C_h) + delta
    assert planner_ref.eq2_reuse(2, 10.0, 1.0, 0.5, 0.0, 0.0) is True      # 10 > 2
    assert planner_ref.eq2_reuse(2, 10.0, 9.0, 0.5, 0.0, 0.0) is False     # 10 > 10 fails
    assert planner_ref.eq2_reuse(1, 10.0, 0.0, 0.0, 0.0, 0.0) is False     # nothing to save
    assert planner_ref.eq2_reuse(5, 1.0, 0.0, 0.0, 0.0, 4.0) is False      # delta blocks
    assert planner_ref.eq2_reuse(5, 1.0, 0.0, 0.0, 0.0, 3.9) is True


def test_break_even_is_two_with_negligible_overheads():
    # Sec. VI (Q4): with negligible materialize/reload cost, N* = 2
    assert planner_ref.break_even_tasks(10.0, 1.0, 1e-9, 1e-9) == 2
    # the 10 % guard pushes a marginal case to abstention
    assert planner_ref.guarded_reuse(2, 1.0, 10.0, 0.0, 0.0, guard=0.10) is False
    assert planner_ref.guarded_reuse(2, 1.0, 10.0, 0.0, 0.0, guard=0.0) is True
