"""GPU tests of the planned workload executor (run_workload): the planned
execution equals direct per-task execution with the same segment cuts bit
for bit (states, expectations, samples), and matches the oracle. Every case
prints its name before running."""
import sys

import numpy as np
import pytest

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu

FID_TOL = 1e-6
EXP_TOL = 1e-5


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2609_23664_amd import binding
    assert torch.cuda.is_available()
    c = binding.Ctx(0)
    yield c
    c.sync()


def _same(ra, rb):
    for x, y in zip(ra.states, rb.states):
        assert np.array_equal(x, y)
    if ra.expectations is not None:
        assert ra.expectations == rb.expectations
    if ra.samples is not None:
        assert np.array_equal(ra.samples, rb.samples)


def test_config1_workload(ctx):
    say("run_workload config1")
    w = gen.config1()
    tasks = [w.task_gates(t) for t in range(w.n_tasks)]
    from paper_2609_23664_amd import planner as P
    plan = P.plan_workload(w.n, tasks)
    assert plan.decision == "REUSE"
    ra, tr, cr = P.run_workload(ctx, w.n, tasks, terms=w.terms, keep_states=True, plan=plan)
    rb, _, _ = P.run_workload(ctx, w.n, tasks, terms=w.terms, keep_states=True, plan=plan, mode="direct")
    _same(ra, rb)
    scale = sum(abs(t[0]) for t in w.terms)
    for t in range(w.n_tasks):
        ref = oracle.simulate(w.n, tasks[t])
        assert 1 - oracle.fidelity(ra.states[t].astype(np.complex128), ref) <= FID_TOL
        assert abs(ra.expectations[t] - oracle.expect(ref, w.n, w.terms)) <= EXP_TOL * scale
    assert tr.decision == "REUSE" and cr.plan == "reuse"


def test_trie_workload_with_sampling(ctx):
    say("run_workload trie 12q")
    from paper_2609_23664_amd import planner as P
    w = gen.small_trie(12, 3, 3, 1, 3, seed=21, shots=256)
    tasks = [w.leaf_path(k) for k in range(len(w.leaves))]
    plan = P.plan_workload(w.n, tasks)
    assert plan.decision == "REUSE" and len(plan.materialized) >= 3
    ra, tr, _ = P.run_workload(ctx, w.n, tasks, shots=256, seed=77, keep_states=True, plan=plan)
    rb, _, _ = P.run_workload(ctx, w.n, tasks, shots=256, seed=77, keep_states=True, plan=plan,
                              mode="direct")
    _same(ra, rb)
    for k in (0, 13, len(tasks) - 1):
        ref = oracle.simulate(w.n, tasks[k])
        assert 1 - oracle.fidelity(ra.states[k].astype(np.complex128), ref) <= FID_TOL
    assert sum(1 for v in tr.nodes if v["decision"] == "REUSE") == len(plan.materialized)


def test_noisy_workload(ctx):
    say("run_workload noisy 12q")
    from paper_2609_23664_amd import planner as P
    w = gen.small_noisy(12, 3, 2, 24, 2e-2, seed=31, shots=128)
    tasks = [list(w.prefix) + list(t) for t in w.trajectories]
    plan = P.plan_workload(w.n, tasks)
    ra, _, _ = P.run_workload(ctx, w.n, tasks, shots=128, seed=5, keep_states=True, plan=plan)
    rb, _, _ = P.run_workload(ctx, w.n, tasks, shots=128, seed=5, keep_states=True, plan=plan,
                              mode="direct")
    _same(ra, rb)
    for t in (0, 5, 23):
        ref = oracle.simulate(w.n, tasks[t])
        assert 1 - oracle.fidelity(ra.states[t].astype(np.complex128), ref) <= FID_TOL


def test_negative_control_abstains_and_is_correct(ctx):
    say("run_workload negative control")
    from paper_2609_23664_amd import planner as P
    w = gen.small_vqe(11, 0, 3, 5, 6, seed=41)
    tasks = [w.task_gates(t) for t in range(w.n_tasks)]
    ra, tr, cr = P.run_workload(ctx, w.n, tasks, terms=w.terms, keep_states=True)
    assert tr.decision == "ABSTAIN" and cr.plan == "abstain"
    scale = sum(abs(t[0]) for t in w.terms)
    for t in range(w.n_tasks):
        ref = oracle.simulate(w.n, tasks[t])
        assert abs(ra.expectations[t] - oracle.expect(ref, w.n, w.terms)) <= EXP_TOL * scale
