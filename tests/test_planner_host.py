"""Host checks of the workload planner (no GPU): prefix trie, Eq. (1)
provenance, Eq. (2) decisions (cross-checked with the oracle's independent
closed form), abstention on negative controls, EXPLAIN records."""
import json

import numpy as np
import pytest

from oracle import planner_ref
from paper_2609_23664_amd import planner as P
from workloads import gen


def _tasks(w):
    return [w.task_gates(t) for t in range(w.n_tasks)]


def test_fingerprint_is_structural():
    g1 = [("RY", (0,), 0.5), ("CNOT", (0, 1), 0.0)]
    g2 = [("RY", (0,), 0.5), ("CNOT", (1, 0), 0.0)]
    g3 = [("RY", (0,), 0.5000000001), ("CNOT", (0, 1), 0.0)]
    assert P.fingerprint(4, g1) == P.fingerprint(4, list(g1))
    assert len({P.fingerprint(4, g) for g in (g1, g2, g3)}) == 3
    assert P.fingerprint(4, g1) != P.fingerprint(5, g1)   # layout is hashed
    assert len(P.fingerprint(4, [])) == 32


def test_config2_one_shared_prefix():
    w = gen.config2()
    tasks = _tasks(w)
    plan = P.plan_workload(24, tasks)
    root = plan.nodes[0]
    assert (root.start, root.end) == (0, len(w.prefix))
    assert len(root.children) == w.n_tasks
    assert plan.decision == "REUSE" and plan.materialized == [0]
    assert all(a == 0 for a in plan.anchor)
    # the node's decision is the oracle's closed form on the same costs
    cost = P.CostModel(24)
    c_prefix = cost.segment(w.prefix)
    c_suffix = np.mean([cost.segment(s) for s in w.suffixes])
    assert root.c_prefix == pytest.approx(c_prefix)
    assert bool(planner_ref.guarded_reuse(w.n_tasks, c_prefix, c_suffix, 0.0, 0.0))
    # byte-model speedup of the plan
    assert plan.est_direct / plan.est_reuse > 3.0


def test_negative_control_abstains():
    w = gen.small_vqe(12, 0, 3, 6, 4, seed=9)   # no shared layer
    plan = P.plan_workload(12, _tasks(w))
    assert plan.decision == "ABSTAIN"
    assert plan.materialized == []
    assert all(a is None for a in plan.anchor)


def test_single_task_abstains():
    w = gen.small_vqe(12, 3, 1, 1, 4, seed=9)
    plan = P.plan_workload(12, _tasks(w))
    assert plan.decision == "ABSTAIN"


@pytest.mark.parametrize("n_tasks,expect", [(2, True), (8, True)])
def test_eq2_matches_oracle_rule(n_tasks, expect):
    w = gen.small_vqe(12, 3, 1, n_tasks, 4, seed=10 + n_tasks)
    plan = P.plan_workload(12, _tasks(w))
    root = plan.nodes[0]
    cost = P.CostModel(12)
    c_suffix = np.mean([cost.segment(s) for s in w.suffixes])
    ref = bool(planner_ref.guarded_reuse(n_tasks, root.c_prefix, c_suffix, 0.0, 0.0))
    assert (root.decision == "REUSE") == ref == expect


def test_guard_pushes_marginal_case_to_abstain():
    """A two-task workload whose shared prefix is tiny next to the suffixes:
    Eq. (2) without the guard says reuse, with delta = 0.1 est_reuse it
    abstains (the paper's conservative margin)."""
    n = 12
    g = np.random.default_rng(1)
    pre = [("RY", (0,), 0.3)]
    # suffixes of 8 segments (each RENORM ends a pass): 8+ passes per task
    suf = [[gg for _ in range(8) for gg in ([("RY", (q,), float(g.uniform(0, 6))) for q in range(n)]
                                               + [("RENORM", (), 0.0)])] for _ in range(2)]
    tasks = [pre + s for s in suf]
    plan0 = P.plan_workload(n, tasks, guard=0.0)
    plan1 = P.plan_workload(n, tasks, guard=0.10)
    assert plan0.nodes[0].decision == "REUSE"
    assert plan1.nodes[0].decision == "ABSTAIN"


def test_trie_levels_and_leaves():
    w = gen.small_trie(12, 3, 3, 1, 3, seed=4, shots=0)
    tasks = [w.leaf_path(k) for k in range(len(w.leaves))]
    plan = P.plan_workload(12, tasks)
    # depth-1 nodes: 3 subtrees of 9 leaves; depth-2: 9 nodes of 3 leaves
    by_depth = {}
    for v in plan.nodes:
        by_depth.setdefault(v.depth, []).append(v)
    assert sorted(len(v.tasks) for v in by_depth[1]) == [9, 9, 9]
    assert sorted(len(v.tasks) for v in by_depth[2]) == [3] * 9
    assert all(len(v.tasks) == 1 for v in by_depth[3])
    # every materialized node is shared and its anchor chain is consistent
    for vid in plan.materialized:
        assert len(plan.nodes[vid].tasks) >= 2
    for t, a in enumerate(plan.anchor):
        if a is not None:
            assert t in plan.nodes[a].tasks


def test_noisy_trajectories_share_jump_free_suffix():
    w = gen.small_noisy(10, 3, 2, 40, 1e-2, seed=5, shots=0)
    tasks = [list(w.prefix) + list(t) for t in w.trajectories]
    plan = P.plan_workload(10, tasks)
    clean = [t for t, tr in enumerate(w.trajectories) if tr == list(w.suffix)]
    assert clean, "seed should give jump-free trajectories"
    # all jump-free trajectories end in one trie node
    ends = {v.id for v in plan.nodes for t in v.ending if t in clean}
    assert len(ends) == 1
    assert plan.decision == "REUSE"


def test_config5_negative_controls_abstain():
    specs = [s for s in gen.config5_specs(200) if s.negative and s.n <= 16][:5]
    assert specs
    for s in specs:
        w = gen.config5_workload(s, max_tasks=8)
        plan = P.plan_workload(w.n, _tasks(w))
        assert plan.decision == "ABSTAIN", s


def test_explain_trace_is_json():
    w = gen.small_vqe(12, 3, 1, 4, 4, seed=2)
    tasks = _tasks(w)
    plan = P.plan_workload(12, tasks)
    tr = P._explain("t", plan, tasks, 12, [])
    d = json.loads(tr.to_json())
    assert d["decision"] == "REUSE"
    root = d["nodes"][0]
    assert root["provenance"] == P.fingerprint(12, w.prefix).hex()
    assert "Eq.(2)" in root["reason"]


class _StubModel:
    """Stands in for the trained perceptron: predicts a fixed correction of
    the analytic log ratio (and log t_reuse)."""

    def __init__(self, pred, lo=-1e9, hi=1e9):
        self.pred, self.lo, self.hi = np.asarray(pred, dtype=np.float32), lo, hi
        self.delta = 0.1

    def in_range(self, f):
        return bool(np.all(np.asarray(f) >= self.lo) and np.all(np.asarray(f) <= self.hi))

    def predict(self, x):
        return np.tile(self.pred, (len(x), 1))


def test_learned_hook_drives_eq2_decision():
    """The learned model's decision replaces Eq. (2) at each trie node; out of
    its training range the analytic rule decides (hook returns None)."""
    from paper_2609_23664_amd import costmodel as CM
    from paper_2609_23664_amd.planner import plan_workload
    w = gen.small_vqe(12, 3, 1, 6, 4, seed=11)
    tasks = [w.task_gates(t) for t in range(w.n_tasks)]
    analytic = plan_workload(w.n, tasks)
    assert analytic.materialized                       # the byte rule reuses here
    never = plan_workload(w.n, tasks, decide=CM.planner_hook(_StubModel([-9.0, 0.0])))
    assert not never.materialized                      # predicted ratio e^-9 x the analytic one
    always = plan_workload(w.n, tasks, decide=CM.planner_hook(_StubModel([5.0, 0.0])))
    assert always.materialized == analytic.materialized
    out_of_range = plan_workload(w.n, tasks, decide=CM.planner_hook(_StubModel([-9.0, 0.0], 0.0, 0.0)))
    assert out_of_range.materialized == analytic.materialized
