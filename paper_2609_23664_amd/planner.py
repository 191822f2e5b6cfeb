"""Workload planner (host side) and workload executor.

Implements the planning layer of the method (Sec. III-A and Sec. IV):

* Eq. (1) structural fingerprints, here of every cumulative prefix, used as
  the provenance of boundary states;
* shared-prefix detection: a radix trie over the tasks' gate records
  (longest common prefixes; two gates match when kind, qubits and bound
  parameter are equal);
* the Eq. (2) materialize-versus-recompute rule, evaluated top-down over
  the trie (a bounded search: each node is either materialized or folded
  into its tasks' suffixes), with an analytic byte-count cost model and
  the safety margin delta = 0.1 * est_reuse; ABSTAIN when no node
  survives (a single task, no shared segment, or no profit);
* execution through the C ABI (``binding``): materialized nodes are run
  once and frozen as exact boundary snapshots, every task continues from
  its nearest one; a legality refusal falls back to direct execution;
* the three output records: ExecutionResult, ExplainTrace, CostRecord.

The plan changes timing only: results are the same for every plan
(bit-identical to direct execution with the same segment cuts).
"""
from __future__ import annotations

import hashlib
import json
import math
import struct
import time
from dataclasses import asdict, dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from .binding import GATE_KIND

Gate = Tuple[str, Tuple[int, ...], float]

DELTA_GUARD = 0.10  # delta = 0.10 * est_reuse (the 10 % guard)


# ---------------------------------------------------------------- Eq. (1)
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


# ---------------------------------------------------------------- trie
@dataclass
class Node:
    """A trie node: gates [start, end) of its tasks are shared by all of
    them (and, for a non-root node, the gate at `start` is where they
    diverged from their siblings)."""
    id: int
    depth: int
    start: int
    end: int
    tasks: List[int]
    parent: Optional[int]
    children: List[int] = field(default_factory=list)
    ending: List[int] = field(default_factory=list)  # tasks whose gates end at `end`
    # planning
    seg_bytes: float = 0.0
    decision: str = "FOLD"
    reason: str = ""
    c_prefix: float = 0.0
    est_direct: float = 0.0
    est_reuse: float = 0.0
    delta: float = 0.0


def build_trie(tasks: Sequence[Sequence[Gate]]) -> List[Node]:
    """Radix trie of the task gate lists (exact gate records). Node 0 is
    the root (start = 0; its segment is the prefix shared by all tasks)."""
    codes: Dict[Tuple, int] = {}
    lens = np.array([len(t) for t in tasks], dtype=np.int64)
    lmax = int(lens.max()) if len(tasks) else 0
    ids = np.full((len(tasks), lmax + 1), -1, dtype=np.int64)
    for i, t in enumerate(tasks):
        for j, (name, qs, p) in enumerate(t):
            key = (name, tuple(qs), float(p))
            c = codes.get(key)
            if c is None:
                c = codes[key] = len(codes)
            ids[i, j] = c
    nodes: List[Node] = []

    def make(group: np.ndarray, start: int, depth: int, parent: Optional[int]) -> int:
        ref = ids[group[0]]
        minlen = int(lens[group].min())
        if len(group) == 1:
            end = int(lens[group[0]])
        elif minlen > start:
            eq = (ids[group, start:minlen] == ref[start:minlen]).all(axis=0)
            end = start + (int(np.argmin(eq)) if not eq.all() else minlen - start)
        else:
            end = start
        node = Node(id=len(nodes), depth=depth, start=start, end=end,
                    tasks=[int(t) for t in group], parent=parent)
        nodes.append(node)
        if len(group) == 1:
            node.ending = [int(group[0])]
            return node.id
        at_end = group[lens[group] == end]
        node.ending = [int(t) for t in at_end]
        rest = group[lens[group] > end]
        if len(rest):
            nxt = ids[rest, end]
            for code in np.unique(nxt):
                sub = rest[nxt == code]
                cid = make(sub, end, depth + 1, node.id)
                node.children.append(cid)
        return node.id

    if len(tasks):
        make(np.arange(len(tasks)), 0, 0, None)
    return nodes


def path_to(nodes: List[Node], v: int) -> List[int]:
    """Node ids from the root to v (inclusive)."""
    out = []
    while v is not None:
        out.append(v)
        v = nodes[v].parent
    return out[::-1]


# ---------------------------------------------------------------- Eq. (2)
def eq2(n_tasks: int, c_prefix: float, c_materialize: float, c_reload: float,
        c_handoff: float, delta: float) -> bool:
    """Eq. (2): (N - 1) C_prefix > C_materialize + N (C_reload + C_handoff) + delta."""
    return (n_tasks - 1) * c_prefix > c_materialize + n_tasks * (c_reload + c_handoff) + delta


@dataclass
class CostModel:
    """Analytic byte-count costs (Sec. IV-C with costs measured in HBM
    bytes). A segment costs the bytes of the tile passes the library runs
    for it; materializing a frozen snapshot costs nothing (the boundary
    slot becomes the artifact); the reload is fused into the first suffix
    pass (it reads the snapshot instead of the slot), except for a task
    with nothing left to run, which costs one copy; a same-backend handoff
    costs nothing."""
    n: int
    tile_bits: int = 14
    _cache: Dict[Tuple, float] = field(default_factory=dict)

    @property
    def state_bytes(self) -> float:
        return 8.0 * (1 << self.n)

    def segment(self, gates: Sequence[Gate]) -> float:
        if not gates:
            return 0.0
        key = tuple((g[0], tuple(g[1]), float(g[2])) for g in gates)
        c = self._cache.get(key)
        if c is None:
            from .binding import plan_cost
            c = plan_cost(self.n, list(gates), self.tile_bits)[1]
            self._cache[key] = c
        return c

    def materialize(self) -> float:
        return 0.0

    def reload(self, remainder_empty: bool) -> float:
        return 2.0 * self.state_bytes if remainder_empty else 0.0

    def handoff(self) -> float:
        return 0.0


@dataclass
class Plan:
    n: int
    nodes: List[Node]
    materialized: List[int]
    anchor: List[Optional[int]]      # per task: nearest materialized node (None: direct)
    decision: str                    # REUSE or ABSTAIN
    reason: str
    est_direct: float
    est_reuse: float
    planning_ms: float
    # marshalled gate segments (task, start, end) -> GateArray, filled on use
    arrays: Dict[Tuple[int, int, int], object] = field(default_factory=dict)
    # Eq. (1) provenance of each node's prefix, filled on use
    fps: Dict[int, bytes] = field(default_factory=dict)

    def node_fingerprint(self, tasks, vid: int) -> bytes:
        """Eq. (1) fingerprint of the gates from |0...0> to the end of node vid."""
        fp = self.fps.get(vid)
        if fp is None:
            v = self.nodes[vid]
            fp = self.fps[vid] = fingerprint(self.n, tasks[v.tasks[0]][:v.end])
        return fp

    def segment_array(self, tasks, t: int, b0: int, b1: int):
        key = (t, b0, b1)
        a = self.arrays.get(key)
        if a is None:
            from .binding import GateArray
            a = self.arrays[key] = GateArray(list(tasks[t][b0:b1]))
        return a


def plan_workload(n: int, tasks: Sequence[Sequence[Gate]], cost: Optional[CostModel] = None,
                  guard: float = DELTA_GUARD,
                  decide: Optional[Callable[[Node, dict], Optional[bool]]] = None,
                  ) -> Plan:
    """Bounded top-down search: a node is materialized when Eq. (2) holds
    for it, C_prefix being the cost from its nearest materialized ancestor.
    `decide(node, info)` may override the rule (a learned cost model; info
    holds n, tasks, c_prefix, suffix_costs, state_bytes, the estimates and
    gate counts); returning None keeps the analytic decision."""
    t0 = time.perf_counter()
    cost = cost or CostModel(n)
    nodes = build_trie(tasks)
    B = cost.state_bytes
    for v in nodes:
        v.seg_bytes = cost.segment(tasks[v.tasks[0]][v.start:v.end])
    # cost of each task's gates below a node (sum of segment costs)
    below: Dict[int, Dict[int, float]] = {}

    def suffix_costs(vid: int) -> Dict[int, float]:
        if vid in below:
            return below[vid]
        v = nodes[vid]
        out = {t: 0.0 for t in v.ending}
        for c in v.children:
            for t, cst in suffix_costs(c).items():
                out[t] = nodes[c].seg_bytes + cst
        below[vid] = out
        return out

    materialized: List[int] = []
    anchor_of: Dict[int, Optional[int]] = {0: None} if nodes else {}
    order = sorted(range(len(nodes)), key=lambda i: nodes[i].depth)
    for vid in order:
        v = nodes[vid]
        a = anchor_of.get(vid)
        # C_prefix: segments from the nearest materialized ancestor to v
        c_prefix, u = 0.0, vid
        while u is not None and u != a:
            c_prefix += nodes[u].seg_bytes
            u = nodes[u].parent
        N = len(v.tasks)
        suf = suffix_costs(vid)
        c_suffix = sum(suf.values()) / max(1, N)
        n_empty = len(v.ending)
        est_direct = N * (c_prefix + c_suffix)
        est_reuse = c_prefix + cost.materialize() + N * (cost.handoff() + c_suffix) + \
            n_empty * cost.reload(True)
        delta = guard * est_reuse
        v.c_prefix, v.est_direct, v.est_reuse, v.delta = c_prefix, est_direct, est_reuse, delta
        if N < 2:
            ok, why = False, "single task below this node"
        elif v.end == v.start and vid != 0:
            ok, why = False, "no shared segment"
        elif c_prefix <= 0.0:
            ok, why = False, "empty shared prefix"
        else:
            c_reload = n_empty * cost.reload(True) / N
            ok = eq2(N, c_prefix, cost.materialize(), c_reload, cost.handoff(), delta)
            why = (f"Eq.(2): (N-1)C_prefix = {(N - 1) * c_prefix:.4g} B "
                   f"{'>' if ok else '<='} C_mat + N(C_reload + C_handoff) + delta = "
                   f"{cost.materialize() + N * (c_reload + cost.handoff()) + delta:.4g} B")
            if decide is not None:
                info = {"n": n, "tasks": N, "c_prefix": c_prefix, "suffix_costs": list(suf.values()),
                        "state_bytes": B, "est_direct": est_direct, "est_reuse": est_reuse,
                        "prefix_gates": v.end - (nodes[a].end if a is not None else 0),
                        "suffix_gates": float(np.mean([len(tasks[t]) - v.end for t in v.tasks]))}
                d = decide(v, info)
                if d is not None:
                    why += f"; learned model: {'reuse' if d else 'abstain'}"
                    ok = bool(d)
        v.decision = "REUSE" if ok else "ABSTAIN"
        v.reason = why
        if ok:
            materialized.append(vid)
        for c in v.children:
            anchor_of[c] = vid if ok else a
        if ok:
            anchor_of[vid] = vid
    anchor: List[Optional[int]] = [None] * len(tasks)
    for v in nodes:
        for t in v.ending:
            anchor[t] = anchor_of.get(v.id) if v.id not in materialized else v.id
    root = nodes[0] if nodes else None
    # whole-workload estimates (direct: every task from |0>)
    est_direct = sum(suffix_costs(0).values()) + (root.seg_bytes * len(tasks) if root else 0.0)
    est_reuse = 0.0
    for vid in materialized:
        est_reuse += nodes[vid].c_prefix
    for t in range(len(tasks)):
        a = anchor[t]
        start = nodes[a].end if a is not None else 0
        est_reuse += cost.segment(tasks[t][start:]) if start < len(tasks[t]) else cost.reload(True)
    decision = "REUSE" if materialized else "ABSTAIN"
    reason = (f"{len(materialized)} boundary state(s) materialized" if materialized else
              ("no node passes Eq.(2)" if len(tasks) > 1 else "single task"))
    return Plan(n=n, nodes=nodes, materialized=materialized, anchor=anchor, decision=decision,
                reason=reason, est_direct=est_direct, est_reuse=est_reuse,
                planning_ms=(time.perf_counter() - t0) * 1e3)


# ---------------------------------------------------------------- records
@dataclass
class ExecutionResult:
    expectations: Optional[List[float]] = None
    samples: Optional[np.ndarray] = None     # [task, shot] basis indices
    states: Optional[List[np.ndarray]] = None

    def to_json(self) -> str:
        d = {"expectations": self.expectations,
             "samples": None if self.samples is None else self.samples.tolist()}
        return json.dumps(d)


@dataclass
class ExplainTrace:
    workload: str
    decision: str
    reason: str
    nodes: List[dict]
    refusals: List[dict]

    def to_json(self) -> str:
        return json.dumps(asdict(self))


@dataclass
class CostRecord:
    plan: str
    predicted_direct_bytes: float
    predicted_reuse_bytes: float
    planning_ms: float
    realized_ms: Dict[str, float]

    def to_json(self) -> str:
        return json.dumps(asdict(self))


def _explain(name: str, plan: Plan, tasks: Sequence[Sequence[Gate]], n: int,
             refusals: List[dict]) -> ExplainTrace:
    rows = []
    for v in plan.nodes:
        fp = plan.node_fingerprint(tasks, v.id).hex() if v.decision == "REUSE" else None
        rows.append({"id": v.id, "depth": v.depth, "parent": v.parent, "gates": [v.start, v.end],
                     "tasks": len(v.tasks), "decision": v.decision, "reason": v.reason,
                     "c_prefix_bytes": v.c_prefix, "est_direct_bytes": v.est_direct,
                     "est_reuse_bytes": v.est_reuse, "delta_bytes": v.delta,
                     "provenance": fp})
    return ExplainTrace(workload=name, decision=plan.decision, reason=plan.reason, nodes=rows,
                        refusals=refusals)


# ---------------------------------------------------------------- executor
def _reset_runs(st, slots) -> None:
    """Set the given slots to |0...0>: one reset per run of consecutive slots.
    Only tasks that start in place need it; a task with a source state has its
    destination written in full by its first pass."""
    ss = sorted(set(slots))
    i = 0
    while i < len(ss):
        j = i + 1
        while j < len(ss) and ss[j] == ss[j - 1] + 1:
            j += 1
        st.reset(ss[i], j - i)
        i = j


def run_workload(ctx, n: int, tasks: Sequence[Sequence[Gate]], terms=None, shots: int = 0,
                 seed: int = 0, name: str = "workload", mode: str = "plan",
                 plan: Optional[Plan] = None, keep_states: bool = False,
                 cost: Optional[CostModel] = None, decide=None,
                 ) -> Tuple[ExecutionResult, ExplainTrace, CostRecord]:
    """Plan and execute a workload of related tasks on the ctx's GPU.

    mode "plan": the planner's decision; "direct": every task from |0...0>
    with the same segment cuts (the reference for bit-identity); "reuse":
    materialize every shared node regardless of cost.

    When the device memory (or the context's QW_OPT_DEVICE_MEM_CAP) cannot
    hold the materialized nodes and every task's state at once, the library
    refuses with QW_E_OOM and the tasks run in chunks of half as many (then a
    quarter, ... down to one) through the same slots, the materialized nodes
    kept: every task runs the same kernels on the same inputs, so states,
    expectations and samples equal those of the unchunked run (samples keep
    each task's own counter-hash stream; with tiered kernels a small chunk may
    take the interpreted path, which gives the same states, and expectations
    within the epilogue tolerance). The chunk used is in realized_ms["chunk"]."""
    from . import binding as B
    t_plan0 = time.perf_counter()
    if plan is None:
        if mode == "reuse":
            plan = plan_workload(n, tasks, cost, decide=lambda *a: True)
        else:
            plan = plan_workload(n, tasks, cost, decide=decide)
    planning_ms = (time.perf_counter() - t_plan0) * 1e3
    T = len(tasks)
    chunk = max(1, T)
    while True:
        try:
            res, refusals, realized = _execute(ctx, n, tasks, terms, shots, seed, mode, plan, keep_states,
                                               chunk)
            break
        except B.QwError as e:
            if e.code != B.QW_E_OOM or chunk <= 1:
                raise
            chunk = (chunk + 1) // 2
    realized["chunk"] = chunk
    trace = _explain(name, plan, tasks, n, refusals)
    rec = CostRecord(plan="direct" if mode == "direct" else plan.decision.lower(),
                     predicted_direct_bytes=plan.est_direct, predicted_reuse_bytes=plan.est_reuse,
                     planning_ms=planning_ms, realized_ms=realized)
    return res, trace, rec


def _execute(ctx, n: int, tasks, terms, shots: int, seed: int, mode: str, plan: Plan,
             keep_states: bool, chunk: int):
    """One execution of `plan` with at most `chunk` task states at a time:
    (ExecutionResult, refusal records, realized milliseconds)."""
    from . import binding as B
    nodes = plan.nodes
    T = len(tasks)
    mats = list(plan.materialized)
    refusals: List[dict] = []
    realized: Dict[str, float] = {}
    slot_of = {vid: i for i, vid in enumerate(mats)}
    chunk = max(1, min(chunk, T)) if T else 1
    st = B.State(ctx, n, len(mats) + (chunk if T else 0))
    snaps: Dict[int, object] = {}
    res = ExecutionResult()
    try:
        def anchor_chain(vid: Optional[int]) -> List[int]:
            """Materialized nodes from the root down to vid."""
            if vid is None:
                return []
            return [u for u in path_to(nodes, vid) if u in slot_of]

        def segment_cuts(t: int) -> List[int]:
            a = plan.anchor[t]
            return [nodes[u].end for u in anchor_chain(a)]

        t0 = time.perf_counter()
        # expectations as the epilogue of the batch that ends every task (part
        # of the terms reduced inside its last pass) when one batch ends them
        # all in both modes: every task has the same number of cuts
        fuse_terms = terms is not None and T > 0 and len({len(segment_cuts(t)) for t in range(T)}) == 1
        if mode != "direct":
            # materialized nodes by depth: each from its nearest materialized ancestor
            by_depth: Dict[int, List[int]] = {}
            for vid in mats:
                by_depth.setdefault(nodes[vid].depth, []).append(vid)
            for d in sorted(by_depth):
                srcs, gl, dsts, provs = [], [], [], []
                for vid in by_depth[d]:
                    chain = anchor_chain(nodes[vid].parent)
                    a = chain[-1] if chain else None
                    b0 = nodes[a].end if a is not None else 0
                    gl.append(plan.segment_array(tasks, nodes[vid].tasks[0], b0, nodes[vid].end))
                    dsts.append(slot_of[vid])
                    srcs.append(snaps.get(a))
                    provs.append(snaps[a].provenance if a is not None else bytes(32))
                _reset_runs(st, [d_ for d_, s_ in zip(dsts, srcs) if s_ is None])
                any_src = any(s is not None for s in srcs)
                B.run_suffix_batch(ctx, srcs if any_src else None, gl, st, dsts,
                                   expect_provs=provs if any_src else None)
                for vid in by_depth[d]:
                    fp = plan.node_fingerprint(tasks, vid)
                    snaps[vid] = st.snapshot(slot_of[vid], fp, B.QW_SNAP_FREEZE)
            ctx.sync()
            realized["prefix"] = (time.perf_counter() - t0) * 1e3
        t1 = time.perf_counter()
        exps: List[float] = []
        samples, states = [], []
        t_red = 0.0
        for c0 in range(0, T, chunk):
            ct = list(range(c0, min(T, c0 + chunk)))
            slots = [len(mats) + i for i in range(len(ct))]
            fused_e = None
            if mode == "direct":
                # each task alone, cut at the same boundaries as the reuse plan
                st.reset(len(mats), len(ct))
                cuts = {t: segment_cuts(t) for t in ct}
                levels = max((len(c) for c in cuts.values()), default=0)
                for lev in range(levels + 1):
                    batch, dsts = [], []
                    for t, sl in zip(ct, slots):
                        if lev > len(cuts[t]):
                            continue
                        b0 = 0 if lev == 0 else cuts[t][lev - 1]
                        b1 = cuts[t][lev] if lev < len(cuts[t]) else len(tasks[t])
                        if b1 > b0:
                            batch.append(plan.segment_array(tasks, t, b0, b1))
                            dsts.append(sl)
                    last = lev == levels and fuse_terms and dsts == slots
                    if batch:
                        e = B.run_suffix_batch(ctx, None, batch, st, dsts, terms=terms if last else None)
                        if last:
                            fused_e = e
            else:
                srcs, gl, provs = [], [], []
                for t, sl in zip(ct, slots):
                    a = plan.anchor[t]
                    b0 = nodes[a].end if a is not None else 0
                    srcs.append(snaps.get(a) if a is not None else None)
                    gl.append(plan.segment_array(tasks, t, b0, len(tasks[t])))
                    provs.append(snaps[a].provenance if a is not None else bytes(32))
                _reset_runs(st, [sl for sl, x in zip(slots, srcs) if x is None])
                n_direct = sum(1 for x in srcs if x is None)
                try:
                    fused_e = B.run_suffix_batch(ctx, srcs if n_direct < len(ct) else None, gl, st, slots,
                                                 expect_provs=provs if n_direct < len(ct) else None,
                                                 terms=terms if fuse_terms else None)
                except B.QwRefused as r:
                    # structured refusal: record it and rerun these tasks from |0...0>
                    refusals.append(r.record)
                    st.reset(len(mats), len(ct))
                    fused_e = B.run_suffix_batch(ctx, None, [plan.segment_array(tasks, t, 0, len(tasks[t]))
                                                             for t in ct], st, slots,
                                                 terms=terms if fuse_terms else None)
            ctx.sync()
            t2 = time.perf_counter()
            if fused_e is not None:
                exps += list(fused_e)
            elif terms is not None:
                exps += list(st.expect(len(mats), len(ct), terms))
            if shots:
                samples.append(st.sample(len(mats), len(ct), seed, c0, shots).reshape(len(ct), shots))
            if keep_states:
                states += [st.host(s) for s in slots]
            ctx.sync()
            t_red += time.perf_counter() - t2
        realized["suffix"] = (time.perf_counter() - t1 - t_red) * 1e3
        realized["reduce"] = t_red * 1e3
        realized["total"] = (time.perf_counter() - t0) * 1e3
        if terms is not None and T:
            res.expectations = exps
        if shots and T:
            import numpy as np
            res.samples = np.concatenate(samples, axis=0)
        if keep_states:
            res.states = states
    finally:
        for s in snaps.values():
            s.free()
        st.free()
    return res, refusals, realized


class RecordedWorkload:
    """A planned workload recorded as one HIP graph (qw_graph_*): replay()
    enqueues the whole execution (prefix nodes, snapshots, suffix batch,
    expectations and samples into device buffers) as one graph launch;
    results() copies the outputs of the latest replay to the host."""

    def __init__(self, ctx, n, T, shots, mode):
        self.ctx, self.n, self.T, self.shots, self.mode = ctx, n, T, shots, mode
        self.graph = None
        self.state = None
        self.snaps: List[object] = []
        self.exp_dev = None
        self.samp_dev = None
        self.task_slots: List[int] = []

    def replay(self) -> None:
        self.graph.replay()

    def results(self) -> ExecutionResult:
        res = ExecutionResult()
        if self.exp_dev is not None:
            res.expectations = [float(v) for v in self.exp_dev.cpu().numpy()]
        if self.samp_dev is not None:
            res.samples = self.samp_dev.cpu().numpy().view(np.uint32).reshape(self.T, self.shots)
        return res

    def state_host(self, t: int):
        return self.state.host(self.task_slots[t])

    def free(self) -> None:
        if self.graph is not None:
            self.graph.free()
            self.graph = None
        for s in self.snaps:
            s.free()
        self.snaps = []
        if self.state is not None:
            self.state.free()
            self.state = None


def record_workload(ctx, n: int, tasks: Sequence[Sequence[Gate]], plan: Plan, terms=None,
                    shots: int = 0, seed: int = 0, mode: str = "plan",
                    tree: bool = False) -> RecordedWorkload:
    """Record the execution of `plan` ("plan": materialized nodes level by
    level, then every task's suffix from its anchor; "direct": every task
    from |0...0> with the same segment cuts) as one graph. Planning,
    fingerprints, legality gates and plan uploads happen here, once; a
    replay is device work only. The caller replays it, then reads results().

    `tree` ("plan" mode): the materialized nodes and the tasks' suffixes are
    one qw_run_tree call (each from its nearest materialized ancestor), a
    single persistent kernel launch when the context has QW_OPT_PERSISTENT;
    expectations then come from a reducer sweep after it."""
    from . import binding as B
    torch = ctx.torch
    nodes = plan.nodes
    T = len(tasks)
    mats = list(plan.materialized) if mode != "direct" else []
    slot_of = {vid: i for i, vid in enumerate(mats)}
    rw = RecordedWorkload(ctx, n, T, shots, mode)
    rw.state = st = B.State(ctx, n, len(mats) + T)
    rw.task_slots = task_slots = [len(mats) + t for t in range(T)]
    dev = f"cuda:{ctx.device}"
    if terms is not None and T:
        rw.exp_dev = torch.zeros(T, dtype=torch.float64, device=dev)
    if shots and T:
        rw.samp_dev = torch.zeros(T * shots, dtype=torch.int32, device=dev)
    torch.cuda.synchronize(ctx.device)

    def anchor_chain(vid: Optional[int]) -> List[int]:
        if vid is None:
            return []
        return [u for u in path_to(nodes, vid) if u in slot_of]

    # expectations as the epilogue of the batch that ends every task, under
    # the same condition as run_workload (so both modes take the same path)
    mat_set = set(plan.materialized)
    ncuts = {len([u for u in path_to(nodes, plan.anchor[t]) if u in mat_set])
             if plan.anchor[t] is not None else 0 for t in range(T)}
    fuse = rw.exp_dev is not None and len(ncuts) == 1
    fused = False
    ctx.begin_graph()
    try:
        if mode == "direct":
            mats_all = list(plan.materialized)
            slot_all = {vid: i for i, vid in enumerate(mats_all)}
            cuts = [[nodes[u].end for u in path_to(nodes, plan.anchor[t]) if u in slot_all]
                    if plan.anchor[t] is not None else [] for t in range(T)]
            st.reset(0, T)
            levels = max((len(c) for c in cuts), default=0)
            for lev in range(levels + 1):
                batch, dsts = [], []
                for t in range(T):
                    if lev > len(cuts[t]):
                        continue
                    b0 = 0 if lev == 0 else cuts[t][lev - 1]
                    b1 = cuts[t][lev] if lev < len(cuts[t]) else len(tasks[t])
                    if b1 > b0:
                        batch.append(plan.segment_array(tasks, t, b0, b1))
                        dsts.append(task_slots[t])
                last = lev == levels and fuse and dsts == task_slots
                if batch:
                    B.run_suffix_batch(ctx, None, batch, st, dsts, terms=terms if last else None,
                                       out_dev=rw.exp_dev if last else None)
                    fused = fused or last
        elif tree and all(len(tasks[t]) > (nodes[plan.anchor[t]].end if plan.anchor[t] is not None else 0)
                          for t in range(T)):
            # one tree call: materialized nodes (parents first, the ones with
            # no materialized ancestor in the first slots, so that one reset
            # clears them), then the tasks
            order = sorted(mats, key=lambda v: (bool(anchor_chain(nodes[v].parent)), nodes[v].depth))
            idx = {vid: i for i, vid in enumerate(order)}
            slot_of.clear()
            slot_of.update(idx)
            gl, parents, dsts, eprov, oprov = [], [], [], [], []
            for vid in order:
                chain = anchor_chain(nodes[vid].parent)
                a = chain[-1] if chain else None
                b0 = nodes[a].end if a is not None else 0
                gl.append(plan.segment_array(tasks, nodes[vid].tasks[0], b0, nodes[vid].end))
                parents.append(idx[a] if a is not None else -1)
                dsts.append(slot_of[vid])
                eprov.append(oprov[idx[a]] if a is not None else bytes(32))
                oprov.append(plan.node_fingerprint(tasks, vid))
            for t in range(T):
                a = plan.anchor[t]
                b0 = nodes[a].end if a is not None else 0
                gl.append(plan.segment_array(tasks, t, b0, len(tasks[t])))
                parents.append(idx[a] if a is not None else -1)
                dsts.append(task_slots[t])
                eprov.append(oprov[idx[a]] if a is not None else bytes(32))
                oprov.append(fingerprint(n, tasks[t]))
            _reset_runs(st, [d for k, d in enumerate(dsts) if parents[k] < 0])
            B.run_tree(ctx, None, gl, parents, st, dsts, expect_provs=eprov, out_provs=oprov)
        else:
            snaps: Dict[int, object] = {}
            by_depth: Dict[int, List[int]] = {}
            for vid in mats:
                by_depth.setdefault(nodes[vid].depth, []).append(vid)
            for d in sorted(by_depth):
                srcs, gl, dsts, provs = [], [], [], []
                for vid in by_depth[d]:
                    chain = anchor_chain(nodes[vid].parent)
                    a = chain[-1] if chain else None
                    b0 = nodes[a].end if a is not None else 0
                    gl.append(plan.segment_array(tasks, nodes[vid].tasks[0], b0, nodes[vid].end))
                    dsts.append(slot_of[vid])
                    srcs.append(snaps.get(a))
                    provs.append(snaps[a].provenance if a is not None else bytes(32))
                _reset_runs(st, [d_ for d_, s_ in zip(dsts, srcs) if s_ is None])
                any_src = any(s is not None for s in srcs)
                B.run_suffix_batch(ctx, srcs if any_src else None, gl, st, dsts,
                                   expect_provs=provs if any_src else None)
                for vid in by_depth[d]:
                    fp = plan.node_fingerprint(tasks, vid)
                    snaps[vid] = st.snapshot(slot_of[vid], fp, B.QW_SNAP_FREEZE)
            rw.snaps = list(snaps.values())
            srcs, gl, dsts, provs = [], [], [], []
            for t in range(T):
                a = plan.anchor[t]
                b0 = nodes[a].end if a is not None else 0
                srcs.append(snaps.get(a) if a is not None else None)
                gl.append(plan.segment_array(tasks, t, b0, len(tasks[t])))
                dsts.append(task_slots[t])
                provs.append(snaps[a].provenance if a is not None else bytes(32))
            direct = [t for t in range(T) if srcs[t] is None]
            _reset_runs(st, [task_slots[t] for t in direct])
            B.run_suffix_batch(ctx, srcs if len(direct) < T else None, gl, st, dsts,
                               expect_provs=provs if len(direct) < T else None,
                               terms=terms if fuse else None, out_dev=rw.exp_dev if fuse else None)
            fused = fuse
        if rw.exp_dev is not None and not fused:
            st.expect(len(mats), T, terms, out_dev=rw.exp_dev)
        if rw.samp_dev is not None:
            st.sample(len(mats), T, seed, 0, shots, out_dev=rw.samp_dev)
    except BaseException:
        try:
            ctx.end_graph().free()
        except Exception:
            pass
        rw.free()
        raise
    rw.graph = ctx.end_graph()
    return rw
