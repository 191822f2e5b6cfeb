"""GPU tests of the persistent launch (QW_OPT_PERSISTENT) and of qw_run_tree:
one kernel runs every pass of a call, and with in-call parents every level
of a task tree, taking claims in order and waiting on completion counters.
Its states and expectations are bitwise those of the per-pass launches (the
same generated pass bodies on the same inputs), a tree run as one launch
equals the same tree run level by level and, through the planner, the
direct execution with the same cuts; sampled states match the oracle. A
wait forced past its bound from the host (spin limit 0) ends the launch
with QW_E_ABANDONED at the next synchronisation, and the context then runs
normally. Every case prints its name first."""
import sys

import numpy as np
import pytest

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu

FID_TOL = 1e-6


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2609_23664_amd import binding
    assert torch.cuda.is_available()
    c = binding.Ctx(0)
    c.set_option(binding.QW_OPT_JIT, 2)
    yield c
    c.set_option(binding.QW_OPT_PERSISTENT, 0)
    c.sync()


def _suffix_batch(ctx, w, persistent, layout):
    """Prefix once, FREEZE snapshot, the tasks' suffixes with the expectation
    epilogue: (states, expectations)."""
    from paper_2609_23664_amd import binding as B
    from paper_2609_23664_amd import planner as P
    ctx.set_option(B.QW_OPT_PERSISTENT, 1 if persistent else 0)
    ctx.set_option(B.QW_OPT_LAYOUT, layout)
    T = w.n_tasks
    st = B.State(ctx, w.n, T + 1)
    snap = None
    try:
        st.reset(0, 1)
        st.apply(0, w.prefix)
        snap = st.snapshot(0, P.fingerprint(w.n, w.prefix), B.QW_SNAP_FREEZE)
        e = B.run_suffix_batch(ctx, [snap] * T, [w.suffixes[t] for t in range(T)], st,
                               list(range(1, T + 1)), terms=w.terms)
        ctx.sync()
        states = [st.host(1 + t) for t in range(T)]
    finally:
        if snap is not None:
            snap.free()
        st.free()
        ctx.set_option(B.QW_OPT_PERSISTENT, 0)
        ctx.set_option(B.QW_OPT_LAYOUT, 1)
    return states, e


@pytest.mark.parametrize("n,tile_bits,layout", [(18, 14, 1), (18, 14, 2), (17, 12, 2), (15, 13, 0)])
def test_persistent_suffix_batch_equals_per_pass(ctx, n, tile_bits, layout):
    say(f"persistent suffix batch {n}q tile_bits={tile_bits} layout={layout}")
    from paper_2609_23664_amd import binding as B
    w = gen.small_vqe(n, 2, 3, 6, 24, seed=400 + n)
    ctx.set_option(B.QW_OPT_TILE_BITS, tile_bits)
    try:
        s0, e0 = _suffix_batch(ctx, w, False, layout)
        say("  per-pass launches done")
        s1, e1 = _suffix_batch(ctx, w, True, layout)
        say("  persistent launch done")
    finally:
        ctx.set_option(B.QW_OPT_TILE_BITS, 14)
    for t in range(w.n_tasks):
        assert np.array_equal(s0[t].view(np.uint32), s1[t].view(np.uint32)), t
    assert np.array_equal(np.array(e0).view(np.uint64), np.array(e1).view(np.uint64))
    for t in (0, w.n_tasks - 1):
        ref = oracle.simulate(n, w.task_gates(t))
        assert 1 - oracle.fidelity(s1[t].astype(np.complex128), ref) <= FID_TOL
        c = sum(abs(term[0]) for term in w.terms)
        assert abs(e1[t] - oracle.expect(ref, n, w.terms)) <= 1e-5 * c


def _tree(w):
    """The trie as qw_run_tree tasks: level nodes (parents first), then the
    leaves; parent indices into that list."""
    from paper_2609_23664_amd import planner as P
    gl, parents, first = [], [], []
    base = 0
    for d, level in enumerate(w.levels):
        first.append(base)
        for p, g in level:
            gl.append(g)
            parents.append(-1 if p < 0 else first[d - 1] + p)
        base += len(level)
    for p, g in w.leaves:
        gl.append(g)
        parents.append(-1 if p < 0 else first[-1] + p)
    # provenance of every task's final state: the fingerprint of its path
    paths = []
    for k, g in enumerate(gl):
        paths.append((paths[parents[k]] if parents[k] >= 0 else []) + list(g))
    provs = [P.fingerprint(w.n, pth) for pth in paths]
    eprov = [provs[p] if p >= 0 else bytes(32) for p in parents]
    return gl, parents, provs, eprov, paths


def _run_tree(ctx, w, persistent):
    from paper_2609_23664_amd import binding as B
    gl, parents, provs, eprov, paths = _tree(w)
    ctx.set_option(B.QW_OPT_PERSISTENT, 1 if persistent else 0)
    st = B.State(ctx, w.n, len(gl))
    try:
        st.reset(0, len(gl))
        B.run_tree(ctx, None, gl, parents, st, list(range(len(gl))), expect_provs=eprov, out_provs=provs)
        ctx.sync()
        states = [st.host(k) for k in range(len(gl))]
    finally:
        st.free()
        ctx.set_option(B.QW_OPT_PERSISTENT, 0)
    return states, paths


def test_tree_one_launch_equals_levels(ctx):
    say("qw_run_tree 15q depth 3 branching 3: persistent vs level by level")
    w = gen.small_trie(15, 3, 3, 1, 3, seed=41, shots=0)
    s_lev, paths = _run_tree(ctx, w, False)
    s_one, _ = _run_tree(ctx, w, True)
    assert len(s_one) == 3 + 9 + 27
    for k in range(len(s_one)):
        assert np.array_equal(s_lev[k].view(np.uint32), s_one[k].view(np.uint32)), k
    for k in (3, 12, len(s_one) - 1):
        ref = oracle.simulate(w.n, paths[k])
        assert 1 - oracle.fidelity(s_one[k].astype(np.complex128), ref) <= FID_TOL, k


def test_tree_refuses_bad_parents_and_provenance(ctx):
    say("qw_run_tree argument checks")
    from paper_2609_23664_amd import binding as B
    w = gen.small_trie(12, 2, 2, 1, 1, seed=42, shots=0)
    gl, parents, provs, eprov, _ = _tree(w)
    st = B.State(ctx, w.n, len(gl))
    try:
        st.reset(0, len(gl))
        bad = list(parents)
        bad[1] = 5   # a parent after its child
        with pytest.raises(B.QwError) as ei:
            B.run_tree(ctx, None, gl, bad, st, list(range(len(gl))), expect_provs=eprov, out_provs=provs)
        assert ei.value.code == B.QW_E_INVALID_ARG
        wrong = list(eprov)
        wrong[-1] = bytes(32)
        with pytest.raises(B.QwRefused) as er:
            B.run_tree(ctx, None, gl, parents, st, list(range(len(gl))), expect_provs=wrong, out_provs=provs)
        assert er.value.record["reason"] == "PROVENANCE_MISMATCH"
    finally:
        st.free()


def test_abandoned_wait_is_reported_and_context_recovers(ctx):
    say("persistent launch with spin limit 0")
    from paper_2609_23664_amd import binding as B
    w = gen.small_vqe(18, 1, 3, 8, 8, seed=43)
    ref, e_ref = _suffix_batch(ctx, w, False, 1)
    ctx.set_option(B.QW_OPT_SPIN_LIMIT, 0)
    try:
        try:
            got, _ = _suffix_batch(ctx, w, True, 1)
            abandoned = False
        except B.QwError as e:
            assert e.code == B.QW_E_ABANDONED, e
            abandoned = True
        say(f"  abandoned={abandoned}")
        if not abandoned:   # no wait was needed: the results are whole
            for t in range(w.n_tasks):
                assert np.array_equal(ref[t].view(np.uint32), got[t].view(np.uint32))
    finally:
        ctx.set_option(B.QW_OPT_SPIN_LIMIT, 1 << 20)
    ctx.sync()
    again, e_again = _suffix_batch(ctx, w, True, 1)
    for t in range(w.n_tasks):
        assert np.array_equal(ref[t].view(np.uint32), again[t].view(np.uint32)), t
    assert np.array_equal(np.array(e_ref).view(np.uint64), np.array(e_again).view(np.uint64))


def _graphs(ctx, w, picks, persistent_plan):
    from paper_2609_23664_amd import binding as B
    from paper_2609_23664_amd import planner as P
    tasks = [w.leaf_path(k) for k in range(len(w.leaves))]
    plan = P.plan_workload(w.n, tasks)
    assert plan.decision == "REUSE"
    out = {}
    for mode in ("plan", "direct"):
        say(f"  recording {mode}")
        ctx.set_option(B.QW_OPT_PERSISTENT, 1 if (mode == "plan" and persistent_plan) else 0)
        rw = P.record_workload(ctx, w.n, tasks, plan, shots=w.shots, seed=w.seed, mode=mode,
                               tree=(mode == "plan" and persistent_plan))
        ctx.set_option(B.QW_OPT_PERSISTENT, 0)
        say(f"  replaying {mode}")
        try:
            nodes = rw.graph.nodes()
            rw.replay()
            res1 = rw.results()
            rw.replay()   # a second replay with the same result
            res = rw.results()
            assert np.array_equal(res1.samples, res.samples)
            states = {k: rw.state_host(k) for k in picks}
        finally:
            rw.free()
        out[mode] = (res.samples, states, nodes)
    return tasks, out


def test_trie_persistent_graph_equals_direct(ctx):
    say("trie 14q 27 leaves, 512 shots: persistent tree graph vs direct graph")
    w = gen.small_trie(14, 3, 3, 1, 4, seed=44, shots=512)
    picks = [0, 13, 26]
    tasks, out = _graphs(ctx, w, picks, True)
    (sp, stp, np_nodes), (sd, std, nd_nodes) = out["plan"], out["direct"]
    say(f"  nodes: plan {np_nodes}, direct {nd_nodes}")
    assert np_nodes <= 8
    assert np.array_equal(sp, sd)
    for k in picks:
        assert np.array_equal(stp[k].view(np.uint32), std[k].view(np.uint32)), k
        ref = oracle.simulate(w.n, tasks[k])
        assert 1 - oracle.fidelity(stp[k].astype(np.complex128), ref) <= FID_TOL


def test_config3_full_size_persistent_graph(ctx):
    say("config3 full size: 20q, 512 leaves, 1024 shots, persistent tree graph vs direct graph")
    w = gen.config3()
    picks = [0, 137, 300, 511]
    tasks, out = _graphs(ctx, w, picks, True)
    (sp, stp, np_nodes), (sd, std, nd_nodes) = out["plan"], out["direct"]
    say(f"  nodes: plan {np_nodes}, direct {nd_nodes}")
    assert np_nodes <= 10
    assert sp.shape == (512, 1024)
    assert np.array_equal(sp, sd)
    for k in picks:
        assert np.array_equal(stp[k].view(np.uint32), std[k].view(np.uint32)), k
        ref = oracle.simulate(w.n, tasks[k])
        assert 1 - oracle.fidelity(stp[k].astype(np.complex128), ref) <= FID_TOL, k


def test_persistent_graph_takes_next_iteration_gates(ctx):
    say("persistent suffix batch recorded, new angles through qw_graph_update_gates")
    import torch
    from paper_2609_23664_amd import binding as B
    from paper_2609_23664_amd.planner import fingerprint
    w = gen.small_vqe(17, 2, 2, 5, 10, seed=71)
    w2 = gen.small_vqe(17, 2, 2, 5, 10, seed=72)   # same gate kinds and qubits, other angles
    st = B.State(ctx, w.n, w.n_tasks + 1)
    slots = list(range(1, w.n_tasks + 1))

    def calls(gw, out_dev=None):
        st.reset(0, 1)
        st.apply(0, gw.prefix)
        snap = st.snapshot(0, fingerprint(w.n, gw.prefix), B.QW_SNAP_FREEZE)
        e = B.run_suffix_batch(ctx, [snap] * w.n_tasks, gw.suffixes, st, slots, terms=w.terms,
                               out_dev=out_dev)
        return snap, e

    snap, e2 = calls(w2)            # per-pass launches, the new angles
    ref2 = [st.host(t + 1) for t in range(w.n_tasks)]
    snap.free()
    out = torch.zeros(w.n_tasks, dtype=torch.float64, device="cuda")
    ctx.set_option(B.QW_OPT_PERSISTENT, 1)
    try:
        ctx.begin_graph()
        snap, _ = calls(w, out_dev=out)
        g = ctx.end_graph()
    finally:
        ctx.set_option(B.QW_OPT_PERSISTENT, 0)
    try:
        g.update_gates(0, 0, w2.prefix)
        for t in range(w.n_tasks):
            g.update_gates(1, t, w2.suffixes[t])
        for rep in range(2):
            g.replay()
            ctx.sync()
            assert out.cpu().tolist() == e2, rep
            for t in range(w.n_tasks):
                assert np.array_equal(st.host(t + 1).view(np.uint32), ref2[t].view(np.uint32)), (rep, t)
    finally:
        g.free()
        snap.free()
        st.free()
