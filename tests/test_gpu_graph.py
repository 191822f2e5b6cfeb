"""GPU tests of recorded workloads (qw_graph_*): a graph replay performs the
recorded calls' device work, so every replay equals the same calls run
directly, bit for bit (states, expectations, samples), with the context's
own direct work and synchronisations between replays; recording runs no
device work; calls that need the host are refused while recording (gate
lists with measurements record: tests/test_gpu_measure.py). Every
case prints its name before running."""
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


def _other_work(ctx):
    """Direct work of the same context between replays (its own buffers,
    plan uploads and a synchronising host read)."""
    from paper_2609_23664_amd import planner as P
    w = gen.small_vqe(13, 2, 1, 3, 5, seed=91)
    tasks = [w.task_gates(t) for t in range(w.n_tasks)]
    P.run_workload(ctx, w.n, tasks, terms=w.terms)


def test_trie_graph_replays_equal_direct_calls(ctx):
    say("graph trie 12q 27 leaves, 256 shots")
    import torch
    from paper_2609_23664_amd import planner as P
    w = gen.small_trie(12, 3, 3, 1, 3, seed=21, shots=256)
    tasks = [w.leaf_path(k) for k in range(len(w.leaves))]
    plan = P.plan_workload(w.n, tasks)
    assert plan.decision == "REUSE"
    ref, _, _ = P.run_workload(ctx, w.n, tasks, shots=256, seed=77, keep_states=True, plan=plan)
    rw = P.record_workload(ctx, w.n, tasks, plan, shots=256, seed=77)
    try:
        torch.cuda.synchronize()
        # recording ran nothing: the device output is still zero
        assert not rw.samp_dev.any().item()
        assert rw.graph.nodes() > 0
        for rep in range(3):
            rw.replay()
            res = rw.results()
            assert np.array_equal(res.samples, ref.samples), rep
            for t in (0, 7, len(tasks) - 1):
                assert np.array_equal(rw.state_host(t), ref.states[t]), (rep, t)
            _other_work(ctx)
            ctx.sync()
    finally:
        rw.free()
    k = 13
    o = oracle.simulate(w.n, tasks[k])
    assert 1 - oracle.fidelity(ref.states[k].astype(np.complex128), o) <= FID_TOL


def test_vqe_graph_reuse_equals_direct_graph_and_oracle(ctx):
    say("graph vqe 18q 6 tasks, plan and direct graphs")
    from paper_2609_23664_amd import planner as P
    w = gen.small_vqe(18, 3, 2, 6, 12, seed=17)
    tasks = [w.task_gates(t) for t in range(w.n_tasks)]
    plan = P.plan_workload(w.n, tasks)
    assert plan.decision == "REUSE"
    ref, _, _ = P.run_workload(ctx, w.n, tasks, terms=w.terms, keep_states=True, plan=plan)
    ga = P.record_workload(ctx, w.n, tasks, plan, terms=w.terms, mode="plan")
    gb = P.record_workload(ctx, w.n, tasks, plan, terms=w.terms, mode="direct")
    try:
        for rep in range(2):
            ga.replay()
            gb.replay()
            ra, rb = ga.results(), gb.results()
            assert ra.expectations == rb.expectations == ref.expectations, rep
            for t in range(w.n_tasks):
                sa = ga.state_host(t)
                assert np.array_equal(sa, gb.state_host(t)), (rep, t)
                assert np.array_equal(sa, ref.states[t]), (rep, t)
            _other_work(ctx)
    finally:
        ga.free()
        gb.free()
    scale = sum(abs(t[0]) for t in w.terms)
    for t in (0, 5):
        o = oracle.simulate(w.n, tasks[t])
        assert 1 - oracle.fidelity(ref.states[t].astype(np.complex128), o) <= FID_TOL
        assert abs(ref.expectations[t] - oracle.expect(o, w.n, w.terms)) <= EXP_TOL * scale


def test_graph_with_fused_epilogue_and_second_buffers(ctx):
    say("graph 20q suffix batch with fused epilogue, generated kernels")
    import torch
    from paper_2609_23664_amd import binding as B
    from paper_2609_23664_amd.planner import fingerprint
    c2 = B.Ctx(0)
    c2.set_option(B.QW_OPT_JIT, 2)
    w = gen.small_vqe(20, 2, 2, 5, 16, seed=23)
    st = B.State(c2, w.n, w.n_tasks + 1)
    fp = fingerprint(w.n, w.prefix)

    def calls(out_dev=None):
        st.reset(0, 1)
        st.apply(0, w.prefix)
        snap = st.snapshot(0, fp, B.QW_SNAP_FREEZE)
        e = B.run_suffix_batch(c2, [snap] * w.n_tasks, w.suffixes, st,
                               list(range(1, w.n_tasks + 1)), terms=w.terms, out_dev=out_dev)
        return snap, e

    snap, e_ref = calls()
    ref_states = [st.host(t + 1) for t in range(w.n_tasks)]
    snap.free()
    out = torch.zeros(w.n_tasks, dtype=torch.float64, device="cuda")
    c2.begin_graph()
    snap, _ = calls(out_dev=out)
    g = c2.end_graph()
    try:
        for rep in range(3):
            g.replay()
            c2.sync()
            assert out.cpu().tolist() == e_ref, rep
            for t in range(w.n_tasks):
                assert np.array_equal(st.host(t + 1), ref_states[t]), (rep, t)
            # direct work that regrows the context's own buffers
            big = gen.small_vqe(20, 1, 1, 12, 30, seed=29)
            st2 = B.State(c2, 20, 12)
            B.run_suffix_batch(c2, None, [big.task_gates(t) for t in range(12)], st2,
                               list(range(12)), terms=big.terms)
            st2.free()
    finally:
        g.free()
        snap.free()
    scale = sum(abs(t[0]) for t in w.terms)
    base = oracle.simulate(w.n, w.prefix)
    for t in (0, 4):
        o = oracle.apply_gates(base.copy(), w.n, w.suffixes[t])
        assert abs(e_ref[t] - oracle.expect(o, w.n, w.terms)) <= EXP_TOL * scale
    st.free()
    c2.close()


def test_recording_refuses_host_calls(ctx):
    say("graph recording refusals")
    import torch
    from paper_2609_23664_amd import binding as B
    st = B.State(ctx, 10, 2)
    terms = [(1.0, 0, 1)]
    ctx.begin_graph()
    try:
        with pytest.raises(B.QwError) as ei:
            st.expect(0, 1, terms)
        assert ei.value.code == B.QW_E_UNSUPPORTED
        with pytest.raises(B.QwError) as ei:
            st.sample(0, 1, 1, 0, 8)
        assert ei.value.code == B.QW_E_UNSUPPORTED
        with pytest.raises(B.QwError) as ei:
            st.sample_noalloc(0, 1, 1, 0, 8)
        assert ei.value.code == B.QW_E_UNSUPPORTED
        with pytest.raises(B.QwError) as ei:
            ctx.sync()
        assert ei.value.code == B.QW_E_UNSUPPORTED
        with pytest.raises(B.QwError):
            ctx.begin_graph()
        st.apply(1, [("H", (0,), 0.0)])
    finally:
        g = ctx.end_graph()
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    st.reset()
    g.replay()
    st.expect(1, 1, [(1.0, 1, 0)], out_dev=out)
    ctx.sync()
    assert abs(out.item() - 1.0) < 1e-6  # <X> of H|0>
    g.free()
    st.free()


def test_autotuner_choice_and_results(ctx):
    say("autotune trie 16q 8 leaves, 4 candidates + the best one as a persistent launch")
    import torch
    from paper_2609_23664_amd import autotune as A
    from paper_2609_23664_amd import binding as B
    from paper_2609_23664_amd import planner as P
    c2 = B.Ctx(0)
    w = gen.small_trie(16, 2, 8, 1, 2, seed=27, shots=64)
    tasks = [w.leaf_path(k) for k in range(len(w.leaves))]
    plan = P.plan_workload(w.n, tasks)
    space = {"tile_bits": (12, 14), "tile_order": (0, 2), "relabel": (1,)}
    r = A.autotune(c2, w.n, tasks, plan, shots=64, seed=3, space=space, reps=2)
    assert len(r.table) == 5 and not r.cached
    assert [row["persistent"] for row in r.table] == [0, 0, 0, 0, 1]
    assert r.choice in [{k: row[k] for k in ("tile_bits", "tile_order", "relabel", "stream_loads", "persistent")}
                        for row in r.table]
    best = min(row["replay_ms"] for row in r.table)
    assert [row for row in r.table if row["replay_ms"] == best][0]["tile_bits"] == r.choice["tile_bits"]
    r2 = A.autotune(c2, w.n, tasks, plan, shots=64, seed=3, space=space)
    assert r2.cached and r2.choice == r.choice
    # under the chosen options: reuse equals direct bitwise, and the oracle agrees
    ra, _, _ = P.run_workload(c2, w.n, tasks, shots=64, seed=3, keep_states=True, plan=plan)
    rb, _, _ = P.run_workload(c2, w.n, tasks, shots=64, seed=3, keep_states=True, plan=plan,
                              mode="direct")
    assert np.array_equal(ra.samples, rb.samples)
    for t in (0, len(tasks) - 1):
        assert np.array_equal(ra.states[t], rb.states[t])
        o = oracle.simulate(w.n, tasks[t])
        assert 1 - oracle.fidelity(ra.states[t].astype(np.complex128), o) <= FID_TOL
    c2.close()


def test_graph_update_gates_next_iteration(ctx):
    say("graph gate update: 16q, 4 tasks, new angles for prefix and suffixes")
    import torch
    from paper_2609_23664_amd import binding as B
    from paper_2609_23664_amd.planner import fingerprint
    w = gen.small_vqe(16, 3, 2, 4, 8, seed=61)
    w2 = gen.small_vqe(16, 3, 2, 4, 8, seed=62)   # same gate kinds and qubits, other angles
    assert [g[:2] for g in w.prefix] == [g[:2] for g in w2.prefix]
    st = B.State(ctx, w.n, w.n_tasks + 1)
    slots = list(range(1, w.n_tasks + 1))

    def calls(gw, out_dev=None):
        st.reset(0, 1)
        st.apply(0, gw.prefix)
        snap = st.snapshot(0, fingerprint(w.n, gw.prefix), B.QW_SNAP_FREEZE)
        e = B.run_suffix_batch(ctx, [snap] * w.n_tasks, gw.suffixes, st, slots, terms=w.terms,
                               out_dev=out_dev)
        return snap, e

    snap, e2 = calls(w2)
    ref2 = [st.host(t + 1) for t in range(w.n_tasks)]
    snap.free()
    out = torch.zeros(w.n_tasks, dtype=torch.float64, device="cuda")
    ctx.begin_graph()
    snap, _ = calls(w, out_dev=out)
    g = ctx.end_graph()
    try:
        g.update_gates(0, 0, w2.prefix)
        for t in range(w.n_tasks):
            g.update_gates(1, t, w2.suffixes[t])
        for rep in range(2):
            g.replay()
            ctx.sync()
            assert out.cpu().tolist() == e2, rep
            for t in range(w.n_tasks):
                assert np.array_equal(st.host(t + 1), ref2[t]), (rep, t)
        bad = list(w2.suffixes[0])
        bad[0] = ("CNOT", (0, 1), 0.0)   # another structure
        with pytest.raises(B.QwError) as ei:
            g.update_gates(1, 0, bad)
        assert ei.value.code == B.QW_E_INVALID_ARG
        with pytest.raises(B.QwError):
            g.update_gates(2, 0, w2.prefix)
        with pytest.raises(B.QwError):
            g.update_gates(1, w.n_tasks, w2.suffixes[0])
        # the refused updates changed nothing
        g.replay()
        ctx.sync()
        assert out.cpu().tolist() == e2
    finally:
        g.free()
        snap.free()
        st.free()
    base = oracle.simulate(w.n, w2.prefix)
    scale = sum(abs(t[0]) for t in w.terms)
    o = oracle.apply_gates(base.copy(), w.n, w2.suffixes[1])
    assert abs(e2[1] - oracle.expect(o, w.n, w.terms)) <= EXP_TOL * scale
