"""The device-memory cap of a context (QW_OPT_DEVICE_MEM_CAP, forced from
the host) and the planner's fallback to fewer task slots: allocations past
the cap are refused with QW_E_OOM before the device work that needs them,
and run_workload then runs the tasks in smaller chunks through the same
slots, with states, expectations and samples equal to the unchunked run.
Every case prints its name."""
import sys

import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_2609_23664_amd import binding
    return binding


@pytest.fixture()
def ctx(B):
    import torch
    assert torch.cuda.is_available()
    c = B.Ctx(0)
    yield c
    c.sync()


def test_cap_refuses_allocations_past_it(ctx, B):
    say("device memory cap: state and snapshot allocations")
    ctx.set_option(B.QW_OPT_DEVICE_MEM_CAP, 3 << 20)
    a = B.State(ctx, 18, 1)                      # 2 MiB: within the cap
    with pytest.raises(B.QwError) as e:
        B.State(ctx, 18, 1)                      # 2 more MiB: past it
    assert e.value.code == B.QW_E_OOM and "cap" in e.value.msg
    with pytest.raises(B.QwError) as e:
        a.snapshot(0, bytes(32), B.QW_SNAP_COPY)  # a copy needs 2 MiB too
    assert e.value.code == B.QW_E_OOM
    a.free()
    b = B.State(ctx, 18, 1)                      # the freed bytes count again
    b.apply(0, [("H", (0,), 0.0)])
    assert abs(abs(b.host(0)[1]) - 2 ** -0.5) < 1e-6
    b.free()
    ctx.set_option(B.QW_OPT_DEVICE_MEM_CAP, 0)


@pytest.mark.parametrize("mode", ["plan", "direct"])
def test_run_workload_falls_back_to_fewer_slots(ctx, B, mode):
    """16 qubits, 12 tasks from a 3-layer shared prefix (1-layer suffixes,
    16 terms, 256 shots): unchunked, then under a cap that holds the
    materialized node and a few task states; generated kernels in both runs
    (QW_OPT_JIT = 2), so the fused expectation epilogue is taken alike."""
    from paper_2609_23664_amd import planner as P
    say("oom fallback", mode)
    w = gen.small_vqe(16, 3, 1, 12, 16, seed=41)
    tasks = [list(w.prefix) + list(s) for s in w.suffixes]
    plan = P.plan_workload(w.n, tasks)
    ctx.set_option(B.QW_OPT_JIT, 2)
    try:
        r0, _, c0 = P.run_workload(ctx, w.n, tasks, terms=w.terms, shots=256, seed=9, plan=plan, mode=mode,
                                   keep_states=True)
        assert c0.realized_ms["chunk"] == 12
        ctx.set_option(B.QW_OPT_DEVICE_MEM_CAP, 5 << 20)   # 512 KiB per state
        r1, _, c1 = P.run_workload(ctx, w.n, tasks, terms=w.terms, shots=256, seed=9, plan=plan, mode=mode,
                                   keep_states=True)
    finally:
        ctx.set_option(B.QW_OPT_DEVICE_MEM_CAP, 0)
        ctx.set_option(B.QW_OPT_JIT, 1)
    say("  chunk", c1.realized_ms["chunk"])
    assert c1.realized_ms["chunk"] < 12
    assert r1.expectations == r0.expectations
    assert np.array_equal(r1.samples, r0.samples)
    for a, b in zip(r1.states, r0.states):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
