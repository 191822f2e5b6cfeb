"""The allocation-free sampler entry point (qw_sample_noalloc) against
qw_sample, through the C ABI: two calls in a row, the second on a smaller
input (fewer qubits, slots and shots, device output), each bitwise equal to
qw_sample on the same states; a request beyond the fixed scratch is refused
before any device work. Every case prints its name."""
import ctypes
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


@pytest.fixture(scope="module")
def ctx(B):
    import torch
    assert torch.cuda.is_available()
    c = B.Ctx(0)
    yield c
    c.sync()


def _states(B, ctx, n, slots, seed):
    st = B.State(ctx, n, slots)
    rng = np.random.default_rng(seed)
    for s in range(slots):
        gates = []
        for _ in range(2):
            gates += gen.hea_layer(n, gen.random_angles(rng, 2 * n))
        st.apply(s, gates)
    return st


def test_noalloc_sampler_equals_sampler_twice(ctx, B):
    import torch
    say("noalloc sampler: 20 qubits x 12 slots x 1024 shots (host out), then 14 x 3 x 100 (device out)")
    st = _states(B, ctx, 20, 12, 7)
    ref = st.sample(0, 12, 1234, 5, 1024)
    got = st.sample_noalloc(0, 12, 1234, 5, 1024)
    assert got.shape == (12, 1024)
    assert np.array_equal(got, ref)
    # a sub-range of slots with its own task base
    assert np.array_equal(st.sample_noalloc(4, 3, 99, 4, 257), st.sample(4, 3, 99, 4, 257))
    st.free()
    st2 = _states(B, ctx, 14, 3, 8)
    ref2 = st2.sample(0, 3, 77, 0, 100)
    out = torch.full((3 * 100,), -1, dtype=torch.int32, device="cuda")
    st2.sample_noalloc(0, 3, 77, 0, 100, out_dev=out)
    ctx.sync()
    got2 = out.cpu().numpy().view(np.uint32).reshape(3, 100)
    assert np.array_equal(got2, ref2)
    st2.free()


def test_noalloc_sampler_refuses_beyond_its_scratch(ctx, B):
    say("noalloc sampler: request beyond the fixed scratch")
    st = _states(B, ctx, 12, 2, 9)
    shots = (64 << 20) // 8 + 1      # 2 slots x shots x 4 B alone exceed the 64 MiB
    out = np.zeros(2 * shots, dtype=np.uint32)
    rc = B.lib().qw_sample_noalloc(st.h, 0, 2, 1, 0, shots, ctypes.c_void_p(out.ctypes.data), 1)
    assert rc == B.QW_E_INVALID_ARG
    assert b"fixed scratch" in B.lib().qw_last_error(ctx.h)
    assert not out.any()
    # the entry point still works after the refusal
    assert np.array_equal(st.sample_noalloc(0, 2, 3, 0, 64), st.sample(0, 2, 3, 0, 64))
    st.free()
