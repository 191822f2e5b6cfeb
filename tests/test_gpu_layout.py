"""Index layouts between passes on the GPU (QW_OPT_LAYOUT): a pass may store
its state with the qubits' index bits permuted so that the next pass's
tiles are contiguous. The layout only moves amplitudes, so every result is
bitwise the one of the standard layout: checked for generated and
interpreted kernels, in place and from a snapshot, for a suffix batch with
the fused expectation epilogue, for renormalised segments, and for a batch
split into chunks by the second-buffer cap (mode 2: layouts at any size),
and for a direct batch large enough for the default mode 1. Every case
prints its name before running."""
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
def B():
    from paper_2609_23664_amd import binding
    return binding


@pytest.fixture(scope="module")
def ctx(B):
    import torch
    assert torch.cuda.is_available()
    c = B.Ctx(0)
    yield c
    c.set_option(B.QW_OPT_JIT, 1)
    c.set_option(B.QW_OPT_LAYOUT, 1)
    c.set_option(B.QW_OPT_TILE_BITS, 14)
    c.set_option(B.QW_OPT_SECOND_BUFFER_CAP, 16 << 30)
    c.sync()


def _permuted(B, n, gates, tile):
    return sum(1 for p in B.plan_describe(n, gates, tile)["passes"] if p["out_pos"])


def _apply(B, ctx, n, gates, jit, layout):
    ctx.set_option(B.QW_OPT_JIT, jit)
    ctx.set_option(B.QW_OPT_LAYOUT, layout)
    try:
        st = B.State(ctx, n, 1)
        st.apply(0, gates)
        out = st.host(0)
        st.free()
    finally:
        ctx.set_option(B.QW_OPT_JIT, 1)
        ctx.set_option(B.QW_OPT_LAYOUT, 1)
    return out


def _hea(n, layers, seed, extra=0):
    g = np.random.default_rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            gates.append(("RY", (q,), float(g.uniform(0, 6.3))))
            gates.append(("RZ", (q,), float(g.uniform(0, 6.3))))
        for q in range(n - 1):
            gates.append(("CNOT", (q, q + 1), 0.0))
        for _ in range(extra):
            a, b = g.choice(n, 2, replace=False)
            gates.append(("CZ", (int(a), int(b)), 0.0))
    return gates


@pytest.mark.parametrize("n,tile,seed", [(16, 10, 1), (18, 12, 2), (20, 14, 3), (22, 14, 4)])
def test_layout_in_place_plan_bitwise(ctx, B, n, tile, seed):
    """A plan applied in place (no snapshot): passes that change the layout
    run out of place through the second buffer."""
    say("layout in-place plan", n, tile, seed)
    gates = _hea(n, 3, 7300 + seed, extra=3)
    assert _permuted(B, n, gates, tile) > 0
    ctx.set_option(B.QW_OPT_TILE_BITS, tile)
    try:
        std = _apply(B, ctx, n, gates, 2, 0)
        gen_ = _apply(B, ctx, n, gates, 2, 2)
        interp = _apply(B, ctx, n, gates, 0, 2)
    finally:
        ctx.set_option(B.QW_OPT_TILE_BITS, 14)
    assert np.array_equal(std, gen_)
    assert np.array_equal(std, interp)
    ref = oracle.simulate(n, gates)
    assert 1 - oracle.fidelity(gen_.astype(np.complex128), ref) <= FID_TOL


def _batch(B, ctx, n, prefix, sufs, terms, layout, cap=None):
    ctx.set_option(B.QW_OPT_LAYOUT, layout)
    if cap is not None:
        ctx.set_option(B.QW_OPT_SECOND_BUFFER_CAP, cap)
    try:
        T = len(sufs)
        st = B.State(ctx, n, T + 1)
        st.reset(0, 1)
        st.apply(0, prefix)
        snap = st.snapshot(0, b"layout-test".ljust(32, b"\0"))
        e = B.run_suffix_batch(ctx, [snap] * T, sufs, st, list(range(1, T + 1)), terms=terms)
        states = [st.host(k) for k in range(1, T + 1)]
        snap.free()
        st.free()
    finally:
        ctx.set_option(B.QW_OPT_LAYOUT, 1)
        ctx.set_option(B.QW_OPT_SECOND_BUFFER_CAP, 16 << 30)
    return np.asarray(e), states


@pytest.mark.parametrize("n,tile", [(18, 12), (20, 14)])
def test_layout_suffix_batch_with_epilogue_bitwise(ctx, B, n, tile):
    """A VQE-like batch from a frozen snapshot with the fused epilogue:
    expectations and states equal bitwise; a second-buffer cap of a few
    states splits the batch into chunks with the same results."""
    say("layout suffix batch", n, tile)
    w = gen.small_vqe(n, 2, 2, 12, 30, seed=5, layer="hea")
    assert _permuted(B, n, w.suffixes[0], tile) > 0
    ctx.set_option(B.QW_OPT_TILE_BITS, tile)
    ctx.set_option(B.QW_OPT_JIT, 2)
    try:
        e0, s0 = _batch(B, ctx, n, w.prefix, w.suffixes, w.terms, 0)
        e1, s1 = _batch(B, ctx, n, w.prefix, w.suffixes, w.terms, 2)
        say("layout suffix batch, chunked", n, tile)
        e2, s2 = _batch(B, ctx, n, w.prefix, w.suffixes, w.terms, 2, cap=3 * (8 << n))
    finally:
        ctx.set_option(B.QW_OPT_JIT, 1)
        ctx.set_option(B.QW_OPT_TILE_BITS, 14)
    assert np.array_equal(e0, e1) and np.array_equal(e0, e2)
    for a, b, c in zip(s0, s1, s2):
        assert np.array_equal(a, b) and np.array_equal(a, c)
    scale = sum(abs(t[0]) for t in w.terms)
    base = oracle.simulate(n, w.prefix)
    for k in (0, len(w.suffixes) - 1):
        ref = oracle.apply_gates(base.copy(), n, w.suffixes[k])
        assert 1 - oracle.fidelity(s1[k].astype(np.complex128), ref) <= FID_TOL
        assert abs(e1[k] - oracle.expect(ref, n, w.terms)) <= 1e-5 * scale


def test_layout_renormalised_segments_bitwise(ctx, B):
    """A projector and a RENORM marker inside a plan: the per-tile norm
    partials and the scale of the next segment's first pass do not depend
    on the layout; the state is the oracle's projected, renormalised one
    followed by the remaining gates (the projection written out from its
    definition, diag(0, f) on the qubit)."""
    n, tile, q, f = 20, 14, 17, 0.6
    say("layout renorm segments", n, tile, q)
    pre, post = _hea(n, 2, 7400), _hea(n, 2, 7401)
    gates = pre + [("PROJ1", (q,), f), ("RENORM", (), 0.0)] + post
    assert _permuted(B, n, gates, tile) > 0
    std = _apply(B, ctx, n, gates, 2, 0)
    lay = _apply(B, ctx, n, gates, 2, 2)
    assert np.array_equal(std, lay)
    ref = oracle.simulate(n, pre)
    idx = np.arange(1 << n)
    ref = np.where(((idx >> q) & 1) == 1, f * ref, 0.0).astype(np.complex128)
    ref /= np.sqrt(oracle.norm2(ref))
    oracle.apply_gates(ref, n, post)
    assert 1 - oracle.fidelity(lay.astype(np.complex128), ref) <= FID_TOL


def test_layout_default_mode_on_a_large_direct_batch(ctx, B):
    """Mode 1 (the default) permutes layouts when the call's states exceed
    128 MiB: 20 tasks of 20 qubits (160 MiB) run from |0...0> in place;
    expectations and states equal those of modes 0 and 2 bitwise."""
    n, T = 20, 20
    say("layout default mode, direct batch", n, T)
    w = gen.small_vqe(n, 2, 2, T, 24, seed=6, layer="hea")
    tasks = [list(w.prefix) + list(s) for s in w.suffixes]
    res = []
    ctx.set_option(B.QW_OPT_JIT, 2)
    try:
        for mode in (0, 1, 2):
            ctx.set_option(B.QW_OPT_LAYOUT, mode)
            st = B.State(ctx, n, T)
            st.reset(0, T)
            e = B.run_suffix_batch(ctx, None, tasks, st, list(range(T)), terms=w.terms)
            res.append((np.asarray(e), [st.host(k) for k in range(T)]))
            st.free()
    finally:
        ctx.set_option(B.QW_OPT_LAYOUT, 1)
        ctx.set_option(B.QW_OPT_JIT, 1)
    for e, states in res[1:]:
        assert np.array_equal(e, res[0][0])
        for a, b in zip(states, res[0][1]):
            assert np.array_equal(a, b)
    ref = oracle.simulate(n, tasks[0])
    assert 1 - oracle.fidelity(res[1][1][0].astype(np.complex128), ref) <= FID_TOL
