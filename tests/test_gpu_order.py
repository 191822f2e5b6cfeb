"""Item order of the persistent generated kernels (QW_OPT_TILE_ORDER) on the
GPU: tile-major (mode 2), descriptor-major (mode 0) and the default mix
(mode 1) give bitwise the same states and expectations, with the per-tile
partials written by tile index.

Covers a suffix batch from a shared snapshot (whose first pass keeps the
descriptor-major order) with a fused epilogue and reducers, and an in-place
batch with a renormalizing pass (norm partials per tile). Every case prints
its name."""
import sys

import numpy as np
import pytest

import oracle
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
    c.set_option(B.QW_OPT_JIT, 1)
    c.set_option(B.QW_OPT_TILE_BITS, 14)
    c.set_option(B.QW_OPT_TILE_ORDER, 1)
    c.sync()


def _run(B, ctx, n, prefix, sufs, terms, order):
    ctx.set_option(B.QW_OPT_TILE_ORDER, order)
    T = len(sufs)
    st = B.State(ctx, n, T + 1)
    st.reset(0, 1)
    st.apply(0, prefix)
    snap = st.snapshot(0, b"order-test".ljust(32, b"\0"))
    e = B.run_suffix_batch(ctx, [snap] * T, sufs, st, list(range(1, T + 1)), terms=terms)
    states = [st.host(k) for k in range(1, T + 1)]
    snap.free()
    st.free()
    return np.asarray(e), states


@pytest.mark.parametrize("n,tile", [(18, 12), (20, 14)])
def test_tile_order_is_bit_identical(ctx, B, n, tile):
    say("tile order vqe", n, tile)
    w = gen.small_vqe(n, 2, 2, 12, 30, seed=11, layer="hea")
    ctx.set_option(B.QW_OPT_TILE_BITS, tile)
    ctx.set_option(B.QW_OPT_JIT, 2)
    try:
        e1, s1 = _run(B, ctx, n, w.prefix, w.suffixes, w.terms, 2)
        e0, s0 = _run(B, ctx, n, w.prefix, w.suffixes, w.terms, 0)
        e_d, s_d = _run(B, ctx, n, w.prefix, w.suffixes, w.terms, 1)
    finally:
        ctx.set_option(B.QW_OPT_JIT, 1)
        ctx.set_option(B.QW_OPT_TILE_BITS, 14)
        ctx.set_option(B.QW_OPT_TILE_ORDER, 1)
    assert np.array_equal(e1, e0) and np.array_equal(e_d, e0)
    for a, b, c in zip(s1, s0, s_d):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        assert np.array_equal(c.view(np.uint32), b.view(np.uint32))
    scale = sum(abs(t[0]) for t in w.terms)
    base = oracle.simulate(n, w.prefix)
    for k in (0, len(w.suffixes) - 1):
        ref = oracle.expect(oracle.apply_gates(base.copy(), n, w.suffixes[k]), n, w.terms)
        assert abs(e1[k] - ref) <= 1e-5 * scale, (k, e1[k], ref)


def test_tile_order_renorm_in_place(ctx, B):
    """In-place tasks (no snapshot) with a renormalization: norm partials and
    the rescale are indexed by tile, so the order does not change them."""
    n, tile, T = 18, 12, 6
    say("tile order renorm", n, tile)
    g = np.random.default_rng(4242)
    tasks = []
    for k in range(T):
        gl = gen.hea_layer(n, gen.random_angles(g, 2 * n)) + gen.hea_layer(n, gen.random_angles(g, 2 * n))
        gl = gl[:60] + [("X", (int(g.integers(n)),), 0.0), ("RENORM", (), 0.0)] + gl[60:]
        tasks.append(gl)
    ctx.set_option(B.QW_OPT_TILE_BITS, tile)
    ctx.set_option(B.QW_OPT_JIT, 2)
    out = {}
    try:
        for order in (2, 0):
            ctx.set_option(B.QW_OPT_TILE_ORDER, order)
            st = B.State(ctx, n, T)
            st.reset(0, T)
            B.run_suffix_batch(ctx, None, tasks, st, list(range(T)))
            out[order] = [st.host(k) for k in range(T)]
            st.free()
    finally:
        ctx.set_option(B.QW_OPT_JIT, 1)
        ctx.set_option(B.QW_OPT_TILE_BITS, 14)
        ctx.set_option(B.QW_OPT_TILE_ORDER, 1)
    for a, b in zip(out[2], out[0]):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    ref = oracle.simulate(n, tasks[0])
    f = abs(np.vdot(ref, out[2][0].astype(np.complex128))) ** 2
    assert 1.0 - f <= 1e-6, f
