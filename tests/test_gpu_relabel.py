"""Output relabelling on the GPU: passes that end with CNOTs whose targets
are not local to the tile, applied as a permutation of the store addresses.

Checked against the oracle (fidelity bar) and for bit-identity between the
generated and interpreted kernels, for the buffer cases of the executor: a
relabelling pass reading a snapshot, relabelling passes in the middle of an
in-place plan, a first pass that relabels in place (copied to the second
buffer first, or made out of place by flipping a later plain pass), and a
batch split into chunks by the second-buffer cap. Every case prints its
name before running."""
import sys

import numpy as np
import pytest

import oracle

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
    c.set_option(B.QW_OPT_RELABEL, 1)
    c.set_option(B.QW_OPT_LAYOUT, 1)
    c.set_option(B.QW_OPT_SECOND_BUFFER_CAP, 16 << 30)
    c.sync()


def _ladder_circuit(n, g, layers, extra=4):
    """Rotation layers with CNOT ladders that climb past the tile, plus
    random long-range CNOTs: plans end passes with relabelling CNOTs whose
    controls are register, wave and non-local bits."""
    gates = []
    for _ in range(layers):
        for q in range(n):
            gates.append(("RY", (q,), float(g.uniform(0, 6.3))))
            gates.append(("RZ", (q,), float(g.uniform(0, 6.3))))
        for q in range(n - 1):
            gates.append(("CNOT", (q, q + 1), 0.0))
        for _ in range(extra):
            a, b = g.choice(n, 2, replace=False)
            gates.append(("CNOT", (int(a), int(b)), 0.0))
    return gates


def _n_relabel(B, n, gates, tile=14):
    return sum(1 for p in B.plan_describe(n, gates, tile)["passes"] if p["out_cx"])


def _run(B, ctx, n, gates, jit):
    ctx.set_option(B.QW_OPT_JIT, jit)
    st = B.State(ctx, n, 1)
    st.apply(0, gates)
    out = st.host(0)
    st.free()
    ctx.set_option(B.QW_OPT_JIT, 1)
    return out


@pytest.mark.parametrize("n,tile,seed", [(16, 10, 1), (18, 12, 2), (20, 14, 3), (22, 14, 4)])
def test_relabel_in_place_plan(ctx, B, n, tile, seed):
    say("relabel in-place plan", n, tile, seed)
    g = np.random.default_rng(7100 + seed)
    gates = _ladder_circuit(n, g, 3)
    assert _n_relabel(B, n, gates, tile) > 0
    ctx.set_option(B.QW_OPT_TILE_BITS, tile)
    try:
        a = _run(B, ctx, n, gates, 0)
        b = _run(B, ctx, n, gates, 2)
        ctx.set_option(B.QW_OPT_RELABEL, 0)
        c = _run(B, ctx, n, gates, 2)
    finally:
        ctx.set_option(B.QW_OPT_RELABEL, 1)
        ctx.set_option(B.QW_OPT_TILE_BITS, 14)
    assert np.array_equal(a, b)
    ref = oracle.simulate(n, gates)
    assert 1 - oracle.fidelity(b.astype(np.complex128), ref) <= FID_TOL
    assert 1 - oracle.fidelity(c.astype(np.complex128), ref) <= FID_TOL


def _first_pass_relabel(n, second_plain):
    # one pass over the low 14 qubits that ends with CNOTs onto high targets
    # (controls 13 and 12: wave/register positions); optionally a second,
    # plain pass on the high qubits
    gates = [("H", (q,), 0.0) for q in range(14)]
    gates += [("RY", (q,), 0.3 + 0.1 * q) for q in range(14)]
    gates += [("CNOT", (13, n - 1), 0.0), ("CNOT", (12, n - 3), 0.0), ("CNOT", (n - 1, n - 2), 0.0)]
    if second_plain:
        gates += [("RX", (q,), 0.2 * q) for q in range(14, n)]
    return gates


@pytest.mark.parametrize("layout", [0, 2])
@pytest.mark.parametrize("second_plain", [False, True])
def test_relabel_first_pass_in_place(ctx, B, second_plain, layout):
    """With the standard layout the second (plain) pass is made out of
    place; with a permuted layout between the two passes both move
    amplitudes and the destination is copied to the second buffer first."""
    n = 20
    say("relabel first pass in place", n, second_plain, layout)
    gates = _first_pass_relabel(n, second_plain)
    plan = B.plan_describe(n, gates)
    assert plan["passes"][0]["out_cx"]
    assert len(plan["passes"]) == (2 if second_plain else 1)
    ctx.set_option(B.QW_OPT_LAYOUT, layout)
    try:
        a = _run(B, ctx, n, gates, 0)
        b = _run(B, ctx, n, gates, 2)
    finally:
        ctx.set_option(B.QW_OPT_LAYOUT, 1)
    assert np.array_equal(a, b)
    ref = oracle.simulate(n, gates)
    assert 1 - oracle.fidelity(b.astype(np.complex128), ref) <= FID_TOL
    # applied twice in a row on the same slot (the slot holds the first result)
    st = B.State(ctx, n, 1)
    st.apply(0, gates)
    st.apply(0, gates)
    twice = st.host(0)
    st.free()
    ref2 = oracle.simulate(n, gates + gates)
    assert 1 - oracle.fidelity(twice.astype(np.complex128), ref2) <= FID_TOL


def test_relabel_suffix_batch_from_snapshot_and_chunks(ctx, B):
    n, T = 20, 5
    say("relabel suffix batch", n, T)
    g = np.random.default_rng(7200)
    prefix = _ladder_circuit(n, g, 2)
    # suffixes 0..2 are plain ladders (relabelling in their last pass, which
    # reads the snapshot's successor buffers), 3..4 add long-range CNOTs
    sufs = [_ladder_circuit(n, np.random.default_rng(7300 + k), 2, extra=0 if k < 3 else 4)
            for k in range(T)]
    assert B.plan_describe(n, sufs[0], 12)["passes"][-1]["out_cx"]
    ctx.set_option(B.QW_OPT_TILE_BITS, 12)
    try:
        full, chunked, direct = _suffix_runs(B, ctx, n, T, prefix, sufs)
    finally:
        ctx.set_option(B.QW_OPT_TILE_BITS, 14)
    for k in range(T):
        assert np.array_equal(full[k], chunked[k])
        ref = oracle.simulate(n, prefix + sufs[k])
        assert 1 - oracle.fidelity(full[k].astype(np.complex128), ref) <= FID_TOL
        assert 1 - oracle.fidelity(direct[k].astype(np.complex128), ref) <= FID_TOL


def _suffix_runs(B, ctx, n, T, prefix, sufs):
    st = B.State(ctx, n, T + 1)
    st.reset(0, 1)
    st.apply(0, prefix)
    snap = st.snapshot(0, b"relabel-test".ljust(32, b"\0"))
    slots = list(range(1, T + 1))
    B.run_suffix_batch(ctx, [snap] * T, sufs, st, slots)
    full = [st.host(s) for s in slots]
    # chunks of one task (cap = one state)
    ctx.set_option(B.QW_OPT_SECOND_BUFFER_CAP, 8 << n)
    try:
        B.run_suffix_batch(ctx, [snap] * T, sufs, st, slots)
        chunked = [st.host(s) for s in slots]
    finally:
        ctx.set_option(B.QW_OPT_SECOND_BUFFER_CAP, 16 << 30)
    # direct: every task from |0..0> through prefix and suffix
    dst = B.State(ctx, n, T)
    dst.reset(0, T)
    B.run_suffix_batch(ctx, None, [prefix + s for s in sufs], dst, list(range(T)))
    direct = [dst.host(k) for k in range(T)]
    snap.free()
    st.free()
    dst.free()
    return full, chunked, direct
