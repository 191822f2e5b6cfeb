"""GPU parity of the HIP path against the CPU complex128 oracle.

Bars (from the target statement): state fidelity 1 - |<psi_o|psi_g>|^2 <= 1e-6
(normalised), expectation error <= 1e-5 * sum_j |c_j|, and the reuse path
bitwise equal to the direct path. Every case prints its name before running.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu

FID_TOL = 1e-6
EXP_TOL = 1e-5
# |<psi|psi> - 1| of a GPU state: every fused op rounds its FP32 factors once
# (relative 2^-24 on amplitudes, 2^-23 on |psi|^2), about one such global
# rounding per pass and diagonal set; measured at most 6.1e-7 over ~900
# gates. 1e-5 leaves room for ~80 systematic roundings and still catches a
# wrong scale (a renormalisation that is missing after a projector, or
# applied with the wrong power of the norm)
NORM_TOL = 1e-5


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


def _fid(a, b):
    return oracle.fidelity(a.astype(np.complex128), b)


def _random_gates(n, g, count, renorm=0.0):
    names1 = ["X", "Y", "Z", "H", "S", "SDG", "T", "TDG", "RX", "RY", "RZ", "P"]
    gates = []
    for _ in range(count):
        if n == 1 or g.random() < 0.65:
            gates.append((names1[g.integers(len(names1))], (int(g.integers(n)),), float(g.uniform(0, 6.3))))
        else:
            a, b = g.choice(n, 2, replace=False)
            gates.append((("CNOT", "CZ")[int(g.integers(2))], (int(a), int(b)), 0.0))
        if g.random() < renorm:
            gates.append(("RENORM", (), 0.0))
    return gates


@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 10, 12, 14, 15, 16, 18])
def test_random_circuits_match_oracle(ctx, B, n):
    say("random circuit", n)
    g = np.random.default_rng(1000 + n)
    gates = _random_gates(n, g, 200, renorm=0.02)
    st = B.State(ctx, n, 2)
    st.apply(1, gates)
    psi = st.host(1)
    ref = oracle.simulate(n, gates)
    assert 1 - _fid(psi, ref) <= FID_TOL
    assert np.array_equal(st.host(0)[:1], np.array([1], dtype=np.complex64))  # slot 0 untouched
    st.free()


@pytest.mark.parametrize("tile", [10, 11, 12, 13, 14])
def test_tile_bits_sweep_17q(ctx, B, tile):
    say("tile sweep", tile)
    n = 17
    w = gen.small_vqe(n, 2, 1, 1, 9, seed=77)
    gates = w.task_gates(0)
    ctx.set_option(B.QW_OPT_TILE_BITS, tile)
    try:
        st = B.State(ctx, n, 1)
        st.apply(0, gates)
        psi = st.host(0)
        e = st.expect(0, 1, w.terms)[0]
    finally:
        ctx.set_option(B.QW_OPT_TILE_BITS, 14)
    ref = oracle.simulate(n, gates)
    assert 1 - _fid(psi, ref) <= FID_TOL
    assert abs(e - oracle.expect(ref, n, w.terms)) <= EXP_TOL * sum(abs(c) for c, _, _ in w.terms)
    st.free()


def run_reuse(B, ctx, w, terms=None, mode=None):
    from paper_2609_23664_amd.planner import fingerprint
    mode = B.QW_SNAP_FREEZE if mode is None else mode
    st = B.State(ctx, w.n, w.n_tasks + 1)
    st.apply(0, w.prefix)
    prov = fingerprint(w.n, w.prefix)
    snap = st.snapshot(0, prov, mode)
    e = B.run_suffix_batch(ctx, [snap] * w.n_tasks, w.suffixes, st,
                           list(range(1, w.n_tasks + 1)), terms=terms)
    return st, snap, e


def run_direct(B, ctx, w, terms=None):
    st = B.State(ctx, w.n, w.n_tasks)
    slots = list(range(w.n_tasks))
    B.run_suffix_batch(ctx, None, [w.prefix] * w.n_tasks, st, slots)
    e = B.run_suffix_batch(ctx, None, w.suffixes, st, slots, terms=terms)
    return st, e


def _check_vqe(B, ctx, w, oracle_tasks, mode=None):
    ctot = sum(abs(c) for c, _, _ in w.terms)
    st_r, snap, e_r = run_reuse(B, ctx, w, w.terms, mode)
    st_d, e_d = run_direct(B, ctx, w, w.terms)
    ctx.sync()
    import torch
    for t in range(w.n_tasks):
        assert torch.equal(st_r.buf[t + 1], st_d.buf[t]), f"task {t}: reuse != direct"
    assert e_r == e_d
    base = oracle.simulate(w.n, w.prefix)
    worst = [0.0, 0.0, 0.0]
    for t in oracle_tasks:
        ref = oracle.apply_gates(base.copy(), w.n, w.suffixes[t])
        psi = st_r.host(t + 1).astype(np.complex128)
        inf = 1 - _fid(psi, ref)
        err = abs(e_r[t] - oracle.expect(ref, w.n, w.terms)) / ctot
        drift = abs(float(np.vdot(psi, psi).real) - 1.0)
        worst = [max(worst[0], inf), max(worst[1], err), max(worst[2], drift)]
        assert inf <= FID_TOL, t
        assert err <= EXP_TOL, t
        assert drift <= NORM_TOL, t
        if w.n >= 20:
            say(f"  task {t}: 1-F={inf:.2e} err/sum|c|={err:.2e} drift={drift:.2e}")
    say(f"  worst over {len(list(oracle_tasks))} tasks: 1-F={worst[0]:.2e} "
        f"err/sum|c|={worst[1]:.2e} drift={worst[2]:.2e}")
    snap.free()
    st_r.free()
    st_d.free()
    return e_r


def test_config1_full(ctx, B):
    say("config1 10q x16 full")
    w = gen.config1()
    _check_vqe(B, ctx, w, range(w.n_tasks))


@pytest.mark.parametrize("mode", ["COPY", "FREEZE"])
def test_vqe_16q_ragged(ctx, B, mode):
    say("vqe 16q ragged", mode)
    w = gen.small_vqe(16, 3, 2, 7, 13, seed=91)
    _check_vqe(B, ctx, w, range(7), getattr(B, "QW_SNAP_" + mode))


def test_vqe_20q_weight4(ctx, B):
    say("vqe 20q")
    w = gen.small_vqe(20, 4, 2, 5, 50, seed=92)
    _check_vqe(B, ctx, w, [0, 4])


def test_config2_full_24q_all_tasks(ctx, B):
    """The 24-qubit, 64-task VQE workload: every task's state and Pauli-sum
    expectation against the oracle (prefix once, each suffix from a copy of
    its state), the reuse path bitwise equal to the direct path, the norm of
    every GPU state within NORM_TOL of 1."""
    say("config2 24q x64 full, all 64 tasks against the oracle")
    w = gen.config2()
    e = _check_vqe(B, ctx, w, range(w.n_tasks))
    assert all(math.isfinite(x) for x in e)


def test_product_state_expectations_24q(ctx, B):
    # closed form at full size: <P> = prod_q Bloch_q(P_q) for a product state
    say("product state 24q")
    n = 24
    w = gen.config2()
    g = np.random.default_rng(5)
    ang = g.uniform(0, 2 * math.pi, 2 * n)
    gates = [gg for gg in gen.hea_layer(n, ang) if gg[0] != "CNOT"]
    st = B.State(ctx, n, 1)
    st.apply(0, gates)
    vals = st.expect(0, 1, [(1.0, x, z) for _, x, z in w.terms[:1]])
    ev = []
    for c, x, z in w.terms:
        ev.append(st.expect(0, 1, [(1.0, x, z)])[0])
    for (c, x, z), v in zip(w.terms, ev):
        s = gen.pauli_string((c, x, z), n)
        e = 1.0
        for q, ch in enumerate(s):
            th, ph = ang[2 * q], ang[2 * q + 1]
            e *= {"X": math.sin(th) * math.cos(ph), "Y": math.sin(th) * math.sin(ph),
                  "Z": math.cos(th), "I": 1.0}[ch]
        assert abs(v - e) <= 1e-5
    assert abs(vals[0] - ev[0]) <= 1e-12
    st.free()


def test_ghz_24q(ctx, B):
    say("ghz 24q")
    n = 24
    ang = [0.0] * (2 * n)
    ang[0] = math.pi / 2
    st = B.State(ctx, n, 1)
    st.apply(0, gen.hea_layer(n, ang))
    psi = st.host(0)
    r = 1 / math.sqrt(2)
    assert abs(psi[0] - r) < 1e-6 and abs(psi[-1] - r) < 1e-6
    nz = np.count_nonzero(psi)
    assert nz == 2
    out = st.sample(0, 1, 7, 0, 1000)
    assert set(np.unique(out).tolist()) <= {0, (1 << n) - 1}
    st.free()


def dyadic_state(n, seed):
    """A state whose probabilities are exact in FP32 and FP64: 2^(n-3)
    amplitudes of modulus 2^-(n/2-1), 2^(n-1) of modulus 2^-(n/2), the rest
    zero, random phases from {1, -1, i, -i}. Every CDF value is a multiple of
    2^-n, so the inverse CDF is exact on both sides."""
    assert n % 2 == 0 and n >= 4
    g = np.random.default_rng(seed)
    perm = g.permutation(1 << n)
    amp = np.zeros(1 << n, dtype=np.complex128)
    ca, cb = 1 << (n - 3), 1 << (n - 1)
    amp[perm[:ca]] = 2.0 ** -(n // 2 - 1)
    amp[perm[ca:ca + cb]] = 2.0 ** -(n // 2)
    amp *= np.array([1, -1, 1j, -1j])[g.integers(0, 4, 1 << n)]
    return amp


@pytest.mark.parametrize("n,shots", [(4, 100), (8, 1000), (14, 1024), (20, 1000), (22, 513)])
def test_sampler_exact_on_dyadic_state(ctx, B, n, shots):
    # integer output: bit-exact against the oracle when the CDF is exact
    say("sampler exact", n, shots)
    amp = dyadic_state(n, 700 + n)
    assert abs(np.sum(np.abs(amp) ** 2) - 1.0) == 0.0
    import torch
    st = B.State(ctx, n, 3)
    st.buf[1].copy_(torch.from_numpy(amp.astype(np.complex64)))
    st.buf[2].copy_(torch.from_numpy(amp[::-1].copy().astype(np.complex64)))
    out = st.sample(1, 2, 99, 5, shots)
    for k, ref in enumerate((amp, amp[::-1].copy())):
        o = oracle.sample(ref, n, 99, 5 + k, shots)
        assert np.array_equal(o, out[k]), (k, np.flatnonzero(o != out[k])[:5])
    st.free()


@pytest.mark.parametrize("n", [3, 7, 12, 16])
def test_sampler_mass_at_the_ends(ctx, B, n):
    # all mass on the first or the last index, or on two indices of the
    # first and last sub-chunk with empty chunks between: every shot must
    # land on an index of non-zero probability, as the oracle's do
    say("sampler edge masses", n)
    import torch
    dim = 1 << n
    cases = []
    for idx in ([0], [dim - 1], [1, dim - 2], [dim // 2 - 1, dim // 2]):
        a = np.zeros(dim, dtype=np.complex128)
        a[idx] = 1.0 / np.sqrt(len(idx))
        cases.append(a)
    st = B.State(ctx, n, len(cases))
    for k, a in enumerate(cases):
        st.buf[k].copy_(torch.from_numpy(a.astype(np.complex64)))
    out = st.sample(0, len(cases), 7, 0, 300)
    for k, a in enumerate(cases):
        o = oracle.sample(a, n, 7, k, 300)
        assert np.array_equal(o, out[k]), (k, np.flatnonzero(o != out[k])[:5])
        assert np.all(np.abs(a[out[k]]) > 0)
    st.free()


@pytest.mark.parametrize("n,shots", [(8, 1000), (14, 1024), (20, 777)])
def test_sampling_matches_oracle(ctx, B, n, shots):
    # FP32 amplitudes shift the CDF by ~1e-9 at 20 qubits, so about
    # 2^n * 1e-9 of the shots may land on a neighbouring index; every GPU
    # shot must still be a valid inverse-CDF pick within eps = 1e-6 of the
    # oracle's CDF, and at least 99% must be identical.
    say("sampling", n, shots)
    w = gen.small_vqe(n, 3, 1, 3, 1, seed=500 + n)
    st_r, snap, _ = run_reuse(B, ctx, w)
    out = st_r.sample(1, 3, 12345, 10, shots)
    base = oracle.simulate(n, w.prefix)
    same = 0
    eps = 1e-6
    for t in range(3):
        ref = oracle.apply_gates(base.copy(), n, w.suffixes[t])
        o = oracle.sample(ref, n, 12345, 10 + t, shots)
        same += int(np.sum(o == out[t]))
        assert np.all(np.abs(ref[out[t]]) > 0)
        cdf = np.cumsum(np.abs(ref) ** 2)
        for s_, i in enumerate(out[t]):
            u = oracle.uniform(12345, 10 + t, s_) * cdf[-1]
            lo = cdf[i - 1] if i > 0 else 0.0
            assert lo - eps <= u <= cdf[i] + eps
    assert same >= 0.99 * 3 * shots
    snap.free()
    st_r.free()


def test_noisy_trajectories_match_oracle(ctx, B):
    say("noisy 14q")
    w = gen.small_noisy(14, 3, 2, 12, 0.02, seed=7, shots=0)
    assert sum(t != w.suffix for t in w.trajectories) >= 3
    from paper_2609_23664_amd.planner import fingerprint
    st = B.State(ctx, w.n, len(w.trajectories) + 1)
    st.apply(0, w.prefix)
    snap = st.snapshot(0, fingerprint(w.n, w.prefix), B.QW_SNAP_FREEZE)
    B.run_suffix_batch(ctx, [snap] * len(w.trajectories), w.trajectories, st,
                       list(range(1, len(w.trajectories) + 1)))
    base = oracle.simulate(w.n, w.prefix)
    for t, traj in enumerate(w.trajectories):
        ref = oracle.apply_gates(base.copy(), w.n, traj)
        psi = st.host(t + 1)
        assert 1 - _fid(psi, ref) <= FID_TOL
        norm = float(np.vdot(psi.astype(np.complex128), psi.astype(np.complex128)).real)
        assert abs(norm - 1.0) < 1e-5
    snap.free()
    st.free()


def test_refusal_then_direct_fallback(ctx, B):
    say("refusal")
    from paper_2609_23664_amd.planner import fingerprint
    w = gen.small_vqe(12, 2, 1, 3, 4, seed=3)
    st = B.State(ctx, w.n, 4)
    st.apply(0, w.prefix)
    snap = st.snapshot(0, fingerprint(w.n, w.prefix), B.QW_SNAP_COPY)
    bad = [bytes(32)] * 3
    with pytest.raises(B.QwRefused) as ei:
        B.run_suffix_batch(ctx, [snap] * 3, w.suffixes, st, [1, 2, 3], expect_provs=bad)
    rec = ei.value.record
    assert rec["reason"] == "PROVENANCE_MISMATCH"
    for f in ("detail", "source_kind", "target_kind", "source_backend", "target_backend"):
        assert f in rec
    # nothing ran: slots 1..3 still |0...0>
    for s in (1, 2, 3):
        h = st.host(s)
        assert h[0] == 1 and np.count_nonzero(h) == 1
    # fallback: direct rerun from scratch equals the reuse result
    st_d, _ = run_direct(B, ctx, w)
    st_r, snap2, _ = run_reuse(B, ctx, w)
    import torch
    for t in range(3):
        assert torch.equal(st_d.buf[t], st_r.buf[t + 1])
    for o in (snap, snap2):
        o.free()
    for o in (st, st_d, st_r):
        o.free()


def test_empty_suffix_copies_snapshot(ctx, B):
    say("empty suffix")
    from paper_2609_23664_amd.planner import fingerprint
    n = 16
    w = gen.small_vqe(n, 2, 1, 1, 1, seed=4)
    st = B.State(ctx, n, 3)
    st.apply(0, w.prefix)
    snap = st.snapshot(0, fingerprint(n, w.prefix), B.QW_SNAP_FREEZE)
    B.run_suffix_batch(ctx, [snap, snap], [[], w.suffixes[0]], st, [1, 2])
    B.run_suffix_batch(ctx, [], [], st, [])  # zero tasks is a no-op
    import torch
    ctx.sync()
    assert torch.equal(st.buf[0], st.buf[1])
    with pytest.raises(B.QwError):  # frozen slot cannot be a destination
        B.run_suffix_batch(ctx, None, [w.suffixes[0]], st, [0])
    snap.free()
    st.free()


def test_run_twice_bitwise(ctx, B):
    say("determinism")
    w = gen.small_vqe(18, 2, 2, 4, 20, seed=11)
    st1, s1, e1 = run_reuse(B, ctx, w, w.terms)
    st2, s2, e2 = run_reuse(B, ctx, w, w.terms)
    import torch
    ctx.sync()
    assert torch.equal(st1.buf, st2.buf) and e1 == e2
    for o in (s1, s2):
        o.free()
    for o in (st1, st2):
        o.free()


@pytest.mark.parametrize("n,q,f", [(14, 3, 2.5), (18, 12, 0.3)])
def test_renorm_after_projector_restores_the_norm(ctx, B, n, q, f):
    """The FP64 renormalisation on a state whose norm is far from 1: a
    projector PROJ1(f) on qubit q leaves |f|^2 P(1) of the norm; RENORM must
    bring it back to 1 (within FP32 rounding), and the state must be the
    oracle's projected, renormalised state followed by the remaining
    gates. The projection is written out here from its definition
    (diag(0, f) on qubit q), the rest is the oracle's."""
    say("renorm after projector", n, q, f)
    g = np.random.default_rng(300 + n)
    pre = _random_gates(n, g, 120)
    post = _random_gates(n, g, 60)
    st = B.State(ctx, n, 1)
    st.apply(0, pre + [("PROJ1", (q,), f), ("RENORM", (), 0.0)] + post)
    psi = st.host(0).astype(np.complex128)
    st.free()
    ref = oracle.simulate(n, pre)
    idx = np.arange(1 << n)
    ref = np.where(((idx >> q) & 1) == 1, f * ref, 0.0).astype(np.complex128)
    ref /= math.sqrt(oracle.norm2(ref))
    oracle.apply_gates(ref, n, post)
    assert abs(float(np.vdot(psi, psi).real) - 1.0) <= 1e-6
    assert 1 - _fid(psi, ref) <= FID_TOL
