"""Host checks of the pass planner (no GPU).

The plan that libqw would execute (qw_plan_describe) is interpreted here with
numpy, op by op with the kernel's op semantics, and compared with the oracle;
this checks fusion, gate reordering, local-bit mapping and phase grouping
independently of the GPU. Structural properties (passes per HEA layer, I/O
phases, register sets) are checked too.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2609_23664_amd import binding as B
from workloads import gen

LOC_REG, LOC_THREAD, LOC_GLOBAL, LOC_LANE = 0, 1, 2, 3
OP_U, OP_DIAG, OP_PERM, OP_CX, OP_CZ, OP_UR, OP_DSET, OP_DTAB, OP_PDIAG, OP_URT = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10


def _local_bits(mask):
    return [q for q in range(64) if (mask >> q) & 1]


def interpret(n, plan, psi):
    psi = psi.astype(np.complex128).copy()
    idx = np.arange(1 << n)
    for p in plan["passes"]:
        lb = _local_bits(p["local_mask"])
        assert len(lb) == plan["tile_bits"]
        if p["scale_in"]:
            psi /= np.sqrt(np.vdot(psi, psi).real)
        phase_of = {}
        for f in p["phases"]:
            for j in range(f["op_begin"], f["op_end"]):
                phase_of[j] = f
        # device records name a non-local qubit by its bit in the layout the
        # pass loads (in_pos); this interpreter keeps the standard layout
        qubit_at = {pos: q for q, pos in enumerate(p.get("in_pos", []))}
        for j, op in enumerate(p["ops"]):
            def gbit(loc, b):
                return qubit_at.get(b, b) if loc == LOC_GLOBAL else lb[b]
            m = op["m"]
            t = op["type"]
            if t == OP_DTAB:
                continue          # read with its OP_DSET header
            if t == OP_DSET:
                if op["sb"]:
                    # register table: entry k = product of the register-bit
                    # factors for register index k of the phase
                    reg = phase_of[j]["reg"]
                    tab = []
                    for r in range(op["sb"]):
                        mm = p["ops"][j + 1 + r]["m"]
                        assert p["ops"][j + 1 + r]["type"] == OP_DTAB
                        tab += [mm[2 * e] + 1j * mm[2 * e + 1] for e in range(4)]
                    k = np.zeros(1 << n, dtype=np.int64)
                    for s_, rb in enumerate(reg):
                        k |= ((idx >> lb[rb]) & 1) << s_
                    psi *= np.asarray(tab)[k]
                continue          # parity members follow as OP_PDIAG
            if t == OP_PDIAG:
                par = np.zeros(1 << n, dtype=np.int64)
                qm = op["qmask"]
                for q in range(n):
                    if (qm >> q) & 1:
                        par ^= (idx >> q) & 1
                psi *= np.where(par == 1, m[2] + 1j * m[3], m[0] + 1j * m[1])
                continue
            if t in (OP_U, OP_PERM, OP_UR, OP_URT):
                assert op["la"] != LOC_GLOBAL
                g = gbit(op["la"], op["a"])
                i0 = idx[((idx >> g) & 1) == 0]
                i1 = i0 | (1 << g)
                x, y = psi[i0].copy(), psi[i1].copy()
                if t == OP_URT:
                    tt = m[0]
                    a, b, c, d = {0: (1, -tt, tt, 1), 1: (1, tt, tt, -1)}[op["b"]]
                    psi[i0], psi[i1] = a * x + b * y, c * x + d * y
                elif t == OP_UR:
                    psi[i0], psi[i1] = m[0] * x + m[1] * y, m[2] * x + m[3] * y
                elif t == OP_U:
                    a, b, c, d = (m[0] + 1j * m[1], m[2] + 1j * m[3], m[4] + 1j * m[5], m[6] + 1j * m[7])
                    psi[i0], psi[i1] = a * x + b * y, c * x + d * y
                else:
                    psi[i0], psi[i1] = (m[0] + 1j * m[1]) * y, (m[2] + 1j * m[3]) * x
            elif t == OP_DIAG:
                g = gbit(op["la"], op["a"])
                d = np.where((idx >> g) & 1, m[2] + 1j * m[3], m[0] + 1j * m[1])
                psi *= d
            elif t == OP_CX:
                assert op["la"] != LOC_GLOBAL
                g = gbit(op["la"], op["a"])
                c = gbit(op["lb"], op["b"])
                sel = (((idx >> c) & 1) == 1) & (((idx >> g) & 1) == 0)
                i0 = idx[sel]
                i1 = i0 | (1 << g)
                psi[i0], psi[i1] = psi[i1].copy(), psi[i0].copy()
            elif t == OP_CZ:
                a = gbit(op["la"], op["a"])
                b = gbit(op["lb"], op["b"])
                psi[((idx >> a) & 1) & ((idx >> b) & 1) == 1] *= -1
            else:
                raise AssertionError(t)
        # output relabelling: the pass stores amplitude j at C(j) for each
        # trailing CNOT C, i.e. the CNOTs act after the pass, in order
        for c, t in p.get("out_cx", []):
            assert not (p["local_mask"] >> t) & 1
            sel = (((idx >> c) & 1) == 1) & (((idx >> t) & 1) == 0)
            i0 = idx[sel]
            i1 = i0 | (1 << t)
            psi[i0], psi[i1] = psi[i1].copy(), psi[i0].copy()
    return psi


def _lanes(m, reg):
    return [b for b in range(m) if b not in reg][:6]


def _check_phases(plan):
    """Layout invariants of the register kernel: 4 register bits per phase,
    first/last phases I/O capable, gate targets in a register or lane bit."""
    m = plan["tile_bits"]
    if m < 10:
        return
    for p in plan["passes"]:
        ph = p["phases"]
        assert ph[0]["op_begin"] == 0 and ph[-1]["op_end"] == len(p["ops"])
        lb = _local_bits(p["local_mask"])
        for c, t in p.get("out_cx", []):
            assert t not in lb                  # relabelling targets are non-local
            if c in lb:
                assert lb.index(c) >= 7         # never a lane bit of the store
        for a, b in zip(ph, ph[1:]):
            assert a["op_end"] == b["op_begin"]
        for k, f in enumerate(ph):
            reg = f["reg"]
            assert len(set(reg)) == 4 and reg == sorted(reg) and max(reg) < m
            lanes = _lanes(m, reg)
            kind = 1 if (0 in reg and lanes == [1, 2, 3, 4, 5, 6]) else (2 if lanes == list(range(6)) else 0)
            assert f["io"] == kind
            if k == 0 or k == len(ph) - 1:
                assert kind != 0
            for op in p["ops"][f["op_begin"]:f["op_end"]]:
                if op["type"] in (OP_U, OP_PERM, OP_CX, OP_UR, OP_URT):
                    assert op["la"] in (LOC_REG, LOC_LANE)
                    if op["la"] == LOC_REG:
                        assert reg[op["sa"]] == op["a"]
                    else:
                        assert lanes[op["sa"]] == op["a"]
                for loc, b, s_ in ((op["la"], op["a"], op["sa"]), (op["lb"], op["b"], op["sb"])):
                    if loc == LOC_REG:
                        assert reg[s_] == b


@pytest.mark.parametrize("n,tile", [(6, 14), (10, 14), (12, 10), (13, 11), (16, 12), (16, 14), (18, 10)])
def test_plan_matches_oracle_hea(n, tile):
    w = gen.small_vqe(n, 3, 2, 1, 1, seed=40 + n)
    gates = w.task_gates(0)
    plan = B.plan_describe(n, gates, tile)
    _check_phases(plan)
    psi = interpret(n, plan, oracle.zero_state(n))
    ref = oracle.simulate(n, gates)
    assert np.max(np.abs(psi - ref)) < 2e-5


@pytest.mark.parametrize("n,tile", [(11, 10), (15, 12)])
def test_plan_matches_oracle_random_gates(n, tile):
    g = np.random.default_rng(n)
    names1 = ["X", "Y", "Z", "H", "S", "SDG", "T", "TDG", "RX", "RY", "RZ", "P"]
    gates = []
    for _ in range(300):
        if g.random() < 0.65:
            gates.append((names1[g.integers(len(names1))], (int(g.integers(n)),), float(g.uniform(0, 6.3))))
        else:
            a, b = g.choice(n, 2, replace=False)
            gates.append((("CNOT", "CZ")[int(g.integers(2))], (int(a), int(b)), 0.0))
        if g.random() < 0.02:
            gates.append(("RENORM", (), 0.0))
    plan = B.plan_describe(n, gates, tile)
    _check_phases(plan)
    psi = interpret(n, plan, oracle.zero_state(n))
    ref = oracle.simulate(n, gates)
    assert np.max(np.abs(psi - ref)) < 5e-5


def test_hea_24q_pass_counts():
    """Two HEA layers on 24 qubits with 14 local bits take 3 passes: the
    trailing CNOT of the chain becomes an output relabelling (4 passes
    without it)."""
    w = gen.config2()
    pre = B.plan_describe(24, w.prefix)
    suf = B.plan_describe(24, w.suffixes[0])
    assert len(suf["passes"]) == 3
    assert suf["passes"][-1]["out_cx"]
    assert len(pre["passes"]) <= 12
    for p in pre["passes"] + suf["passes"]:
        assert p["local_mask"] & 0xF == 0xF   # 128-byte runs


def test_renorm_marks_norm_and_scale():
    gates = [("RY", (0,), 0.3), ("RENORM", (), 0.0), ("RY", (1,), 0.2), ("RENORM", (), 0.0)]
    plan = B.plan_describe(12, gates)
    ps = plan["passes"]
    assert ps[0]["norm_out"] == 1 and ps[1]["scale_in"] == 1 and ps[1]["norm_out"] == 1
    assert ps[-1]["scale_in"] == 1


def test_plan_is_deterministic():
    w = gen.small_vqe(20, 2, 2, 1, 1, seed=3)
    a = B.plan_describe(20, w.task_gates(0))
    b = B.plan_describe(20, w.task_gates(0))
    assert a == b


def test_vqe_tasks_share_one_pass_structure():
    """Suffixes that differ only in angles lower to the same ops and layouts
    (so one generated kernel serves every task)."""
    w = gen.config2()

    def shape(pl):
        return [[(o["type"], o["a"], o["b"], o["la"], o["lb"], o["sa"], o["sb"]) for o in p["ops"]]
                for p in pl["passes"]]
    ref = shape(B.plan_describe(24, w.suffixes[0]))
    for t in range(1, w.n_tasks):
        assert shape(B.plan_describe(24, w.suffixes[t])) == ref


def test_trie_leaves_of_equal_length_share_structure():
    """Leaf segments with the same gate kinds and qubits but different
    angles lower to the same ops (rotations in a factor-free form whose
    factors are folded per group into diagonal ops, real matrices split
    without sign-dependent phases)."""
    w = gen.small_trie(20, 2, 6, 2, 3, seed=303, shots=0)

    def shape(pl):
        return [[(o["type"], o["a"], o["b"], o["la"], o["lb"], o["sa"], o["sb"]) for o in p["ops"]]
                for p in pl["passes"]]
    by = {}
    for _, gates in w.leaves:
        key = tuple((g[0], tuple(g[1])) for g in gates)
        by.setdefault(key, []).append(gates)
    checked = 0
    for group in by.values():
        ref = shape(B.plan_describe(20, group[0]))
        for gates in group[1:]:
            assert shape(B.plan_describe(20, gates)) == ref
            checked += 1
    assert checked >= 3


def _to_layout(v, pos):
    """Standard-layout index bits of v at their places in layout pos (qubit q
    at bit pos[q]; an empty list is the standard layout)."""
    if not pos:
        return v
    r = np.zeros_like(v)
    for q, b in enumerate(pos):
        r |= ((v >> q) & 1) << b
    return r


def _from_layout(v, pos):
    if not pos:
        return v
    r = np.zeros_like(v)
    for q, b in enumerate(pos):
        r |= ((v >> b) & 1) << q
    return r


def _io_addresses(n, m, p, side, tile_bases):
    """Index of every element (tile, wave, lane, register) by the register
    kernel's address arithmetic of the pass's load (side "io_in") or store
    ("io_out", with output relabelling) record and the given tile origins,
    and the element's index in the standard layout before relabelling."""
    io = p[side]
    pos = p["in_pos"] if side == "io_in" else p["out_pos"]
    g4, g5, g6 = io["g"]
    lane = np.arange(64)
    if io["kind"] == 1:
        lane_off = ((lane & 7) << 1) | (((lane >> 3) & 1) << g4) | (((lane >> 4) & 1) << g5) | (((lane >> 5) & 1) << g6)
    else:
        lane_off = (lane & 15) | (((lane >> 4) & 1) << g4) | (((lane >> 5) & 1) << g5)
    nl = [q for q in range(n) if not (p["local_mask"] >> q) & 1]
    waves = 1 << (m - 10)
    addr, logical = [], []
    for ti in range(1 << (n - m)):
        base = sum(1 << nl[b] for b in range(len(nl)) if (ti >> b) & 1)
        for w in range(waves):
            for k in range(16):
                lo = io["wave_off"][w] | io["reg_off"][k]
                logical.append(base | _from_layout(lo | lane_off, pos))
                hi = tile_bases[ti]
                if side == "io_out":
                    hi = hi ^ io["wave_xor"][w] ^ io["reg_xor"][k]
                addr.append(hi | lo | lane_off)
    return np.concatenate(addr), np.concatenate(logical)


def _tile_origins(n, m, p, side):
    """The executor's tile origin tables: tile ti is the ti-th value of the
    non-local qubits in counting order, relabelled (stores) and placed in
    the side's layout."""
    nl = [q for q in range(n) if not (p["local_mask"] >> q) & 1]
    img = p["out_img"] if side == "io_out" else []
    pos = p["in_pos"] if side == "io_in" else p["out_pos"]
    out = []
    for ti in range(1 << (n - m)):
        o = 0
        for b, q in enumerate(nl):
            if (ti >> b) & 1:
                o ^= img[q] if img else (1 << q)
        out.append(int(_to_layout(np.int64(o), pos)))
    return out


def _relabel(v, out_cx):
    r = v.copy()
    for c, t in out_cx:
        r ^= ((r >> c) & 1) << t
    return r


def test_relabel_store_addresses_are_the_cnot_permutation():
    """For passes with output relabelling, the store index computed from the
    plan's store record and relabelled tile origins equals L(j), the image
    of the element's logical index under the pass's trailing CNOTs, placed
    in the layout the pass stores, and the stores are a permutation of the
    state."""
    from tests.test_gpu_relabel import _ladder_circuit
    checked = 0
    for n, tile, seed in [(16, 10, 1), (18, 12, 2), (20, 14, 3)]:
        gates = _ladder_circuit(n, np.random.default_rng(7100 + seed), 3)
        plan = B.plan_describe(n, gates, tile)
        m = plan["tile_bits"]
        for p in plan["passes"]:
            if not p["out_cx"]:
                continue
            img = p["out_img"]
            assert len(img) == n
            addr, logical = _io_addresses(n, m, p, "io_out", _tile_origins(n, m, p, "io_out"))
            assert np.array_equal(np.sort(addr), np.arange(1 << n))
            want = np.zeros_like(logical)
            for q in range(n):
                want ^= np.where((logical >> q) & 1, img[q], 0)
            # L from the CNOT list directly
            ref = _relabel(logical, p["out_cx"])
            assert np.array_equal(want, ref)
            assert np.array_equal(addr, _to_layout(ref, p["out_pos"]))
            checked += 1
    assert checked >= 3


def test_layouts_between_passes():
    """Index layouts between the passes of a plan: a plan loads and stores
    the standard layout at its ends; pass k stores the layout pass k + 1
    loads; qubits 0..3 keep bits 0..3; at each permuted boundary one side's
    local qubits are the lowest index bits (contiguous tiles). Every pass's
    load and store records, with the executor's tile origins, address each
    amplitude at its index in the side's layout (after relabelling, for
    stores), and both are permutations of the state. A config-2 suffix gets
    whole-tile stores in its middle pass and half-tile loads in its last."""
    from tests.test_gpu_relabel import _ladder_circuit
    w2 = gen.config2()
    cases = [(20, w2.suffixes[0], 14), (20, w2.prefix, 14),
             (16, _ladder_circuit(16, np.random.default_rng(7101), 3), 10),
             (18, gen.small_vqe(18, 3, 2, 1, 1, seed=58).task_gates(0), 12)]
    permuted = 0
    for n, gates, tile in cases:
        gates = [g for g in gates if max(g[1]) < n]
        plan = B.plan_describe(n, gates, tile)
        m = plan["tile_bits"]
        ps = plan["passes"]
        assert ps[0]["in_pos"] == [] and ps[-1]["out_pos"] == []
        for k, p in enumerate(ps):
            if k + 1 < len(ps):
                assert p["out_pos"] == ps[k + 1]["in_pos"]
            for pos in (p["in_pos"], p["out_pos"]):
                if pos:
                    assert sorted(pos) == list(range(n)) and pos[:4] == [0, 1, 2, 3]
            if p["out_pos"]:
                permuted += 1
                nxt = ps[k + 1]
                low = (1 << m) - 1
                sides = [int(_to_layout(np.int64(q["local_mask"]), p["out_pos"])) for q in (p, nxt)]
                assert low in sides
            for side in ("io_in", "io_out"):
                addr, logical = _io_addresses(n, m, p, side, _tile_origins(n, m, p, side))
                assert np.array_equal(np.sort(addr), np.arange(1 << n))
                pos = p["in_pos"] if side == "io_in" else p["out_pos"]
                want = logical if side == "io_in" else _relabel(logical, p["out_cx"])
                assert np.array_equal(addr, _to_layout(want, pos))
    assert permuted >= 3
    # config 2's suffix at 24 qubits: the middle pass stores whole tiles and
    # the last pass loads runs of 2^13 amplitudes (instead of 16 each)
    plan = B.plan_describe(24, w2.suffixes[0], 14)
    mid, last = plan["passes"][1], plan["passes"][2]
    assert int(_to_layout(np.int64(mid["local_mask"]), mid["out_pos"])) == (1 << 14) - 1
    run = int(~_to_layout(np.int64(last["local_mask"]), last["in_pos"]) & ((1 << 24) - 1))
    assert (run & -run).bit_length() - 1 >= 13


def test_special_angles_keep_the_structure_of_an_hea_suffix():
    """One RY of a config-2 suffix set to pi, pi/2, 2 pi or -pi gives the
    pass structure of generic angles: the one-FMA rotation form is chosen
    from the gate kinds, and one rotation's scale (at most 2^53.9, at
    exactly pi) is within the 2^60 bound. The documented exceptions change
    the structure: every RY at pi (several rotations near pi between two
    diagonal ops) and an angle of exactly 0 (RY(0) is exactly the identity
    and drops out of the plan)."""
    w = gen.config2()

    def shape(pl):
        return [[(o["type"], o["a"], o["b"], o["la"], o["lb"], o["sa"], o["sb"]) for o in p["ops"]]
                for p in pl["passes"]]
    ref = shape(B.plan_describe(24, w.suffixes[0]))
    ry = [k for k, g in enumerate(w.suffixes[0]) if g[0] == "RY"]
    for special in (math.pi, math.pi / 2, 2 * math.pi, -math.pi):
        for k in (ry[0], ry[17], ry[-1]):
            gates = list(w.suffixes[0])
            gates[k] = (gates[k][0], gates[k][1], special)
            assert shape(B.plan_describe(24, gates)) == ref, (special, k)
    for special in (math.pi, 0.0):
        gates = [(g[0], g[1], special if g[0] == "RY" else g[2]) for g in w.suffixes[0]]
        assert shape(B.plan_describe(24, gates)) != ref, special


@pytest.mark.parametrize("angles", [(math.pi, math.pi, math.pi), (1.0, 2.0, 0.5), (0.0, math.pi, 0.0)])
def test_degenerate_angles_still_give_the_oracle_state(angles):
    """Where angle values change the plan (several rotations near pi
    between diagonal ops, exact identities), the described plan still
    computes the oracle's state."""
    n = 12
    g = np.random.default_rng(2)
    gates = [("RY", (q,), float(g.uniform(0, 2 * math.pi))) for q in range(n)]
    gates += [("RY", (3,), angles[0]), ("RY", (5,), angles[1]), ("CNOT", (3, 5), 0.0),
              ("RY", (7,), angles[2]), ("RZ", (7,), 0.3), ("RY", (7,), angles[0])]
    for tile in (10, 12):
        plan = B.plan_describe(n, gates, tile)
        psi = interpret(n, plan, oracle.zero_state(n))
        ref = oracle.simulate(n, gates)
        assert oracle.fidelity(psi, ref) >= 1 - 1e-12
