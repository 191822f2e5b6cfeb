// Host planner of libqw: gate lists -> pass plans over local-bit tiles.
//
// A pass streams the whole state once (read + write of every amplitude):
// each workgroup owns a tile of 2^m amplitudes whose indices differ only in
// the pass's m "local" bits, so every gate whose operands are local (or that
// is diagonal, or a CNOT whose target is local) runs on data held on chip.
// High-order qubits become local by choosing the local bit set per pass
// (index-bit remapping); the low 4 bits are always local so that every tile
// is made of 128-byte contiguous runs.
//
// Inside a pass, the register kernel keeps 16 amplitudes per thread; the
// ops are split into phases, each with 4 local bits held in registers; an
// LDS exchange moves between phases.
//
// The plan is a pure function of (n, gates, tile bits); the reuse path and
// the direct path therefore execute the same arithmetic on the same values
// as long as both cut the gate list at the same prefix boundary.
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <cstring>
#include <complex>
#include <cmath>
#include <complex>
#include <cstdio>
#include <sstream>

#include "../../include/qw.h"
#include "qw_internal.h"

namespace qw {
namespace {

constexpr size_t kMaxPassGates = 8192;

using cd = std::complex<double>;

enum GClass { C_MIX, C_DIAG, C_PERM, C_CX, C_CZ, C_RENORM, C_DYN };

struct G {
    int kind;
    int q0, q1;
    double param;
    GClass cls;
};

struct M2 {
    cd a, b, c, d;  // [[a, b], [c, d]]
};

M2 mul(const M2 &x, const M2 &y) {  // x * y
    return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d,
            x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}

M2 gate_matrix(int kind, double t) {
    const cd I(0.0, 1.0);
    const double r2 = 1.0 / std::sqrt(2.0);
    const double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
    switch (kind) {
    case QW_GATE_X: return {0.0, 1.0, 1.0, 0.0};
    case QW_GATE_Y: return {0.0, -I, I, 0.0};
    case QW_GATE_Z: return {1.0, 0.0, 0.0, -1.0};
    case QW_GATE_H: return {r2, r2, r2, -r2};
    case QW_GATE_S: return {1.0, 0.0, 0.0, I};
    case QW_GATE_SDG: return {1.0, 0.0, 0.0, -I};
    case QW_GATE_T: return {1.0, 0.0, 0.0, std::polar(1.0, M_PI / 4.0)};
    case QW_GATE_TDG: return {1.0, 0.0, 0.0, std::polar(1.0, -M_PI / 4.0)};
    case QW_GATE_RX: return {c, -I * s, -I * s, c};
    case QW_GATE_RY: return {c, -s, s, c};
    case QW_GATE_RZ: return {std::polar(1.0, -0.5 * t), 0.0, 0.0, std::polar(1.0, 0.5 * t)};
    case QW_GATE_P: return {1.0, 0.0, 0.0, std::polar(1.0, t)};
    case QW_GATE_PROJ0: return {t, 0.0, 0.0, 0.0};
    case QW_GATE_PROJ1: return {0.0, 0.0, 0.0, t};
    default: return {1.0, 0.0, 0.0, 1.0};
    }
}

bool classify(int kind, GClass *cls) {
    switch (kind) {
    case QW_GATE_H: case QW_GATE_RX: case QW_GATE_RY: *cls = C_MIX; return true;
    case QW_GATE_X: case QW_GATE_Y: *cls = C_PERM; return true;
    case QW_GATE_Z: case QW_GATE_S: case QW_GATE_SDG: case QW_GATE_T:
    case QW_GATE_TDG: case QW_GATE_RZ: case QW_GATE_P:
    case QW_GATE_PROJ0: case QW_GATE_PROJ1: *cls = C_DIAG; return true;
    case QW_GATE_CNOT: *cls = C_CX; return true;
    case QW_GATE_CZ: *cls = C_CZ; return true;
    case QW_GATE_RENORM: *cls = C_RENORM; return true;
    default: return false;
    }
}

uint64_t qubit_mask(const G &g) {
    switch (g.cls) {
    case C_CX: case C_CZ: return (1ull << g.q0) | (1ull << g.q1);
    case C_RENORM: return 0;
    default: return 1ull << g.q0;
    }
}

// Qubits that must be local for the gate to run inside a tile.
uint64_t local_need(const G &g) {
    switch (g.cls) {
    case C_MIX: case C_PERM: case C_DYN: return 1ull << g.q0;
    case C_CX: return 1ull << g.q1;  // target only; the control may be global
    default: return 0;
    }
}

// One pass picked by the greedy construction: the gates run inside the tile
// (in order), the CNOTs applied as the output relabelling after them, and
// the local set.
struct PassPick {
    std::vector<int> gates;
    std::vector<int> out_cx;
    uint64_t mask = 0;
};

// Lowest local position a relabelling control may take: positions 0..6 can
// be lane bits of an I/O layout, whose addresses are per-lane, not uniform.
constexpr int kMinRelabelPos = 7;

// Greedy pass construction over one RENORM-free segment. Gates are taken in
// order; a gate that cannot run in the current pass is deferred and blocks
// its qubits, so later gates on those qubits are deferred too (this keeps
// the order of every pair of non-commuting gates). Gates on other qubits may
// overtake a deferred gate, which is valid since they act on disjoint
// qubits. `horizon` bounds how many gates are scanned past the first
// deferral (a negative horizon means no bound).
//
// With `relabel`, a CNOT whose target cannot be made local is taken as an
// output relabelling gate instead of being deferred: the pass stores the
// amplitude of index j at C(j) = j ^ (j_c << t), which is exactly the CNOT
// applied after everything the pass computes. Such a gate must therefore
// follow every in-tile gate of the pass on its two qubits: its qubits are
// closed to in-tile gates from then on (later relabelling CNOTs on them are
// still taken, composing the map in order), its target stays non-local
// (the padding skips it), and its control, if local, must sit at a local
// position >= kMinRelabelPos; a relabelling gate that fails that last test
// is deferred after all, with every later relabelling gate that shares a
// qubit with it.
std::vector<PassPick> greedy_passes(int n, int m, const std::vector<G> &gs, long horizon,
                                    bool relabel) {
    std::vector<PassPick> passes;
    std::vector<int> remaining(gs.size());
    for (size_t i = 0; i < gs.size(); ++i) remaining[i] = (int)i;
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    const int low = std::min(n, 4);
    while (!remaining.empty()) {
        uint64_t L = (n <= m) ? all : ((1ull << low) - 1);
        uint64_t blocked = 0, closed = 0, targets = 0;
        std::vector<int> acc, def, rel;
        long since_defer = -1;
        for (int idx : remaining) {
            const G &g = gs[idx];
            if (acc.size() >= kMaxPassGates) {  // keeps op indices in 16 bits
                def.push_back(idx);
                continue;
            }
            if (since_defer >= 0) {
                ++since_defer;
                if (horizon >= 0 && since_defer > horizon) {
                    def.push_back(idx);
                    continue;
                }
            }
            uint64_t qm = qubit_mask(g);
            if (qm & blocked) {
                def.push_back(idx);
                blocked |= qm;
                continue;
            }
            const uint64_t tbit = (g.cls == C_CX) ? (1ull << g.q1) : 0;
            if (qm & closed) {
                // only a further relabelling CNOT may touch a closed qubit
                if (tbit && !(tbit & L) && popc64(targets | tbit) <= n - m) {
                    rel.push_back(idx);
                    closed |= qm;
                    targets |= tbit;
                } else {
                    def.push_back(idx);
                    blocked |= qm;
                    if (since_defer < 0) since_defer = 0;
                }
                continue;
            }
            uint64_t need = local_need(g);
            if ((need & ~L) == 0) {
                acc.push_back(idx);
            } else if (!(need & targets) && popc64(L | need) <= m) {
                L |= need;
                acc.push_back(idx);
            } else if (relabel && tbit && !(tbit & L) && popc64(targets | tbit) <= n - m) {
                rel.push_back(idx);
                closed |= qm;
                targets |= tbit;
            } else {
                def.push_back(idx);
                blocked |= qm;
                if (since_defer < 0) since_defer = 0;
            }
        }
        // Pad the local set to exactly m bits with the lowest free bits that
        // are not relabelling targets.
        for (int q = 0; q < n && popc64(L) < m; ++q)
            if (!((targets >> q) & 1ull)) L |= 1ull << q;
        // Relabelling controls must not be local bits at lane positions.
        std::vector<int> keep;
        uint64_t dropped = 0;
        for (int idx : rel) {
            const G &g = gs[idx];
            const uint64_t qm = qubit_mask(g);
            bool ok = !(qm & dropped);
            if (ok && ((L >> g.q0) & 1ull))
                ok = popc64(L & ((1ull << g.q0) - 1)) >= kMinRelabelPos;
            if (ok) {
                keep.push_back(idx);
            } else {
                dropped |= qm;
                def.push_back(idx);
            }
        }
        std::sort(def.begin(), def.end());
        PassPick pk;
        pk.gates.swap(acc);
        pk.out_cx.swap(keep);
        pk.mask = L;
        passes.push_back(std::move(pk));
        remaining.swap(def);
    }
    return passes;
}

// Split a 2x2 unitary M into D2 * R * D1 with R real and D1, D2 diagonal;
// returns false if no such split was found (M is then kept complex).
// The phases are taken from fixed entries (a, d), falling back to the other
// entry of the row/column only when that one is negligible, so the form of
// the split (and of the kernels built from it) depends on the gate kinds,
// not on the angles. The fallback phase carries the sign that keeps R in the
// rotation pattern [[c, -s], [s, c]] (s >= 0) that the fixed entries give a
// unitary, so a rotation whose cosine is negligible (an angle of pi) still
// lowers to a rotation, not a reflection.
bool split_real(const M2 &M, M2 *D2, M2 *R, M2 *D1) {
    auto ph = [](cd z) { return z / std::abs(z); };
    auto small = [](double x) { return std::fabs(x) < 1e-13; };
    auto pick = [&](cd first, cd other, double sgn) {
        return std::abs(first) > 1e-9 ? ph(first) : sgn * ph(other);
    };
    // a real matrix is its own R (no sign-dependent phase factors)
    if (M.a.imag() == 0.0 && M.b.imag() == 0.0 && M.c.imag() == 0.0 && M.d.imag() == 0.0) {
        *D2 = {1.0, 0.0, 0.0, 1.0};
        *R = M;
        *D1 = {1.0, 0.0, 0.0, 1.0};
        return true;
    }
    // row phases: M = diag(p0, p1) * R
    {
        cd p0 = pick(M.a, M.b, -1.0);
        cd p1 = pick(M.d, M.c, 1.0);
        cd r00 = M.a / p0, r01 = M.b / p0, r10 = M.c / p1, r11 = M.d / p1;
        if (small(r00.imag()) && small(r01.imag()) && small(r10.imag()) && small(r11.imag())) {
            *D2 = {p0, 0.0, 0.0, p1};
            *R = {r00.real(), r01.real(), r10.real(), r11.real()};
            *D1 = {1.0, 0.0, 0.0, 1.0};
            return true;
        }
    }
    // column phases: M = R * diag(q0, q1)
    {
        cd q0 = pick(M.a, M.c, 1.0);
        cd q1 = pick(M.d, M.b, -1.0);
        cd r00 = M.a / q0, r01 = M.b / q1, r10 = M.c / q0, r11 = M.d / q1;
        if (small(r00.imag()) && small(r01.imag()) && small(r10.imag()) && small(r11.imag())) {
            *D2 = {1.0, 0.0, 0.0, 1.0};
            *R = {r00.real(), r01.real(), r10.real(), r11.real()};
            *D1 = {q0, 0.0, 0.0, q1};
            return true;
        }
    }
    // general: c = |M00|, s = |M10|, D2 = diag(M00/c, M10/s), D1 = diag(1, e)
    const double c = std::abs(M.a), s = std::abs(M.c);
    if (c < 1e-12 || s < 1e-12) return false;
    const cd p0 = M.a / c, p1 = M.c / s;
    const cd e = M.d / (p1 * c);
    *D2 = {p0, 0.0, 0.0, p1};
    *R = {c, -s, s, c};
    *D1 = {1.0, 0.0, 0.0, e};
    const M2 chk = mul(mul(*D2, *R), *D1);
    return std::abs(chk.a - M.a) + std::abs(chk.b - M.b) + std::abs(chk.c - M.c) +
               std::abs(chk.d - M.d) < 1e-12;
}

bool is_identity(const M2 &u) { return u.a == 1.0 && u.d == 1.0 && u.b == 0.0 && u.c == 0.0; }

// Fuse runs of single-qubit gates per qubit (FP64 products, rounded once to
// FP32 when lowered) and emit ops in an order equivalent to the gate order.
// Each mixing run becomes a real 2x2 rotation framed by diagonal factors.
// Diagonal factors stay pending as parity factors d[parity(x & mask)]: they
// commute with each other and with CZ, and a CNOT (control c, target t) is
// moved in front of them by rewriting every mask that holds t to mask ^ c
// (D(x) followed by CNOT equals CNOT followed by D(CNOT x)). All pending
// factors are emitted together, as one OP_DSET, before the first gate that
// mixes a qubit of one of their masks.
std::vector<HostOp> fuse_ops(int n, const std::vector<G> &gs, const std::vector<int> &idx) {
    std::vector<HostOp> ops;
    std::vector<M2> pend(n);
    std::vector<char> has(n, 0);
    // pending parity factors: mask -> (d0, d1), ordered by mask
    std::map<uint64_t, std::pair<cd, cd>> terms;
    auto add_term = [&](uint64_t mask, cd d0, cd d1) {
        auto it = terms.find(mask);
        if (it == terms.end()) {
            terms.emplace(mask, std::make_pair(d0, d1));
        } else {
            it->second.first *= d0;
            it->second.second *= d1;
        }
    };
    auto add_diag = [&](int q, const M2 &d) {
        if (is_identity(d)) return;
        add_term(1ull << q, d.a, d.d);
    };
    auto touches = [&](int q) {
        for (auto &t : terms)
            if ((t.first >> q) & 1ull) return true;
        return false;
    };
    auto emit_dset = [&]() {
        HostOp set;
        set.type = OP_DSET;
        for (auto &t : terms) {
            const cd d0 = t.second.first, d1 = t.second.second;
            if (d0 == 1.0 && d1 == 1.0) continue;
            HostOp d;
            d.type = OP_PDIAG;
            d.mask = t.first;
            d.m[0] = d0.real(); d.m[1] = d0.imag();
            d.m[2] = d1.real(); d.m[3] = d1.imag();
            set.members.push_back(d);
        }
        terms.clear();
        if (set.members.size() == 1 && popc64(set.members[0].mask) == 1) {
            HostOp d = set.members[0];
            d.type = OP_DIAG;
            d.a = __builtin_ctzll(d.mask);
            ops.push_back(d);
        } else if (!set.members.empty()) {
            ops.push_back(set);
        }
    };
    // CNOT moved in front of the pending factors
    auto cx_through = [&](int c, int t) {
        std::map<uint64_t, std::pair<cd, cd>> next;
        for (auto &e : terms) {
            const uint64_t m = ((e.first >> t) & 1ull) ? (e.first ^ (1ull << c)) : e.first;
            auto it = next.find(m);
            if (it == next.end()) {
                next.emplace(m, e.second);
            } else {
                it->second.first *= e.second.first;
                it->second.second *= e.second.second;
            }
        }
        terms.swap(next);
    };
    auto flush = [&](int q) {
        if (!has[q]) return;
        has[q] = 0;
        const M2 &u = pend[q];
        if (u.b == 0.0 && u.c == 0.0) {  // diagonal run
            add_diag(q, u);
            return;
        }
        HostOp op;
        op.a = q;
        if (u.a == 0.0 && u.d == 0.0) {  // exact swap with phases
            if (touches(q)) emit_dset();
            op.type = OP_PERM;
            op.m[0] = u.b.real(); op.m[1] = u.b.imag();
            op.m[2] = u.c.real(); op.m[3] = u.c.imag();
            ops.push_back(op);
            return;
        }
        M2 D2, R, D1;
        if (split_real(u, &D2, &R, &D1)) {
            add_diag(q, D1);
            if (touches(q)) emit_dset();
            op.type = OP_UR;
            op.m[0] = R.a.real(); op.m[1] = R.b.real();
            op.m[2] = R.c.real(); op.m[3] = R.d.real();
            ops.push_back(op);
            add_diag(q, D2);
            return;
        }
        if (touches(q)) emit_dset();
        op.type = OP_U;
        op.m[0] = u.a.real(); op.m[1] = u.a.imag();
        op.m[2] = u.b.real(); op.m[3] = u.b.imag();
        op.m[4] = u.c.real(); op.m[5] = u.c.imag();
        op.m[6] = u.d.real(); op.m[7] = u.d.imag();
        ops.push_back(op);
    };
    for (int i : idx) {
        const G &g = gs[i];
        if (g.cls == C_DYN) {
            // an operator whose entries the device writes at run time: the
            // run on its qubit and the pending factors on it go first; it is
            // never fused with other gates
            flush(g.q0);
            if (touches(g.q0)) emit_dset();
            HostOp op;
            op.type = OP_URD;
            op.a = g.q0;
            op.m[0] = g.param;  // the address bits of the entries
            ops.push_back(op);
            continue;
        }
        if (g.cls == C_CX || g.cls == C_CZ) {
            flush(g.q0);
            flush(g.q1);
            HostOp op;
            if (g.cls == C_CX) {
                cx_through(g.q0, g.q1);
                op.type = OP_CX;
                op.a = g.q1;  // target
                op.b = g.q0;  // control
            } else {
                op.type = OP_CZ;
                op.a = g.q0;
                op.b = g.q1;
            }
            ops.push_back(op);
        } else {
            M2 u = gate_matrix(g.kind, g.param);
            if (has[g.q0]) {
                pend[g.q0] = mul(u, pend[g.q0]);
            } else {
                pend[g.q0] = u;
                has[g.q0] = 1;
            }
        }
    }
    for (int q = 0; q < n; ++q) flush(q);
    emit_dset();
    return ops;
}

// Rewrite real rotations [[p, -q], [q, p]] as p * [[1, -t], [t, 1]] and
// reflections [[p, q], [q, -p]] as p * [[1, t], [t, -1]] (t = q / p). The
// factors p of the rotations between two diagonal ops are multiplied (in
// FP64) into the next diagonal op (else the previous one, else a new one at
// the end of the pass): a global factor, so where it is applied does not
// matter, and the FP32 amplitudes in between grow by at most the product
// of those 1/|p|. The form never depends on the angle, so tasks that differ
// only in angles keep one kernel; a large t costs no accuracy (the FMA
// rounds x - t y once and t's rounding weighs |q y|, as in the plain
// product). Only a group whose growth would pass 2^96 keeps its remaining
// rotations in the plain form: one rotation grows by at most 2^53.9 (at
// exactly pi, cos(pi/2) rounding to 6.1e-17), so that takes two rotations
// within ~1e-9 of pi between two diagonal ops. The bound keeps amplitudes
// below 2^96 (FP32 holds 2^128) and the folded factor above 2^-96 (FP32
// normals reach 2^-126).
void tangent_form(std::vector<HostOp> &ops) {
    double pending = 1.0, growth = 0.0;  // growth in log2, since the last diagonal op
    HostOp *last_diag = nullptr;
    auto scale_op = [](HostOp &op, double f) {
        HostOp *d = op.type == OP_DSET ? &op.members[0] : &op;
        for (int k = 0; k < 4; ++k) d->m[k] *= f;
    };
    for (HostOp &op : ops) {
        if (op.type == OP_DSET || op.type == OP_DIAG) {
            if (pending != 1.0) scale_op(op, pending);
            pending = 1.0;
            growth = 0.0;
            last_diag = &op;
            continue;
        }
        if (op.type != OP_UR) continue;
        const double a = op.m[0], b = op.m[1], c = op.m[2], d = op.m[3];
        const double tol = 1e-14 * (std::fabs(a) + std::fabs(b) + std::fabs(c) + std::fabs(d));
        int form = -1;
        double t = 0.0;
        if (std::fabs(a - d) <= tol && std::fabs(b + c) <= tol) {
            form = 0;
            t = c / a;
        } else if (std::fabs(a + d) <= tol && std::fabs(b - c) <= tol) {
            form = 1;
            t = b / a;
        }
        if (form < 0 || a == 0.0) continue;
        const double g = std::max(-std::log2(std::fabs(a)), 0.0);
        if (growth + g > 96.0) continue;
        growth += g;
        op.type = OP_URT;
        op.b = form;
        op.m[0] = t;
        op.m[1] = op.m[2] = op.m[3] = 0.0;
        pending *= a;
    }
    if (pending == 1.0) return;
    if (last_diag) {
        scale_op(*last_diag, pending);
        return;
    }
    HostOp set, d;
    set.type = OP_DSET;
    d.type = OP_PDIAG;
    d.mask = 0;
    d.m[0] = pending;
    d.m[2] = pending;
    set.members.push_back(d);
    ops.push_back(set);
}

int local_index(uint64_t mask, int g) { return popc64(mask & ((1ull << g) - 1)); }

// Layout helpers (see IoKind in qw_internal.h).
uint32_t lane_bits_of(int m, uint32_t R) {
    uint32_t lanes = 0;
    int c = 0;
    for (int b = 0; b < m && c < 6; ++b)
        if (!((R >> b) & 1u)) {
            lanes |= 1u << b;
            ++c;
        }
    return lanes;
}

uint8_t io_kind_of(int m, uint32_t R) {
    const uint32_t lanes = lane_bits_of(m, R);
    if ((R & 1u) && lanes == 0x7Eu) return IO_F4;
    if (lanes == 0x3Fu) return IO_F2;
    return IO_NONE;
}

// Fill R up to 4 bits with the highest unused local bits (keeps the lowest
// bits as lanes, which makes the layout I/O capable when possible).
uint32_t pad_high(int m, uint32_t R) {
    for (int b = m - 1; b >= 0 && popc64(R) < kRegBits; --b) R |= 1u << b;
    return R;
}

// Split a lowered pass into phases (register kernel only, m >= 10). In a
// phase, an op whose target bit is a register or lane bit runs without any
// data exchange; moving to a layout with other wave bits costs one LDS
// exchange. Within a phase ops are taken in order and a blocked op blocks
// its bits; the sequence of layouts comes from a small beam search under an
// instruction-count cost model (below).
void plan_phases(int m, HostPass &p, std::vector<DevOp> &lops_in, const std::vector<int> &unit_len,
                 const std::vector<std::array<double, 8>> &md_in) {
    // units: a single op, or an OP_DSET header with its members
    std::vector<size_t> ustart;
    {
        size_t pos = 0;
        for (int len : unit_len) {
            ustart.push_back(pos);
            pos += (size_t)len;
        }
    }
    struct Info { int need; uint32_t bits; };
    std::vector<Info> info(unit_len.size());
    for (size_t u = 0; u < unit_len.size(); ++u) {
        Info in{-1, 0};
        for (int j = 0; j < unit_len[u]; ++j) {
            const DevOp &o = lops_in[ustart[u] + j];
            bool a_loc = o.la != LOC_GLOBAL, b_loc = o.lb != LOC_GLOBAL;
            switch (o.type) {
            case OP_U: case OP_PERM: case OP_UR: case OP_URT: case OP_URD:
                in.need = o.a;
                in.bits |= 1u << o.a;
                break;
            case OP_CX: in.need = o.a; in.bits |= (1u << o.a) | (b_loc ? (1u << o.b) : 0u); break;
            case OP_DIAG: in.bits |= a_loc ? (1u << o.a) : 0u; break;
            case OP_PDIAG: in.bits |= o.tmask; break;
            case OP_CZ: in.bits |= (a_loc ? (1u << o.a) : 0u) | (b_loc ? (1u << o.b) : 0u); break;
            default: break;
            }
        }
        info[u] = in;
    }
    // Accept ops for layout R from `rem`; returns accepted / deferred. With
    // lanes_ok false only ops whose target is a register bit are taken (ops
    // without a target always are).
    auto run = [&](uint32_t R, bool lanes_ok, const std::vector<int> &rem, std::vector<int> *acc,
                   std::vector<int> *def) {
        const uint32_t intra = lanes_ok ? (R | lane_bits_of(m, R)) : R;
        uint32_t blocked = 0;
        acc->clear();
        def->clear();
        for (int i : rem) {
            const Info &in = info[i];
            if ((in.bits & blocked) || (in.need >= 0 && !((intra >> in.need) & 1u))) {
                def->push_back(i);
                blocked |= in.bits;
            } else {
                acc->push_back(i);
            }
        }
    };
    // Cost model (thread instructions per tile pass, 16 amplitudes per
    // thread): a register-target op costs its arithmetic; a lane target adds
    // the partner fetch of 32 floats (DPP for lane bits 0..3, twice that for
    // the ds_bpermute of bits 4..5); a CNOT on registers is a renaming, a
    // register target with a non-register control a select; each layout
    // change costs one LDS exchange (32 LDS accesses, address arithmetic and
    // two barriers).
    constexpr double kExchange = 100.0;
    constexpr double kWaveExchange = 50.0;  // same wave bits: no workgroup barrier
    auto wave_of = [&](uint32_t R) {
        return ((1u << m) - 1u) & ~R & ~lane_bits_of(m, R);
    };
    auto unit_cost = [&](int u, uint32_t R) -> double {
        const uint32_t lanes = lane_bits_of(m, R);
        double c = 0.0;
        for (int j = 0; j < unit_len[u]; ++j) {
            const DevOp &o = lops_in[ustart[u] + j];
            auto lane_extra = [&](int bit) -> double {
                if ((R >> bit) & 1u) return 0.0;
                int J = 0;
                for (int b = 0; b < bit; ++b) J += (lanes >> b) & 1u;
                return J < 4 ? 32.0 : 64.0;
            };
            switch (o.type) {
            case OP_URT: case OP_UR: case OP_URD: c += 32.0 + lane_extra(o.a); break;
            case OP_U: c += 64.0 + lane_extra(o.a); break;
            case OP_PERM: c += 16.0 + lane_extra(o.a); break;
            case OP_CX: {
                const bool creg = o.lb != LOC_GLOBAL && ((R >> o.b) & 1u);
                if ((R >> o.a) & 1u) c += creg ? 0.0 : 32.0;
                else c += 32.0 + lane_extra(o.a);
                break;
            }
            case OP_DIAG: c += 32.0; break;
            case OP_CZ: c += 16.0; break;
            case OP_DSET: c += 64.0; break;
            case OP_PDIAG: c += 16.0; break;
            default: break;
            }
        }
        return c;
    };
    const uint32_t R_F4 = (1u << 0) | (1u << 7) | (1u << 8) | (1u << 9);
    const uint32_t R_F2 = (1u << (m - 1)) | (1u << (m - 2)) | (1u << (m - 3)) | (1u << (m - 4));
    // Beam search over phase sequences: each step tries candidate layouts
    // (the I/O layouts, the registers wanted next in program order, with or
    // without the lane positions) under both acceptance policies; states
    // are ranked by cost so far plus the register-only cost of what remains.
    struct St {
        std::vector<int> rem;
        std::vector<std::vector<int>> ops;
        std::vector<uint32_t> R;
        double cost = 0.0;
        double rank = 0.0;
    };
    std::vector<double> reg_cost(unit_len.size());
    for (size_t i = 0; i < unit_len.size(); ++i) {
        const int nb = info[i].need;
        reg_cost[i] = unit_cost((int)i, nb >= 0 ? pad_high(m, 1u << nb) : R_F2);
    }
    auto lower_bound = [&](const std::vector<int> &rem) {
        double c = 0.0;
        for (int i : rem) c += reg_cost[i];
        return c;
    };
    const size_t beam = unit_len.size() > 512 ? 1 : 6;
    std::vector<St> states(1), done;
    for (size_t i = 0; i < unit_len.size(); ++i) states[0].rem.push_back((int)i);
    while (!states.empty()) {
        std::vector<St> next;
        for (const St &st : states) {
            const bool first = st.R.empty();
            std::vector<uint32_t> cands;
            if (first) {
                cands = {R_F4, R_F2};
            } else {
                uint32_t want_hi = 0, want_any = 0;
                for (int i : st.rem) {
                    const int nb = info[i].need;
                    if (nb < 0) continue;
                    if (nb >= 6 && !((want_hi >> nb) & 1u) && popc64(want_hi) < kRegBits) want_hi |= 1u << nb;
                    if (!((want_any >> nb) & 1u) && popc64(want_any) < kRegBits) want_any |= 1u << nb;
                }
                cands = {pad_high(m, want_hi), pad_high(m, want_any), R_F2, R_F4};
                for (int i : st.rem)
                    if (info[i].need >= 0) {
                        cands.push_back(pad_high(m, 1u << info[i].need));
                        break;
                    }
            }
            std::sort(cands.begin(), cands.end());
            cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
            std::vector<int> acc, def;
            for (uint32_t R : cands) {
                for (int pol = 0; pol < 2; ++pol) {
                    run(R, pol == 0, st.rem, &acc, &def);
                    if (acc.empty() && !(first && st.rem.empty())) continue;
                    St ns;
                    ns.rem = def;
                    ns.ops = st.ops;
                    ns.ops.push_back(acc);
                    ns.R = st.R;
                    ns.R.push_back(R);
                    ns.cost = st.cost;
                    if (!first)
                        ns.cost += (st.R.size() > 1 && wave_of(st.R.back()) == wave_of(R)) ? kWaveExchange
                                                                                      : kExchange;
                    for (int i : acc) ns.cost += unit_cost(i, R);
                    if (ns.rem.empty()) {
                        if (io_kind_of(m, R) == IO_NONE) {
                            ns.ops.push_back({});
                            ns.R.push_back(R_F2);
                            ns.cost += kExchange;
                        }
                        done.push_back(std::move(ns));
                    } else {
                        ns.rank = ns.cost + lower_bound(ns.rem);
                        next.push_back(std::move(ns));
                    }
                }
            }
        }
        std::stable_sort(next.begin(), next.end(), [](const St &a, const St &b) { return a.rank < b.rank; });
        // one state per remaining set (the cheapest), then the best `beam`
        std::vector<St> keep;
        for (St &st : next) {
            bool dup = false;
            for (const St &k : keep) dup |= k.rem == st.rem && k.R.back() == st.R.back();
            if (!dup) keep.push_back(std::move(st));
            if (keep.size() == beam) break;
        }
        states.swap(keep);
    }
    size_t bi = 0;
    for (size_t i = 1; i < done.size(); ++i)
        if (done[i].cost < done[bi].cost) bi = i;
    std::vector<std::vector<int>> phase_ops = std::move(done[bi].ops);
    std::vector<uint32_t> phase_R = std::move(done[bi].R);
    // Emit ops grouped by phase with operand locations resolved.
    std::vector<DevOp> out;
    p.dev_phases.clear();
    for (size_t ph = 0; ph < phase_R.size(); ++ph) {
        const uint32_t R = phase_R[ph];
        int reg[4], k = 0;
        for (int b = 0; b < m; ++b)
            if ((R >> b) & 1u) reg[k++] = b;
        const uint32_t lanes = lane_bits_of(m, R);
        int lane_idx[32];
        {
            int j = 0;
            for (int b = 0; b < m; ++b)
                if ((lanes >> b) & 1u) lane_idx[b] = j++;
        }
        DevPhase dp{};
        for (int s2 = 0; s2 < kRegBits; ++s2) dp.reg[s2] = (uint8_t)reg[s2];
        dp.io = io_kind_of(m, R);
        for (int kk = 0; kk < 16; ++kk) {
            uint32_t l = 0;
            for (int s2 = 0; s2 < 4; ++s2)
                if ((kk >> s2) & 1) l |= 1u << reg[s2];
            dp.lds_off[kk] = lds_swizzle(l) << 3;
        }
        dp.op_begin = (uint16_t)out.size();
        auto slot_of = [&](int b) -> int {
            for (int s2 = 0; s2 < kRegBits; ++s2)
                if (reg[s2] == b) return s2;
            return -1;
        };
        for (int ui : phase_ops[ph]) {
        if (lops_in[ustart[ui]].type == OP_DSET) {
            // members split by where their mask bits live in this phase:
            // register bits only -> 16-entry FP64 product table; no register
            // bits -> per-thread factor; both -> mixed member
            std::complex<double> tab[16];
            for (auto &t : tab) t = 1.0;
            bool has_tab = false;
            std::vector<DevOp> tg, mixed;
            for (int uj = 1; uj < unit_len[ui]; ++uj) {
                DevOp o = lops_in[ustart[ui] + uj];
                const auto &md = md_in[ustart[ui] + uj];
                uint8_t rmask = 0;
                for (int s2 = 0; s2 < kRegBits; ++s2)
                    if ((o.tmask >> reg[s2]) & 1u) rmask |= (uint8_t)(1u << s2);
                const uint32_t tpart = o.tmask & ~R;
                if (tpart == 0 && o.gmask == 0) {
                    const std::complex<double> d0(md[0], md[1]), d1(md[2], md[3]);
                    for (int kk = 0; kk < 16; ++kk) tab[kk] *= (popc64((uint64_t)(kk & rmask)) & 1) ? d1 : d0;
                    has_tab = true;
                    continue;
                }
                o.rmask = rmask;
                o.tmask = tpart;
                o.la = o.lb = LOC_GLOBAL;
                (rmask ? mixed : tg).push_back(o);
            }
            DevOp hd = lops_in[ustart[ui]];
            hd.b = (uint8_t)tg.size();
            hd.a = (uint8_t)mixed.size();
            hd.sb = has_tab ? 4 : 0;
            out.push_back(hd);
            if (has_tab) {
                for (int r = 0; r < 4; ++r) {
                    DevOp t{};
                    t.type = OP_DTAB;
                    t.la = t.lb = LOC_GLOBAL;
                    for (int e = 0; e < 4; ++e) {
                        t.m[2 * e] = (float)tab[4 * r + e].real();
                        t.m[2 * e + 1] = (float)tab[4 * r + e].imag();
                    }
                    out.push_back(t);
                }
            }
            for (const DevOp &o : tg) out.push_back(o);
            for (const DevOp &o : mixed) out.push_back(o);
            continue;
        }
        for (int uj = 0; uj < unit_len[ui]; ++uj) {
            DevOp o = lops_in[ustart[ui] + uj];
            const bool target_op =
                (o.type == OP_U || o.type == OP_PERM || o.type == OP_CX || o.type == OP_UR ||
                 o.type == OP_URT || o.type == OP_URD);
            if (o.la != LOC_GLOBAL) {
                int sl = slot_of(o.a);
                if (sl >= 0) {
                    o.la = LOC_REG;
                    o.sa = (uint8_t)sl;
                } else if (target_op) {
                    o.la = LOC_LANE;  // planner invariant: intra-wave target
                    o.sa = (uint8_t)lane_idx[o.a];
                } else {
                    o.la = LOC_THREAD;
                    o.sa = 0;
                }
            }
            if ((o.type == OP_CX || o.type == OP_CZ) && o.lb != LOC_GLOBAL) {
                int sl = slot_of(o.b);
                o.lb = sl >= 0 ? LOC_REG : LOC_THREAD;
                o.sb = (uint8_t)(sl >= 0 ? sl : 0);
            }
            out.push_back(o);
        }
        }
        dp.op_end = (uint16_t)out.size();
        p.dev_phases.push_back(dp);
    }
    lops_in.swap(out);
}

// Host form of the uniform address arithmetic of an I/O phase, for the
// index layout `pos` of the state it loads or stores.
IoRec make_iorec(int m, uint64_t lmask, const DevPhase &ph, const std::vector<uint8_t> &pos) {
    IoRec r{};
    r.kind = ph.io;
    std::vector<int> gpos;
    for (int q = 0; q < 64; ++q)
        if ((lmask >> q) & 1ull) gpos.push_back(pos.empty() ? q : pos[q]);
    r.g4 = (uint8_t)gpos[4];
    r.g5 = (uint8_t)gpos[5];
    r.g6 = (uint8_t)gpos[6];
    uint32_t R = 0;
    for (int s = 0; s < 4; ++s) R |= 1u << ph.reg[s];
    for (int k = 0; k < 16; ++k) {
        uint32_t off = 0;
        for (int s = 0; s < 4; ++s)
            if ((k >> s) & 1) off |= 1u << gpos[ph.reg[s]];
        r.reg_off[k] = off;
    }
    // wave bits: non-register local bits above the 6 lanes, ascending
    std::vector<int> wbits;
    int lanes = 0;
    for (int b = 0; b < m; ++b) {
        if ((R >> b) & 1u) continue;
        if (lanes < 6) {
            ++lanes;
            continue;
        }
        wbits.push_back(b);
    }
    for (int w = 0; w < 16; ++w) {
        uint32_t off = 0;
        for (size_t j = 0; j < wbits.size(); ++j)
            if ((w >> j) & 1) off |= 1u << gpos[wbits[j]];
        r.wave_off[w] = off;
    }
    return r;
}

// Output relabelling terms of the store record: the non-local part of the
// image of each local bit, combined per register index and per wave.
// Returns false if a lane bit would need one (the planner prevents that).
bool fill_relabel(int m, const HostPass &p, const DevPhase &ph, IoRec *r) {
    std::vector<int> gpos;
    for (int q = 0; q < 64; ++q)
        if ((p.local_mask >> q) & 1ull) gpos.push_back(q);
    auto dpart = [&](int b) -> uint32_t {
        const int q = gpos[b];
        return (uint32_t)to_layout(p.out_img[q] ^ (1ull << q), p.out_pos);
    };
    uint32_t R = 0;
    for (int s = 0; s < 4; ++s) R |= 1u << ph.reg[s];
    std::vector<int> wbits;
    int lanes = 0;
    for (int b = 0; b < m; ++b) {
        if ((R >> b) & 1u) continue;
        if (lanes < 6) {
            ++lanes;
            if (dpart(b)) return false;
            continue;
        }
        wbits.push_back(b);
    }
    for (int k = 0; k < 16; ++k) {
        uint32_t x = 0;
        for (int s = 0; s < 4; ++s)
            if ((k >> s) & 1) x ^= dpart(ph.reg[s]);
        r->reg_xor[k] = x;
    }
    for (int w = 0; w < 16; ++w) {
        uint32_t x = 0;
        for (size_t j = 0; j < wbits.size(); ++j)
            if ((w >> j) & 1) x ^= dpart(wbits[j]);
        r->wave_xor[w] = x;
    }
    return true;
}

// Convert a pass's ops to local bit numbers and device form. An OP_DSET
// becomes a header (b = member count) followed by its OP_DIAG members.
bool lower_pass(int n, int m, HostPass &p) {
    (void)n;
    std::vector<DevOp> lops;
    std::vector<std::array<double, 8>> lmd;  // FP64 entries, parallel to lops
    std::vector<int> unit_len;
    auto lower_one = [&](const HostOp &h) {
        DevOp o{};
        o.type = h.type;
        if (h.type == OP_URD) {
            // the device address of the entries, bit for bit
            std::memcpy(&o.m[0], &h.m[0], sizeof(double));
        } else {
            for (int k = 0; k < 8; ++k) o.m[k] = (float)h.m[k];
        }
        auto put = [&](int g, uint8_t *bit, uint8_t *loc) {
            if (g < 0) { *bit = 0; *loc = LOC_GLOBAL; return; }
            if ((p.local_mask >> g) & 1ull) {
                *bit = (uint8_t)local_index(p.local_mask, g);
                *loc = LOC_THREAD;  // resolved per phase
            } else {
                // read from the tile origin, an index in the load layout
                *bit = (uint8_t)(p.in_pos.empty() ? g : p.in_pos[g]);
                *loc = LOC_GLOBAL;
            }
        };
        if (h.type == OP_PDIAG) {
            o.tmask = (uint32_t)pext64(h.mask & p.local_mask, p.local_mask);
            o.gmask = (uint32_t)to_layout(h.mask & ~p.local_mask, p.in_pos);
            o.la = o.lb = LOC_GLOBAL;
            return o;
        }
        put(h.a, &o.a, &o.la);
        if (h.type == OP_CX || h.type == OP_CZ) put(h.b, &o.b, &o.lb);
        else o.lb = LOC_GLOBAL;
        if (h.type == OP_URT) o.b = (uint8_t)h.b;
        return o;
    };
    for (const HostOp &h : p.ops) {
        if (h.type == OP_DSET) {
            DevOp hd{};
            hd.type = OP_DSET;
            hd.la = LOC_GLOBAL;
            hd.lb = LOC_GLOBAL;
            hd.b = (uint8_t)h.members.size();
            lops.push_back(hd);
            lmd.push_back({});
            for (const HostOp &mm : h.members) {
                lops.push_back(lower_one(mm));
                std::array<double, 8> md;
                for (int k = 0; k < 8; ++k) md[k] = mm.m[k];
                lmd.push_back(md);
            }
            unit_len.push_back(1 + (int)h.members.size());
        } else {
            lops.push_back(lower_one(h));
            std::array<double, 8> md;
            for (int k = 0; k < 8; ++k) md[k] = h.m[k];
            lmd.push_back(md);
            unit_len.push_back(1);
        }
    }
    if (m >= kMinTileBits) {
        plan_phases(m, p, lops, unit_len, lmd);
        p.io_in = make_iorec(m, p.local_mask, p.dev_phases.front(), p.in_pos);
        p.io_out = make_iorec(m, p.local_mask, p.dev_phases.back(), p.out_pos);
        if (!p.out_img.empty() && !fill_relabel(m, p, p.dev_phases.back(), &p.io_out))
            return false;
    } else {
        // small-state kernel: whole state is one tile, no phases needed
        p.dev_phases.clear();
        DevPhase dp{};
        dp.op_begin = 0;
        dp.op_end = (uint16_t)lops.size();
        p.dev_phases.push_back(dp);
    }
    p.dev_ops.swap(lops);
    return true;
}

// Index layouts between the passes of a plan. A tile of a pass is one
// contiguous run of 2^m amplitudes when its local qubits are the lowest m
// index bits; two consecutive passes with different local sets cannot both
// have that, so each boundary favours one side: its local qubits in
// ascending order, then the other side's remaining local qubits, then the
// rest. The other side's run is then 2^r amplitudes, r the number of lowest
// index bits that it holds locally. The boundary takes the side that leaves
// the longer run to the other; at equal runs the pass with fewer ops (the
// one more bound by memory) gets the contiguous tiles. Qubits 0..3 stay at
// bits 0..3 (the lane part of every access), so a boundary is permuted only
// when both passes hold them, and only when that lengthens the runs.
// A pass that changes the layout stores to another buffer than it loads;
// an in-place plan whose first pass would then have to store into the
// buffer it loads keeps the standard layout at its first boundary.
void assign_layouts(int n, int m, Plan &plan, bool in_place) {
    auto favour = [&](uint64_t first, uint64_t second) {
        std::vector<uint8_t> pos(n);
        int next = 0;
        for (int q = 0; q < n; ++q)
            if ((first >> q) & 1ull) pos[q] = (uint8_t)next++;
        for (int q = 0; q < n; ++q)
            if (!((first >> q) & 1ull) && ((second >> q) & 1ull)) pos[q] = (uint8_t)next++;
        for (int q = 0; q < n; ++q)
            if (!(((first | second) >> q) & 1ull)) pos[q] = (uint8_t)next++;
        bool ident = true;
        for (int q = 0; q < n && ident; ++q) ident = pos[q] == q;
        if (ident) pos.clear();
        return pos;
    };
    // run length in index bits, counted up to 2 KiB runs (longer ones
    // stream no faster)
    auto run_bits = [&](uint64_t lmask, const std::vector<uint8_t> &pos) {
        return std::min(__builtin_ctzll(~to_layout(lmask, pos)), 8);
    };
    const size_t P = plan.passes.size();
    for (size_t k = 0; k + 1 < P; ++k) {
        HostPass &a = plan.passes[k], &b = plan.passes[k + 1];
        if ((a.local_mask & 15ull) != 15ull || (b.local_mask & 15ull) != 15ull) continue;
        if (a.local_mask == b.local_mask) continue;
        std::vector<uint8_t> w = favour(a.local_mask, b.local_mask);
        std::vector<uint8_t> r = favour(b.local_mask, a.local_mask);
        const int rw = run_bits(b.local_mask, w), rr = run_bits(a.local_mask, r);
        const bool reader = rr != rw ? rr > rw : a.ops.size() > b.ops.size();
        std::vector<uint8_t> &pos = reader ? r : w;
        const int std_runs = run_bits(a.local_mask, {}) + run_bits(b.local_mask, {});
        if (pos.empty() || run_bits(a.local_mask, pos) + run_bits(b.local_mask, pos) <= std_runs) continue;
        a.out_pos = pos;
        b.in_pos = pos;
    }
    if (in_place && P >= 2 && plan.passes[0].moves()) {
        size_t later = 0;
        for (size_t k = 1; k < P; ++k) later += plan.passes[k].moves();
        if (later % 2 == 0) {
            plan.passes[0].out_pos.clear();
            plan.passes[1].in_pos.clear();
        }
    }
}

}  // namespace

std::string build_plan(int n, const void *gates_v, size_t n_gates, int tile_bits, Plan *out,
                       bool relabel, bool lower, bool allow_dyn, bool layout, bool in_place) {
    const qw_gate *gates = static_cast<const qw_gate *>(gates_v);
    if (n < 1 || n > kMaxQubits) return "qubit count out of range 1..30";
    if (tile_bits < kMinTileBits || tile_bits > kMaxTileBits) return "tile bits out of range 10..14";
    if (n_gates > 0 && gates == nullptr) return "gates == NULL with n_gates > 0";
    const int m = tile_bits_for(n, tile_bits);
    std::vector<G> all;
    all.reserve(n_gates);
    for (size_t i = 0; i < n_gates; ++i) {
        const qw_gate &q = gates[i];
        G g{(int)q.kind, (int)q.q0, (int)q.q1, q.param, C_MIX};
        char buf[160];
        if (q.kind == QW_GATE_MEASURE || q.kind == QW_GATE_RESET) {
            // executed between segments (qw_apply_prefix, qw_run_suffix_batch)
            snprintf(buf, sizeof buf, "gate %zu: a measurement cannot be inside a pass plan", i);
            return buf;
        }
        if (q.kind == kGateDyn && allow_dyn) {
            g.cls = C_DYN;
        } else if (!classify(g.kind, &g.cls)) {
            snprintf(buf, sizeof buf, "gate %zu: unknown kind 0x%x", i, (unsigned)q.kind);
            return buf;
        }
        if (q.reserved != 0) {
            snprintf(buf, sizeof buf, "gate %zu: reserved field must be 0", i);
            return buf;
        }
        if (g.cls != C_RENORM) {
            if (q.q0 >= (uint32_t)n) {
                snprintf(buf, sizeof buf, "gate %zu: qubit %u >= n = %d", i, q.q0, n);
                return buf;
            }
            if ((g.cls == C_CX || g.cls == C_CZ) && (q.q1 >= (uint32_t)n || q.q1 == q.q0)) {
                snprintf(buf, sizeof buf, "gate %zu: bad second qubit %u", i, q.q1);
                return buf;
            }
            if (g.cls != C_DYN && !std::isfinite(q.param)) {
                snprintf(buf, sizeof buf, "gate %zu: non-finite parameter", i);
                return buf;
            }
        }
        all.push_back(g);
    }
    Plan plan;
    plan.n = n;
    plan.m = m;
    plan.n_gates = n_gates;
    // Split at RENORM markers: the pass ending a segment writes FP64 norm
    // partials, the first pass of the next segment applies 1/sqrt(norm).
    std::vector<std::vector<G>> segs(1);
    std::vector<char> renorm_after;
    for (const G &g : all) {
        if (g.cls == C_RENORM) {
            renorm_after.push_back(1);
            segs.emplace_back();
        } else {
            segs.back().push_back(g);
        }
    }
    renorm_after.push_back(0);
    bool pending_scale = false;
    for (size_t s = 0; s < segs.size(); ++s) {
        const std::vector<G> &gs = segs[s];
        std::vector<PassPick> best;
        if (!gs.empty()) {
            const long horizons[] = {-1, 0, 8, 32, 128, 512};
            for (long h : horizons) {
                auto ps = greedy_passes(n, m, gs, h, relabel);
                if (best.empty() || ps.size() < best.size()) best.swap(ps);
            }
        }
        // A segment with no gates still needs a pass if it must carry a
        // scale (renorm right after renorm / at the end) or a norm.
        if (best.empty() && (pending_scale || renorm_after[s])) {
            PassPick pk;
            pk.mask = n <= m ? ((1ull << n) - 1) : ((1ull << m) - 1);
            best.push_back(pk);
        }
        for (size_t k = 0; k < best.size(); ++k) {
            HostPass hp;
            hp.local_mask = best[k].mask;
            hp.ops = fuse_ops(n, gs, best[k].gates);
            tangent_form(hp.ops);
            if (!best[k].out_cx.empty()) {
                hp.out_img.resize(n);
                for (int q = 0; q < n; ++q) hp.out_img[q] = 1ull << q;
                for (int gi : best[k].out_cx) {
                    const G &g = gs[gi];
                    hp.out_cx.push_back({g.q0, g.q1});
                    for (int q = 0; q < n; ++q)
                        hp.out_img[q] ^= ((hp.out_img[q] >> g.q0) & 1ull) << g.q1;
                }
            }
            if (k == 0 && pending_scale) hp.scale_in = true;
            if (k + 1 == best.size() && renorm_after[s]) hp.norm_out = true;
            plan.passes.push_back(std::move(hp));
        }
        pending_scale = renorm_after[s] != 0;
    }
    plan.in_place = in_place;
    plan.layout = layout;
    if (layout && m >= kMinTileBits && n > m) assign_layouts(n, m, plan, in_place);
    if (lower)
        for (HostPass &p : plan.passes)
            if (!lower_pass(n, m, p)) return "internal: relabelling control on a lane bit";
    *out = std::move(plan);
    return "";
}

std::string plan_json(const Plan &p) {
    std::ostringstream o;
    o.precision(17);
    o << "{\"n\":" << p.n << ",\"tile_bits\":" << p.m << ",\"n_gates\":" << p.n_gates
      << ",\"passes\":[";
    for (size_t i = 0; i < p.passes.size(); ++i) {
        const HostPass &h = p.passes[i];
        if (i) o << ",";
        o << "{\"local_mask\":" << h.local_mask << ",\"scale_in\":" << (h.scale_in ? 1 : 0)
          << ",\"norm_out\":" << (h.norm_out ? 1 : 0) << ",\"out_cx\":[";
        for (size_t k = 0; k < h.out_cx.size(); ++k)
            o << (k ? "," : "") << "[" << h.out_cx[k].first << "," << h.out_cx[k].second << "]";
        o << "],\"out_img\":[";
        for (size_t k = 0; k < h.out_img.size(); ++k) o << (k ? "," : "") << h.out_img[k];
        o << "],\"in_pos\":[";
        for (size_t k = 0; k < h.in_pos.size(); ++k) o << (k ? "," : "") << (int)h.in_pos[k];
        o << "],\"out_pos\":[";
        for (size_t k = 0; k < h.out_pos.size(); ++k) o << (k ? "," : "") << (int)h.out_pos[k];
        // load and store records of the register kernel (address arithmetic
        // of the first and the last phase)
        o << "]";
        for (int side = 0; side < 2; ++side) {
            const IoRec &r = side ? h.io_out : h.io_in;
            o << (side ? ",\"io_out\"" : ",\"io_in\"") << ":{\"kind\":" << (int)r.kind << ",\"g\":["
              << (int)r.g4 << "," << (int)r.g5 << "," << (int)r.g6 << "]";
            const uint32_t *arrs[4] = {r.reg_off, r.wave_off, r.reg_xor, r.wave_xor};
            const char *names[4] = {"reg_off", "wave_off", "reg_xor", "wave_xor"};
            for (int a = 0; a < (side ? 4 : 2); ++a) {
                o << ",\"" << names[a] << "\":[";
                for (int k = 0; k < 16; ++k) o << (k ? "," : "") << arrs[a][k];
                o << "]";
            }
            o << "}";
        }
        o << ",\"ops\":[";
        for (size_t k = 0; k < h.dev_ops.size(); ++k) {
            const DevOp &d = h.dev_ops[k];
            if (k) o << ",";
            o << "{\"type\":" << (int)d.type << ",\"a\":" << (int)d.a << ",\"b\":" << (int)d.b
              << ",\"la\":" << (int)d.la << ",\"lb\":" << (int)d.lb << ",\"sa\":" << (int)d.sa
              << ",\"sb\":" << (int)d.sb;
            if (d.type == OP_PDIAG) {
                // qubit mask of the parity factor (register slots resolved with
                // the layout of the op's phase; non-local qubits by number, not
                // by their bit in the load layout)
                uint64_t g = d.gmask;
                if (!h.in_pos.empty()) {
                    g = 0;
                    for (int q2 = 0; q2 < p.n; ++q2)
                        if ((d.gmask >> h.in_pos[q2]) & 1u) g |= 1ull << q2;
                }
                uint64_t q = g | pdep64(d.tmask, h.local_mask);
                for (const DevPhase &f : h.dev_phases)
                    if (k >= f.op_begin && k < f.op_end)
                        for (int s2 = 0; s2 < 4; ++s2)
                            if ((d.rmask >> s2) & 1) q |= pdep64(1ull << f.reg[s2], h.local_mask);
                o << ",\"qmask\":" << q;
            }
            o << ",\"m\":[";
            for (int j = 0; j < 8; ++j) o << (j ? "," : "") << (double)d.m[j];
            o << "]}";
        }
        o << "],\"phases\":[";
        for (size_t k = 0; k < h.dev_phases.size(); ++k) {
            const DevPhase &d = h.dev_phases[k];
            if (k) o << ",";
            o << "{\"reg\":[" << (int)d.reg[0] << "," << (int)d.reg[1] << "," << (int)d.reg[2]
              << "," << (int)d.reg[3] << "],\"op_begin\":" << d.op_begin
              << ",\"op_end\":" << d.op_end << ",\"io\":" << (int)d.io << "}";
        }
        o << "]}";
    }
    o << "]}";
    return o.str();
}

// Greedy grouping of terms taken in `order`: each group takes every term
// (in order) whose X/Y support still fits m local bits with the group's.
std::vector<TermGroup> group_in_order(int n, int m, const uint64_t *x, const std::vector<uint32_t> &order) {
    std::vector<TermGroup> groups;
    const uint64_t all = (1ull << n) - 1;
    const uint64_t low = (1ull << std::min(n, 4)) - 1;
    std::vector<uint32_t> rem = order;
    while (!rem.empty()) {
        uint64_t L = low;
        std::vector<uint32_t> take, left;
        for (uint32_t t : rem) {
            if (take.size() < (size_t)kMaxGroupTerms && popc64(L | x[t]) <= m) {
                L |= x[t];
                take.push_back(t);
            } else {
                left.push_back(t);
            }
        }
        for (int q = 0; q < n && popc64(L) < m; ++q) L |= 1ull << q;
        std::sort(take.begin(), take.end());
        groups.push_back({L & all, take});
        rem.swap(left);
    }
    return groups;
}

static std::vector<TermGroup> group_terms_search(int n, int m, const uint64_t *x, size_t n_terms);

// Term grouping, memoized: the seeded search below costs about half a
// millisecond for 50 terms, and a VQE loop asks for the same grouping at
// every batch (it is a pure function of n, m and the X/Y masks).
std::vector<TermGroup> group_terms(int n, int m, const uint64_t *x, size_t n_terms) {
    static std::mutex mu;
    static std::map<std::vector<uint64_t>, std::vector<TermGroup>> memo;
    std::vector<uint64_t> key;
    key.reserve(n_terms + 2);
    key.push_back((uint64_t)n);
    key.push_back((uint64_t)m);
    key.insert(key.end(), x, x + n_terms);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
    }
    std::vector<TermGroup> groups = group_terms_search(n, m, x, n_terms);
    std::lock_guard<std::mutex> lk(mu);
    if (memo.size() >= 256) memo.clear();
    memo.emplace(std::move(key), groups);
    return groups;
}

static std::vector<TermGroup> group_terms_search(int n, int m, const uint64_t *x, size_t n_terms) {
    std::vector<TermGroup> groups;
    const uint64_t all = (1ull << n) - 1;
    if (n <= m) {
        for (size_t i = 0; i < n_terms; i += kMaxGroupTerms) {
            TermGroup g{all, {}};
            for (size_t k = i; k < std::min(n_terms, i + (size_t)kMaxGroupTerms); ++k)
                g.terms.push_back((uint32_t)k);
            groups.push_back(g);
        }
        return groups;
    }
    const uint64_t low = (1ull << std::min(n, 4)) - 1;
    std::vector<uint32_t> order(n_terms);
    for (size_t i = 0; i < n_terms; ++i) order[i] = (uint32_t)i;
    // hardest terms (most high X/Y bits) first
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return popc64(x[a] & ~low) > popc64(x[b] & ~low);
    });
    groups = group_in_order(n, m, x, order);
    // Every group is one sweep over the states: retry with seeded shuffles
    // of the order and keep the first grouping with fewer groups.
    uint32_t st = 0x2545F491u;
    for (int trial = 0; trial < 256 && groups.size() > 1; ++trial) {
        std::vector<uint32_t> o = order;
        for (size_t i = o.size(); i > 1; --i) {
            st ^= st << 13;
            st ^= st >> 17;
            st ^= st << 5;
            std::swap(o[i - 1], o[st % i]);
        }
        std::vector<TermGroup> g2 = group_in_order(n, m, x, o);
        if (g2.size() < groups.size()) groups.swap(g2);
    }
    return groups;
}

RedPlan plan_reduce_group(int n, int m, const TermGroup &g, const uint64_t *x,
                          const uint64_t *z, const uint8_t *diag_reg) {
    (void)n;
    RedPlan rp;
    const uint64_t L = g.local_mask;
    const size_t nt = g.terms.size();
    std::vector<uint32_t> xl(nt), zl(nt);
    for (size_t i = 0; i < nt; ++i) {
        xl[i] = (uint32_t)pext64(x[g.terms[i]], L);
        zl[i] = (uint32_t)pext64(z[g.terms[i]], L);
    }
    // first-fit decreasing packing of X/Y supports into 4-bit register sets
    std::vector<size_t> order(nt);
    for (size_t i = 0; i < nt; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return popc64(xl[a]) > popc64(xl[b]); });
    std::vector<uint32_t> R;
    std::vector<std::vector<size_t>> mem;
    std::vector<size_t> diag;
    for (size_t i : order) {
        if (xl[i] == 0) {
            diag.push_back(i);
            continue;
        }
        int best = -1, best_sz = 99;
        for (size_t p = 0; p < R.size(); ++p) {
            int sz = popc64(R[p] | xl[i]);
            if (sz <= kRegBits && sz < best_sz) {
                best = (int)p;
                best_sz = sz;
            }
        }
        if (best < 0) {
            R.push_back(xl[i]);
            mem.push_back({i});
        } else {
            R[best] |= xl[i];
            mem[best].push_back(i);
        }
    }
    // diagonal terms: one phase, first, in the I/O layout (register bits 0,
    // 7, 8, 9) or the given one
    std::vector<char> is_diag(R.size(), 0);
    if (!diag.empty()) {
        uint32_t dr = (1u << 0) | (1u << 7) | (1u << 8) | (1u << 9);
        if (diag_reg) {
            dr = 0;
            for (int s2 = 0; s2 < 4; ++s2) dr |= 1u << diag_reg[s2];
        }
        R.insert(R.begin(), dr);
        mem.insert(mem.begin(), diag);
        is_diag.insert(is_diag.begin(), 1);
    }
    for (size_t p = 0; p < R.size(); ++p) {
        for (int b = 0; b < m && popc64(R[p]) < kRegBits; ++b) R[p] |= 1u << b;
        int reg[4], k = 0;
        for (int b = 0; b < m; ++b)
            if ((R[p] >> b) & 1u) reg[k++] = b;
        RedPhase ph{};
        for (int s = 0; s < 4; ++s) ph.reg[s] = (uint8_t)reg[s];
        ph.t_begin = (uint16_t)rp.terms.size();
        for (size_t i : mem[p]) {
            TermDev t{};
            for (int s = 0; s < 4; ++s)
                if ((xl[i] >> reg[s]) & 1u) t.xr |= (uint8_t)(1u << s);
            for (int kk = 0; kk < 16; ++kk) {
                uint32_t l = 0;
                for (int s = 0; s < 4; ++s)
                    if ((kk >> s) & 1) l |= 1u << reg[s];
                if (popc64(l & zl[i]) & 1) t.smask |= (uint16_t)(1u << kk);
            }
            const int ny = popc64(x[g.terms[i]] & z[g.terms[i]]) & 3;
            t.odd = (uint8_t)(ny & 1);
            t.neg = (uint8_t)((ny == 1 || ny == 2) ? 1 : 0);
            t.zt = zl[i] & ~R[p];
            t.zg = z[g.terms[i]] & ~L;
            t.col = (uint16_t)i;
            rp.terms.push_back(t);
        }
        ph.t_end = (uint16_t)rp.terms.size();
        ph.diag = is_diag[p] ? 1u : 0u;
        rp.phases.push_back(ph);
    }
    rp.cols.assign(g.terms.begin(), g.terms.end());
    return rp;
}

}  // namespace qw
