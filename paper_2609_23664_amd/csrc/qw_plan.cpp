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

enum GClass { C_MIX, C_DIAG, C_PERM, C_CX, C_CZ, C_RENORM };

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
    default: return {1.0, 0.0, 0.0, 1.0};
    }
}

bool classify(int kind, GClass *cls) {
    switch (kind) {
    case QW_GATE_H: case QW_GATE_RX: case QW_GATE_RY: *cls = C_MIX; return true;
    case QW_GATE_X: case QW_GATE_Y: *cls = C_PERM; return true;
    case QW_GATE_Z: case QW_GATE_S: case QW_GATE_SDG: case QW_GATE_T:
    case QW_GATE_TDG: case QW_GATE_RZ: case QW_GATE_P: *cls = C_DIAG; return true;
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
    case C_MIX: case C_PERM: return 1ull << g.q0;
    case C_CX: return 1ull << g.q1;  // target only; the control may be global
    default: return 0;
    }
}

// Greedy pass construction over one RENORM-free segment. Gates are taken in
// order; a gate that cannot run in the current pass is deferred and blocks
// its qubits, so later gates on those qubits are deferred too (this keeps
// the order of every pair of non-commuting gates). Gates on other qubits may
// overtake a deferred gate, which is valid since they act on disjoint
// qubits. `horizon` bounds how many gates are scanned past the first
// deferral (a negative horizon means no bound).
std::vector<std::vector<int>> greedy_passes(int n, int m, const std::vector<G> &gs,
                                            long horizon, std::vector<uint64_t> *masks) {
    std::vector<std::vector<int>> passes;
    masks->clear();
    std::vector<int> remaining(gs.size());
    for (size_t i = 0; i < gs.size(); ++i) remaining[i] = (int)i;
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    const int low = std::min(n, 4);
    while (!remaining.empty()) {
        uint64_t L = (n <= m) ? all : ((1ull << low) - 1);
        uint64_t blocked = 0;
        std::vector<int> acc, def;
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
            uint64_t need = local_need(g);
            if ((need & ~L) == 0) {
                acc.push_back(idx);
            } else if (popc64(L | need) <= m) {
                L |= need;
                acc.push_back(idx);
            } else {
                def.push_back(idx);
                blocked |= qm;
                if (since_defer < 0) since_defer = 0;
            }
        }
        // Pad the local set to exactly m bits with the lowest free bits.
        for (int q = 0; q < n && popc64(L) < m; ++q) L |= 1ull << q;
        passes.push_back(acc);
        masks->push_back(L);
        remaining.swap(def);
    }
    return passes;
}

// Fuse runs of single-qubit gates per qubit (FP64 products, rounded once to
// FP32 when lowered) and emit ops in an order equivalent to the gate order.
std::vector<HostOp> fuse_ops(int n, const std::vector<G> &gs, const std::vector<int> &idx) {
    std::vector<HostOp> ops;
    std::vector<M2> pend(n);
    std::vector<char> has(n, 0);
    auto flush = [&](int q) {
        if (!has[q]) return;
        has[q] = 0;
        const M2 &u = pend[q];
        HostOp op;
        op.a = q;
        if (u.b == 0.0 && u.c == 0.0) {
            if (u.a == 1.0 && u.d == 1.0) return;  // exact identity
            op.type = OP_DIAG;
            op.m[0] = u.a.real(); op.m[1] = u.a.imag();
            op.m[2] = u.d.real(); op.m[3] = u.d.imag();
        } else if (u.a == 0.0 && u.d == 0.0) {
            op.type = OP_PERM;
            op.m[0] = u.b.real(); op.m[1] = u.b.imag();
            op.m[2] = u.c.real(); op.m[3] = u.c.imag();
        } else {
            op.type = OP_U;
            op.m[0] = u.a.real(); op.m[1] = u.a.imag();
            op.m[2] = u.b.real(); op.m[3] = u.b.imag();
            op.m[4] = u.c.real(); op.m[5] = u.c.imag();
            op.m[6] = u.d.real(); op.m[7] = u.d.imag();
        }
        ops.push_back(op);
    };
    for (int i : idx) {
        const G &g = gs[i];
        if (g.cls == C_CX || g.cls == C_CZ) {
            flush(g.q0);
            flush(g.q1);
            HostOp op;
            op.type = (g.cls == C_CX) ? OP_CX : OP_CZ;
            if (g.cls == C_CX) {
                op.a = g.q1;  // target
                op.b = g.q0;  // control
            } else {
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
    return ops;
}

int local_index(uint64_t mask, int g) { return popc64(mask & ((1ull << g) - 1)); }

bool io_ok(const std::vector<int> &R) {
    // slot 0 is local bit 0; no register bit among the lane bits 1..6
    bool has0 = false;
    for (int b : R) {
        if (b == 0) has0 = true;
        if (b >= kIoLaneLo && b <= kIoLaneHi) return false;
    }
    return has0 || (int)R.size() < kRegBits;
}

// Split a lowered pass into register phases (register kernel only, m >= 10).
void plan_phases(int m, HostPass &p, std::vector<DevOp> &lops) {
    // Per op: register need (local bit or -1) and blocking bits (local).
    struct Info { int need; uint32_t bits; };
    std::vector<Info> info(lops.size());
    for (size_t i = 0; i < lops.size(); ++i) {
        const DevOp &o = lops[i];
        Info in{-1, 0};
        bool a_loc = o.la != LOC_GLOBAL, b_loc = o.lb != LOC_GLOBAL;
        switch (o.type) {
        case OP_U: case OP_PERM: in.need = o.a; in.bits = 1u << o.a; break;
        case OP_CX: in.need = o.a; in.bits = (1u << o.a) | (b_loc ? (1u << o.b) : 0u); break;
        case OP_DIAG: in.bits = a_loc ? (1u << o.a) : 0u; break;
        case OP_CZ: in.bits = (a_loc ? (1u << o.a) : 0u) | (b_loc ? (1u << o.b) : 0u); break;
        default: break;
        }
        info[i] = in;
    }
    std::vector<int> remaining(lops.size());
    for (size_t i = 0; i < lops.size(); ++i) remaining[i] = (int)i;
    std::vector<std::vector<int>> phase_ops;
    std::vector<std::vector<int>> phase_regs;
    bool first = true;
    while (!remaining.empty() || first) {
        std::vector<int> R;
        if (first) R.push_back(0);
        uint32_t blocked = 0;
        std::vector<int> acc, def;
        for (int i : remaining) {
            const Info &in = info[i];
            if (in.bits & blocked) {
                def.push_back(i);
                blocked |= in.bits;
                continue;
            }
            if (in.need < 0 || std::find(R.begin(), R.end(), in.need) != R.end()) {
                acc.push_back(i);
                continue;
            }
            bool allowed = !first || in.need < kIoLaneLo || in.need > kIoLaneHi;
            if ((int)R.size() < kRegBits && allowed) {
                R.push_back(in.need);
                acc.push_back(i);
            } else {
                def.push_back(i);
                blocked |= in.bits;
            }
        }
        phase_ops.push_back(acc);
        phase_regs.push_back(R);
        remaining.swap(def);
        first = false;
    }
    // The last phase must be I/O capable; otherwise append an empty one.
    if (!io_ok(phase_regs.back())) {
        phase_ops.push_back({});
        phase_regs.push_back({0});
    } else if (std::find(phase_regs.back().begin(), phase_regs.back().end(), 0) ==
               phase_regs.back().end()) {
        phase_regs.back().push_back(0);
    }
    // Pad every phase to 4 register bits. I/O phases (first and last) take
    // pads from bits >= 7; others from any free bit.
    const size_t np = phase_regs.size();
    for (size_t ph = 0; ph < np; ++ph) {
        std::vector<int> &R = phase_regs[ph];
        bool io = (ph == 0 || ph + 1 == np);
        for (int b = 0; b < m && (int)R.size() < kRegBits; ++b) {
            if (std::find(R.begin(), R.end(), b) != R.end()) continue;
            if (io && b >= kIoLaneLo && b <= kIoLaneHi) continue;
            R.push_back(b);
        }
        std::sort(R.begin(), R.end());
    }
    // Emit ops grouped by phase with register slots resolved.
    std::vector<DevOp> out;
    p.dev_phases.clear();
    for (size_t ph = 0; ph < np; ++ph) {
        const std::vector<int> &R = phase_regs[ph];
        DevPhase dp{};
        for (int s = 0; s < kRegBits; ++s) dp.reg[s] = (uint8_t)R[s];
        dp.op_begin = (uint16_t)out.size();
        for (int i : phase_ops[ph]) {
            DevOp o = lops[i];
            auto slot_of = [&](int b) -> int {
                for (int s = 0; s < kRegBits; ++s)
                    if (R[s] == b) return s;
                return -1;
            };
            if (o.la != LOC_GLOBAL) {
                int s = slot_of(o.a);
                o.la = s >= 0 ? LOC_REG : LOC_THREAD;
                o.sa = (uint8_t)(s >= 0 ? s : 0);
            }
            if ((o.type == OP_CX || o.type == OP_CZ) && o.lb != LOC_GLOBAL) {
                int s = slot_of(o.b);
                o.lb = s >= 0 ? LOC_REG : LOC_THREAD;
                o.sb = (uint8_t)(s >= 0 ? s : 0);
            }
            out.push_back(o);
        }
        dp.op_end = (uint16_t)out.size();
        p.dev_phases.push_back(dp);
    }
    lops.swap(out);
}

// Convert a pass's ops to local bit numbers and device form.
void lower_pass(int n, int m, HostPass &p) {
    std::vector<DevOp> lops;
    for (const HostOp &h : p.ops) {
        DevOp o{};
        o.type = h.type;
        for (int k = 0; k < 8; ++k) o.m[k] = (float)h.m[k];
        auto put = [&](int g, uint8_t *bit, uint8_t *loc) {
            if (g < 0) { *bit = 0; *loc = LOC_GLOBAL; return; }
            if ((p.local_mask >> g) & 1ull) {
                *bit = (uint8_t)local_index(p.local_mask, g);
                *loc = LOC_THREAD;  // resolved per phase
            } else {
                *bit = (uint8_t)g;
                *loc = LOC_GLOBAL;
            }
        };
        put(h.a, &o.a, &o.la);
        if (h.type == OP_CX || h.type == OP_CZ) put(h.b, &o.b, &o.lb);
        else o.lb = LOC_GLOBAL;
        lops.push_back(o);
    }
    if (m >= kMinTileBits) {
        plan_phases(m, p, lops);
    } else {
        // small-state kernel: whole state is one tile, no phases needed
        p.dev_phases.clear();
        DevPhase dp{};
        dp.op_begin = 0;
        dp.op_end = (uint16_t)lops.size();
        p.dev_phases.push_back(dp);
    }
    p.dev_ops.swap(lops);
}

}  // namespace

std::string build_plan(int n, const void *gates_v, size_t n_gates, int tile_bits, Plan *out) {
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
        if (!classify(g.kind, &g.cls)) {
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
            if (!std::isfinite(q.param)) {
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
        std::vector<std::vector<int>> best;
        std::vector<uint64_t> best_masks;
        if (!gs.empty()) {
            const long horizons[] = {-1, 0, 8, 32, 128, 512};
            for (long h : horizons) {
                std::vector<uint64_t> masks;
                auto ps = greedy_passes(n, m, gs, h, &masks);
                if (best.empty() || ps.size() < best.size()) {
                    best = ps;
                    best_masks = masks;
                }
            }
        }
        // A segment with no gates still needs a pass if it must carry a
        // scale (renorm right after renorm / at the end) or a norm.
        if (best.empty() && (pending_scale || renorm_after[s])) {
            best.push_back({});
            best_masks.push_back(n <= m ? ((1ull << n) - 1) : ((1ull << m) - 1));
        }
        for (size_t k = 0; k < best.size(); ++k) {
            HostPass hp;
            hp.local_mask = best_masks[k];
            hp.ops = fuse_ops(n, gs, best[k]);
            if (k == 0 && pending_scale) hp.scale_in = true;
            if (k + 1 == best.size() && renorm_after[s]) hp.norm_out = true;
            plan.passes.push_back(std::move(hp));
        }
        pending_scale = renorm_after[s] != 0;
    }
    for (HostPass &p : plan.passes) lower_pass(n, m, p);
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
          << ",\"norm_out\":" << (h.norm_out ? 1 : 0) << ",\"ops\":[";
        for (size_t k = 0; k < h.dev_ops.size(); ++k) {
            const DevOp &d = h.dev_ops[k];
            if (k) o << ",";
            o << "{\"type\":" << (int)d.type << ",\"a\":" << (int)d.a << ",\"b\":" << (int)d.b
              << ",\"la\":" << (int)d.la << ",\"lb\":" << (int)d.lb << ",\"sa\":" << (int)d.sa
              << ",\"sb\":" << (int)d.sb << ",\"m\":[";
            for (int j = 0; j < 8; ++j) o << (j ? "," : "") << (double)d.m[j];
            o << "]}";
        }
        o << "],\"phases\":[";
        for (size_t k = 0; k < h.dev_phases.size(); ++k) {
            const DevPhase &d = h.dev_phases[k];
            if (k) o << ",";
            o << "{\"reg\":[" << (int)d.reg[0] << "," << (int)d.reg[1] << "," << (int)d.reg[2]
              << "," << (int)d.reg[3] << "],\"op_begin\":" << d.op_begin
              << ",\"op_end\":" << d.op_end << "}";
        }
        o << "]}";
    }
    o << "]}";
    return o.str();
}

std::vector<TermGroup> group_terms(int n, int m, const uint64_t *x, size_t n_terms) {
    std::vector<TermGroup> groups;
    const uint64_t all = (1ull << n) - 1;
    if (n <= m) {
        TermGroup g{all, {}};
        for (size_t i = 0; i < n_terms; ++i) g.terms.push_back((uint32_t)i);
        if (n_terms) groups.push_back(g);
        return groups;
    }
    const uint64_t low = (1ull << std::min(n, 4)) - 1;
    std::vector<uint32_t> rem(n_terms);
    for (size_t i = 0; i < n_terms; ++i) rem[i] = (uint32_t)i;
    // hardest terms (most high X/Y bits) first
    std::stable_sort(rem.begin(), rem.end(), [&](uint32_t a, uint32_t b) {
        return popc64(x[a] & ~low) > popc64(x[b] & ~low);
    });
    while (!rem.empty()) {
        uint64_t L = low;
        std::vector<uint32_t> take, left;
        for (uint32_t t : rem) {
            if (popc64(L | x[t]) <= m) {
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

}  // namespace qw
