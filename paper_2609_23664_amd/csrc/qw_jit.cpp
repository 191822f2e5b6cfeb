// Generated pass kernels: source generation, hipRTC compilation, caching
// and launch. See qw_jit.h.
#include "qw_jit.h"

#include <algorithm>
#include <hip/hiprtc.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <thread>
#include <unordered_map>

#include <sys/stat.h>

namespace qw {
namespace {

// Text of qw_desc.h and qw_dev.h (written into the build folder by the
// package build step), handed to hipRTC as named headers.
#include "qw_embed.inc"

// Options of every generated kernel: the flags of the ahead-of-time build.
const char *const kOpts[] = {
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
};
constexpr int kNumOpts = sizeof(kOpts) / sizeof(kOpts[0]);

// ---------------------------------------------------------------- source
struct Gen {
    std::ostringstream o;
    template <typename T>
    Gen &operator<<(const T &v) {
        o << v;
        return *this;
    }
};

std::string hex(uint64_t v) {
    char b[32];
    std::snprintf(b, sizeof b, "0x%llxull", (unsigned long long)v);
    return b;
}


// Lane part (amplitude units) and wave bit positions of an I/O layout.
void emit_io_helpers(Gen &g, const char *name, const IoRec &r, int m) {
    g << "__device__ __forceinline__ uint32_t " << name << "_lane(uint32_t lane) {\n";
    if (r.kind == IO_F4)
        g << "    return (((lane & 7u) << 1) | (((lane >> 3) & 1u) << " << (int)r.g4
          << ") | (((lane >> 4) & 1u) << " << (int)r.g5 << ") | (((lane >> 5) & 1u) << "
          << (int)r.g6 << ")) * 8u;\n";
    else
        g << "    return ((lane & 15u) | (((lane >> 4) & 1u) << " << (int)r.g4
          << ") | (((lane >> 5) & 1u) << " << (int)r.g5 << ")) * 8u;\n";
    g << "}\n";
    g << "__device__ __forceinline__ uint64_t " << name << "_wave(uint32_t w) {\n    return 0ull";
    const int nw = m - 10;
    for (int j = 0; j < nw; ++j) g << " | ((uint64_t)((w >> " << j << ") & 1u) * " << hex(r.wave_off[1u << j]) << ")";
    g << ";\n}\n";
}

// Loads of registers [k0, k1) of the first phase (k0, k1 even) into v[k - k0].
void emit_load(Gen &g, const IoRec &r, const char *name, int k0, int k1) {
    g << "__device__ __forceinline__ void " << name << "(float2 (&v)[" << std::max(1, k1 - k0)
      << "], const void *src, uint64_t ub, uint32_t lb) {\n    (void)v; (void)src; (void)ub; (void)lb;\n";
    if (r.kind == IO_F4) {
        for (int k = k0; k < k1; k += 2)
            g << "    { const float4 q = buf_ld4(src, ub + " << hex(r.reg_off[k]) << ", lb); v["
              << k - k0 << "] = make_float2(q.x, q.y); v[" << k + 1 - k0
              << "] = make_float2(q.z, q.w); }\n";
    } else {
        for (int k = k0; k < k1; ++k)
            g << "    v[" << k - k0 << "] = buf_ld2(src, ub + " << hex(r.reg_off[k]) << ", lb);\n";
    }
    g << "}\n";
}

// Store of the last phase. `ub` is the tile's output base with the wave
// part; with output relabelling a register's non-local xor term is applied
// to it before its local offset is added (the two never share bits).
void emit_store(Gen &g, const IoRec &r, bool remap, int m) {
    auto idx = [&](int k) {
        std::string e = "ub";
        if (remap && r.reg_xor[k]) e = "(ub ^ " + hex(r.reg_xor[k]) + ")";
        return e + " + " + hex(r.reg_off[k]);
    };
    g << "__device__ __forceinline__ void store_out(const float2 (&v)[16], void *dst, uint64_t ub, "
         "uint32_t lb) {\n";
    if (r.kind == IO_F4) {
        for (int k2 = 0; k2 < 8; ++k2)
            g << "    buf_st4(dst, " << idx(2 * k2) << ", lb, v[" << 2 * k2 << "], v[" << 2 * k2 + 1
              << "]);\n";
    } else {
        for (int k = 0; k < 16; ++k)
            g << "    buf_st2(dst, " << idx(k) << ", lb, v[" << k << "]);\n";
    }
    g << "}\n";
    // per-wave xor term of the output relabelling
    g << "__device__ __forceinline__ uint64_t io_out_wxor(uint32_t w) {\n    (void)w;\n    return 0ull";
    if (remap)
        for (int j = 0; j < m - 10; ++j)
            if (r.wave_xor[1u << j])
                g << " ^ ((uint64_t)((w >> " << j << ") & 1u) * " << hex(r.wave_xor[1u << j]) << ")";
    g << ";\n}\n";
}

// Value of a thread or global operand bit in phase ph.
std::string bitval(uint8_t loc, uint8_t bit, size_t ph) {
    std::ostringstream s;
    if (loc == LOC_THREAD)
        s << "(((tl" << ph << " >> " << (int)bit << ") & 1u) != 0u)";
    else
        s << "(((base >> " << (int)bit << ") & 1ull) != 0ull)";
    return s.str();
}

// Parity of the thread/global part of a parity member in phase ph.
// Parity of the thread and global part of a parity factor (the boolean of
// pdiag_tg). A thread mask of one bit, or of two adjacent bits (the parities
// a CNOT ladder leaves), is read as one bit of tl or of tl ^ (tl >> 1).
std::string pbit(const DevOp &mm, size_t ph) {
    std::ostringstream s;
    s << "((0u";
    const uint32_t t = mm.tmask;
    const int lo = t ? __builtin_ctz(t) : 0;
    if (t && (t & (t - 1)) == 0)
        s << " ^ (tl" << ph << " >> " << lo << ")";
    else if (t && t == (3u << lo))
        s << " ^ ((tl" << ph << " ^ (tl" << ph << " >> 1)) >> " << lo << ")";
    else if (t)
        s << " ^ (uint32_t)__popc(tl" << ph << " & " << t << "u)";
    if (mm.gmask) s << " ^ (uint32_t)__popcll(base & " << hex(mm.gmask) << ")";
    s << ") & 1u) != 0u";
    return s.str();
}

// The same parity as an all-ones / zero mask (for dset_fold_m): one signed
// bit-field extract for the one- and two-adjacent-bit thread masks.
std::string pmask(const DevOp &mm, size_t ph) {
    std::ostringstream s;
    const uint32_t t = mm.tmask;
    const int lo = t ? __builtin_ctz(t) : 0;
    std::string src;
    if (t && (t & (t - 1)) == 0)
        src = "tl" + std::to_string(ph);
    else if (t && t == (3u << lo))
        src = "(tl" + std::to_string(ph) + " ^ (tl" + std::to_string(ph) + " >> 1))";
    s << "(0u";
    if (!src.empty())
        s << " ^ (uint32_t)((int32_t)(" << src << " << " << 31 - lo << ") >> 31)";
    else if (t)
        s << " ^ (0u - ((uint32_t)__popc(tl" << ph << " & " << t << "u) & 1u))";
    if (mm.gmask) s << " ^ (0u - ((uint32_t)__popcll(base & " << hex(mm.gmask) << ") & 1u))";
    s << ")";
    return s.str();
}

std::string mr(size_t j) {  // 4 real entries of record j
    std::ostringstream s;
    s << "opm(ops, " << j << ", 0), opm(ops, " << j << ", 1), opm(ops, " << j << ", 2), opm(ops, "
      << j << ", 3)";
    return s.str();
}
std::string mc(size_t j, int n) {  // n complex entries of record j
    std::ostringstream s;
    for (int i = 0; i < n; ++i) s << (i ? ", " : "") << "opc(ops, " << j << ", " << i << ")";
    return s.str();
}

// Basic blocks of a generated body. A very long pass would be one basic
// block of tens of thousands of instructions, whose instruction selection
// and scheduling time grows faster than linearly; such passes are cut into
// blocks of kOpsPerBlock ops separated by a branch on an opaque always-true
// scalar. The cut costs register copies where the block's values merge with
// the untaken path's (about 5 % of a pass's VALU at 8-op blocks), so passes
// of up to kSplitAbove ops stay one block (at most a few seconds to compile).
constexpr int kOpsPerBlock = 32;
constexpr size_t kSplitAbove = 320;
const char *kBlockOpen = "    { uint32_t qw_g; __asm__ volatile(\"s_mov_b32 %0, 1\" : \"=s\"(qw_g)); if (qw_g) {\n";
const char *kBlockClose = "    } }\n";

// Diagonal sets of a pass whose thread members carry no non-local bits:
// their folded per-thread factor depends only on the thread and the op
// records, so a workgroup computes it once per descriptor (dset_factors)
// instead of on every tile, with the same sequence of operations. Maps the
// set's op index to its slot in the factor array; `phase` holds each slot's
// phase.
struct Hoisted {
    std::map<size_t, int> slot;
    std::vector<size_t> op, phase;
};

Hoisted hoisted_sets(const HostPass &p) {
    Hoisted h;
    const auto &ops = p.dev_ops;
    for (size_t k = 0; k < p.dev_phases.size(); ++k) {
        for (size_t j = p.dev_phases[k].op_begin; j < p.dev_phases[k].op_end;) {
            const DevOp &o = ops[j];
            if (o.type != OP_DSET) {
                ++j;
                continue;
            }
            const size_t m0 = j + 1 + o.sb;
            bool ok = o.b > 0;
            for (size_t q = 0; q < o.b && ok; ++q) ok = ops[m0 + q].gmask == 0;
            if (ok) {
                h.slot[j] = (int)h.op.size();
                h.op.push_back(j);
                h.phase.push_back(k);
            }
            j = m0 + o.b + o.a;
        }
    }
    return h;
}

// The fold of a diagonal set's thread members into its per-thread factor ft.
std::string emit_fold(const std::vector<DevOp> &ops, size_t j, size_t ph, const char *ind) {
    std::ostringstream g;
    const DevOp &o = ops[j];
    const size_t m0 = j + 1 + o.sb;
    g << ind << "float2 ft = make_float2(1.0f, 0.0f); (void)ft;\n";
    for (size_t q = 0; q < o.b; ++q) {
        const DevOp &mm = ops[m0 + q];
        g << ind << "ft = dset_fold_m(ft, " << pmask(mm, ph) << ", " << mc(m0 + q, 2) << ");\n";
    }
    return g.str();
}

// CNOTs of a phase with a register target and a thread or non-local
// control that every later op of the phase commutes with. Each is a
// conditional swap of the register pairs of its target slot (4 selects per
// pair); the exchange after the phase applies it instead as a per-thread
// flip of the write addresses (one select for the exchange): writing v[r]
// where register r ^ e_S would go is the swap. An op commutes with it if it
// is a CNOT with a register target whose control is not the slot, a one-bit
// op on another register slot, a diagonal on a thread or non-local bit, or a
// CZ off the slot.
// With `before`, the CNOTs that every earlier op of the phase commutes
// with: the exchange into the phase applies them to its read addresses.
std::vector<size_t> folded_cx(const std::vector<DevOp> &ops, size_t b, size_t e, bool before,
                              const std::vector<size_t> &taken = {}) {
    std::vector<size_t> top, out;
    for (size_t j = b; j < e;) {
        top.push_back(j);
        j = ops[j].type == OP_DSET ? j + 1 + ops[j].sb + ops[j].b + ops[j].a : j + 1;
    }
    for (size_t i = 0; i < top.size(); ++i) {
        const DevOp &o = ops[top[i]];
        if (o.type != OP_CX || o.la != LOC_REG || o.lb == LOC_REG) continue;
        if (std::find(taken.begin(), taken.end(), top[i]) != taken.end()) continue;
        const int S = o.sa;
        bool ok = true;
        const size_t i_lo = before ? 0 : i + 1, i_hi = before ? i : top.size();
        for (size_t i2 = i_lo; i2 < i_hi && ok; ++i2) {
            const DevOp &q = ops[top[i2]];
            if (before && std::find(out.begin(), out.end(), top[i2]) != out.end()) continue;
            const bool a_on = q.la == LOC_REG && q.sa == S;
            const bool b_on = q.lb == LOC_REG && q.sb == S;
            switch (q.type) {
            case OP_CX: ok = q.la == LOC_REG && !b_on; break;
            case OP_URT: case OP_UR: case OP_U: case OP_PERM: case OP_URD: ok = q.la == LOC_REG && !a_on; break;
            case OP_DIAG: ok = !a_on && q.la != LOC_LANE; break;
            case OP_CZ: ok = !a_on && !b_on && q.la != LOC_LANE && q.lb != LOC_LANE; break;
            default: ok = false; break;
            }
        }
        if (ok) out.push_back(top[i]);
    }
    return out;
}

// Straight-line code of ops [b, e) of a pass in phase ph (`split`: cut into
// opaque blocks; `hoist`: diagonal sets whose factor is read from ftc;
// `skip`: CNOTs the next exchange applies).
std::string emit_ops(const std::vector<DevOp> &ops, size_t b, size_t e, size_t ph, bool split,
                     const Hoisted *hoist = nullptr, const std::vector<size_t> *skip = nullptr) {
    std::ostringstream g;
    int in_block = 0;
    for (size_t j = b; j < e;) {
        const DevOp &o = ops[j];
        if (skip && std::find(skip->begin(), skip->end(), j) != skip->end()) {
            ++j;
            continue;
        }
        if (split && in_block == kOpsPerBlock) {
            g << kBlockClose;
            in_block = 0;
        }
        if (split && in_block == 0) g << kBlockOpen;
        ++in_block;
        const bool lane = o.la == LOC_LANE;
        switch (o.type) {
        case OP_URT:
            if (lane)
                g << "    urt_l<" << (int)o.sa << ", " << (int)o.b << ">(v, opm(ops, " << j << ", 0), lane);\n";
            else
                g << "    urt_r<" << (int)o.sa << ", " << (int)o.b << ">(v, opm(ops, " << j << ", 0));\n";
            ++j;
            break;
        case OP_UR:
            if (lane) g << "    ur_l<" << (int)o.sa << ">(v, " << mr(j) << ", lane);\n";
            else g << "    ur_r<" << (int)o.sa << ">(v, " << mr(j) << ");\n";
            ++j;
            break;
        case OP_URD:
            g << "    { const Urd e = urd_entries(ops, " << j << "); ";
            if (lane) g << "ur_l<" << (int)o.sa << ">(v, e.a, e.b, e.c, e.d, lane); }\n";
            else g << "ur_r<" << (int)o.sa << ">(v, e.a, e.b, e.c, e.d); }\n";
            ++j;
            break;
        case OP_U:
            if (lane) g << "    u_l<" << (int)o.sa << ">(v, " << mc(j, 4) << ", lane);\n";
            else g << "    u_r<" << (int)o.sa << ">(v, " << mc(j, 4) << ");\n";
            ++j;
            break;
        case OP_PERM:
            if (lane) g << "    perm_l<" << (int)o.sa << ">(v, " << mc(j, 2) << ", lane);\n";
            else g << "    perm_r<" << (int)o.sa << ">(v, " << mc(j, 2) << ");\n";
            ++j;
            break;
        case OP_CX:
            if (lane) {
                if (o.lb == LOC_REG) g << "    cx_lr<" << (int)o.sa << ", " << (int)o.sb << ">(v);\n";
                else g << "    cx_lb<" << (int)o.sa << ">(v, " << bitval(o.lb, o.b, ph) << ");\n";
            } else {
                if (o.lb == LOC_REG) g << "    cx_rr<" << (int)o.sa << ", " << (int)o.sb << ">(v);\n";
                else g << "    cx_rb<" << (int)o.sa << ">(v, " << bitval(o.lb, o.b, ph) << ");\n";
            }
            ++j;
            break;
        case OP_DIAG:
            if (o.la == LOC_REG) g << "    diag_r<" << (int)o.sa << ">(v, " << mc(j, 2) << ");\n";
            else g << "    diag_b(v, " << bitval(o.la, o.a, ph) << ", " << mc(j, 2) << ");\n";
            ++j;
            break;
        case OP_CZ:
            if (o.la == LOC_REG && o.lb == LOC_REG)
                g << "    cz_rr<" << (int)o.sa << ", " << (int)o.sb << ">(v);\n";
            else if (o.la == LOC_REG)
                g << "    cz_rb<" << (int)o.sa << ">(v, " << bitval(o.lb, o.b, ph) << ");\n";
            else if (o.lb == LOC_REG)
                g << "    cz_rb<" << (int)o.sb << ">(v, " << bitval(o.la, o.a, ph) << ");\n";
            else
                g << "    cz_bb(v, " << bitval(o.la, o.a, ph) << " && " << bitval(o.lb, o.b, ph)
                  << ");\n";
            ++j;
            break;
        case OP_DSET: {
            const size_t m0 = j + 1 + o.sb;
            g << "    {\n";
            if (hoist && hoist->slot.count(j))
                g << "        const float2 ft = ftc[" << hoist->slot.at(j) << "];\n";
            else
                g << emit_fold(ops, j, ph, "        ");
            // with a table or thread members, the first mixed member is
            // merged into the application (the interpreted kernels do the same)
            const size_t merged = (o.a && (o.sb || o.b)) ? 1 : 0;
            if (merged) {
                const DevOp &mm = ops[m0 + o.b];
                g << "        dset_apply_m(v, " << (o.sb ? "ops + " + std::to_string(j + 1) : std::string("ops"))
                  << ", " << (o.sb ? "true" : "false") << ", ft, " << pbit(mm, ph) << ", "
                  << mc(m0 + o.b, 2) << ", " << (int)mm.rmask << "u);\n";
            } else if (o.sb) {
                g << "        dset_apply(v, ops + " << j + 1 << ", true, ft, " << (o.b ? "true" : "false")
                  << ");\n";
            } else if (o.b) {
                g << "        dset_apply(v, ops, false, ft, true);\n";
            }
            for (size_t q = merged; q < o.a; ++q) {
                const DevOp &mm = ops[m0 + o.b + q];
                g << "        pdiag_mixed_c<" << (int)mm.rmask << ">(v, " << pbit(mm, ph) << ", "
                  << mc(m0 + o.b + q, 2) << ");\n";
            }
            g << "    }\n";
            j = m0 + o.b + o.a;
            break;
        }
        default:
            ++j;
            break;
        }
    }
    if (split && in_block) g << kBlockClose;
    return g.str();
}

// Local bits of a phase that select the wave (above the register and lane bits).
uint32_t wave_bits(int m, const DevPhase &f) {
    uint32_t R = 0, w = 0;
    for (int s = 0; s < 4; ++s) R |= 1u << f.reg[s];
    int lanes = 0;
    for (int b = 0; b < m; ++b) {
        if ((R >> b) & 1u) continue;
        if (lanes < 6) {
            ++lanes;
            continue;
        }
        w |= 1u << b;
    }
    return w;
}

// LDS address map of one exchange: element l is stored at l ^ T(l) with
// T(l) = XOR of terms ((l >> s) & mask), s >= 1 and mask within the low 5
// bits. Every term moves a bit to a lower position, so the map is bijective
// (triangular), and it keeps every bit >= 5: wave bits (all >= 6) are kept
// and wave-local exchanges stay race-free. T is chosen so that the 64-bit
// accesses of both layouts of the exchange spread over the banks: the first
// 5 (and the first 4) lane bits of each layout map to independent bank bits
// (the low 5, and the low 4, bits of the address).
struct ExSwz {
    std::vector<std::pair<int, uint32_t>> terms;
    uint32_t apply(uint32_t l) const {
        uint32_t t = 0;
        for (const auto &x : terms) t ^= (l >> x.first) & x.second;
        return l ^ t;
    }
};

int gf2_rank(std::vector<uint32_t> v) {
    int r = 0;
    for (int bit = 4; bit >= 0; --bit) {
        size_t piv = v.size();
        for (size_t i = (size_t)r; i < v.size(); ++i)
            if ((v[i] >> bit) & 1u) {
                piv = i;
                break;
            }
        if (piv == v.size()) continue;
        std::swap(v[(size_t)r], v[piv]);
        for (size_t i = 0; i < v.size(); ++i)
            if (i != (size_t)r && ((v[i] >> bit) & 1u)) v[i] ^= v[(size_t)r];
        ++r;
    }
    return r;
}

std::vector<int> lane_list(int m, const uint8_t *reg) {
    uint32_t R = 0;
    for (int s = 0; s < 4; ++s) R |= 1u << reg[s];
    std::vector<int> lanes;
    for (int b = 0; b < m && lanes.size() < 6; ++b)
        if (!((R >> b) & 1u)) lanes.push_back(b);
    return lanes;
}

// The kernels' fixed swizzle in this form: bits 5..9 and 10..13 folded
// onto bits 0..4.
ExSwz fixed_swizzle() {
    ExSwz d;
    d.terms = {{5, 31u}, {10, 31u}};
    return d;
}

// A map for which every layout in `regs` (register slots of each layout
// that writes or reads the LDS copy) spreads its accesses over the banks;
// `found` (optional) tells whether one was found (else the fixed map).
ExSwz choose_swizzle_for(int m, const std::vector<const uint8_t *> &regs, bool *found = nullptr) {
    std::vector<std::vector<int>> lanes;
    for (const uint8_t *r : regs) lanes.push_back(lane_list(m, r));
    auto good = [&](const ExSwz &x) {
        for (const std::vector<int> &ln : lanes) {
            std::vector<uint32_t> v5, v4;
            for (size_t j = 0; j < 5; ++j) {
                const uint32_t bank = x.apply(1u << ln[j]) & 31u;
                v5.push_back(bank);
                if (j < 4) v4.push_back(bank & 15u);
            }
            if (gf2_rank(v5) < 5 || gf2_rank(v4) < 4) return false;
        }
        return true;
    };
    if (found) *found = true;
    const ExSwz d = fixed_swizzle();
    if (good(d)) return d;
    std::vector<std::pair<int, uint32_t>> cands;
    for (int sh = 1; sh < m; ++sh)
        for (uint32_t mk = 1; mk < 32; ++mk) cands.push_back({sh, mk});
    ExSwz x;
    for (const auto &c : cands) {
        x.terms = {c};
        if (good(x)) return x;
    }
    for (size_t i = 0; i < cands.size(); ++i)
        for (size_t j = i + 1; j < cands.size(); ++j) {
            x.terms = {cands[i], cands[j]};
            if (good(x)) return x;
        }
    if (found) *found = false;
    return d;
}

ExSwz choose_swizzle(int m, const DevPhase &a, const DevPhase &b) {
    return choose_swizzle_for(m, {a.reg, b.reg});
}

// Address expression (bytes) of thread-local index t under map x.
std::string swz_addr(const ExSwz &x, const std::string &t) {
    std::ostringstream e;
    e << "((" << t << " ^ (0u";
    for (const auto &tm : x.terms) e << " ^ ((" << t << " >> " << tm.first << ") & " << tm.second << "u)";
    e << ")) << 3)";
    return e.str();
}

bool same_reg(const DevPhase &a, const DevPhase &b) { return std::equal(a.reg, a.reg + 4, b.reg); }

// Local offset of register k of a layout.
uint32_t reg_off(const uint8_t *reg, int k) {
    uint32_t l = 0;
    for (int s2 = 0; s2 < 4; ++s2)
        if ((k >> s2) & 1) l |= 1u << reg[s2];
    return l;
}

// `in_place_first`: the tile's first exchange may also skip the barrier
// before its writes (see below).
std::string emit_body(int m, const HostPass &p, const Hoisted &hs, bool in_place_first) {
    std::ostringstream g;
    g << "__device__ __forceinline__ void body(float2 (&v)[16], const DevOp *__restrict__ ops, "
         "uint32_t tid, uint32_t lane, uint64_t base, char *lb, const float2 *ftc) {\n";
    g << "    (void)lane; (void)base; (void)lb; (void)ftc;\n";
    const auto &ph = p.dev_phases;
    // A phase's thread index (and the LDS addresses derived from it) is
    // computed when the phase starts, from a copy of tid that the compiler
    // must treat as new: otherwise it hoists the index arithmetic of every
    // phase out of the persistent tile loop and keeps it in VGPRs, which
    // pushes the prefetched tile into scratch.
    auto tl_def = [&](size_t k) {
        std::ostringstream t;
        t << "    uint32_t tid" << k << " = tid; __asm__ volatile(\"\" : \"+v\"(tid" << k << "));\n"
          << "    const uint32_t tl" << k << " = thread_local_index(tid" << k << ", " << (int)ph[k].reg[0] << "u, "
          << (int)ph[k].reg[1] << "u, " << (int)ph[k].reg[2] << "u, " << (int)ph[k].reg[3] << "u); (void)tl"
          << k << ";\n";
        return t.str();
    };
    g << tl_def(0);
    // One LDS map for all layouts of the pass, when one spreads them all
    // over the banks: a thread then writes each exchange's values to the
    // addresses it read them from in the exchange before (the same local
    // indices under the same map), which no other thread reads, so a full
    // exchange after the tile's first one needs only the barrier between
    // its writes and its reads, and early waves write while late ones still
    // compute. The tile's first exchange is in the same position when the
    // pass starts and ends in one layout and nothing else uses the LDS
    // between tiles (`in_place_first`): the previous tile's last reads were
    // then at the same addresses, by the same threads.
    std::vector<const uint8_t *> lays;
    for (const DevPhase &f : ph) lays.push_back(f.reg);
    bool one_map = false;
    const ExSwz xall = choose_swizzle_for(m, lays, &one_map);
    auto roff = [&](const DevPhase &f, int r) {
        uint32_t l = 0;
        for (int s2 = 0; s2 < 4; ++s2)
            if ((r >> s2) & 1) l |= 1u << f.reg[s2];
        return l;
    };
    // CNOTs applied by the exchange into their phase (in) or out of it (out)
    std::vector<std::vector<size_t>> fold_in(ph.size()), fold(ph.size()), skip(ph.size());
    for (size_t k = 0; k < ph.size(); ++k) {
        if (k > 0) fold_in[k] = folded_cx(p.dev_ops, ph[k].op_begin, ph[k].op_end, true);
        if (k + 1 < ph.size()) fold[k] = folded_cx(p.dev_ops, ph[k].op_begin, ph[k].op_end, false, fold_in[k]);
        skip[k] = fold_in[k];
        skip[k].insert(skip[k].end(), fold[k].begin(), fold[k].end());
    }
    for (size_t k = 0; k < ph.size(); ++k) {
        if (k > 0) g << tl_def(k);
        if (k > 0) {
            // an exchange between layouts with the same wave bits moves data
            // only within each wave (the first exchange of a tile stays a
            // full one: the previous tile's reads may still be in flight)
            const bool local = k > 1 && wave_bits(m, ph[k - 1]) == wave_bits(m, ph[k]);
            const ExSwz x = one_map ? xall : choose_swizzle(m, ph[k - 1], ph[k]);
            auto thread_addr = [&](const std::string &t) { return swz_addr(x, t); };
            g << "    {   // exchange " << k - 1 << " -> " << k << (local ? " (within waves)" : "") << "\n";
            g << "        const uint32_t s8 = " << thread_addr("tl" + std::to_string(k - 1));
            for (size_t j : fold[k - 1]) {
                const DevOp &o = p.dev_ops[j];
                g << " ^ ((0u - (uint32_t)" << bitval(o.lb, o.b, k - 1) << ") & "
                  << (x.apply(1u << ph[k - 1].reg[o.sa]) << 3) << "u)";
            }
            g << ";\n";
            if (local)
                g << "        lds_wave_sync();\n";
            else if (!one_map || (k == 1 && !(in_place_first && same_reg(ph[0], ph.back()))))
                g << "        lds_barrier();\n";
            for (int r = 0; r < 16; ++r)
                g << "        *reinterpret_cast<float2 *>(lb + (s8 ^ " << (x.apply(roff(ph[k - 1], r)) << 3)
                  << "u)) = v[" << r << "];\n";
            g << (local ? "        lds_wave_sync();\n" : "        lds_barrier();\n");
            g << "        const uint32_t t8 = " << thread_addr("tl" + std::to_string(k));
            for (size_t j : fold_in[k]) {
                const DevOp &o = p.dev_ops[j];
                g << " ^ ((0u - (uint32_t)" << bitval(o.lb, o.b, k) << ") & "
                  << (x.apply(1u << ph[k].reg[o.sa]) << 3) << "u)";
            }
            g << ";\n";
            for (int r = 0; r < 16; ++r)
                g << "        v[" << r << "] = *reinterpret_cast<const float2 *>(lb + (t8 ^ "
                  << (x.apply(roff(ph[k], r)) << 3) << "u));\n";
            g << "    }\n";
        }
        g << "    // phase " << k << ": registers " << (int)ph[k].reg[0] << "," << (int)ph[k].reg[1] << ","
          << (int)ph[k].reg[2] << "," << (int)ph[k].reg[3] << "\n";
        g << emit_ops(p.dev_ops, ph[k].op_begin, ph[k].op_end, k, p.dev_ops.size() > kSplitAbove, &hs,
                      &skip[k]);
    }
    g << "}\n";
    // the hoisted per-thread factors, from each set's phase layout
    g << "__device__ __forceinline__ void dset_factors(float2 *ftc, const DevOp *__restrict__ ops, "
         "uint32_t tid) {\n    (void)ftc; (void)ops; (void)tid;\n";
    for (size_t i = 0; i < hs.op.size(); ++i) {
        const size_t k = hs.phase[i];
        g << "    {\n        uint32_t tid" << k << " = tid; __asm__ volatile(\"\" : \"+v\"(tid" << k << "));\n"
          << "        const uint32_t tl" << k << " = thread_local_index(tid" << k << ", " << (int)ph[k].reg[0]
          << "u, " << (int)ph[k].reg[1] << "u, " << (int)ph[k].reg[2] << "u, " << (int)ph[k].reg[3] << "u);\n"
          << emit_fold(p.dev_ops, hs.op[i], k, "        ") << "        ftc[" << i << "] = ft;\n    }\n";
    }
    g << "}\n";
    (void)m;
    return g.str();
}

const char *kScaleIn =
    "    {\n"
    "        const double s = *gin<double>(ldu(&d->scale_in));\n"
    "        #pragma unroll\n"
    "        for (int k = 0; k < 16; ++k)\n"
    "            v[k] = make_float2((float)((double)v[k].x * s), (float)((double)v[k].y * s));\n"
    "    }\n";

}  // namespace

std::string jit_pass_key(int n, int m, const HostPass &p, bool use_lds) {
    std::string k;
    k.reserve(64 + 8 * p.dev_ops.size() + 12 * p.dev_phases.size());
    auto put = [&](uint64_t v, int bytes) {
        for (int i = 0; i < bytes; ++i) k.push_back((char)((v >> (8 * i)) & 0xFF));
    };
    put((uint64_t)n, 1);
    put((uint64_t)m, 1);
    put(use_lds ? 1 : 0, 1);
    put((p.scale_in ? 1 : 0) | (p.norm_out ? 2 : 0) | (p.moves() ? 4 : 0), 1);
    put(p.local_mask, 8);
    // index layouts of the load and the store (their bit positions are
    // compiled into the address arithmetic)
    put(p.in_pos.size(), 1);
    for (uint8_t b : p.in_pos) put(b, 1);
    put(p.out_pos.size(), 1);
    for (uint8_t b : p.out_pos) put(b, 1);
    if (!p.out_img.empty()) {
        // the local-bit part of the relabelling is compiled in; its tile
        // part comes from the per-tile output bases
        for (int k = 0; k < 16; ++k) put(p.io_out.reg_xor[k], 4);
        for (int w = 0; w < 16; ++w) put(p.io_out.wave_xor[w], 4);
    }
    put(p.dev_phases.size(), 2);
    for (const DevPhase &f : p.dev_phases) {
        for (int s = 0; s < 4; ++s) put(f.reg[s], 1);
        put(f.io, 1);
        put(f.op_begin, 2);
        put(f.op_end, 2);
    }
    put(p.dev_ops.size(), 2);
    for (const DevOp &o : p.dev_ops) {
        put(o.type, 1);
        put(o.a, 1);
        put(o.b, 1);
        put(o.sa, 1);
        put(o.sb, 1);
        put(o.la, 1);
        put(o.lb, 1);
        if (o.type == OP_PDIAG) {
            put(o.rmask, 1);
            put(o.tmask, 4);
            put(o.gmask, 4);
        }
    }
    return k;
}

static void emit_reduce_tile(std::ostringstream &o, int m, const RedPlan &rp, const DevPhase *stage,
                             const char *name);

std::string jit_epilogue_key(int n, int m, const HostPass &p, const RedPlan &epi) {
    TermGroup g{p.local_mask, {}};
    return "E" + jit_reduce_key(n, m, g, epi);
}

// Definitions of one pass structure, shared by its own kernel and by the
// persistent kernel of a call: I/O address helpers, the loads (all 16
// registers; the first `PF` of a tile ahead; the rest), the store, the body
// and, with an epilogue, its term evaluation. Returns the number of hoisted
// diagonal sets (the size of the per-thread factor array).
static size_t emit_pass_defs(Gen &g, int n, int m, const HostPass &p, bool use_lds, int PF,
                             const RedPlan *epi) {
    emit_io_helpers(g, "io_in", p.io_in, m);
    emit_io_helpers(g, "io_out", p.io_out, m);
    emit_load(g, p.io_in, "load_in", 0, 16);
    emit_load(g, p.io_in, "load_pre", 0, PF);
    emit_load(g, p.io_in, "load_rest", PF, 16);
    emit_store(g, p.io_out, p.moves(), m);
    const Hoisted hs = hoisted_sets(p);
    g << emit_body(m, p, hs, use_lds && !epi);
    if (epi) {
        // fused expectation epilogue: the tile's terms, evaluated after the
        // store from the last phase's registers (staged through LDS)
        std::ostringstream e;
        e << "constexpr int ENT = " << epi->cols.size() << ";\n";
        // items are (descriptor, row of RT consecutive tiles), run in order
        e << "constexpr uint32_t RT = " << red_row_tiles(1u << (n - m)) << "u;\n";
        emit_reduce_tile(e, m, *epi, &p.dev_phases.back(), "epi_tile");
        e << "__device__ const uint32_t kECols[ENT] = {";
        for (size_t c = 0; c < epi->cols.size(); ++c) e << (c ? ", " : "") << epi->cols[c] << "u";
        e << "};\n";
        g << e.str();
    }
    return hs.op.size();
}

std::string jit_pass_source(int n, int m, const HostPass &p, bool use_lds, int prefetch,
                            const RedPlan *epi, bool stream_loads) {
    Gen g;
    const int T = 1 << (m - 4);
    const int WG = T < 256 ? T : 256;
    g << "// generated pass kernel: " << n << " qubits, tile bits " << m << ", " << p.dev_ops.size()
      << " op records, " << p.dev_phases.size() << " phases, "
      << (use_lds ? "persistent LDS form" : "flat form") << "\n";
    g << "#define QW_ST_AUX 2\n";
    if (stream_loads) g << "#define QW_LD_AUX 2\n";
    g << "#include \"qw_dev.h\"\nusing namespace qw;\n";
    g << "constexpr int M = " << m << ", T = " << T << ", WG = " << WG << ", PARTS = T / WG;\n";
    const bool remap = p.moves();
    // persistent form: registers [0, PF) of the next tile are loaded while
    // the current one is worked on, the rest when it starts
    const int PF = use_lds ? prefetch : 0;
    // output base of the tile: the relabelled one, or the load base
    const char *obase = remap ? "uni(ldu(ldu(&d->tile_base_out) + tile))" : "base";
    const size_t K = emit_pass_defs(g, n, m, p, use_lds, PF, epi);
    if (!use_lds) {
        g << "extern \"C\" __global__ __launch_bounds__(WG) void qw_pass(const PassDesc *__restrict__ "
             "descs, uint32_t n_descs, uint32_t items, int remap, uint32_t tmaj) {\n"
             "    (void)tmaj;\n"
             "    const uint32_t wg_item = item_of(blockIdx.x, gridDim.x, remap);\n"
             "    const uint32_t item = wg_item / PARTS;\n"
             "    if (item >= items) return;\n"
             "    const uint32_t part = wg_item % PARTS;\n"
             "    const uint32_t p = item % n_descs, tile = item / n_descs;\n"
             "    const PassDesc *d = descs + p;\n"
             "    const uint64_t base = uni(ldu(ldu(&d->tile_base) + tile));\n"
             "    const uint32_t tid = part * WG + threadIdx.x;\n"
             "    const uint32_t lane = threadIdx.x & 63u;\n"
             "    const uint32_t wave = uni(tid >> 6);\n"
             "    float2 v[16];\n"
             "    load_in(v, ldu(&d->src), base | io_in_wave(wave), io_in_lane(lane));\n";
        if (p.scale_in) g << kScaleIn;
        g << "    float2 ftc[" << std::max<size_t>(1, K) << "];\n";
        if (K) g << "    dset_factors(ftc, ldu(&d->ops), tid);\n";
        g << "    body(v, ldu(&d->ops), tid, lane, base, nullptr, ftc);\n"
             "    store_out(v, ldu(&d->dst), ((uint64_t)" << obase << " ^ io_out_wxor(wave)) | io_out_wave(wave), io_out_lane(lane));\n"
             "}\n";
    } else {
        g << "extern \"C\" __global__ __launch_bounds__(T) void qw_pass(const PassDesc *__restrict__ "
             "descs, uint32_t n_descs, uint32_t items, int remap, uint32_t tmaj) {\n"
             "    (void)remap;\n"
             "    // item -> (descriptor, tile" << (epi ? " row" : "") << "): tmaj = 0 descriptor-fastest, else\n"
             "    // tile-fastest with 1 << (tmaj - 1) items per descriptor\n"
             "    const uint32_t tg = tmaj ? tmaj - 1u : 0u;\n"
             "    auto desc_of = [=](uint32_t it) { return tmaj ? (it >> tg) : (it % n_descs); };\n"
             "    auto tile_of = [=](uint32_t it) { return tmaj ? (it & ((1u << tg) - 1u)) : (it / n_descs); };\n"
             "    __shared__ float2 lds[1 << M];\n"
             "    __shared__ double red[" << (epi ? "(T / 64) * ENT + 1" : "T / 64 + 1") << "];\n"
             "    (void)red;\n"
             "    const uint32_t w = blockIdx.x, x = w & 7u, j = w >> 3, wpx = gridDim.x >> 3;\n"
             "    const uint32_t per = (items + 7u) >> 3;\n"
             "    const uint32_t first = x * per;\n"
             "    const uint32_t last = (first + per < items) ? first + per : items;\n"
             "    uint32_t item = first + j;\n"
             "    if (item >= last) return;\n"
             "    // this workgroup's items are first + j + wpx k (k < K); descriptor-\n"
             "    // fastest, their descriptor repeats with period P in k, and they\n"
             "    // run as the P sequences k = r, r + P, r + 2 P, ... so that one\n"
             "    // descriptor's items run back to back\n"
             "    const uint32_t K = (last - item + wpx - 1u) / wpx;\n"
             "    uint32_t P = 1u;\n"
             "    if (!tmaj) {\n"
             "        uint32_t a = wpx, b = n_descs;\n"
             "        while (b) {\n"
             "            const uint32_t t = a % b;\n"
             "            a = b;\n"
             "            b = t;\n"
             "        }\n"
             "        P = n_descs / a;\n"
             "    }\n"
             "    uint32_t rr = 0u, kk = 0u;\n"
             "    auto advance = [&](uint32_t &r_, uint32_t &k_) {\n"
             "        k_ += P;\n"
             "        if (k_ >= K) {\n"
             "            r_ += 1u;\n"
             "            k_ = r_;\n"
             "        }\n"
             "        return r_ < P && k_ < K;\n"
             "    };\n"
             "    const uint32_t tid = threadIdx.x;\n"
             "    const uint32_t lane = tid & 63u;\n"
             "    const uint32_t wave = uni(tid >> 6);\n"
             "    const uint64_t wi = io_in_wave(wave), wo = io_out_wave(wave), wx = io_out_wxor(wave);\n"
             "    const uint32_t li = io_in_lane(lane), lo = io_out_lane(lane);\n"
             "    char *lb = reinterpret_cast<char *>(lds);\n"
             "    float2 ftc[" << std::max<size_t>(1, K) << "];   // per-thread factors of the hoisted diagonal sets\n"
             "    uint32_t ft_desc = 0xFFFFFFFFu;   // descriptor they were computed for\n"
             "    (void)ft_desc;\n";
        if (epi)
            g << "    uint32_t rk = 0;   // tile of the row\n"
                 "    float acc[ENT];\n"
                 "    #pragma unroll\n"
                 "    for (int i = 0; i < ENT; ++i) acc[i] = 0.f;\n";
        const char *tile0 = epi ? "tile_of(item) * RT" : "tile_of(item)";
        g << "    float2 nv[" << std::max(1, PF) << "];\n"
             "    {\n"
             "        const PassDesc *d0 = descs + desc_of(item);\n"
             "        load_pre(nv, ldu(&d0->src), uni(ldu(ldu(&d0->tile_base) + " << tile0 << ")) | wi, li);\n"
             "    }\n"
             "    while (true) {\n"
             "        float2 v[16];\n"
             "        #pragma unroll\n"
             "        for (int k = 0; k < " << PF << "; ++k) v[k] = nv[k];\n"
             "        const uint32_t p = desc_of(item), tile = " << (epi ? "tile_of(item) * RT + rk" : "tile_of(item)")
          << ";\n"
             "        const PassDesc *d = descs + p;\n"
             "        const uint64_t base = uni(ldu(ldu(&d->tile_base) + tile));\n"
             "        {\n"
             "            float2 rest[" << std::max(1, 16 - PF) << "];\n"
             "            load_rest(rest, ldu(&d->src), base | wi, li);\n"
             "            #pragma unroll\n"
             "            for (int k = " << PF << "; k < 16; ++k) v[k] = rest[k - " << PF << "];\n"
             "        }\n"
             "";
        if (epi)
            g << "        uint32_t next = item, nk = rk + 1u, nr = rr, nkk = kk;\n"
                 "        bool has_next = true;\n"
                 "        if (nk == RT) {\n"
                 "            nk = 0u;\n"
                 "            has_next = advance(nr, nkk);\n"
                 "            next = first + j + wpx * nkk;\n"
                 "        }\n";
        else
            g << "        uint32_t nr = rr, nkk = kk;\n"
                 "        const bool has_next = advance(nr, nkk);\n"
                 "        const uint32_t next = first + j + wpx * nkk;\n";
        g << "        if (has_next) {\n"
             "            const PassDesc *dn = descs + desc_of(next);\n"
             "            load_pre(nv, ldu(&dn->src), uni(ldu(ldu(&dn->tile_base) + "
          << (epi ? "tile_of(next) * RT + nk" : "tile_of(next)") << ")) | wi, li);\n"
             "        }\n";
        if (p.scale_in) g << kScaleIn;
        if (K)
            g << "        if (p != ft_desc) {\n"
                 "            dset_factors(ftc, ldu(&d->ops), tid);\n"
                 "            ft_desc = p;\n"
                 "        }\n";
        g << "        body(v, ldu(&d->ops), tid, lane, base, lb, ftc);\n";
        if (p.norm_out)
            g << "        {\n"
                 "            double s = 0.0;\n"
                 "            #pragma unroll\n"
                 "            for (int k = 0; k < 16; ++k) {\n"
                 "                const double xx = v[k].x, yy = v[k].y;\n"
                 "                s = fma(xx, xx, s);\n"
                 "                s = fma(yy, yy, s);\n"
                 "            }\n"
                 "            s = block_sum<T>(s, red);\n"
                 "            if (tid == 0) gout<double>(ldu(&d->norm_part))[tile] = s;\n"
                 "        }\n";
        g << "        store_out(v, ldu(&d->dst), ((uint64_t)" << obase << " ^ wx) | wo, lo);\n";
        if (epi)
            g << "        epi_tile(v, tid, lane, base, lb, acc);\n"
                 "        if (rk == RT - 1u) {\n"
                 "            epi_tile_flush(acc, lane, wave, red);\n"
                 "            __syncthreads();\n"
                 "            double *part = ldu(&d->red_part) + (uint64_t)tile_of(item) * ldu(&d->red_nt);\n"
                 "            for (uint32_t c = tid; c < (uint32_t)ENT; c += T) {\n"
                 "                double s = 0.0;\n"
                 "                for (int ww = 0; ww < T / 64; ++ww) s += red[ww * ENT + c];\n"
                 "                gout<double>(part)[kECols[c]] = s;\n"
                 "            }\n"
                 "        }\n";
        g << "        if (!has_next) break;\n"
             "        item = next;\n"
             "        rr = nr;\n"
             "        kk = nkk;\n";
        if (epi) g << "        rk = nk;\n";
        g << "    }\n"
             "}\n";
    }
    return g.o.str();
}


// ---------------------------------------------------------- persistent
std::string jit_persist_key(const std::vector<PersistPart> &parts) {
    std::string k = "P";
    for (const PersistPart &q : parts) {
        const std::string e = q.epi_key ? *q.epi_key : std::string();
        const std::string pk = jit_pass_key(q.n, q.m, *q.pass, true) + e;
        const uint32_t len = (uint32_t)pk.size();
        k.append(reinterpret_cast<const char *>(&len), sizeof len);
        k += pk;
        k.push_back(q.stream_loads ? 'S' : 'T');
    }
    return k;
}

std::string jit_persist_source(const std::vector<PersistPart> &parts, int prefetch) {
    Gen g;
    const int n = parts[0].n, m = parts[0].m;
    const int T = 1 << (m - 4);
    bool all_stream = true;
    size_t red_words = T / 64 + 1;
    for (const PersistPart &q : parts) {
        all_stream &= q.stream_loads;
        if (q.epi) red_words = std::max(red_words, (size_t)(T / 64) * q.epi->cols.size() + 1);
    }
    g << "// generated persistent kernel: " << n << " qubits, tile bits " << m << ", " << parts.size()
      << " pass structures\n";
    g << "#define QW_ST_AUX 2\n";
    if (all_stream) g << "#define QW_LD_AUX 2\n";
    g << "#include \"qw_dev.h\"\nusing namespace qw;\n";
    g << "constexpr int M = " << m << ", T = " << T << ";\n";
    g << "__shared__ float2 qw_lds[1 << M];\n__shared__ double qw_red[" << red_words << "];\n";
    const int PF = prefetch;
    for (size_t s = 0; s < parts.size(); ++s) {
        const PersistPart &q = parts[s];
        const HostPass &p = *q.pass;
        g << "namespace s" << s << " {\n";
        const size_t K = emit_pass_defs(g, n, m, p, true, PF, q.epi);
        const char *obase = p.moves() ? "uni(ldu(ldu(&d->tile_base_out) + tile))" : "base";
        // units [u0, u1) of one descriptor (tiles, or rows of RT tiles), the
        // first PF registers of each next tile loaded during the current one
        g << "__device__ __forceinline__ void run(const PassDesc *__restrict__ d, uint32_t u0, uint32_t u1) {\n"
             "    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = uni(tid >> 6);\n"
             "    const uint64_t wi = io_in_wave(wave), wo = io_out_wave(wave), wx = io_out_wxor(wave);\n"
             "    const uint32_t li = io_in_lane(lane), lo = io_out_lane(lane);\n"
             "    char *lb = reinterpret_cast<char *>(qw_lds);\n"
             "    double *red = qw_red;\n"
             "    (void)red;\n"
             "    const void *src = ldu(&d->src);\n"
             "    void *dst = ldu(&d->dst);\n"
             "    const uint32_t *tb = ldu(&d->tile_base);\n";
        if (q.epi)
            g << "    const uint32_t t0 = u0 * RT, t1 = u1 * RT;\n"
                 "    float acc[ENT];\n"
                 "    #pragma unroll\n"
                 "    for (int i = 0; i < ENT; ++i) acc[i] = 0.f;\n";
        else
            g << "    const uint32_t t0 = u0, t1 = u1;\n";
        g << "    float2 ftc[" << std::max<size_t>(1, K) << "];\n";
        if (K) g << "    dset_factors(ftc, ldu(&d->ops), tid);\n";
        g << "    float2 nv[" << std::max(1, PF) << "];\n"
             "    load_pre(nv, src, uni(ldu(tb + t0)) | wi, li);\n"
             "    for (uint32_t tile = t0; tile < t1; ++tile) {\n"
             "        float2 v[16];\n"
             "        #pragma unroll\n"
             "        for (int k = 0; k < " << PF << "; ++k) v[k] = nv[k];\n"
             "        const uint64_t base = uni(ldu(tb + tile));\n"
             "        {\n"
             "            float2 rest[" << std::max(1, 16 - PF) << "];\n"
             "            load_rest(rest, src, base | wi, li);\n"
             "            #pragma unroll\n"
             "            for (int k = " << PF << "; k < 16; ++k) v[k] = rest[k - " << PF << "];\n"
             "        }\n"
             "        if (tile + 1u < t1) load_pre(nv, src, uni(ldu(tb + tile + 1u)) | wi, li);\n";
        if (p.scale_in) g << kScaleIn;
        g << "        body(v, ldu(&d->ops), tid, lane, base, lb, ftc);\n"
             "        store_out(v, dst, ((uint64_t)" << obase << " ^ wx) | wo, lo);\n";
        if (q.epi)
            g << "        epi_tile(v, tid, lane, base, lb, acc);\n"
                 "        if ((tile + 1u) % RT == 0u) {\n"
                 "            epi_tile_flush(acc, lane, wave, red);\n"
                 "            __syncthreads();\n"
                 "            double *part = ldu(&d->red_part) + (uint64_t)(tile / RT) * ldu(&d->red_nt);\n"
                 "            for (uint32_t c = tid; c < (uint32_t)ENT; c += T) {\n"
                 "                double sum = 0.0;\n"
                 "                for (int ww = 0; ww < T / 64; ++ww) sum += red[ww * ENT + c];\n"
                 "                gout<double>(part)[kECols[c]] = sum;\n"
                 "            }\n"
                 "        }\n";
        g << "    }\n}\n}  // namespace s" << s << "\n";
    }
    // The claim loop. Claims are taken in increasing order from one counter
    // and a claim only waits for descriptors of earlier claims, so the
    // earliest unfinished claim never waits: the launch completes whether or
    // not all its workgroups are resident at once. A wait is bounded in time
    // (spin_limit microseconds of the 100 MHz real-time counter) and ends
    // early when another workgroup has abandoned the launch or the host has
    // set host_flag[0]; an abandoned launch skips all further claims and
    // sets host_flag[1].
    // Wave 0 claims, waits and releases as a whole (a branch on the wave
    // index, every lane active, one lane's value counted in each atomic):
    // no lane-divergent region may enclose or follow the workgroup barriers
    // of the loop, or the compiler may let the other lanes of wave 0 go
    // round the barriers while its claiming lane waits to run.
    g << "__device__ __forceinline__ uint32_t seg_of(const PSeg *__restrict__ segs, uint32_t n_segs, uint32_t c) {\n"
         "    uint32_t lo = 0u, hi = n_segs;\n"
         "    while (hi - lo > 1u) {\n"
         "        const uint32_t mid = (lo + hi) >> 1;\n"
         "        if (ldu(&segs[mid].claim0) <= c) lo = mid; else hi = mid;\n"
         "    }\n"
         "    return lo;\n"
         "}\n"
         "__device__ __forceinline__ void claim_desc(const PSeg *__restrict__ sg, uint32_t c, uint32_t *gi, uint32_t *u0) {\n"
         "    const uint32_t lc = c - ldu(&sg->claim0), chunk = ldu(&sg->chunk);\n"
         "    const uint32_t per = ldu(&sg->units) / chunk, nd = ldu(&sg->n_descs);\n"
         "    const uint32_t dl = ldu(&sg->tmaj) ? lc / per : lc % nd;\n"
         "    const uint32_t ul = ldu(&sg->tmaj) ? lc % per : lc / nd;\n"
         "    *gi = ldu(&sg->desc0) + dl;\n"
         "    *u0 = ul * chunk;\n"
         "}\n";
    g << "extern \"C\" __global__ __launch_bounds__(T) void qw_persist(const PSeg *__restrict__ segs, uint32_t n_segs, "
         "const PassDesc *__restrict__ descs, const PDep *__restrict__ deps, uint32_t *sync, uint32_t claims, "
         "uint32_t spin_limit, uint32_t *host_flag) {\n"
         "    __shared__ uint32_t s_claim;\n"
         "    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = uni(tid >> 6);\n"
         "    const uint32_t one = lane == 0u ? 1u : 0u;\n"
         "    uint32_t done_gi = kNoDep, done_units = 0u;   // the claim just finished (wave 0)\n"
         "    while (true) {\n"
         "        // every wave's stores of the finished claim have completed\n"
         "        __builtin_amdgcn_s_waitcnt(0);\n"
         "        __syncthreads();\n"
         "        if (wave == 0u) {\n"
         "            if (done_gi != kNoDep) {\n"
         "                __builtin_amdgcn_fence(__ATOMIC_RELEASE, \"agent\");\n"
         "                __hip_atomic_fetch_add(&sync[kSyncCounters + done_gi], one * done_units, __ATOMIC_RELAXED,\n"
         "                                       __HIP_MEMORY_SCOPE_AGENT);\n"
         "            }\n"
         "            uint32_t c = claims;\n"
         "            if (uni(__hip_atomic_load(&sync[kSyncAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0u)\n"
         "                c = uni(__hip_atomic_fetch_add(&sync[kSyncClaim], one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));\n"
         "            if (c < claims) {\n"
         "                uint32_t gi, u0;\n"
         "                claim_desc(segs + seg_of(segs, n_segs, c), c, &gi, &u0);\n"
         "                const uint32_t dep = ldu(&deps[gi].dep), need = ldu(&deps[gi].need);\n"
         "                if (dep != kNoDep) {\n"
         "                    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();\n"
         "                    const uint64_t limit = (uint64_t)spin_limit * 100ull;\n"
         "                    while (uni(__hip_atomic_load(&sync[kSyncCounters + dep], __ATOMIC_RELAXED,\n"
         "                                                 __HIP_MEMORY_SCOPE_AGENT)) < need) {\n"
         "                        const bool give_up =\n"
         "                            __builtin_amdgcn_s_memrealtime() - t0 >= limit ||\n"
         "                            uni(__hip_atomic_load(&sync[kSyncAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0u ||\n"
         "                            uni(__hip_atomic_load(&host_flag[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) != 0u;\n"
         "                        if (give_up) {\n"
         "                            __hip_atomic_fetch_or(&sync[kSyncAbort], one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);\n"
         "                            __hip_atomic_fetch_or(&host_flag[1], one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);\n"
         "                            c = claims;\n"
         "                            break;\n"
         "                        }\n"
         "                        __builtin_amdgcn_s_sleep(2);\n"
         "                    }\n"
         "                    // the producers' stores, released before their counter updates\n"
         "                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, \"agent\");\n"
         "                }\n"
         "            }\n"
         "            s_claim = c;   // the same value from every lane of wave 0\n"
         "        }\n"
         "        __syncthreads();\n"
         "        const uint32_t c = uni(s_claim);\n"
         "        if (c >= claims) break;\n"
         "        const PSeg *sg = segs + seg_of(segs, n_segs, c);\n"
         "        uint32_t gi, u0;\n"
         "        claim_desc(sg, c, &gi, &u0);\n"
         "        const uint32_t u1 = u0 + ldu(&sg->chunk);\n"
         "        switch (ldu(&sg->kind)) {\n";
    for (size_t s = 0; s < parts.size(); ++s)
        g << "        case " << s << "u: s" << s << "::run(descs + gi, u0, u1); break;\n";
    g << "        default: break;\n"
         "        }\n"
         "        done_gi = gi;\n"
         "        done_units = u1 - u0;\n"
         "    }\n"
         "}\n";
    return g.o.str();
}


// ---------------------------------------------------------------- reducer
std::string jit_reduce_key(int n, int m, const TermGroup &g, const RedPlan &rp) {
    std::string k = "R";
    auto put = [&](uint64_t v, int bytes) {
        for (int i = 0; i < bytes; ++i) k.push_back((char)((v >> (8 * i)) & 0xFF));
    };
    put((uint64_t)n, 1);
    put((uint64_t)m, 1);
    put(g.local_mask, 8);
    put(rp.phases.size(), 2);
    for (const RedPhase &f : rp.phases) {
        for (int s = 0; s < 4; ++s) put(f.reg[s], 1);
        put(f.t_begin, 2);
        put(f.t_end, 2);
        put(f.diag, 1);
    }
    put(rp.terms.size(), 2);
    for (const TermDev &t : rp.terms) {
        put(t.xr, 1);
        put(t.neg, 1);
        put(t.odd, 1);
        put(t.smask, 2);
        put(t.col, 2);
        put(t.zt, 4);
        put(t.zg, 8);
    }
    for (uint32_t c : rp.cols) put(c, 4);
    return k;
}

// Term evaluation of one tile for a reducer plan (shared by the generated
// reducers and the fused expectation epilogue of pass kernels): adds each
// term's per-thread FP32 value into acc[column]. Without `stage`, v holds
// the tile in the I/O layout (register slots = local bits 0, 7, 8, 9); with
// `stage`, v holds the tile in that phase layout (the last phase of a
// pass). A diagonal phase (the first phase, when there is one) in the layout
// v already holds is evaluated on v; the other phases read the tile from an
// LDS copy staged first. `name`_flush sums a row's accumulators over the
// wave 8 at a time in FP64 (each term's wave sum is the same butterfly
// whatever its position) into red[wave * NT + column] and clears them.
static void emit_reduce_tile(std::ostringstream &o, int m, const RedPlan &rp, const DevPhase *stage,
                             const char *name) {
    static const uint8_t io_reg[4] = {0, 7, 8, 9};
    const uint8_t *held = stage ? stage->reg : io_reg;
    std::vector<char> from_lds(rp.phases.size(), 1);
    for (size_t pi = 0; pi < rp.phases.size(); ++pi) {
        const RedPhase &f = rp.phases[pi];
        if (pi == 0 && f.diag && std::equal(f.reg, f.reg + 4, held)) from_lds[pi] = 0;
    }
    bool any_lds = false;
    for (char c : from_lds) any_lds |= c != 0;
    // one LDS address map for the writing layout and every reading phase
    std::vector<const uint8_t *> lay{held};
    for (size_t pi = 0; pi < rp.phases.size(); ++pi)
        if (from_lds[pi]) lay.push_back(rp.phases[pi].reg);
    const ExSwz x = choose_swizzle_for(m, lay);
    const size_t nt = rp.cols.size();
    o << "__device__ __forceinline__ void " << name << "(float2 (&v)[16], uint32_t tid, uint32_t lane, "
         "uint64_t base, char *lb, float (&acc)[" << nt << "]) {\n";
    o << "    (void)lb; (void)base; (void)lane;\n";
    if (stage && any_lds) {
        o << "    {\n        uint32_t tids = tid; __asm__ volatile(\"\" : \"+v\"(tids));\n"
          << "        const uint32_t tls = thread_local_index(tids, " << (int)stage->reg[0] << "u, "
          << (int)stage->reg[1] << "u, " << (int)stage->reg[2] << "u, " << (int)stage->reg[3] << "u);\n"
          << "        const uint32_t s8 = " << swz_addr(x, "tls") << ";\n"
          << "        lds_barrier();\n";
        for (int k = 0; k < 16; ++k)
            o << "        *reinterpret_cast<float2 *>(lb + (s8 ^ " << (x.apply(reg_off(stage->reg, k)) << 3)
              << "u)) = v[" << k << "];\n";
        o << "    }\n    lds_barrier();\n";
    } else if (!stage) {
        o << "    const uint32_t tlio = thread_local_index(tid, " << (int)io_reg[0] << "u, " << (int)io_reg[1] << "u, "
          << (int)io_reg[2] << "u, " << (int)io_reg[3] << "u);\n";
        if (any_lds) {
            o << "    {\n        const uint32_t s8 = " << swz_addr(x, "tlio") << ";\n";
            for (int k = 0; k < 16; ++k)
                o << "        *reinterpret_cast<float2 *>(lb + (s8 ^ " << (x.apply(reg_off(io_reg, k)) << 3)
                  << "u)) = v[" << k << "];\n";
            o << "    }\n    lds_barrier();\n";
        }
    }
    for (size_t pi = 0; pi < rp.phases.size(); ++pi) {
        const RedPhase &f = rp.phases[pi];
        o << "    {   // phase " << pi << (f.diag ? " (diagonal terms)" : "") << "\n";
        // (an opaque copy of tid keeps the index arithmetic inside the tile loop)
        o << "        uint32_t tidp = tid; __asm__ volatile(\"\" : \"+v\"(tidp));\n";
        o << "        const uint32_t tl = thread_local_index(tidp, " << (int)f.reg[0] << "u, " << (int)f.reg[1]
          << "u, " << (int)f.reg[2] << "u, " << (int)f.reg[3] << "u); (void)tl;\n";
        if (from_lds[pi]) {
            o << "        const uint32_t t8 = " << swz_addr(x, "tl") << ";\n";
            for (int k = 0; k < 16; ++k)
                o << "        v[" << k << "] = *reinterpret_cast<const float2 *>(lb + (t8 ^ "
                  << (x.apply(reg_off(f.reg, k)) << 3) << "u));\n";
        }
        if (f.diag)
            o << "        float pr[16];\n        #pragma unroll\n        for (int k = 0; k < 16; ++k) pr[k] = "
                 "fmaf(v[k].x, v[k].x, v[k].y * v[k].y);\n";
        for (uint32_t j = f.t_begin; j < f.t_end; ++j) {
            const TermDev &t = rp.terms[j];
            o << "        {\n";
            if (f.diag)
                o << "            float a = diag_sum(pr, " << t.smask << "u);\n";
            else
                o << "            float a = pair_sum<" << (int)t.xr << ", " << (t.odd ? "true" : "false")
                  << ">(v, " << t.smask << "u);\n            a *= 2.0f;\n";
            o << "            const uint32_t par = (" << (int)t.neg << "u";
            if (t.zt) o << " ^ (uint32_t)__popc(tl & " << t.zt << "u)";
            if (t.zg) o << " ^ (uint32_t)__popcll(base & " << hex(t.zg) << ")";
            o << ") & 1u;\n            if (par) a = -a;\n";
            o << "            acc[" << t.col << "] += a;\n        }\n";
        }
        o << "    }\n";
    }
    o << "}\n";
    o << "__device__ __forceinline__ void " << name << "_flush(float (&acc)[" << nt
      << "], uint32_t lane, uint32_t wave, double *red) {\n";
    for (size_t c0 = 0; c0 < nt; c0 += 8) {
        o << "    {\n        float q[8] = {";
        for (size_t i = 0; i < 8; ++i) {
            if (i) o << ", ";
            if (c0 + i < nt) o << "acc[" << c0 + i << "]";
            else o << "0.f";
        }
        o << "};\n        const double h = wave_reduce8(q, lane);\n"
          << "        const uint32_t pos = 4u * (lane & 1u) + 2u * ((lane >> 1) & 1u) + ((lane >> 2) & 1u);\n"
          << "        if (lane < 8u && pos < " << std::min<size_t>(8, nt - c0) << "u) red[wave * " << nt << " + "
          << c0 << "u + pos] = h;\n    }\n";
    }
    o << "    #pragma unroll\n    for (int i = 0; i < " << nt << "; ++i) acc[i] = 0.f;\n}\n";
}

std::string jit_reduce_source(int n, int m, const TermGroup &g, const RedPlan &rp) {
    std::ostringstream o;
    const int T = 1 << (m - 4);
    const size_t NT = rp.cols.size();
    o << "// generated expectation reducer: " << n << " qubits, tile bits " << m << ", " << NT
      << " terms, " << rp.phases.size() << " phases\n";
    o << "#define QW_LD_AUX 2\n";  // each state is swept once per term group
    o << "#include \"qw_dev.h\"\nusing namespace qw;\n";
    o << "constexpr int M = " << m << ", T = " << T << ", W = T / 64, NT = " << NT << ";\n";
    // I/O layout of the tile: register slots = local bits {0, 7, 8, 9}
    std::vector<int> gpos;
    for (int q = 0; q < 64; ++q)
        if ((g.local_mask >> q) & 1ull) gpos.push_back(q);
    auto gbit = [&](int l) { return 1ull << gpos[l]; };
    const int io_reg[4] = {0, 7, 8, 9};
    o << "__device__ __forceinline__ uint32_t io_lane(uint32_t lane) {\n"
      << "    return (((lane & 7u) << 1) | (((lane >> 3) & 1u) << " << gpos[4] << ") | (((lane >> 4) & 1u) << "
      << gpos[5] << ") | (((lane >> 5) & 1u) << " << gpos[6] << ")) * 8u;\n}\n";
    {
        // wave bits: local bits >= 10 (not registers, above the lanes 1..6)
        o << "__device__ __forceinline__ uint64_t io_wave(uint32_t w) {\n    return 0ull";
        for (int j = 0; j < m - 10; ++j) o << " | ((uint64_t)((w >> " << j << ") & 1u) * " << hex(gbit(10 + j)) << ")";
        o << ";\n}\n";
    }
    o << "__device__ __forceinline__ void load_in(float2 (&v)[16], const void *src, uint64_t ub, uint32_t lb) {\n";
    for (int k2 = 0; k2 < 8; ++k2) {
        uint64_t off = 0;
        for (int s = 1; s < 4; ++s)
            if (((2 * k2) >> s) & 1) off |= gbit(io_reg[s]);
        o << "    { const float4 q = buf_ld4(src, ub + " << hex(off) << ", lb); v[" << 2 * k2
          << "] = make_float2(q.x, q.y); v[" << 2 * k2 + 1 << "] = make_float2(q.z, q.w); }\n";
    }
    o << "}\n";
    emit_reduce_tile(o, m, rp, nullptr, "tile");
    o << "__device__ const uint32_t kCols[NT] = {";
    for (size_t c = 0; c < NT; ++c) o << (c ? ", " : "") << rp.cols[c] << "u";
    o << "};\n";
    // items are (descriptor, row of RT consecutive tiles); the row's tiles
    // run in order on one workgroup, the next tile's load in flight
    o << "constexpr uint32_t RT = " << red_row_tiles(1u << (n - m)) << "u;\n";
    o << "extern \"C\" __global__ __launch_bounds__(T) void qw_reduce(const ReduceDesc *__restrict__ descs, "
         "uint32_t n_descs, uint32_t items, uint32_t tmaj) {\n"
         "    __shared__ float2 lds[1 << M];\n"
         "    __shared__ double red[W * NT];\n"
         "    const uint32_t tg = tmaj ? tmaj - 1u : 0u;\n"
         "    auto desc_of = [=](uint32_t it) { return tmaj ? (it >> tg) : (it % n_descs); };\n"
         "    auto row_of = [=](uint32_t it) { return tmaj ? (it & ((1u << tg) - 1u)) : (it / n_descs); };\n"
         "    const uint32_t w = blockIdx.x, x = w & 7u, j = w >> 3, wpx = gridDim.x >> 3;\n"
         "    const uint32_t per = (items + 7u) >> 3;\n"
         "    const uint32_t first = x * per;\n"
         "    const uint32_t last = (first + per < items) ? first + per : items;\n"
         "    uint32_t item = first + j, k = 0;\n"
         "    if (item >= last) return;\n"
         "    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = uni(tid >> 6);\n"
         "    const uint64_t wi = io_wave(wave);\n"
         "    const uint32_t li = io_lane(lane);\n"
         "    char *lb = reinterpret_cast<char *>(lds);\n"
         "    float acc[NT];\n"
         "    #pragma unroll\n"
         "    for (int i = 0; i < NT; ++i) acc[i] = 0.f;\n"
         "    float2 nv[16];\n"
         "    {\n"
         "        const ReduceDesc *d0 = descs + desc_of(item);\n"
         "        load_in(nv, ldu(&d0->psi), uni(ldu(ldu(&d0->tile_base) + row_of(item) * RT)) | wi, li);\n"
         "    }\n"
         "    while (true) {\n"
         "        float2 v[16];\n"
         "        #pragma unroll\n"
         "        for (int r = 0; r < 16; ++r) v[r] = nv[r];\n"
         "        const uint32_t p = desc_of(item), row = row_of(item);\n"
         "        const ReduceDesc *d = descs + p;\n"
         "        const uint64_t base = uni(ldu(ldu(&d->tile_base) + row * RT + k));\n"
         "        uint32_t ni = item, nk = k + 1u;\n"
         "        if (nk == RT) {\n"
         "            ni = item + wpx;\n"
         "            nk = 0u;\n"
         "        }\n"
         "        const bool has_next = ni < last;\n"
         "        if (has_next) {\n"
         "            const ReduceDesc *dn = descs + desc_of(ni);\n"
         "            load_in(nv, ldu(&dn->psi), uni(ldu(ldu(&dn->tile_base) + row_of(ni) * RT + nk)) | wi, li);\n"
         "        }\n"
         "        __syncthreads();  // the previous tile's LDS and partial reads are done\n"
         "        tile(v, tid, lane, base, lb, acc);\n"
         "        if (k == RT - 1u) {\n"
         "            tile_flush(acc, lane, wave, red);\n"
         "            __syncthreads();\n"
         "            double *part = ldu(&d->part);\n"
         "            const uint32_t ntt = ldu(&d->n_terms_total);\n"
         "            for (uint32_t c = tid; c < (uint32_t)NT; c += T) {\n"
         "                double s = 0.0;\n"
         "                for (int ww = 0; ww < W; ++ww) s += red[ww * NT + c];\n"
         "                gout<double>(part)[(uint64_t)row * ntt + kCols[c]] = s;\n"
         "            }\n"
         "        }\n"
         "        if (!has_next) break;\n"
         "        item = ni;\n"
         "        k = nk;\n"
         "    }\n"
         "}\n";
    return o.str();
}

// ---------------------------------------------------------------- compile
namespace {

struct Registry {
    std::mutex mu;
    // (device, key) -> kernel
    std::map<std::pair<int, std::string>, std::unique_ptr<JitKernel>> kernels;
    // key -> code object
    std::unordered_map<std::string, std::vector<char>> code;
};

Registry &reg() {
    static Registry *r = new Registry();  // never destroyed: modules live until exit
    return *r;
}

std::atomic<uint64_t> g_compiled{0}, g_hits{0};
std::atomic<uint64_t> g_compile_us{0};

uint64_t fnv1a(const std::string &s, uint64_t h) {
    for (unsigned char c : s) {
        h ^= c;
        h *= 0x100000001b3ull;
    }
    return h;
}

std::string cache_dir() {
    const char *e = std::getenv("QW_JIT_CACHE");
    if (e) {
        if (!std::strcmp(e, "off") || !*e) return "";
        return e;
    }
    const char *h = std::getenv("HOME");
    if (!h || !*h) return "";
    return std::string(h) + "/.cache/qw_jit";
}

// Identity of a code object: the kernel source plus fingerprints of the two
// headers it includes and of the compile options, so that a library built
// with other record layouts never loads a stale entry.
std::string cache_text(const std::string &src) {
    static const std::string tag = [] {
        std::string opts;
        for (int i = 0; i < kNumOpts; ++i) opts += std::string(kOpts[i]) + " ";
        char b[96];
        std::snprintf(b, sizeof b, "\n// qw headers %016llx %016llx options %016llx\n",
                      (unsigned long long)fnv1a(kEmbedDescH, 0xcbf29ce484222325ull),
                      (unsigned long long)fnv1a(kEmbedDevH, 0xcbf29ce484222325ull),
                      (unsigned long long)fnv1a(opts, 0xcbf29ce484222325ull));
        return std::string(b);
    }();
    return src + tag;
}

std::string cache_path(const std::string &dir, const std::string &src) {
    const std::string t = cache_text(src);
    char b[64];
    std::snprintf(b, sizeof b, "/%016llx%016llx.co",
                  (unsigned long long)fnv1a(t, 0xcbf29ce484222325ull),
                  (unsigned long long)fnv1a(t, 0x84222325cbf29ce4ull));
    return dir + b;
}

// Disk cache entry: text length, identity text (cache_text), code object.
// The stored text must equal the requested one (no trust in the hash alone).
bool cache_load(const std::string &src_in, std::vector<char> *code) {
    const std::string dir = cache_dir();
    if (dir.empty()) return false;
    const std::string src = cache_text(src_in);
    std::ifstream f(cache_path(dir, src_in), std::ios::binary);
    if (!f) return false;
    uint64_t len = 0;
    if (!f.read(reinterpret_cast<char *>(&len), sizeof len) || len != src.size()) return false;
    std::string s(len, '\0');
    if (!f.read(&s[0], (std::streamsize)len) || s != src) return false;
    std::vector<char> c((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    if (c.empty()) return false;
    code->swap(c);
    return true;
}

void cache_store(const std::string &src_in, const std::vector<char> &code) {
    const std::string dir = cache_dir();
    if (dir.empty()) return;
    const std::string src = cache_text(src_in);
    std::string cmd_dir = dir;
    // create the directory chain (best effort, no shell)
    for (size_t i = 1; i <= cmd_dir.size(); ++i) {
        if (i == cmd_dir.size() || cmd_dir[i] == '/') {
            std::string part = cmd_dir.substr(0, i);
            ::mkdir(part.c_str(), 0755);
        }
    }
    const std::string path = cache_path(dir, src_in);
    const std::string tmp = path + ".tmp" + std::to_string((unsigned long long)std::hash<std::thread::id>()(std::this_thread::get_id()));
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f) return;
        const uint64_t len = src.size();
        f.write(reinterpret_cast<const char *>(&len), sizeof len);
        f.write(src.data(), (std::streamsize)src.size());
        f.write(code.data(), (std::streamsize)code.size());
        if (!f) return;
    }
    std::rename(tmp.c_str(), path.c_str());
}

std::string compile_one(const std::string &src, std::vector<char> *code) {
    hiprtcProgram prog = nullptr;
    const char *hdr_src[2] = {kEmbedDescH, kEmbedDevH};
    const char *hdr_name[2] = {"qw_desc.h", "qw_dev.h"};
    hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), "qw_pass.hip", 2, hdr_src, hdr_name);
    if (r != HIPRTC_SUCCESS) return std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r);
    r = hiprtcCompileProgram(prog, kNumOpts, kOpts);
    if (r != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return std::string("hiprtcCompileProgram: ") + hiprtcGetErrorString(r) + "\n" + log;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code->resize(cs);
    hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    return "";
}

// Private segment (scratch) bytes per lane of the kernel `name` in an
// AMDGPU code object: field 1 (offset 4) of its kernel descriptor `name.kd`.
// Returns -1 if the descriptor is not found.
long code_scratch_bytes(const std::vector<char> &code, const char *name) {
    auto rd = [&](size_t off, size_t n) -> uint64_t {
        uint64_t v = 0;
        if (off + n > code.size()) return 0;
        std::memcpy(&v, code.data() + off, n);
        return v;
    };
    if (code.size() < 64 || std::memcmp(code.data(), "\x7f" "ELF", 4) != 0) return -1;
    const uint64_t shoff = rd(0x28, 8), shentsize = rd(0x3A, 2), shnum = rd(0x3C, 2);
    const std::string want = std::string(name) + ".kd";
    for (uint64_t i = 0; i < shnum; ++i) {
        const size_t sh = shoff + i * shentsize;
        if (rd(sh + 4, 4) != 2) continue;  // SHT_SYMTAB
        const uint64_t off = rd(sh + 0x18, 8), size = rd(sh + 0x20, 8), link = rd(sh + 0x28, 4);
        const uint64_t stroff = rd(shoff + link * shentsize + 0x18, 8);
        for (uint64_t j = 0; j + 24 <= size; j += 24) {
            const uint64_t nm = stroff + rd(off + j, 4);
            if (nm >= code.size()) continue;
            const char *sname = code.data() + nm;
            if (std::strncmp(sname, want.c_str(), code.size() - nm) != 0) continue;
            const uint64_t shndx = rd(off + j + 6, 2), value = rd(off + j + 8, 8);
            const size_t ds = shoff + shndx * shentsize;
            const uint64_t fo = value - rd(ds + 0x10, 8) + rd(ds + 0x18, 8);
            return (long)rd(fo + 4, 4);
        }
    }
    return -1;
}

}  // namespace

namespace {
// Kernel source of a request with `prefetch` registers of the next tile.
std::string req_source(const JitReq &r, int prefetch) {
    if (r.persist) return jit_persist_source(*r.persist, prefetch);
    if (r.pass) return jit_pass_source(r.n, r.m, *r.pass, r.use_lds, prefetch, r.epi, r.stream_loads);
    return jit_reduce_source(r.n, r.m, *r.group, *r.rplan);
}
const char *req_kernel_name(const JitReq &r) {
    return r.persist ? "qw_persist" : (r.pass ? "qw_pass" : "qw_reduce");
}
}  // namespace

bool jit_available(int device, const JitReq &r) {
    Registry &R = reg();
    {
        std::lock_guard<std::mutex> lk(R.mu);
        if (R.kernels.count({device, r.key}) || R.code.count(r.key)) return true;
    }
    const std::string dir = cache_dir();
    if (dir.empty()) return false;
    const std::string src = req_source(r, 16);
    struct stat sb;
    return ::stat(cache_path(dir, src).c_str(), &sb) == 0;
}

std::string jit_precompile(const std::vector<JitReq> &ks) {
    Registry &R = reg();
    // code objects still missing (in memory): disk cache, else compile in parallel
    std::vector<size_t> need;
    {
        std::lock_guard<std::mutex> lk(R.mu);
        for (size_t i = 0; i < ks.size(); ++i) {
            if (R.code.count(ks[i].key)) continue;
            bool dup = false;
            for (size_t q : need) dup |= ks[q].key == ks[i].key;
            if (!dup) need.push_back(i);
        }
    }
    if (need.empty()) return "";
    std::vector<std::vector<char>> codes(need.size());
    std::vector<std::string> errs(need.size());
    std::vector<std::string> srcs(need.size());
    const char *dump = std::getenv("QW_JIT_DUMP");  // debugging: write sources to this folder
    for (size_t q = 0; q < need.size(); ++q) {
        const JitReq &r = ks[need[q]];
        srcs[q] = req_source(r, 16);
        if (dump && *dump) {
            std::ofstream f(cache_path(dump, srcs[q]) + ".hip");
            f << srcs[q];
        }
    }
    std::atomic<size_t> next{0};
    auto work = [&]() {
        for (size_t q; (q = next.fetch_add(1)) < need.size();) {
            const std::string &src = srcs[q];
            if (cache_load(src, &codes[q])) {
                g_hits.fetch_add(1);
                continue;
            }
            const auto t0 = std::chrono::steady_clock::now();
            errs[q] = compile_one(src, &codes[q]);
            // persistent pass kernels: if the full register prefetch of the
            // next tile spills, prefetch half of it, else none (stored under
            // the identity of the requested source)
            const JitReq &r = ks[need[q]];
            const char *kname = req_kernel_name(r);
            if (errs[q].empty() && ((r.pass && r.use_lds) || r.persist) &&
                code_scratch_bytes(codes[q], kname) > 0) {
                for (int pf : {8, 0}) {
                    std::vector<char> c2;
                    const std::string e2 = compile_one(req_source(r, pf), &c2);
                    if (!e2.empty()) break;
                    codes[q].swap(c2);
                    if (code_scratch_bytes(codes[q], kname) == 0) break;
                }
            }
            const auto t1 = std::chrono::steady_clock::now();
            g_compile_us.fetch_add(
                (uint64_t)std::chrono::duration_cast<std::chrono::microseconds>(t1 - t0).count());
            if (errs[q].empty()) {
                g_compiled.fetch_add(1);
                cache_store(src, codes[q]);
            }
        }
    };
    const unsigned hw = std::thread::hardware_concurrency();
    const size_t nth = std::min<size_t>(need.size(), std::max(1u, std::min(hw, 16u)));
    std::vector<std::thread> th;
    for (size_t t = 1; t < nth; ++t) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
    std::lock_guard<std::mutex> lk(R.mu);
    for (size_t q = 0; q < need.size(); ++q) {
        if (!errs[q].empty()) return "generated kernel failed to compile: " + errs[q];
        R.code[ks[need[q]].key] = std::move(codes[q]);
    }
    return "";
}

std::string jit_get(int device, const std::vector<JitReq> &reqs, std::vector<const JitKernel *> *out) {
    Registry &R = reg();
    const std::vector<JitReq> &ks = reqs;
    out->assign(ks.size(), nullptr);
    {
        // fast path: every kernel already loaded on this device
        std::lock_guard<std::mutex> lk(R.mu);
        bool all = true;
        for (size_t i = 0; i < ks.size(); ++i) {
            auto it = R.kernels.find({device, ks[i].key});
            if (it == R.kernels.end()) {
                all = false;
                continue;
            }
            (*out)[i] = it->second.get();
        }
        if (all) return "";
    }
    {
        std::vector<JitReq> miss;
        for (size_t i = 0; i < ks.size(); ++i)
            if (!(*out)[i]) miss.push_back(ks[i]);
        const std::string e = jit_precompile(miss);
        if (!e.empty()) return e;
    }
    std::lock_guard<std::mutex> lk(R.mu);
    for (size_t i = 0; i < ks.size(); ++i) {
        if ((*out)[i]) continue;
        auto it = R.kernels.find({device, ks[i].key});
        if (it != R.kernels.end()) {
            (*out)[i] = it->second.get();
            continue;
        }
        const std::vector<char> &code = R.code[ks[i].key];
        const int m = ks[i].m;
        const bool use_lds = ks[i].use_lds || !ks[i].pass || ks[i].persist;
        hipModule_t mod = nullptr;
        hipError_t e = hipModuleLoadData(&mod, code.data());
        if (e != hipSuccess) return std::string("hipModuleLoadData: ") + hipGetErrorString(e);
        auto k = std::make_unique<JitKernel>();
        e = hipModuleGetFunction(&k->fn, mod, req_kernel_name(ks[i]));
        if (e != hipSuccess) return std::string("hipModuleGetFunction: ") + hipGetErrorString(e);
        const int T = 1 << (m - 4);
        k->use_lds = use_lds;
        k->m = m;
        k->wg = use_lds ? T : (T < 256 ? T : 256);
        k->parts = use_lds ? 1 : T / k->wg;
        k->blocks_per_cu = 1;
        if ((!ks[i].pass && !ks[i].persist) || ks[i].epi) k->row_tiles = (int)red_row_tiles(1u << (ks[i].n - m));
        if (use_lds) {
            int nb = 0;
            if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k->fn, k->wg, 0) == hipSuccess &&
                nb > 0)
                k->blocks_per_cu = nb;
        }
        (*out)[i] = k.get();
        R.kernels[{device, ks[i].key}] = std::move(k);
    }
    return "";
}

// Item-order argument of the persistent kernels: 0 for descriptor-fastest,
// else 1 + log2(items per descriptor) for tile-fastest (a power of two).
static uint32_t tile_order_arg(uint32_t tiles, bool tile_major) {
    if (!tile_major || tiles == 0 || (tiles & (tiles - 1)) != 0) return 0u;
    return 1u + (uint32_t)__builtin_ctz(tiles);
}

hipError_t jit_launch(hipStream_t st, const JitKernel &k, const PassDesc *descs, uint32_t n_descs,
                      uint32_t tiles, int remap, uint32_t cu_count, bool tile_major) {
    const uint32_t rows = tiles / (uint32_t)k.row_tiles;
    const uint32_t items = n_descs * rows;
    uint32_t tmaj = k.use_lds ? tile_order_arg(rows, tile_major) : 0u;
    uint32_t grid;
    if (k.use_lds) {
        const uint32_t full = cu_count * (uint32_t)k.blocks_per_cu;
        const uint32_t want = ((items + 7u) / 8u) * 8u;
        grid = want < full ? want : (full / 8u) * 8u;
        if (grid < 8u) grid = 8u;
    } else {
        grid = items * (uint32_t)k.parts;
        if (remap && (grid & 7u)) remap = 0;
    }
    uint32_t items_arg = items;
    void *args[] = {&descs, &n_descs, &items_arg, &remap, &tmaj};
    return hipModuleLaunchKernel(k.fn, grid, 1, 1, (uint32_t)k.wg, 1, 1, 0, st, args, nullptr);
}

hipError_t jit_launch_reduce(hipStream_t st, const JitKernel &k, const ReduceDesc *descs,
                             uint32_t n_descs, uint32_t tiles, uint32_t cu_count, bool tile_major) {
    const uint32_t rows = tiles / (uint32_t)k.row_tiles;
    uint32_t tmaj = tile_order_arg(rows, tile_major);
    const uint32_t items = n_descs * rows;
    const uint32_t full = cu_count * (uint32_t)k.blocks_per_cu;
    const uint32_t want = ((items + 7u) / 8u) * 8u;
    uint32_t grid = want < full ? want : (full / 8u) * 8u;
    if (grid < 8u) grid = 8u;
    uint32_t items_arg = items;
    void *args[] = {&descs, &n_descs, &items_arg, &tmaj};
    return hipModuleLaunchKernel(k.fn, grid, 1, 1, (uint32_t)k.wg, 1, 1, 0, st, args, nullptr);
}

hipError_t jit_launch_persist(hipStream_t st, const JitKernel &k, const PSeg *segs, uint32_t n_segs,
                              const PassDesc *descs, const PDep *deps, uint32_t *sync, uint32_t claims,
                              uint32_t grid, uint32_t spin_limit, uint32_t *host_flag) {
    if (grid == 0u) grid = 1u;
    void *args[] = {&segs, &n_segs, &descs, &deps, &sync, &claims, &spin_limit, &host_flag};
    return hipModuleLaunchKernel(k.fn, grid, 1, 1, (uint32_t)k.wg, 1, 1, 0, st, args, nullptr);
}

void jit_stats(uint64_t *compiled, uint64_t *cache_hits, double *compile_s) {
    if (compiled) *compiled = g_compiled.load();
    if (cache_hits) *cache_hits = g_hits.load();
    if (compile_s) *compile_s = (double)g_compile_us.load() * 1e-6;
}

}  // namespace qw
