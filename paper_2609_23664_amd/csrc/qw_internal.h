// Internal types shared by the host planner, the C ABI and the gfx950
// kernels of libqw. Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "qw_desc.h"
#include "../../include/qw.h"

namespace qw {

// ---------------------------------------------------------------- host plan
struct HostOp {
    OpType type;
    int a = -1, b = -1;         // global qubits
    uint64_t mask = 0;          // OP_PDIAG: qubit mask of the parity factor
    double m[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // FP64 complex entries
    std::vector<HostOp> members;  // OP_DSET: the OP_DIAG ops of the set
};

struct HostPass {
    uint64_t local_mask = 0;
    IoRec io_in{}, io_out{};      // filled by lower_pass() (register kernel)
    std::vector<HostOp> ops;    // global-qubit form, execution order
    bool scale_in = false;
    bool norm_out = false;
    // Output relabelling: CNOTs (control, target) with non-local targets that
    // end the pass, applied as a linear map L of the store addresses.
    // out_img[q] = L(e_q) for every qubit q (empty: no relabelling).
    std::vector<std::pair<int, int>> out_cx;
    std::vector<uint64_t> out_img;
    // Index layouts of the state the pass loads and of the one it stores:
    // qubit q is index bit in_pos[q] / out_pos[q] (empty: bit q). A plan
    // starts and ends in the standard layout; between two of its passes the
    // qubits may be permuted so that more of a tile is one contiguous run.
    // Device records name non-local qubits by their bit in the load layout.
    std::vector<uint8_t> in_pos, out_pos;
    // the pass stores to other addresses than the ones it loads
    bool moves() const { return !out_img.empty() || in_pos != out_pos; }
    // filled by lower_pass():
    std::vector<DevOp> dev_ops;
    std::vector<DevPhase> dev_phases;
    mutable std::string jit_key;  // generated-kernel key, computed on first use
};

struct Plan {
    int n = 0;
    int m = 0;                  // tile bits
    std::vector<HostPass> passes;
    size_t n_gates = 0;
    bool in_place = false;      // planned for a first pass that loads its own destination
    bool layout = false;        // planned with permuted layouts allowed
};

// Validates and plans `gates` on n qubits with at most tile_bits local bits
// per pass; `relabel` allows output relabelling (trailing CNOTs with
// non-local targets applied as store-address maps). Without `lower` the
// passes keep their host ops only (no device records or phases: enough to
// count passes). Returns "" on success, otherwise an error message.
// `layout` allows permuted index layouts between passes (HostPass::in_pos);
// `in_place`: the first pass will load the state from its own destination
// (no separate source), which the layouts take into account.
std::string build_plan(int n, const void *gates /* qw_gate* */, size_t n_gates,
                       int tile_bits, Plan *out, bool relabel = true, bool lower = true,
                       bool allow_dyn = false, bool layout = true, bool in_place = false);

// Internal gate kind (never accepted from callers): a real 2x2 operator on
// q0 whose 4 FP32 entries the device writes at run time at the address held
// in the bits of `param` (lowered to OP_URD, never fused with other gates).
// The library opens a segment after a measurement with one per measured
// qubit: its projector (and the X of a RESET with outcome 1).
constexpr uint32_t kGateDyn = 0x86;
inline double dyn_param(const void *addr) {
    double d;
    const uint64_t a = reinterpret_cast<uint64_t>(addr);
    __builtin_memcpy(&d, &a, sizeof d);
    return d;
}

// JSON form of a plan (for qw_plan_describe).
std::string plan_json(const Plan &p);

// Effective tile bits for an n-qubit state.
inline int tile_bits_for(int n, int max_bits) {
    return n < max_bits ? n : max_bits;
}

// Term grouping for the reducer: splits terms into groups whose X/Y support
// fits one local set. Each group lists term indices and its local mask.
struct TermGroup {
    uint64_t local_mask;
    std::vector<uint32_t> terms;
};
std::vector<TermGroup> group_terms(int n, int m, const uint64_t *x, size_t n_terms);

// Register-phase layout of one term group for the reducer kernel.
struct RedPlan {
    std::vector<RedPhase> phases;
    std::vector<TermDev> terms;   // ordered by phase
    std::vector<uint32_t> cols;   // group-local column -> global term index
};
// `diag_reg` (optional): register slots of the diagonal phase (default: the
// I/O layout, local bits 0, 7, 8, 9).
RedPlan plan_reduce_group(int n, int m, const TermGroup &g, const uint64_t *x,
                          const uint64_t *z, const uint8_t *diag_reg = nullptr);

// Stabilizer tableau (qw_tableau.cpp): rows (x, z, r) of the destabilizers
// (0..n-1) and stabilizer generators (n..2n-1), n <= 63.
struct StabExport {
    uint64_t x0 = 0;                 // a basis state of the support
    std::vector<uint64_t> x, z;      // X-type generators in reduced echelon form
    std::vector<uint8_t> phase;      // their i-powers: 2 r + |x & z| (mod 4)
    std::vector<uint32_t> pivot;     // X pivot qubit of each
};
struct Tableau {
    int n = 0;
    std::vector<uint64_t> x, z;
    std::vector<uint8_t> r;
    explicit Tableau(int n_);
    void rowsum(int h, int i);
    void h(int a);
    void s(int a);
    void cx(int a, int b);
    void pauli(uint64_t px, uint64_t pz);
    // Applies Clifford gates (X Y Z H S SDG CNOT CZ); "" or an error.
    std::string apply(const qw_gate *g, uint64_t count);
    // The data of the dense export.
    StabExport export_form() const;
};

// Persistent launch (qw_persist.cpp): the claim schedule of a call's
// descriptors. `descs` lists every (task t, pass k) once; parent[t] is -1 or
// an earlier task whose last pass task t's first pass waits for; passes[t]
// is task t's pass count. Claims are ordered by level (the passes that must
// have run before a descriptor), then pass structure, then task, so every
// dependency lies in an earlier level. Returns "" or an error.
struct PersistDesc {
    uint32_t t = 0, k = 0;  // task and pass index
    uint32_t kind = 0;      // pass structure (case of the persistent kernel)
    uint32_t units = 0;     // tiles, or rows of an epilogue pass (a power of two)
    uint64_t src = 0;       // identity of the state its tiles load
    bool relabel = false;   // the pass stores to relabelled addresses
};
struct PersistSchedule {
    std::vector<uint32_t> order;  // claim-order position -> index into descs
    std::vector<PSeg> segs;
    std::vector<PDep> deps;       // per claim-order position
    uint32_t claims = 0;
};
std::string persist_schedule(const std::vector<int> &parent, const std::vector<uint32_t> &passes,
                             const std::vector<PersistDesc> &descs, int tile_order, uint32_t chunk_max,
                             uint32_t grid, PersistSchedule *out);

// bit helpers
inline uint64_t pdep64(uint64_t v, uint64_t mask) {
    uint64_t r = 0;
    for (uint64_t bb = 1; mask; bb <<= 1) {
        uint64_t low = mask & (~mask + 1);
        if (v & bb) r |= low;
        mask &= mask - 1;
    }
    return r;
}
inline uint64_t pext64(uint64_t v, uint64_t mask) {
    uint64_t r = 0, bb = 1;
    while (mask) {
        uint64_t low = mask & (~mask + 1);
        if (v & low) r |= bb;
        bb <<= 1;
        mask &= mask - 1;
    }
    return r;
}
inline int popc64(uint64_t v) { return __builtin_popcountll(v); }
// Bits of a standard-layout index v at their places in layout `pos`.
inline uint64_t to_layout(uint64_t v, const std::vector<uint8_t> &pos) {
    if (pos.empty()) return v;
    uint64_t r = 0;
    for (; v; v &= v - 1) r |= 1ull << pos[__builtin_ctzll(v)];
    return r;
}

// The non-local bits of `nonlocal` in counting order: the k-th value is
// pdep64(k, nonlocal) (a tile's origin), and each next one comes from
// adding one through the other bits, ((v | ~nonlocal) + 1) & nonlocal.
inline uint64_t next_in_mask(uint64_t v, uint64_t nonlocal) { return ((v | ~nonlocal) + 1) & nonlocal; }

}  // namespace qw
