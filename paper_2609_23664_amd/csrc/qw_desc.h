// Device-visible records of libqw: pass and reducer descriptors, ops and
// phase layouts. Shared by the host planner, the ahead-of-time kernels and
// the kernels generated at run time (this text is compiled by hipRTC too,
// so it includes nothing). Not part of the public ABI.
#pragma once

#if defined(__HIPCC_RTC__)
using __hip_internal::uint8_t;
using __hip_internal::uint16_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
using __hip_internal::int32_t;
#endif

namespace qw {

// ---------------------------------------------------------------- limits
constexpr int kMaxQubits = 30;      // 8 GiB per complex64 state
constexpr int kRegBits = 4;         // amplitudes per thread = 2^kRegBits
constexpr int kMinTileBits = 10;    // register/lane/wave layout needs >= 10
constexpr int kMaxTileBits = 14;    // 2^14 complex64 = 128 KiB of LDS
constexpr int kIoLaneLo = 1;        // lanes cover local bits 1..6 at I/O
constexpr int kIoLaneHi = 6;

// ---------------------------------------------------------------- ops
// Operations executed on a tile. Bit operands are *local* bit positions
// (0..m-1) unless the matching GLOBAL flag is set, in which case they are
// global qubit indices (bits that are constant over the tile).
enum OpType : uint8_t {
    OP_U = 1,     // 2x2 complex matrix on local bit a (register slot s)
    OP_DIAG = 2,  // diag(d0, d1) on bit a
    OP_PERM = 3,  // [[0, p01], [p10, 0]] on local bit a (register slot s)
    OP_CX = 4,    // swap the pair on local target a (slot s) where control b is 1
    OP_CZ = 5,    // negate where bits a and b are both 1
    OP_UR = 6,    // real 2x2 matrix [[m0, m1], [m2, m3]] on local bit a
    OP_DSET = 7,  // header of a diagonal set applied at once: a product of
                  // parity factors d[parity(index & mask)]. Register kernel:
                  // sb = number of OP_DTAB records that follow (0 or 4: for
                  // each register k, the product of the factors whose mask
                  // lies in the register bits, computed in FP64 on the host),
                  // then b OP_PDIAG members without register bits (folded into
                  // one per-thread factor), then a OP_PDIAG members with both
                  // register and other bits. Small-state kernel: sb = a = 0 and
                  // the b members are applied one by one.
    OP_DTAB = 8,  // 4 complex entries (m[0..7]) of an OP_DSET register table
    OP_URT = 10,  // real rotation or reflection with its factor p dropped
                  // (the pass folds the product of the factors into one of
                  // its diagonal ops): target local bit a (slot sa), form b,
                  // t = m[0]:  0: [[1, -t], [t, 1]]   1: [[1, t], [t, -1]]
                  // one FMA per output component
    OP_URD = 11,  // real 2x2 matrix [[e0, e1], [e2, e3]] on local bit a (slot sa)
                  // whose 4 FP32 entries are read at run time from the device
                  // address held in the bytes of m[0..1] (written there by an
                  // earlier kernel: a measurement's projector, decided on the
                  // device)
    OP_PDIAG = 9, // parity factor (member of an OP_DSET): d0 = m[0..1] where
                  // the parity of (index & mask) is even, d1 = m[2..3] where odd;
                  // mask = register slots rmask + thread bits tmask (local bit
                  // numbers) + non-local bits gmask (qubit numbers)
};

// Where an operand bit lives inside a phase of the register kernel.
enum BitLoc : uint8_t {
    LOC_REG = 0,     // register slot (index in `slot` fields)
    LOC_THREAD = 1,  // a thread-index bit (local bit number in a/b)
    LOC_GLOBAL = 2,  // non-local: global qubit index in a/b
    LOC_LANE = 3,    // target on a lane bit: lane index bit in `sa` (0..5)
};

// Layout of a phase: 4 register bits R; the 6 lowest local bits not in R
// are the lane bits of the 64-wide wavefront; the rest are wave bits.
// I/O kinds: IO_F4 = R holds local bit 0 and the lanes are local bits
// 1..6 (16-byte accesses); IO_F2 = the lanes are local bits 0..5 (8-byte
// accesses). Loads happen in phase 0 and stores in the last phase, both of
// which must have an I/O kind.
enum IoKind : uint8_t { IO_NONE = 0, IO_F4 = 1, IO_F2 = 2 };

struct alignas(16) DevOp {
    uint8_t type;
    uint8_t a, b;          // local or global bit numbers (see loc)
    uint8_t sa, sb;        // register slots of a and b when LOC_REG
    uint8_t la, lb;        // BitLoc of a and b
    uint8_t rmask;         // OP_PDIAG: register-slot part of the mask
    uint32_t tmask;        // OP_PDIAG: thread part (local bit numbers)
    uint32_t gmask;        // OP_PDIAG: non-local part (qubit numbers)
    float m[8];            // U: m00 m01 m10 m11 (re, im); DIAG/PDIAG: d0 d1;
                           // PERM: p01 p10
};
static_assert(sizeof(DevOp) == 48, "DevOp layout");

// One phase of a pass: the 4 local bits held in registers and the ops run
// while that mapping is live. Phase 0 and the last phase are I/O capable:
// register slot 0 is local bit 0 and no register bit lies in the lane bits.
struct alignas(16) DevPhase {
    uint8_t reg[4];        // local bit of register slot 0..3 (ascending)
    uint16_t op_begin;
    uint16_t op_end;
    uint8_t io;            // IoKind
    uint8_t pad[7];
    uint32_t lds_off[16];  // byte offset in LDS of register k (swizzled)
};
static_assert(sizeof(DevPhase) == 80, "DevPhase layout");

// LDS element swizzle (see the kernels): the low 5 bits of the element index
// are XORed with bits 5..9 and 10..13. It is linear over GF(2).
#if !defined(__HIPCC_RTC__)
inline uint32_t lds_swizzle(uint32_t l) { return l ^ (((l >> 5) ^ (l >> 10)) & 31u); }
#endif

// Pass descriptor flags
enum : uint32_t {
    PD_SCALE_IN = 1u,    // multiply loaded amplitudes by *scale (FP64)
    PD_NORM_OUT = 2u,    // write per-tile FP64 sums of |psi|^2
    PD_REMAP_OUT = 4u,   // stores go through the pass's output relabelling
};

// Uniform address record of an I/O phase, computed on the host: global
// index bits of the lane part (shifts), of each register and of each wave.
// Output relabelling (a pass whose last gates are CNOTs with non-local
// targets, applied as a permutation of the store addresses): the amplitude
// of global index j is stored at index L(j) with L linear over GF(2), equal
// to the identity on the local bits. L(j) = tile_base_out[tile] ^ reg_xor[k]
// ^ wave_xor[w] combined with the local part of j, where the two xor terms
// are the non-local images of the local bits that register k and wave w
// carry. Lane bits never carry such a bit (the planner keeps relabelling
// controls out of the lane positions).
struct alignas(16) IoRec {
    uint8_t kind;          // IoKind
    uint8_t g4, g5, g6;    // global positions of local bits 4, 5, 6
    uint32_t pad[3];
    uint32_t reg_off[16];  // global index bits of register k
    uint32_t wave_off[16]; // global index bits of wave w (tile bits >= 10)
    uint32_t reg_xor[16];  // output relabelling: non-local bits flipped by register k
    uint32_t wave_xor[16]; // output relabelling: non-local bits flipped by wave w
};
static_assert(sizeof(IoRec) == 272, "IoRec layout");

// One (task, pass): a tile sweep over a state slot.
struct alignas(16) PassDesc {
    const void *src;       // float2 amplitudes read (may equal dst)
    void *dst;             // float2 amplitudes written
    const DevOp *ops;
    const DevPhase *phases;
    uint64_t local_mask;   // global bits that are local to a tile
    const double *scale_in;  // PD_SCALE_IN: factor applied on load
    double *norm_part;     // PD_NORM_OUT: [tiles] FP64 sums of |psi|^2
    double *scale_out;     // PD_NORM_OUT: 1/sqrt(sum) written by finalize
    const uint32_t *tile_base;  // global index of local index 0, per tile
    const uint32_t *tile_base_out;  // PD_REMAP_OUT: L(tile_base), per tile
    const IoRec *io_in;    // address record of phase 0
    const IoRec *io_out;   // address record of the last phase
    double *red_part;      // fused expectation epilogue: [rows][red_nt] FP64 partials
    uint32_t n_ops;
    uint32_t n_phases;
    uint32_t flags;
    uint32_t red_nt;       // fused expectation epilogue: columns per row (all terms)
};
static_assert(sizeof(PassDesc) == 128, "PassDesc layout");

// Persistent launch of a whole call (every pass of every task, and with
// in-call parents every level of a task tree): the work is a list of claims
// taken in increasing order from one device counter. A segment is one pass
// structure at one pass index: its descriptors are consecutive in the call's
// descriptor array and each is swept in units (tiles, or rows of
// red_row_tiles tiles for a pass with an expectation epilogue), `chunk`
// units per claim.
struct alignas(16) PSeg {
    uint32_t claim0;       // first claim of the segment
    uint32_t n_claims;
    uint32_t desc0;        // index of its first descriptor
    uint32_t n_descs;
    uint32_t chunk;        // units per claim (divides units)
    uint32_t kind;         // pass structure (case of the generated kernel)
    uint32_t tmaj;         // 1: one descriptor's claims are consecutive
    uint32_t units;        // units per descriptor
};
static_assert(sizeof(PSeg) == 32, "PSeg layout");

// Dependency of one descriptor of a persistent launch: its sweep starts when
// the completion counter of descriptor `dep` has reached `need` units (the
// pass before it, or the last pass of the parent task). dep = kNoDep: none.
constexpr uint32_t kNoDep = 0xFFFFFFFFu;
struct alignas(8) PDep {
    uint32_t dep;
    uint32_t need;
};

// Words of a persistent launch's synchronisation area (cleared by a kernel
// before the launch): the claim counter, the abandon flag, then one
// completion counter per descriptor.
constexpr uint32_t kSyncClaim = 0, kSyncAbort = 1, kSyncCounters = 2;

// Expectation partials are kept per row of kRedRowTiles consecutive tiles of
// a state (all of its tiles when it has fewer): each thread adds its FP32
// term values over the row's tiles, in tile order, before the FP64 sum
// across lanes and waves, so a row's partials do not depend on which
// workgroup processed it or on the launch's item order.
constexpr uint32_t kRedRowTiles = 4;
constexpr uint32_t red_row_tiles(uint32_t tiles) { return tiles < kRedRowTiles ? tiles : kRedRowTiles; }

// Expectation reducer, small states (n < 10): the whole state is one tile
// staged in LDS; one descriptor per slot.
struct alignas(16) TermSmall {
    uint32_t x;            // X/Y support
    uint32_t z;            // Z/Y support
    uint32_t ny_mod4;      // number of Y factors mod 4
    uint32_t out_index;    // column of the term in the partial array
};

struct alignas(16) ReduceDescSmall {
    const void *psi;
    const TermSmall *terms;
    double *part;          // [n_terms] of this slot
    uint32_t n_terms;
    uint32_t pad;
};

// Expectation reducer, register kernel (tile bits >= 10). A term group is a
// set of terms whose X/Y support lies in the group's local bits; its terms
// are split into phases whose 4 register bits contain each term's X/Y
// support, so every pair (l, l ^ x) of a term is inside one thread.
constexpr int kMaxGroupTerms = 64;

struct alignas(16) TermDev {
    uint8_t xr;            // X/Y support as register-slot mask
    uint8_t neg;           // 1: negate the pair sum (phase i^ny)
    uint8_t odd;           // 1: ny odd, use Im(conj(b) a)
    uint8_t pad0;
    uint16_t smask;        // bit k: parity of the Z/Y bits at register index k
    uint16_t col;          // group-local column (0..n_terms-1)
    uint32_t zt;           // Z/Y support on the phase's thread bits (local numbering)
    uint32_t pad1;
    uint64_t zg;           // Z/Y support on global (non-local) bits
};
static_assert(sizeof(TermDev) == 32, "TermDev layout");

struct alignas(16) RedPhase {
    uint8_t reg[4];        // local bits of register slots 0..3 (ascending)
    uint16_t t_begin;
    uint16_t t_end;
    uint32_t diag;         // 1: diagonal terms only, evaluated in the I/O layout
    uint32_t pad;
};
static_assert(sizeof(RedPhase) == 16, "RedPhase layout");

struct alignas(16) ReduceDesc {
    const void *psi;       // float2 state slot
    const TermDev *terms;
    const RedPhase *phases;
    const uint32_t *cols;  // group-local column -> column of the partial array
    double *part;          // [rows][n_terms_total] of this slot (see kRedRowTiles)
    const uint32_t *tile_base;  // global index of local index 0, per tile
    uint64_t local_mask;
    uint32_t n_phases;
    uint32_t n_terms;      // terms of this group
    uint32_t n_terms_total;
    uint32_t pad;
};

}  // namespace qw
