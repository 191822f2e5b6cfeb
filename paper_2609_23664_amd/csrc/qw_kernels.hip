// gfx950 kernels of libqw.
//
// Layout: a state slot is 2^n complex64 amplitudes (float2, interleaved),
// qubit q = bit q of the index.
//
// Gate pass (pass_kernel<M>): one workgroup owns one tile of 2^M amplitudes
// per (task, pass); the tile is the set of indices that differ only in the
// pass's M local bits. 2^(M-4) threads hold 16 amplitudes each in registers.
// A "phase" maps 4 local bits to the 16 register slots and the remaining
// M-4 local bits to the thread index (its 6 lowest bits to the lanes of a
// 64-wide wavefront). Ops whose target bit sits in a register slot run in
// registers; between phases the tile is exchanged through LDS (XOR-swizzled
// to spread LDS banks). The first and last phases are I/O phases: slot 0 is
// local bit 0 and the lanes are local bits 1..6, so every load/store is a
// 16-byte access and eight consecutive lanes cover one 128-byte run.
//
// All reductions are FP64 and use a fixed order (per-thread sequential,
// then a fixed shuffle tree, then the waves in order), so results do not
// depend on how many tasks share a launch.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qw_internal.h"
#include "qw_kernels.h"

namespace qw {

// ------------------------------------------------------------- helpers
// Descriptors, ops, phases and terms are written by a host-to-device copy
// before a launch and only read during it; reading them through the
// constant address space lets uniform accesses use scalar loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define QW_CONST __attribute__((address_space(4)))
#define QW_GLOBAL __attribute__((address_space(1)))
#else
#define QW_CONST
#define QW_GLOBAL
#endif

template <typename T>
__device__ __forceinline__ T ldu(const T *p) {
    return *(const QW_CONST T *)(p);
}

// Force a wave-uniform 32-bit value into a scalar register.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float unif(float v) {
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}

// Uniform loads of the small plan records, kept in scalar registers.
struct PhaseHead {
    uint8_t reg[4];
    uint16_t op_begin, op_end;
    uint8_t io;
};

__device__ __forceinline__ PhaseHead ld_phase_head(const DevPhase *p) {
    const QW_CONST uint32_t *w = (const QW_CONST uint32_t *)(p);
    const uint32_t w0 = uni(w[0]), w1 = uni(w[1]), w2 = uni(w[2]);
    PhaseHead h;
    h.reg[0] = (uint8_t)w0;
    h.reg[1] = (uint8_t)(w0 >> 8);
    h.reg[2] = (uint8_t)(w0 >> 16);
    h.reg[3] = (uint8_t)(w0 >> 24);
    h.op_begin = (uint16_t)w1;
    h.op_end = (uint16_t)(w1 >> 16);
    h.io = (uint8_t)w2;
    return h;
}

template <typename T>
__device__ __forceinline__ T ld_words(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "word record");
    uint32_t w[sizeof(T) / 4];
    #pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = uni(((const QW_CONST uint32_t *)p)[i]);
    T r;
    __builtin_memcpy(&r, w, sizeof r);
    return r;
}

template <typename T>
__device__ __forceinline__ const QW_GLOBAL T *gin(const void *p) {
    return (const QW_GLOBAL T *)(p);
}

template <typename T>
__device__ __forceinline__ QW_GLOBAL T *gout(void *p) {
    return (QW_GLOBAL T *)(p);
}

__device__ __forceinline__ uint64_t dpdep(uint64_t v, uint64_t mask) {
    uint64_t r = 0;
    uint64_t bb = 1;
    while (mask) {
        uint64_t low = mask & (~mask + 1);
        if (v & bb) r |= low;
        bb <<= 1;
        mask &= mask - 1;
    }
    return r;
}

__device__ __forceinline__ uint32_t dpdep32(uint32_t v, uint32_t mask) {
    uint32_t r = 0;
    uint32_t bb = 1;
    while (mask) {
        uint32_t low = mask & (~mask + 1);
        if (v & bb) r |= low;
        bb <<= 1;
        mask &= mask - 1;
    }
    return r;
}

// LDS address swizzle: the low 5 bits of the element index are XORed with
// bits 5..9 and 10..13, which keeps every phase's 64 lanes on distinct bank
// groups for the phase layouts the planner produces.
__device__ __forceinline__ uint32_t swz(uint32_t l) {
    return l ^ (((l >> 5) ^ (l >> 10)) & 31u);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// u * x + v * y for complex u, v, x, y
__device__ __forceinline__ float2 cmad2(float2 u, float2 x, float2 v, float2 y) {
    float re = u.x * x.x;
    re = fmaf(-u.y, x.y, re);
    re = fmaf(v.x, y.x, re);
    re = fmaf(-v.y, y.y, re);
    float im = u.x * x.y;
    im = fmaf(u.y, x.x, im);
    im = fmaf(v.x, y.y, im);
    im = fmaf(v.y, y.x, im);
    return make_float2(re, im);
}

// Item index for workgroup b: with remapping, the workgroups that the
// hardware places on one XCD (b mod 8) process consecutive items.
__device__ __forceinline__ uint32_t item_of(uint32_t b, uint32_t grid, int remap) {
    if (!remap) return b;
    uint32_t per = grid >> 3;
    return (b & 7u) * per + (b >> 3);
}

// Fixed-order block sum of one double per thread; result valid in thread 0.
template <int T>
__device__ double block_sum(double v, double *red) {
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    constexpr int W = (T + 63) / 64;
    if constexpr (W == 1) {
        return v;
    } else {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        __syncthreads();
        if (lane == 0) red[w] = v;
        __syncthreads();
        double s = 0.0;
        if (threadIdx.x == 0) {
            for (int k = 0; k < W; ++k) s += red[k];
        }
        return s;
    }
}

// ------------------------------------------------------------- register ops
template <int S>
__device__ __forceinline__ void op_u(float2 (&v)[16], const float *m) {
    const float2 a = make_float2(m[0], m[1]), b = make_float2(m[2], m[3]);
    const float2 c = make_float2(m[4], m[5]), d = make_float2(m[6], m[7]);
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k & (1 << S)) continue;
        const float2 x = v[k], y = v[k | (1 << S)];
        v[k] = cmad2(a, x, b, y);
        v[k | (1 << S)] = cmad2(c, x, d, y);
    }
}

// Real 2x2 matrix on a register slot: 4 FP32 ops per output amplitude.
template <int S>
__device__ __forceinline__ void op_ur(float2 (&v)[16], const float *m) {
    const float a = m[0], b = m[1], c = m[2], d = m[3];
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k & (1 << S)) continue;
        const float2 x = v[k], y = v[k | (1 << S)];
        v[k] = make_float2(fmaf(a, x.x, b * y.x), fmaf(a, x.y, b * y.y));
        v[k | (1 << S)] = make_float2(fmaf(c, x.x, d * y.x), fmaf(c, x.y, d * y.y));
    }
}

template <int S>
__device__ __forceinline__ void op_perm(float2 (&v)[16], const float *m) {
    const float2 p01 = make_float2(m[0], m[1]), p10 = make_float2(m[2], m[3]);
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k & (1 << S)) continue;
        const float2 x = v[k], y = v[k | (1 << S)];
        v[k] = cmul(p01, y);
        v[k | (1 << S)] = cmul(p10, x);
    }
}

// Value (0/1) of operand bit for register k.
__device__ __forceinline__ uint32_t opbit(uint8_t loc, uint8_t bit, uint8_t slot, int k,
                                          uint32_t tl, uint64_t base) {
    if (loc == LOC_REG) return ((uint32_t)k >> slot) & 1u;
    if (loc == LOC_THREAD) return (tl >> bit) & 1u;
    return (uint32_t)(base >> bit) & 1u;
}

template <int S>
__device__ __forceinline__ void op_cx(float2 (&v)[16], const DevOp &op, uint32_t tl,
                                      uint64_t base) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k & (1 << S)) continue;
        const uint32_t c = opbit(op.lb, op.b, op.sb, k, tl, base);
        const float2 x = v[k], y = v[k | (1 << S)];
        v[k] = c ? y : x;
        v[k | (1 << S)] = c ? x : y;
    }
}

__device__ __forceinline__ void op_diag(float2 (&v)[16], const DevOp &op, uint32_t tl,
                                        uint64_t base) {
    const float2 d0 = make_float2(op.m[0], op.m[1]), d1 = make_float2(op.m[2], op.m[3]);
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t b = opbit(op.la, op.a, op.sa, k, tl, base);
        v[k] = cmul(b ? d1 : d0, v[k]);
    }
}

__device__ __forceinline__ void op_cz(float2 (&v)[16], const DevOp &op, uint32_t tl,
                                      uint64_t base) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t b = opbit(op.la, op.a, op.sa, k, tl, base) &
                           opbit(op.lb, op.b, op.sb, k, tl, base);
        if (b) v[k] = make_float2(-v[k].x, -v[k].y);
    }
}

// Value of lane (lane ^ 2^J) for the 64-wide wavefront: DPP for J < 4
// (quad permutes and row mirrors), cross-row shuffles for J = 4, 5.
template <int J>
__device__ __forceinline__ float lane_xor(float x) {
    int v = __float_as_int(x);
    if constexpr (J == 0) {
        v = __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);   // quad_perm 1,0,3,2
    } else if constexpr (J == 1) {
        v = __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);   // quad_perm 2,3,0,1
    } else if constexpr (J == 2) {
        v = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);  // row_half_mirror: ^7
        v = __builtin_amdgcn_mov_dpp(v, 0x1B, 0xF, 0xF, true);   // quad_perm 3,2,1,0: ^3
    } else if constexpr (J == 3) {
        v = __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true);  // row_mirror: ^15
        v = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);  // row_half_mirror: ^7
    } else {
        v = __shfl_xor(v, 1 << J, 64);
    }
    return __int_as_float(v);
}

template <int J>
__device__ __forceinline__ float2 lane_xor2(float2 a) {
    return make_float2(lane_xor<J>(a.x), lane_xor<J>(a.y));
}

// 2x2 op on a lane bit: each lane keeps its own component of the pair.
template <int J>
__device__ __forceinline__ void op_u_lane(float2 (&v)[16], const float *m, uint32_t lane) {
    const bool b = (lane >> J) & 1u;
    // the matrix entries are wave-uniform; select per lane between scalars
    const float m0 = unif(m[0]), m1 = unif(m[1]), m2 = unif(m[2]), m3 = unif(m[3]);
    const float m4 = unif(m[4]), m5 = unif(m[5]), m6 = unif(m[6]), m7 = unif(m[7]);
    const float2 cs = make_float2(b ? m6 : m0, b ? m7 : m1);
    const float2 co = make_float2(b ? m4 : m2, b ? m5 : m3);
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float2 pk = lane_xor2<J>(v[k]);
        v[k] = cmad2(cs, v[k], co, pk);
    }
}

template <int J>
__device__ __forceinline__ void op_ur_lane(float2 (&v)[16], const float *m, uint32_t lane) {
    const bool b = (lane >> J) & 1u;
    const float m0 = unif(m[0]), m1 = unif(m[1]), m2 = unif(m[2]), m3 = unif(m[3]);
    const float cs = b ? m3 : m0, co = b ? m2 : m1;
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float2 pk = lane_xor2<J>(v[k]);
        v[k] = make_float2(fmaf(cs, v[k].x, co * pk.x), fmaf(cs, v[k].y, co * pk.y));
    }
}

template <int J>
__device__ __forceinline__ void op_perm_lane(float2 (&v)[16], const float *m, uint32_t lane) {
    const bool b = (lane >> J) & 1u;
    const float m0 = unif(m[0]), m1 = unif(m[1]), m2 = unif(m[2]), m3 = unif(m[3]);
    const float2 co = make_float2(b ? m2 : m0, b ? m3 : m1);
    #pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = cmul(co, lane_xor2<J>(v[k]));
}

template <int J>
__device__ __forceinline__ void op_cx_lane(float2 (&v)[16], const DevOp &op, uint32_t tl,
                                           uint64_t base) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t c = opbit(op.lb, op.b, op.sb, k, tl, base);
        const float2 pk = lane_xor2<J>(v[k]);
        v[k] = c ? pk : v[k];
    }
}

__device__ __forceinline__ void run_op(float2 (&v)[16], const DevOp &op, uint32_t tl,
                                       uint64_t base) {
    const uint32_t lane = threadIdx.x & 63u;
    if (op.la == LOC_LANE) {
        switch (op.type) {
        case OP_U:
            switch (op.sa) {
            case 0: op_u_lane<0>(v, op.m, lane); break;
            case 1: op_u_lane<1>(v, op.m, lane); break;
            case 2: op_u_lane<2>(v, op.m, lane); break;
            case 3: op_u_lane<3>(v, op.m, lane); break;
            case 4: op_u_lane<4>(v, op.m, lane); break;
            default: op_u_lane<5>(v, op.m, lane); break;
            }
            return;
        case OP_UR:
            switch (op.sa) {
            case 0: op_ur_lane<0>(v, op.m, lane); break;
            case 1: op_ur_lane<1>(v, op.m, lane); break;
            case 2: op_ur_lane<2>(v, op.m, lane); break;
            case 3: op_ur_lane<3>(v, op.m, lane); break;
            case 4: op_ur_lane<4>(v, op.m, lane); break;
            default: op_ur_lane<5>(v, op.m, lane); break;
            }
            return;
        case OP_PERM:
            switch (op.sa) {
            case 0: op_perm_lane<0>(v, op.m, lane); break;
            case 1: op_perm_lane<1>(v, op.m, lane); break;
            case 2: op_perm_lane<2>(v, op.m, lane); break;
            case 3: op_perm_lane<3>(v, op.m, lane); break;
            case 4: op_perm_lane<4>(v, op.m, lane); break;
            default: op_perm_lane<5>(v, op.m, lane); break;
            }
            return;
        case OP_CX:
            switch (op.sa) {
            case 0: op_cx_lane<0>(v, op, tl, base); break;
            case 1: op_cx_lane<1>(v, op, tl, base); break;
            case 2: op_cx_lane<2>(v, op, tl, base); break;
            case 3: op_cx_lane<3>(v, op, tl, base); break;
            case 4: op_cx_lane<4>(v, op, tl, base); break;
            default: op_cx_lane<5>(v, op, tl, base); break;
            }
            return;
        default: return;
        }
    }
    switch (op.type) {
    case OP_UR:
        switch (op.sa) {
        case 0: op_ur<0>(v, op.m); break;
        case 1: op_ur<1>(v, op.m); break;
        case 2: op_ur<2>(v, op.m); break;
        default: op_ur<3>(v, op.m); break;
        }
        break;
    case OP_U:
        switch (op.sa) {
        case 0: op_u<0>(v, op.m); break;
        case 1: op_u<1>(v, op.m); break;
        case 2: op_u<2>(v, op.m); break;
        default: op_u<3>(v, op.m); break;
        }
        break;
    case OP_PERM:
        switch (op.sa) {
        case 0: op_perm<0>(v, op.m); break;
        case 1: op_perm<1>(v, op.m); break;
        case 2: op_perm<2>(v, op.m); break;
        default: op_perm<3>(v, op.m); break;
        }
        break;
    case OP_CX:
        switch (op.sa) {
        case 0: op_cx<0>(v, op, tl, base); break;
        case 1: op_cx<1>(v, op, tl, base); break;
        case 2: op_cx<2>(v, op, tl, base); break;
        default: op_cx<3>(v, op, tl, base); break;
        }
        break;
    case OP_DIAG: op_diag(v, op, tl, base); break;
    case OP_CZ: op_cz(v, op, tl, base); break;
    default: break;
    }
}

// Local index offset of register k for a phase with register bits reg[].
__device__ __forceinline__ uint32_t roff(const uint8_t *reg, int k) {
    return ((k & 1) ? (1u << reg[0]) : 0u) | ((k & 2) ? (1u << reg[1]) : 0u) |
           ((k & 4) ? (1u << reg[2]) : 0u) | ((k & 8) ? (1u << reg[3]) : 0u);
}

__device__ __forceinline__ uint32_t regmask(const uint8_t *reg) {
    return (1u << reg[0]) | (1u << reg[1]) | (1u << reg[2]) | (1u << reg[3]);
}

// ------------------------------------------------------------- pass kernel
// Insert a zero bit at each register position (ascending) of tid: the
// phase's local index of the thread's register 0.
__device__ __forceinline__ uint32_t thread_local_index(uint32_t tid, const uint8_t *reg) {
    uint32_t x = tid;
    #pragma unroll
    for (int s = 0; s < 4; ++s) {
        const uint32_t r = reg[s];
        x = ((x >> r) << (r + 1)) | (x & ((1u << r) - 1u));
    }
    return x;
}

// Position of the k-th set bit of mask (k counted from 0). Called with
// wave-uniform arguments, so it compiles to scalar code.
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t mask, uint32_t k) {
    for (uint32_t i = 0; i < k; ++i) mask &= mask - 1;
    return (uint32_t)__builtin_ctzll(mask);
}

// Global offsets of an I/O layout. IO_F4: register slot 0 = local bit 0,
// lanes = local bits 1..6, one 16-byte access per register pair. IO_F2:
// lanes = local bits 0..5, one 8-byte access per register. Waves are the
// remaining non-register local bits. The per-lane part is computed in vector
// registers, everything else is wave-uniform.
struct IoLayout {
    uint32_t lane_off;     // global index bits contributed by the lane
    uint32_t uni_off[16];  // tile base | wave part | register part, per register
};

__device__ __forceinline__ IoLayout io_layout(uint64_t lmask, const uint8_t *reg, uint8_t kind,
                                              uint32_t lane, uint32_t wave, uint32_t m,
                                              uint32_t base) {
    IoLayout io;
    const uint32_t rmask = (1u << reg[0]) | (1u << reg[1]) | (1u << reg[2]) | (1u << reg[3]);
    uint32_t wmask;
    if (kind == IO_F4) {
        const uint32_t g4 = nth_set_bit(lmask, 4), g5 = nth_set_bit(lmask, 5),
                       g6 = nth_set_bit(lmask, 6);
        io.lane_off = ((lane & 7u) << 1) | (((lane >> 3) & 1u) << g4) |
                      (((lane >> 4) & 1u) << g5) | (((lane >> 5) & 1u) << g6);
        wmask = (((1u << m) - 1u) & ~0x7Fu) & ~rmask;
    } else {
        const uint32_t g4 = nth_set_bit(lmask, 4), g5 = nth_set_bit(lmask, 5);
        io.lane_off = (lane & 15u) | (((lane >> 4) & 1u) << g4) | (((lane >> 5) & 1u) << g5);
        wmask = (((1u << m) - 1u) & ~0x3Fu) & ~rmask;
    }
    const uint32_t wl = dpdep32(wave, wmask);
    const uint32_t woff = (uint32_t)dpdep(wl, lmask);
    const uint32_t r0 = 1u << nth_set_bit(lmask, reg[0]);
    const uint32_t r1 = 1u << nth_set_bit(lmask, reg[1]);
    const uint32_t r2 = 1u << nth_set_bit(lmask, reg[2]);
    const uint32_t r3 = 1u << nth_set_bit(lmask, reg[3]);
    #pragma unroll
    for (int k = 0; k < 16; ++k)
        io.uni_off[k] = base | woff | ((k & 1) ? r0 : 0u) | ((k & 2) ? r1 : 0u) |
                        ((k & 4) ? r2 : 0u) | ((k & 8) ? r3 : 0u);
    return io;
}

// I/O layout from a host-computed record: 8 VALU for the lane part, the
// rest is uniform (scalar loads from the record).
__device__ __forceinline__ IoLayout io_from_rec(const IoRec *rec, uint32_t lane, uint32_t wave,
                                                uint32_t base) {
    IoLayout io;
    const uint32_t w0 = uni(*(const QW_CONST uint32_t *)rec);
    const uint32_t kind = w0 & 0xFFu, g4 = (w0 >> 8) & 0xFFu, g5 = (w0 >> 16) & 0xFFu,
                   g6 = w0 >> 24;
    if (kind == IO_F4)
        io.lane_off = ((lane & 7u) << 1) | (((lane >> 3) & 1u) << g4) |
                      (((lane >> 4) & 1u) << g5) | (((lane >> 5) & 1u) << g6);
    else
        io.lane_off = (lane & 15u) | (((lane >> 4) & 1u) << g4) | (((lane >> 5) & 1u) << g5);
    const uint32_t bw = base | uni(ldu(rec->wave_off + wave));
    #pragma unroll
    for (int k = 0; k < 16; ++k) io.uni_off[k] = bw | uni(ldu(rec->reg_off + k));
    return io;
}

__device__ __forceinline__ void io_load(float2 (&v)[16], const void *src_v, const IoLayout &io,
                                        uint8_t kind) {
    if (kind == IO_F4) {
        const QW_GLOBAL float4 *src = gin<float4>(src_v);
        float4 q[8];
        #pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) q[k2] = src[(io.uni_off[2 * k2] >> 1) + (io.lane_off >> 1)];
        #pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
            v[2 * k2] = make_float2(q[k2].x, q[k2].y);
            v[2 * k2 + 1] = make_float2(q[k2].z, q[k2].w);
        }
    } else {
        const QW_GLOBAL float2 *src = gin<float2>(src_v);
        #pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = src[io.uni_off[k] + io.lane_off];
    }
}

__device__ __forceinline__ void io_store(const float2 (&v)[16], void *dst_v, const IoLayout &io,
                                         uint8_t kind) {
    if (kind == IO_F4) {
        QW_GLOBAL float4 *dst = gout<float4>(dst_v);
        #pragma unroll
        for (int k2 = 0; k2 < 8; ++k2)
            dst[(io.uni_off[2 * k2] >> 1) + (io.lane_off >> 1)] =
                make_float4(v[2 * k2].x, v[2 * k2].y, v[2 * k2 + 1].x, v[2 * k2 + 1].y);
    } else {
        QW_GLOBAL float2 *dst = gout<float2>(dst_v);
        #pragma unroll
        for (int k = 0; k < 16; ++k) dst[io.uni_off[k] + io.lane_off] = v[k];
    }
}

// LDS byte address of register k of a thread: swz is linear over GF(2), so
// swz(tl | roff(k)) = swz(tl) ^ swz(roff(k)) with the second part uniform.
__device__ __forceinline__ uint32_t lds_off(uint32_t stl8, const uint8_t *reg, int k) {
    return stl8 ^ (swz(roff(reg, k)) << 3);
}

// Workgroup barrier for LDS exchanges only: waits for this wave's LDS
// operations, not for its global loads/stores, so prefetched loads stay in
// flight across exchanges.
__device__ __forceinline__ void lds_barrier() {
    __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Run the ops of one op range [o, end) on the registers. The next op record
// is requested before the current one is executed (scalar-load prefetch).
__device__ __forceinline__ void run_ops(float2 (&v)[16], const DevOp *ops, uint32_t o,
                                        uint32_t end, uint32_t tl, uint64_t base) {
    if (o >= end) return;
    DevOp nxt = ld_words(ops + o);
    while (o < end) {
        const DevOp op = nxt;
        const uint32_t step = (op.type == OP_DSET) ? 1u + op.b : 1u;
        if (o + step < end) nxt = ld_words(ops + o + step);
        if (op.type == OP_DSET) {
            // diagonal set: register-bit factors per amplitude, all other
            // factors folded into one per-thread complex factor
            float2 ft = make_float2(1.0f, 0.0f);
            DevOp mn = ld_words(ops + o + 1);
            for (uint32_t j = 1; j <= op.b; ++j) {
                const DevOp mm = mn;
                if (j < op.b) mn = ld_words(ops + o + j + 1);
                if (mm.la == LOC_REG) {
                    op_diag(v, mm, tl, base);
                } else {
                    const uint32_t bit = (mm.la == LOC_THREAD) ? ((tl >> mm.a) & 1u)
                                                               : ((uint32_t)(base >> mm.a) & 1u);
                    const float2 f = bit ? make_float2(mm.m[2], mm.m[3])
                                         : make_float2(mm.m[0], mm.m[1]);
                    ft = cmul(f, ft);
                }
            }
            #pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = cmul(ft, v[k]);
        } else {
            run_op(v, op, tl, base);
        }
        o += step;
    }
}

// One-phase passes: no LDS, 256-thread workgroups (a tile is split over
// several workgroups since no data crosses threads), high occupancy.
template <int M>
__global__ __launch_bounds__((1 << (M - 4)) < 256 ? (1 << (M - 4)) : 256)
void pass_kernel_flat(const PassDesc *__restrict__ descs, uint32_t n_descs, uint32_t n,
                      uint32_t items, int remap) {
    constexpr int T = 1 << (M - 4);
    constexpr int WG = T < 256 ? T : 256;
    constexpr int PARTS = T / WG;
    const uint32_t wg_item = item_of(blockIdx.x, gridDim.x, remap);
    const uint32_t item = wg_item / PARTS;
    if (item >= items) return;
    const uint32_t part = wg_item % PARTS;
    const uint32_t p = item % n_descs;
    const uint32_t tile = item / n_descs;
    const PassDesc d = ld_words(descs + p);
    const uint32_t base = uni(ldu(d.tile_base + tile));
    const uint32_t tid = part * WG + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = uni(tid >> 6);
    float2 v[16];
    const PhaseHead ph = ld_phase_head(d.phases);
    const uint32_t tl = thread_local_index(tid, ph.reg);
    const IoLayout io = io_from_rec(d.io_in, lane, wave, base);
    io_load(v, d.src, io, ph.io);
    if (d.flags & PD_SCALE_IN) {
        const double s = *gin<double>(d.scale_in);
        #pragma unroll
        for (int k = 0; k < 16; ++k)
            v[k] = make_float2((float)((double)v[k].x * s), (float)((double)v[k].y * s));
    }
    run_ops(v, d.ops, ph.op_begin, ph.op_end, tl, base);
    io_store(v, d.dst, io_from_rec(d.io_out, lane, wave, base), ph.io);
}

// Multi-phase passes: one 1024-thread workgroup per CU owns a whole tile in
// LDS for exchanges. Workgroups are persistent: each walks a list of items
// and loads the next tile into registers before working on the current one,
// so HBM traffic overlaps the exchanges and arithmetic. The items of XCD x
// (workgroups b with b mod 8 == x) are one contiguous range, so the tasks
// that read the same snapshot tile run on one XCD at about the same time.
template <int M>
__global__ __launch_bounds__(1 << (M - 4)) void pass_kernel_lds(const PassDesc *__restrict__ descs,
                                                                uint32_t n_descs, uint32_t n,
                                                                uint32_t items) {
    constexpr int T = 1 << (M - 4);
    __shared__ float2 lds[1 << M];
    __shared__ double red[T / 64 + 1];
    const uint32_t w = blockIdx.x, x = w & 7u, j = w >> 3, wpx = gridDim.x >> 3;
    const uint32_t per = (items + 7u) >> 3;
    const uint32_t first = x * per;
    const uint32_t last = (first + per < items) ? first + per : items;
    uint32_t item = first + j;
    if (item >= last) return;
    const uint64_t full = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = uni(tid >> 6);
    char *lb = reinterpret_cast<char *>(lds);

    float2 nv[16];
    {
        const PassDesc d0 = ld_words(descs + item % n_descs);
        const uint32_t base0 = uni(ldu(d0.tile_base + item / n_descs));
        const IoLayout io0 = io_from_rec(d0.io_in, lane, wave, base0);
        io_load(nv, d0.src, io0, ld_phase_head(d0.phases).io);
    }
    while (true) {
        float2 v[16];
        #pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = nv[k];
        const uint32_t p = item % n_descs;
        const uint32_t tile = item / n_descs;
        const PassDesc d = ld_words(descs + p);
        const uint32_t base = uni(ldu(d.tile_base + tile));
        const uint32_t next = item + wpx;
        const bool has_next = next < last;
        if (has_next) {
            const PassDesc dn = ld_words(descs + next % n_descs);
            const uint32_t basen = uni(ldu(dn.tile_base + next / n_descs));
            const IoLayout ion = io_from_rec(dn.io_in, lane, wave, basen);
            io_load(nv, dn.src, ion, ld_phase_head(dn.phases).io);
        }
        if (d.flags & PD_SCALE_IN) {
            const double s = *gin<double>(d.scale_in);
            #pragma unroll
            for (int k = 0; k < 16; ++k)
                v[k] = make_float2((float)((double)v[k].x * s), (float)((double)v[k].y * s));
        }
        PhaseHead ph = ld_phase_head(d.phases);
        uint32_t tl = thread_local_index(tid, ph.reg);
        const uint32_t nph = d.n_phases;
        for (uint32_t pi = 0; pi < nph; ++pi) {
            if (pi > 0) {
                const uint32_t *off_prev = d.phases[pi - 1].lds_off;
                const uint32_t *off_next = d.phases[pi].lds_off;
                const uint32_t stl8 = swz(tl) << 3;
                lds_barrier();
                #pragma unroll
                for (int k = 0; k < 16; ++k)
                    *reinterpret_cast<float2 *>(lb + (stl8 ^ uni(ldu(off_prev + k)))) = v[k];
                lds_barrier();
                ph = ld_phase_head(d.phases + pi);
                tl = thread_local_index(tid, ph.reg);
                const uint32_t ntl8 = swz(tl) << 3;
                #pragma unroll
                for (int k = 0; k < 16; ++k)
                    v[k] = *reinterpret_cast<const float2 *>(lb + (ntl8 ^ uni(ldu(off_next + k))));
            }
            run_ops(v, d.ops, ph.op_begin, ph.op_end, tl, base);
        }
        if (d.flags & PD_NORM_OUT) {
            double s = 0.0;
            #pragma unroll
            for (int k = 0; k < 16; ++k) {
                const double xx = v[k].x, yy = v[k].y;
                s = fma(xx, xx, s);
                s = fma(yy, yy, s);
            }
            s = block_sum<T>(s, red);
            if (tid == 0) gout<double>(d.norm_part)[tile] = s;
        }
        io_store(v, d.dst, io_from_rec(d.io_out, lane, wave, base), ph.io);
        if (!has_next) break;
        item = next;
        lds_barrier();  // the next tile's first exchange reuses the LDS buffer
    }
}

// ------------------------------------------------------------- small states
// n < 10: one workgroup of 64 threads holds the whole state in LDS and runs
// the ops one at a time (every bit is local).
__global__ __launch_bounds__(64) void small_pass_kernel(const PassDesc *__restrict__ descs,
                                                        uint32_t n) {
    __shared__ float2 s[512];
    __shared__ double red[2];
    const PassDesc &d = descs[blockIdx.x];
    const uint32_t dim = 1u << n;
    const uint32_t tid = threadIdx.x;
    const float2 *src = reinterpret_cast<const float2 *>(d.src);
    float2 *dst = reinterpret_cast<float2 *>(d.dst);
    const double sc = (d.flags & PD_SCALE_IN) ? *d.scale_in : 1.0;
    for (uint32_t i = tid; i < dim; i += 64) {
        float2 a = src[i];
        if (d.flags & PD_SCALE_IN) a = make_float2((float)((double)a.x * sc), (float)((double)a.y * sc));
        s[i] = a;
    }
    __syncthreads();
    for (uint32_t o = 0; o < d.n_ops; ++o) {
        const DevOp op = d.ops[o];
        if (op.type == OP_DSET) continue;  // members follow as plain diagonal ops
        if (op.type == OP_U || op.type == OP_PERM || op.type == OP_CX || op.type == OP_UR) {
            const uint32_t bit = 1u << op.a;
            for (uint32_t pr = tid; pr < dim / 2; pr += 64) {
                const uint32_t i0 = ((pr >> op.a) << (op.a + 1)) | (pr & (bit - 1));
                const uint32_t i1 = i0 | bit;
                const float2 x = s[i0], y = s[i1];
                if (op.type == OP_U) {
                    s[i0] = cmad2(make_float2(op.m[0], op.m[1]), x, make_float2(op.m[2], op.m[3]), y);
                    s[i1] = cmad2(make_float2(op.m[4], op.m[5]), x, make_float2(op.m[6], op.m[7]), y);
                } else if (op.type == OP_UR) {
                    s[i0] = make_float2(fmaf(op.m[0], x.x, op.m[1] * y.x), fmaf(op.m[0], x.y, op.m[1] * y.y));
                    s[i1] = make_float2(fmaf(op.m[2], x.x, op.m[3] * y.x), fmaf(op.m[2], x.y, op.m[3] * y.y));
                } else if (op.type == OP_PERM) {
                    s[i0] = cmul(make_float2(op.m[0], op.m[1]), y);
                    s[i1] = cmul(make_float2(op.m[2], op.m[3]), x);
                } else if ((i0 >> op.b) & 1u) {
                    s[i0] = y;
                    s[i1] = x;
                }
            }
        } else if (op.type == OP_DIAG) {
            const float2 d0 = make_float2(op.m[0], op.m[1]), d1 = make_float2(op.m[2], op.m[3]);
            for (uint32_t i = tid; i < dim; i += 64) s[i] = cmul(((i >> op.a) & 1u) ? d1 : d0, s[i]);
        } else if (op.type == OP_CZ) {
            for (uint32_t i = tid; i < dim; i += 64)
                if (((i >> op.a) & 1u) && ((i >> op.b) & 1u)) s[i] = make_float2(-s[i].x, -s[i].y);
        }
        __syncthreads();
    }
    if (d.flags & PD_NORM_OUT) {
        double acc = 0.0;
        for (uint32_t i = tid; i < dim; i += 64) {
            const double x = s[i].x, y = s[i].y;
            acc = fma(x, x, acc);
            acc = fma(y, y, acc);
        }
        acc = block_sum<64>(acc, red);
        if (tid == 0) d.norm_part[0] = acc;
    }
    for (uint32_t i = tid; i < dim; i += 64) dst[i] = s[i];
}

// ------------------------------------------------------------- renorm
// For every descriptor with PD_NORM_OUT: scale_out = 1/sqrt(sum of tiles).
__global__ __launch_bounds__(256) void norm_finalize_kernel(const PassDesc *__restrict__ descs,
                                                            uint32_t tiles) {
    __shared__ double red[5];
    const PassDesc &d = descs[blockIdx.x];
    if (!(d.flags & PD_NORM_OUT)) return;
    double s = 0.0;
    for (uint32_t t = threadIdx.x; t < tiles; t += 256) s += d.norm_part[t];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) *d.scale_out = 1.0 / sqrt(s);
}

// ------------------------------------------------------------- init / copy
__global__ __launch_bounds__(256) void init_kernel(float4 *base, uint64_t slot_f4,
                                                   uint64_t total_f4) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < total_f4;
         i += (uint64_t)gridDim.x * 256) {
        base[i] = make_float4((i % slot_f4) == 0 ? 1.0f : 0.0f, 0.0f, 0.0f, 0.0f);
    }
}

__global__ __launch_bounds__(256) void copy_kernel(float4 *__restrict__ dst,
                                                   const float4 *__restrict__ src,
                                                   uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * 256)
        dst[i] = src[i];
}

// ------------------------------------------------------------- expectation
// Small states (n < 10): one workgroup per slot, the state staged in LDS;
// every term is summed over all amplitudes in FP64.
__global__ __launch_bounds__(64) void reduce_small_kernel(const ReduceDescSmall *__restrict__ descs,
                                                          uint32_t n) {
    __shared__ float2 s[512];
    __shared__ double red[2];
    const ReduceDescSmall &d = descs[blockIdx.x];
    const uint32_t dim = 1u << n;
    const float2 *psi = reinterpret_cast<const float2 *>(d.psi);
    for (uint32_t i = threadIdx.x; i < dim; i += 64) s[i] = psi[i];
    __syncthreads();
    for (uint32_t j = 0; j < d.n_terms; ++j) {
        const TermSmall t = d.terms[j];
        double acc = 0.0;
        for (uint32_t l = threadIdx.x; l < dim; l += 64) {
            const float2 a = s[l], b = s[l ^ t.x];
            const double re = fma((double)b.x, (double)a.x, (double)b.y * (double)a.y);
            const double im = fma((double)b.x, (double)a.y, -((double)b.y * (double)a.x));
            double val;
            switch (t.ny_mod4) {
            case 0: val = re; break;
            case 1: val = -im; break;
            case 2: val = -re; break;
            default: val = im; break;
            }
            acc += (__popc(l & t.z) & 1u) ? -val : val;
        }
        acc = block_sum<64>(acc, red);
        if (threadIdx.x == 0) d.part[t.out_index] = acc;
    }
}

// Sum over one thread's register pairs of sign_k * Re or Im of
// conj(v[k ^ X]) v[k]; each unordered pair is counted once (the caller
// doubles it). FP32 products and an FP32 sum over at most 16 values.
template <int X, bool ODD>
__device__ __forceinline__ float pair_sum(const float2 (&v)[16], uint32_t smask) {
    static_assert(X > 0 && X < 16, "off-diagonal register mask");
    constexpr int lead = (X & 8) ? 8 : (X & 4) ? 4 : (X & 2) ? 2 : 1;
    float acc = 0.0f;
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k & lead) continue;
        const float2 a = v[k], b = v[k ^ X];
        float t;
        if constexpr (ODD) t = fmaf(b.x, a.y, -(b.y * a.x));
        else t = fmaf(b.x, a.x, b.y * a.y);
        const float sg = ((smask >> k) & 1u) ? -1.0f : 1.0f;
        acc = fmaf(sg, t, acc);
    }
    return acc;
}

template <bool ODD>
__device__ __forceinline__ float pair_sum_x(uint32_t xr, const float2 (&v)[16], uint32_t smask) {
    switch (xr) {
    case 1: return pair_sum<1, ODD>(v, smask);
    case 2: return pair_sum<2, ODD>(v, smask);
    case 3: return pair_sum<3, ODD>(v, smask);
    case 4: return pair_sum<4, ODD>(v, smask);
    case 5: return pair_sum<5, ODD>(v, smask);
    case 6: return pair_sum<6, ODD>(v, smask);
    case 7: return pair_sum<7, ODD>(v, smask);
    case 8: return pair_sum<8, ODD>(v, smask);
    case 9: return pair_sum<9, ODD>(v, smask);
    case 10: return pair_sum<10, ODD>(v, smask);
    case 11: return pair_sum<11, ODD>(v, smask);
    case 12: return pair_sum<12, ODD>(v, smask);
    case 13: return pair_sum<13, ODD>(v, smask);
    case 14: return pair_sum<14, ODD>(v, smask);
    default: return pair_sum<15, ODD>(v, smask);
    }
}

// Signed sum of |v[k]|^2 (diagonal terms).
__device__ __forceinline__ float diag_sum(const float (&pr)[16], uint32_t smask) {
    float acc = 0.0f;
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float sg = ((smask >> k) & 1u) ? -1.0f : 1.0f;
        acc = fmaf(sg, pr[k], acc);
    }
    return acc;
}

// Butterfly reduction of 8 per-lane partials (positions 0..7) across the
// wave in FP64: after the xor 1/2/4 steps lane l holds position
// 4(l&1) + 2((l>>1)&1) + ((l>>2)&1); xor 8/16/32 complete the wave sum.
__device__ __forceinline__ double wave_reduce8(const float (&q)[8], uint32_t lane) {
    double e[8];
    #pragma unroll
    for (int i = 0; i < 8; ++i) e[i] = (double)q[i];
    const bool b0 = lane & 1u, b1 = lane & 2u, b2 = lane & 4u;
    double f[4];
    #pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double mine = b0 ? e[4 + i] : e[i];
        const double other = b0 ? e[i] : e[4 + i];
        f[i] = mine + __shfl_xor(other, 1, 64);
    }
    double g[2];
    #pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double mine = b1 ? f[2 + i] : f[i];
        const double other = b1 ? f[i] : f[2 + i];
        g[i] = mine + __shfl_xor(other, 2, 64);
    }
    double h;
    {
        const double mine = b2 ? g[1] : g[0];
        const double other = b2 ? g[0] : g[1];
        h = mine + __shfl_xor(other, 4, 64);
    }
    h += __shfl_xor(h, 8, 64);
    h += __shfl_xor(h, 16, 64);
    h += __shfl_xor(h, 32, 64);
    return h;
}


// Register-phase reducer. One workgroup per (slot, group, tile): the tile is
// loaded with the I/O layout, staged once in LDS, and re-read with each
// phase's layout. For up to 8 terms at a time every thread holds one FP32
// partial per term; they are converted to FP64 and summed across the wave
// by a butterfly that halves the number of values per lane at each of the
// first three steps (fixed order); wave sums are added in wave order.
template <int M>
__global__ __launch_bounds__(1 << (M - 4)) void reduce_kernel(const ReduceDesc *__restrict__ descs,
                                                              uint32_t n_descs, uint32_t n,
                                                              uint32_t items) {
    constexpr int T = 1 << (M - 4);
    constexpr int W = T / 64;
    __shared__ float2 lds[1 << M];
    __shared__ double red[W * kMaxGroupTerms];
    const uint32_t item = blockIdx.x;
    if (item >= items) return;
    const uint32_t p = item % n_descs;
    const uint64_t tile = item / n_descs;
    const ReduceDesc d = ld_words(descs + p);
    const uint64_t lmask = d.local_mask;
    const uint64_t full = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    const uint64_t base = dpdep(tile, full & ~lmask);
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;

    float2 v[16];
    {
        // I/O layout: register slots = local bits {0, 7, 8, 9}
        const uint8_t io[4] = {0, 7, 8, 9};
        const uint32_t tl = thread_local_index(tid, io);
        const IoLayout lay = io_layout(lmask, io, IO_F4, lane, uni(tid >> 6), M, (uint32_t)base);
        io_load(v, d.psi, lay, IO_F4);
        const uint32_t stl8 = swz(tl) << 3;
        char *lb = reinterpret_cast<char *>(lds);
        #pragma unroll
        for (int k = 0; k < 16; ++k)
            *reinterpret_cast<float2 *>(lb + lds_off(stl8, io, k)) = v[k];
    }
    __syncthreads();

    for (uint32_t pi = 0; pi < d.n_phases; ++pi) {
        const RedPhase ph = ld_words(d.phases + pi);
        const uint32_t tl = thread_local_index(tid, ph.reg);
        if (!ph.diag) {
            const uint32_t stl8 = swz(tl) << 3;
            const char *lb = reinterpret_cast<const char *>(lds);
            #pragma unroll
            for (int k = 0; k < 16; ++k)
                v[k] = *reinterpret_cast<const float2 *>(lb + lds_off(stl8, ph.reg, k));
        }
        float pr[16];
        if (ph.diag) {
            #pragma unroll
            for (int k = 0; k < 16; ++k) pr[k] = fmaf(v[k].x, v[k].x, v[k].y * v[k].y);
        }
        for (uint32_t j0 = ph.t_begin; j0 < ph.t_end; j0 += 8) {
            const uint32_t nb = (ph.t_end - j0 < 8u) ? (ph.t_end - j0) : 8u;
            float q[8];
            #pragma unroll
            for (int i = 0; i < 8; ++i) q[i] = 0.0f;
            for (uint32_t j = 0; j < nb; ++j) {
                const TermDev t = ld_words(d.terms + j0 + j);
                float a;
                if (ph.diag) {
                    a = diag_sum(pr, t.smask);
                } else {
                    a = t.odd ? pair_sum_x<true>(t.xr, v, t.smask)
                              : pair_sum_x<false>(t.xr, v, t.smask);
                    a *= 2.0f;
                }
                const uint32_t par = (t.neg ^ __popc(tl & t.zt) ^ (uint32_t)__popcll(base & t.zg)) & 1u;
                if (par) a = -a;
                #pragma unroll
                for (int i = 7; i > 0; --i) q[i] = q[i - 1];
                q[0] = a;
            }
            const double h = wave_reduce8(q, lane);
            if (lane < 8u) {
                const uint32_t pos = 4u * (lane & 1u) + 2u * ((lane >> 1) & 1u) + ((lane >> 2) & 1u);
                if (pos < nb) {
                    const uint32_t j = nb - 1u - pos;
                    red[wave * kMaxGroupTerms + gin<TermDev>(d.terms)[j0 + j].col] = h;
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t c = tid; c < d.n_terms; c += T) {
        double s = 0.0;
        for (int w = 0; w < W; ++w) s += red[w * kMaxGroupTerms + c];
        gout<double>(d.part)[tile * d.n_terms_total + gin<uint32_t>(d.cols)[c]] = s;
    }
}

// out[s] = sum_j coeff[j] * (sum over tiles of part[s][tile][j]); one
// workgroup per slot; term sums use a fixed tree, terms are added in order.
__global__ __launch_bounds__(256) void expect_finalize_kernel(const double *__restrict__ part,
                                                              const double *__restrict__ coeff,
                                                              uint32_t n_terms, uint32_t tiles,
                                                              double *__restrict__ out) {
    __shared__ double red[5];
    const uint32_t s = blockIdx.x;
    const double *ps = part + (uint64_t)s * tiles * n_terms;
    double e = 0.0;
    for (uint32_t j = 0; j < n_terms; ++j) {
        double acc = 0.0;
        for (uint32_t t = threadIdx.x; t < tiles; t += 256) acc += ps[(uint64_t)t * n_terms + j];
        acc = block_sum<256>(acc, red);
        if (threadIdx.x == 0) e = fma(coeff[j], acc, e);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[s] = e;
}

// ------------------------------------------------------------- sampling
// SplitMix64 output function (Steele, Lea and Flood 2014) used as a hash of
// the counter (seed, task, shot).
__device__ __forceinline__ uint64_t splitmix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// chunk sums of |psi|^2 (FP64), chunk = 2^C amplitudes; grid (chunks, slots)
__global__ __launch_bounds__(256) void chunk_sum_kernel(const float2 *const *__restrict__ slots,
                                                        uint32_t C, uint32_t chunks,
                                                        double *__restrict__ csum) {
    __shared__ double red[5];
    const uint32_t c = blockIdx.x, s = blockIdx.y;
    const float2 *psi = slots[s] + ((uint64_t)c << C);
    const uint32_t len = 1u << C;
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < len; i += 256) {
        const double x = psi[i].x, y = psi[i].y;
        acc = fma(x, x, acc);
        acc = fma(y, y, acc);
    }
    acc = block_sum<256>(acc, red);
    if (threadIdx.x == 0) csum[(uint64_t)s * chunks + c] = acc;
}

// exclusive prefix of chunk sums per slot (in place into cpre) + total
__global__ __launch_bounds__(256) void chunk_scan_kernel(const double *__restrict__ csum,
                                                         uint32_t chunks,
                                                         double *__restrict__ cpre,
                                                         double *__restrict__ total) {
    __shared__ double seg[256];
    const uint32_t s = blockIdx.x;
    const double *in = csum + (uint64_t)s * chunks;
    double *outp = cpre + (uint64_t)s * chunks;
    const uint32_t per = (chunks + 255) / 256;
    const uint32_t b0 = threadIdx.x * per;
    const uint32_t b1 = (b0 + per < chunks) ? b0 + per : chunks;
    double acc = 0.0;
    for (uint32_t c = b0; c < b1; ++c) acc += in[c];
    seg[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int k = 0; k < 256; ++k) {
            const double t = seg[k];
            seg[k] = run;
            run += t;
        }
        total[s] = run;
    }
    __syncthreads();
    double run = seg[threadIdx.x];
    for (uint32_t c = b0; c < b1; ++c) {
        outp[c] = run;
        run += in[c];
    }
}

// one thread per (slot, shot)
__global__ __launch_bounds__(256) void draw_kernel(const float2 *const *__restrict__ slots,
                                                   uint32_t n_slots, uint32_t n, uint32_t C,
                                                   uint32_t chunks, const double *__restrict__ cpre,
                                                   const double *__restrict__ total,
                                                   uint64_t seed, uint64_t task_base,
                                                   uint32_t shots, uint32_t *__restrict__ out) {
    const uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (uint64_t)n_slots * shots) return;
    const uint32_t s = (uint32_t)(gid / shots), sh = (uint32_t)(gid % shots);
    const uint64_t h = splitmix(seed ^ (((task_base + s) << 32) + sh));
    const double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
    const double target = u * total[s];
    const double *pre = cpre + (uint64_t)s * chunks;
    // last chunk with pre[c] <= target
    uint32_t lo = 0, hi = chunks - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= target) lo = mid;
        else hi = mid - 1;
    }
    const float2 *psi = slots[s];
    const uint64_t dim = 1ull << n;
    uint64_t last_nz = 0;
    uint64_t i = (uint64_t)lo << C;
    double run = pre[lo];
    uint32_t result = 0xFFFFFFFFu;
    for (; i < dim; ++i) {
        const double x = psi[i].x, y = psi[i].y;
        const double pr = fma(x, x, y * y);
        if (pr > 0.0) last_nz = i;
        run += pr;
        if (run > target) {
            result = (uint32_t)i;
            break;
        }
        if (((i + 1) & ((1ull << C) - 1)) == 0 && (i + 1) < dim) {
            // crossed into the next chunk: resynchronise with its prefix
            const uint64_t nc = (i + 1) >> C;
            if (pre[nc] > target) {
                result = (uint32_t)last_nz;
                break;
            }
            run = pre[nc];
        }
    }
    if (result == 0xFFFFFFFFu) result = (uint32_t)last_nz;
    out[gid] = result;
}

// ------------------------------------------------------------- launchers
static_assert(sizeof(float2) == 8, "float2");

template <int M>
static hipError_t launch_pass_m(hipStream_t st, const PassDesc *d, uint32_t n_descs, uint32_t n,
                                uint32_t tiles, int remap, bool use_lds, uint32_t n_cu) {
    const uint64_t items64 = (uint64_t)n_descs * tiles;
    if (items64 == 0) return hipSuccess;
    constexpr int T = 1 << (M - 4);
    constexpr int WG_FLAT = T < 256 ? T : 256;
    if (items64 * (T / WG_FLAT) > 0x7FFFFFF8ull) return hipErrorInvalidValue;
    const uint32_t items = (uint32_t)items64;
    if (use_lds) {
        // one persistent workgroup per CU (a multiple of 8 for the XCD split)
        uint32_t grid = n_cu;
        const uint32_t need = ((items + 7u) / 8u) * 8u;
        if (need < grid) grid = need;
        grid = ((grid + 7u) / 8u) * 8u;
        hipLaunchKernelGGL(pass_kernel_lds<M>, dim3(grid), dim3(T), 0, st, d, n_descs, n, items);
    } else {
        uint32_t grid = (uint32_t)(items64 * (T / WG_FLAT));
        if (remap) grid = ((grid + 7u) / 8u) * 8u;
        hipLaunchKernelGGL(pass_kernel_flat<M>, dim3(grid), dim3(WG_FLAT), 0, st, d, n_descs, n,
                           items, remap);
    }
    return hipGetLastError();
}

static uint32_t cu_count() {
    static uint32_t cached = 0;
    if (cached) return cached;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
        cached = (uint32_t)cus;
    else
        cached = 256;
    return cached;
}

hipError_t launch_pass(hipStream_t st, const PassDesc *d, uint32_t n_descs, uint32_t n,
                       uint32_t m, int remap, bool use_lds) {
    if (n_descs == 0) return hipSuccess;
    if (m < (uint32_t)kMinTileBits) {
        hipLaunchKernelGGL(small_pass_kernel, dim3(n_descs), dim3(64), 0, st, d, n);
        return hipGetLastError();
    }
    const uint32_t tiles = 1u << (n - m);
    const uint32_t ncu = cu_count();
    switch (m) {
    case 10: return launch_pass_m<10>(st, d, n_descs, n, tiles, remap, use_lds, ncu);
    case 11: return launch_pass_m<11>(st, d, n_descs, n, tiles, remap, use_lds, ncu);
    case 12: return launch_pass_m<12>(st, d, n_descs, n, tiles, remap, use_lds, ncu);
    case 13: return launch_pass_m<13>(st, d, n_descs, n, tiles, remap, use_lds, ncu);
    case 14: return launch_pass_m<14>(st, d, n_descs, n, tiles, remap, use_lds, ncu);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_norm_finalize(hipStream_t st, const PassDesc *d, uint32_t n_descs,
                                uint32_t tiles) {
    if (n_descs == 0) return hipSuccess;
    hipLaunchKernelGGL(norm_finalize_kernel, dim3(n_descs), dim3(256), 0, st, d, tiles);
    return hipGetLastError();
}

hipError_t launch_init(hipStream_t st, void *base, uint32_t n, uint32_t n_slots) {
    const uint64_t slot_f4 = (1ull << n) / 2;
    if (slot_f4 == 0) {
        // n == 0 is rejected by the host; keep the kernel safe anyway
        return hipErrorInvalidValue;
    }
    const uint64_t total = slot_f4 * n_slots;
    uint64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(init_kernel, dim3((uint32_t)blocks), dim3(256), 0, st,
                       reinterpret_cast<float4 *>(base), slot_f4, total);
    return hipGetLastError();
}

hipError_t launch_copy(hipStream_t st, void *dst, const void *src, uint64_t bytes) {
    const uint64_t count = bytes / 16;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_kernel, dim3((uint32_t)blocks), dim3(256), 0, st,
                       reinterpret_cast<float4 *>(dst), reinterpret_cast<const float4 *>(src),
                       count);
    return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t st, const ReduceDesc *d, uint32_t n_descs, uint32_t n,
                         uint32_t M) {
    const uint64_t tiles = 1ull << (n - M);
    const uint64_t items = (uint64_t)n_descs * tiles;
    if (items == 0) return hipSuccess;
    if (items > 0x7FFFFFFFull) return hipErrorInvalidValue;
    switch (M) {
#define QW_RED(MM)                                                                       \
    case MM:                                                                             \
        hipLaunchKernelGGL(reduce_kernel<MM>, dim3((uint32_t)items), dim3(1 << (MM - 4)), 0, st, \
                           d, n_descs, n, (uint32_t)items);                              \
        break;
        QW_RED(10) QW_RED(11) QW_RED(12) QW_RED(13) QW_RED(14)
#undef QW_RED
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_small(hipStream_t st, const ReduceDescSmall *d, uint32_t n_descs,
                               uint32_t n) {
    if (n_descs == 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_small_kernel, dim3(n_descs), dim3(64), 0, st, d, n);
    return hipGetLastError();
}

hipError_t launch_expect_finalize(hipStream_t st, const double *part, const double *coeff,
                                  uint32_t n_terms, uint32_t tiles, uint32_t n_slots,
                                  double *out) {
    if (n_slots == 0) return hipSuccess;
    hipLaunchKernelGGL(expect_finalize_kernel, dim3(n_slots), dim3(256), 0, st, part, coeff,
                       n_terms, tiles, out);
    return hipGetLastError();
}

hipError_t launch_sample(hipStream_t st, const float2 *const *slots, uint32_t n_slots,
                         uint32_t n, double *csum, double *cpre, double *total, uint64_t seed,
                         uint64_t task_base, uint32_t shots, uint32_t *out) {
    const uint32_t C = n < 10 ? n : 10;
    const uint32_t chunks = 1u << (n - C);
    hipLaunchKernelGGL(chunk_sum_kernel, dim3(chunks, n_slots), dim3(256), 0, st, slots, C, chunks,
                       csum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(chunk_scan_kernel, dim3(n_slots), dim3(256), 0, st, csum, chunks, cpre,
                       total);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t threads = (uint64_t)n_slots * shots;
    if (threads == 0) return hipSuccess;
    hipLaunchKernelGGL(draw_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, st,
                       slots, n_slots, n, C, chunks, cpre, total, seed, task_base, shots, out);
    return hipGetLastError();
}

hipError_t kernels_init() { return hipSuccess; }

}  // namespace qw
