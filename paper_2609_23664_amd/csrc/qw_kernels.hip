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

#include <algorithm>
#include <cstdint>

#include "qw_internal.h"
#include "qw_dev.h"
#include "qw_kernels.h"

namespace qw {

// ------------------------------------------------------------- interpreter
// The interpreted pass kernels read each op record at run time and branch to
// the matching tile operation of qw_dev.h; generated kernels call the same
// operations with the record contents fixed at compile time.

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

// Value of a thread or global operand bit (never a register bit).
__device__ __forceinline__ bool opbit_tg(uint8_t loc, uint8_t bit, uint32_t tl, uint64_t base) {
    return loc == LOC_THREAD ? ((tl >> bit) & 1u) : ((uint32_t)(base >> bit) & 1u);
}

#define QW_SLOT4(FN, SEL, ...)                                    \
    switch (SEL) {                                                \
    case 0: FN<0>(__VA_ARGS__); break;                            \
    case 1: FN<1>(__VA_ARGS__); break;                            \
    case 2: FN<2>(__VA_ARGS__); break;                            \
    default: FN<3>(__VA_ARGS__); break;                           \
    }
#define QW_LANE6(FN, SEL, ...)                                    \
    switch (SEL) {                                                \
    case 0: FN<0>(__VA_ARGS__); break;                            \
    case 1: FN<1>(__VA_ARGS__); break;                            \
    case 2: FN<2>(__VA_ARGS__); break;                            \
    case 3: FN<3>(__VA_ARGS__); break;                            \
    case 4: FN<4>(__VA_ARGS__); break;                            \
    default: FN<5>(__VA_ARGS__); break;                           \
    }

// CX / CZ with a register control slot chosen at run time.
template <int S>
__device__ __forceinline__ void cx_rr_s(float2 (&v)[16], uint32_t c) {
    switch (c) {
    case 0: cx_rr<S, 0>(v); break;
    case 1: cx_rr<S, 1>(v); break;
    case 2: cx_rr<S, 2>(v); break;
    default: cx_rr<S, 3>(v); break;
    }
}
template <int J>
__device__ __forceinline__ void cx_lr_s(float2 (&v)[16], uint32_t c) {
    switch (c) {
    case 0: cx_lr<J, 0>(v); break;
    case 1: cx_lr<J, 1>(v); break;
    case 2: cx_lr<J, 2>(v); break;
    default: cx_lr<J, 3>(v); break;
    }
}
template <int S>
__device__ __forceinline__ void cz_rr_s(float2 (&v)[16], uint32_t c) {
    switch (c) {
    case 0: cz_rr<S, 0>(v); break;
    case 1: cz_rr<S, 1>(v); break;
    case 2: cz_rr<S, 2>(v); break;
    default: cz_rr<S, 3>(v); break;
    }
}

template <int F>
__device__ __forceinline__ void urt_r_s(float2 (&v)[16], uint32_t slot, float t) {
    switch (slot) {
    case 0: urt_r<0, F>(v, t); break;
    case 1: urt_r<1, F>(v, t); break;
    case 2: urt_r<2, F>(v, t); break;
    default: urt_r<3, F>(v, t); break;
    }
}
template <int F>
__device__ __forceinline__ void urt_l_s(float2 (&v)[16], uint32_t j, float t, uint32_t lane) {
    switch (j) {
    case 0: urt_l<0, F>(v, t, lane); break;
    case 1: urt_l<1, F>(v, t, lane); break;
    case 2: urt_l<2, F>(v, t, lane); break;
    case 3: urt_l<3, F>(v, t, lane); break;
    case 4: urt_l<4, F>(v, t, lane); break;
    default: urt_l<5, F>(v, t, lane); break;
    }
}

// One op record (not OP_DSET) on the registers of a phase.
__device__ __forceinline__ void run_op(float2 (&v)[16], const DevOp &op, const DevOp *ops,
                                       uint32_t j, uint32_t tl, uint64_t base) {
    const uint32_t lane = threadIdx.x & 63u;
    if (op.la == LOC_LANE) {
        switch (op.type) {
        case OP_U:
            QW_LANE6(u_l, op.sa, v, opc(ops, j, 0), opc(ops, j, 1), opc(ops, j, 2), opc(ops, j, 3), lane)
            return;
        case OP_UR:
            QW_LANE6(ur_l, op.sa, v, opm(ops, j, 0), opm(ops, j, 1), opm(ops, j, 2), opm(ops, j, 3), lane)
            return;
        case OP_URD: {
            const Urd e = urd_entries(ops, j);
            QW_LANE6(ur_l, op.sa, v, e.a, e.b, e.c, e.d, lane)
            return;
        }
        case OP_URT:
            if (op.b) urt_l_s<1>(v, op.sa, opm(ops, j, 0), lane);
            else urt_l_s<0>(v, op.sa, opm(ops, j, 0), lane);
            return;
        case OP_PERM:
            QW_LANE6(perm_l, op.sa, v, opc(ops, j, 0), opc(ops, j, 1), lane)
            return;
        case OP_CX:
            if (op.lb == LOC_REG) {
                QW_LANE6(cx_lr_s, op.sa, v, op.sb)
            } else {
                const bool c = opbit_tg(op.lb, op.b, tl, base);
                QW_LANE6(cx_lb, op.sa, v, c)
            }
            return;
        default: return;
        }
    }
    switch (op.type) {
    case OP_URT:
        if (op.b) urt_r_s<1>(v, op.sa, opm(ops, j, 0));
        else urt_r_s<0>(v, op.sa, opm(ops, j, 0));
        break;
    case OP_UR:
        QW_SLOT4(ur_r, op.sa, v, opm(ops, j, 0), opm(ops, j, 1), opm(ops, j, 2), opm(ops, j, 3))
        break;
    case OP_URD: {
        const Urd e = urd_entries(ops, j);
        QW_SLOT4(ur_r, op.sa, v, e.a, e.b, e.c, e.d)
        break;
    }
    case OP_U:
        QW_SLOT4(u_r, op.sa, v, opc(ops, j, 0), opc(ops, j, 1), opc(ops, j, 2), opc(ops, j, 3))
        break;
    case OP_PERM:
        QW_SLOT4(perm_r, op.sa, v, opc(ops, j, 0), opc(ops, j, 1))
        break;
    case OP_CX:
        if (op.lb == LOC_REG) {
            QW_SLOT4(cx_rr_s, op.sa, v, op.sb)
        } else {
            const bool c = opbit_tg(op.lb, op.b, tl, base);
            QW_SLOT4(cx_rb, op.sa, v, c)
        }
        break;
    case OP_DIAG:
        if (op.la == LOC_REG) {
            QW_SLOT4(diag_r, op.sa, v, opc(ops, j, 0), opc(ops, j, 1))
        } else {
            diag_b(v, opbit_tg(op.la, op.a, tl, base), opc(ops, j, 0), opc(ops, j, 1));
        }
        break;
    case OP_CZ:
        if (op.la == LOC_REG && op.lb == LOC_REG) {
            QW_SLOT4(cz_rr_s, op.sa, v, op.sb)
        } else if (op.la == LOC_REG) {
            const bool c = opbit_tg(op.lb, op.b, tl, base);
            QW_SLOT4(cz_rb, op.sa, v, c)
        } else if (op.lb == LOC_REG) {
            const bool c = opbit_tg(op.la, op.a, tl, base);
            QW_SLOT4(cz_rb, op.sb, v, c)
        } else {
            cz_bb(v, opbit_tg(op.la, op.a, tl, base) && opbit_tg(op.lb, op.b, tl, base));
        }
        break;
    default: break;
    }
}

// ------------------------------------------------------------- pass kernel
__device__ __forceinline__ uint32_t thread_local_index(uint32_t tid, const uint8_t *reg) {
    return thread_local_index(tid, reg[0], reg[1], reg[2], reg[3]);
}

// Global offsets of an I/O layout. IO_F4: register slot 0 = local bit 0,
// lanes = local bits 1..6, one 16-byte access per register pair. IO_F2:
// lanes = local bits 0..5, one 8-byte access per register. Waves are the
// remaining non-register local bits.
struct IoLayout {
    uint32_t lane_off;     // global index bits contributed by the lane
    uint32_t uni_off[16];  // tile base | wave part | register part, per register
};

// Position of the k-th set bit of mask (k counted from 0). Called with
// wave-uniform arguments, so it compiles to scalar code.
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t mask, uint32_t k) {
    for (uint32_t i = 0; i < k; ++i) mask &= mask - 1;
    return (uint32_t)__builtin_ctzll(mask);
}

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

// Local index offset of register k for a phase with register bits reg[].
__device__ __forceinline__ uint32_t roff(const uint8_t *reg, int k) {
    return ((k & 1) ? (1u << reg[0]) : 0u) | ((k & 2) ? (1u << reg[1]) : 0u) |
           ((k & 4) ? (1u << reg[2]) : 0u) | ((k & 8) ? (1u << reg[3]) : 0u);
}

// LDS byte address of register k of a thread: swz is linear over GF(2), so
// swz(tl | roff(k)) = swz(tl) ^ swz(roff(k)) with the second part uniform.
__device__ __forceinline__ uint32_t lds_off(uint32_t stl8, const uint8_t *reg, int k) {
    return stl8 ^ (swz(roff(reg, k)) << 3);
}

// I/O layout from a host-computed record: a few VALU for the lane part, the
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

// Store layout of a pass: with PD_REMAP_OUT the non-local bits follow the
// pass's output relabelling (tile_base_out, and the per-wave and
// per-register xor terms of the record), otherwise those of the load.
__device__ __forceinline__ IoLayout io_out_layout(const PassDesc &d, uint32_t tile, uint32_t lane,
                                                  uint32_t wave, uint32_t base) {
    if (!(d.flags & PD_REMAP_OUT)) return io_from_rec(d.io_out, lane, wave, base);
    const uint32_t bo = uni(ldu(d.tile_base_out + tile)) ^ uni(ldu(d.io_out->wave_xor + wave));
    IoLayout io = io_from_rec(d.io_out, lane, wave, bo);
    #pragma unroll
    for (int k = 0; k < 16; ++k) io.uni_off[k] ^= uni(ldu(d.io_out->reg_xor + k));
    return io;
}

__device__ __forceinline__ void io_load(float2 (&v)[16], const void *src, const IoLayout &io,
                                        uint8_t kind) {
    const uint32_t lb = io.lane_off * 8u;
    if (kind == IO_F4) {
        #pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
            const float4 q = buf_ld4(src, io.uni_off[2 * k2], lb);
            v[2 * k2] = make_float2(q.x, q.y);
            v[2 * k2 + 1] = make_float2(q.z, q.w);
        }
    } else {
        #pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = buf_ld2(src, io.uni_off[k], lb);
    }
}

__device__ __forceinline__ void io_store(const float2 (&v)[16], void *dst, const IoLayout &io,
                                         uint8_t kind) {
    const uint32_t lb = io.lane_off * 8u;
    if (kind == IO_F4) {
        #pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) buf_st4(dst, io.uni_off[2 * k2], lb, v[2 * k2], v[2 * k2 + 1]);
    } else {
        #pragma unroll
        for (int k = 0; k < 16; ++k) buf_st2(dst, io.uni_off[k], lb, v[k]);
    }
}

// Run the ops of one op range [o, end) on the registers. The next op record
// is requested before the current one is executed (scalar-load prefetch).
__device__ __forceinline__ void run_ops(float2 (&v)[16], const DevOp *ops, uint32_t o,
                                        uint32_t end, uint32_t tl, uint64_t base) {
    if (o >= end) return;
    DevOp nxt = ld_words(ops + o);
    while (o < end) {
        const DevOp op = nxt;
        const uint32_t step = (op.type == OP_DSET) ? 1u + op.sb + op.b + op.a : 1u;
        if (o + step < end) nxt = ld_words(ops + o + step);
        if (op.type == OP_DSET) {
            // thread/global members -> one factor; table; mixed members
            float2 ft = make_float2(1.0f, 0.0f);
            const uint32_t m0 = o + 1 + op.sb;
            for (uint32_t j = 0; j < op.b; ++j) {
                const DevOp mm = ld_words(ops + m0 + j);
                ft = dset_fold(ft, pdiag_tg(tl, base, mm.tmask, mm.gmask), opc(ops, m0 + j, 0),
                               opc(ops, m0 + j, 1));
            }
            // with a table or thread members, the first mixed member is
            // merged into the application
            const uint32_t merged = (op.a && (op.sb || op.b)) ? 1u : 0u;
            if (merged) {
                const DevOp mm = ld_words(ops + m0 + op.b);
                dset_apply_m(v, op.sb ? ops + o + 1 : ops, op.sb != 0, ft,
                             pdiag_tg(tl, base, mm.tmask, mm.gmask), opc(ops, m0 + op.b, 0),
                             opc(ops, m0 + op.b, 1), mm.rmask);
            } else if (op.sb) {
                dset_apply(v, ops + o + 1, true, ft, op.b != 0);
            } else if (op.b) {
                dset_apply(v, ops, false, ft, true);
            }
            for (uint32_t j = merged; j < op.a; ++j) {
                const DevOp mm = ld_words(ops + m0 + op.b + j);
                pdiag_mixed(v, pdiag_tg(tl, base, mm.tmask, mm.gmask), opc(ops, m0 + op.b + j, 0),
                            opc(ops, m0 + op.b + j, 1), mm.rmask);
            }
        } else {
            run_op(v, op, ops, o, tl, base);
        }
        o += step;
    }
}

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
    io_store(v, d.dst, io_out_layout(d, tile, lane, wave, base), ph.io);
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
        io_store(v, d.dst, io_out_layout(d, tile, lane, wave, base), ph.io);
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
        if (op.type == OP_DSET) continue;  // members follow as plain parity factors
        if (op.type == OP_PDIAG) {
            const float2 d0 = make_float2(op.m[0], op.m[1]), d1 = make_float2(op.m[2], op.m[3]);
            for (uint32_t i = tid; i < dim; i += 64)
                s[i] = cmul((__popc(i & op.tmask) & 1u) ? d1 : d0, s[i]);
            __syncthreads();
            continue;
        }
        if (op.type == OP_U || op.type == OP_PERM || op.type == OP_CX || op.type == OP_UR ||
            op.type == OP_URT || op.type == OP_URD) {
            float e0 = op.m[0], e1 = op.m[1], e2 = op.m[2], e3 = op.m[3];
            if (op.type == OP_URD) {
                const Urd e = urd_entries(d.ops, o);
                e0 = e.a; e1 = e.b; e2 = e.c; e3 = e.d;
            }
            const uint32_t bit = 1u << op.a;
            for (uint32_t pr = tid; pr < dim / 2; pr += 64) {
                const uint32_t i0 = ((pr >> op.a) << (op.a + 1)) | (pr & (bit - 1));
                const uint32_t i1 = i0 | bit;
                const float2 x = s[i0], y = s[i1];
                if (op.type == OP_U) {
                    s[i0] = cmad2(make_float2(op.m[0], op.m[1]), x, make_float2(op.m[2], op.m[3]), y);
                    s[i1] = cmad2(make_float2(op.m[4], op.m[5]), x, make_float2(op.m[6], op.m[7]), y);
                } else if (op.type == OP_URT) {
                    float2 a = x, b = y;
                    if (op.b) urt_pair<1>(op.m[0], a, b);
                    else urt_pair<0>(op.m[0], a, b);
                    s[i0] = a;
                    s[i1] = b;
                } else if (op.type == OP_UR || op.type == OP_URD) {
                    s[i0] = make_float2(fmaf(e0, x.x, e1 * y.x), fmaf(e0, x.y, e1 * y.y));
                    s[i1] = make_float2(fmaf(e2, x.x, e3 * y.x), fmaf(e2, x.y, e3 * y.y));
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


// Register-phase reducer. One workgroup per (slot, group, row of tiles):
// each tile is loaded with the I/O layout, staged in LDS, and re-read with
// each phase's layout. Terms are taken 8 at a time (in phase order): every
// thread adds each term's FP32 value over the row's tiles in tile order,
// then the 8 sums are converted to FP64 and summed across the wave by a
// butterfly that halves the number of values per lane at each of the first
// three steps (fixed order); wave sums are added in wave order. A term's
// result does not depend on the other terms of its chunk, so the generated
// reducers (all terms of a tile at once) round identically. The row's tiles
// are re-read for each chunk of 8 terms.
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
    const uint32_t tiles = 1u << (n - M), rt = red_row_tiles(tiles);
    const uint64_t row = item / n_descs;
    const ReduceDesc d = ld_words(descs + p);
    const uint64_t lmask = d.local_mask;
    const uint64_t full = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint8_t io[4] = {0, 7, 8, 9};   // I/O layout: register slots = local bits 0, 7, 8, 9

    for (uint32_t j0 = 0; j0 < d.n_terms; j0 += 8u) {
        const uint32_t j1 = j0 + 8u < d.n_terms ? j0 + 8u : d.n_terms;
        float q[8];
        #pragma unroll
        for (int i = 0; i < 8; ++i) q[i] = 0.0f;
        for (uint32_t k = 0; k < rt; ++k) {
            const uint64_t tile = row * rt + k;
            const uint64_t base = dpdep(tile, full & ~lmask);
            float2 v[16];
            {
                const uint32_t tl = thread_local_index(tid, io);
                const IoLayout lay = io_layout(lmask, io, IO_F4, lane, uni(tid >> 6), M, (uint32_t)base);
                io_load(v, d.psi, lay, IO_F4);
                __syncthreads();   // the previous tile's LDS reads are done
                const uint32_t stl8 = swz(tl) << 3;
                char *lb = reinterpret_cast<char *>(lds);
                #pragma unroll
                for (int r = 0; r < 16; ++r)
                    *reinterpret_cast<float2 *>(lb + lds_off(stl8, io, r)) = v[r];
            }
            __syncthreads();
            for (uint32_t pi = 0; pi < d.n_phases; ++pi) {
                const RedPhase ph = ld_words(d.phases + pi);
                if (ph.t_end <= j0 || ph.t_begin >= j1) continue;
                const uint32_t tl = thread_local_index(tid, ph.reg);
                if (!ph.diag) {
                    const uint32_t stl8 = swz(tl) << 3;
                    const char *lb = reinterpret_cast<const char *>(lds);
                    #pragma unroll
                    for (int r = 0; r < 16; ++r)
                        v[r] = *reinterpret_cast<const float2 *>(lb + lds_off(stl8, ph.reg, r));
                }
                float pr[16];
                if (ph.diag) {
                    #pragma unroll
                    for (int r = 0; r < 16; ++r) pr[r] = fmaf(v[r].x, v[r].x, v[r].y * v[r].y);
                }
                const uint32_t jb = ph.t_begin > j0 ? ph.t_begin : j0;
                const uint32_t je = ph.t_end < j1 ? ph.t_end : j1;
                for (uint32_t j = jb; j < je; ++j) {
                    const TermDev t = ld_words(d.terms + j);
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
                    // q[j - j0] += a, with constant register indices
                    #pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if ((uint32_t)i == j - j0) q[i] += a;
                }
            }
        }
        const double h = wave_reduce8(q, lane);
        if (lane < 8u) {
            const uint32_t pos = 4u * (lane & 1u) + 2u * ((lane >> 1) & 1u) + ((lane >> 2) & 1u);
            if (j0 + pos < j1) {
                // a per-lane load (ld_words reads wave-uniform records)
                const uint32_t col = d.terms[j0 + pos].col;
                red[wave * kMaxGroupTerms + col] = h;
            }
        }
    }
    __syncthreads();
    for (uint32_t c = tid; c < d.n_terms; c += T) {
        double s = 0.0;
        for (int w = 0; w < W; ++w) s += red[w * kMaxGroupTerms + c];
        gout<double>(d.part)[row * d.n_terms_total + gin<uint32_t>(d.cols)[c]] = s;
    }
}

// out[s] = sum_j coeff[j] * (sum over rows of part[s][row][j]); one
// workgroup per slot; term sums use a fixed tree, terms are added in order.
__global__ __launch_bounds__(256) void expect_finalize_kernel(const double *__restrict__ part,
                                                              const double *__restrict__ coeff,
                                                              uint32_t n_terms, uint32_t rows,
                                                              double *__restrict__ out) {
    __shared__ double red[5];
    const uint32_t s = blockIdx.x;
    const double *ps = part + (uint64_t)s * rows * n_terms;
    double e = 0.0;
    for (uint32_t j = 0; j < n_terms; ++j) {
        double acc = 0.0;
        for (uint32_t t = threadIdx.x; t < rows; t += 256) acc += ps[(uint64_t)t * n_terms + j];
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

// Measurement sums of slot s over chunk c of 2^C amplitudes: the FP64 sum
// of |psi_i|^2 and the same sum over the indices with bit qubit[s] set
// (fixed order: per thread in index order, then the block sum).
__global__ __launch_bounds__(256) void measure_sum_kernel(const float2 *const *__restrict__ slots,
                                                          const uint32_t *__restrict__ qubit,
                                                          uint32_t C, uint32_t chunks,
                                                          double *__restrict__ part) {
    __shared__ double red[5];
    const uint32_t c = blockIdx.x, s = blockIdx.y;
    const uint64_t first = (uint64_t)c << C;
    const float2 *psi = slots[s] + first;
    const uint32_t q = qubit[s];
    const uint32_t len = 1u << C;
    double acc = 0.0, acc1 = 0.0;
    for (uint32_t i = threadIdx.x; i < len; i += 256) {
        const double x = psi[i].x, y = psi[i].y;
        const double w = fma(x, x, y * y);
        acc += w;
        if (((first + i) >> q) & 1ull) acc1 += w;
    }
    acc = block_sum<256>(acc, red);
    acc1 = block_sum<256>(acc1, red);
    if (threadIdx.x == 0) {
        part[2 * ((uint64_t)s * chunks + c)] = acc;
        part[2 * ((uint64_t)s * chunks + c) + 1] = acc1;
    }
}

// Chunk sums of slot s added in a fixed order: out[2 s] = S, out[2 s + 1] = S1.
__global__ __launch_bounds__(256) void measure_finalize_kernel(const double *__restrict__ part,
                                                               uint32_t chunks,
                                                               double *__restrict__ out) {
    __shared__ double red[5];
    const uint32_t s = blockIdx.x;
    const double *in = part + 2 * (uint64_t)s * chunks;
    const uint32_t per = (chunks + 255) / 256;
    const uint32_t b0 = threadIdx.x * per;
    const uint32_t b1 = (b0 + per < chunks) ? b0 + per : chunks;
    double a = 0.0, a1 = 0.0;
    for (uint32_t c = b0; c < b1; ++c) {
        a += in[2 * c];
        a1 += in[2 * c + 1];
    }
    a = block_sum<256>(a, red);
    a1 = block_sum<256>(a1, red);
    if (threadIdx.x == 0) {
        out[2 * s] = a;
        out[2 * s + 1] = a1;
    }
}

// Joint measurement masses: chunk c of slot s (2^C amplitudes, FP64 sum
// csum[s * chunks + c]) lies in one outcome bin when every measured qubit is
// >= C; bin b of slot s (its measured bits in ascending qubit order) is the
// sum of its chunks in increasing chunk order. mq[s]: measured-qubit mask of
// slot s shifted down by C (a mask over chunk-index bits).
__global__ __launch_bounds__(256) void bin_mass_kernel(const double *__restrict__ csum,
                                                       uint32_t chunks_log2,
                                                       const uint64_t *__restrict__ mq,
                                                       uint32_t bin_stride,
                                                       double *__restrict__ out) {
    const uint32_t s = blockIdx.x;
    const uint64_t M = mq[s];
    const uint32_t k = (uint32_t)__popcll(M);
    const uint64_t all = (chunks_log2 >= 64) ? ~0ull : ((1ull << chunks_log2) - 1ull);
    const uint64_t F = all & ~M;
    const uint64_t nfree = 1ull << (chunks_log2 - k);
    const double *in = csum + ((uint64_t)s << chunks_log2);
    for (uint32_t b = threadIdx.x; b < (1u << k); b += 256) {
        // chunk bits of the bin: deposit b into M
        uint64_t cb = 0;
        {
            uint32_t j = 0;
            for (uint32_t p = 0; p < chunks_log2; ++p)
                if ((M >> p) & 1ull) cb |= (uint64_t)((b >> j++) & 1u) << p;
        }
        double a = 0.0;
        for (uint64_t f = 0; f < nfree; ++f) {
            uint64_t c = cb;
            uint32_t j = 0;
            for (uint32_t p = 0; p < chunks_log2; ++p)
                if ((F >> p) & 1ull) c |= ((f >> j++) & 1ull) << p;
            a += in[c];
        }
        out[(uint64_t)s * bin_stride + b] = a;
    }
}

// Dense export of a stabilizer state (STAB -> SV): amplitude k is
// 2^{-r/2} i^e when k = x0 ^ (sum of the X parts x_i of the generators whose
// pivot bit p_i is set in k ^ x0), e collecting each such generator's phase
// (ph_i, then (-1)^{z_i . cur} as it acts on the current basis state cur in
// increasing i), else 0.
__global__ __launch_bounds__(256) void stab_export_kernel(float2 *__restrict__ psi, uint32_t n,
                                                          uint64_t x0, uint32_t r,
                                                          const uint64_t *__restrict__ xs,
                                                          const uint64_t *__restrict__ zs,
                                                          const uint32_t *__restrict__ ph,
                                                          const uint32_t *__restrict__ piv,
                                                          float norm) {
    __shared__ uint64_t sx[64], sz[64];
    __shared__ uint32_t sp[64], sv[64];
    for (uint32_t i = threadIdx.x; i < r; i += 256) {
        sx[i] = xs[i];
        sz[i] = zs[i];
        sp[i] = ph[i];
        sv[i] = piv[i];
    }
    __syncthreads();
    const uint64_t total = 1ull << n;
    for (uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (uint64_t)gridDim.x * 256) {
        const uint64_t d = k ^ x0;
        uint64_t cur = x0;
        uint32_t e = 0;
        for (uint32_t i = 0; i < r; ++i)
            if ((d >> sv[i]) & 1ull) {
                e += sp[i] + 2u * (uint32_t)__popcll(sz[i] & cur);
                cur ^= sx[i];
            }
        float2 a = make_float2(0.0f, 0.0f);
        if (cur == k) {
            switch (e & 3u) {
            case 0: a = make_float2(norm, 0.0f); break;
            case 1: a = make_float2(0.0f, norm); break;
            case 2: a = make_float2(-norm, 0.0f); break;
            default: a = make_float2(0.0f, -norm); break;
            }
        }
        psi[k] = a;
    }
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

// Sub-chunk and chunk sums of |psi|^2 (FP64) for the sampler; grid (chunks,
// slots), chunk = 2^C amplitudes, sub-chunk = 2^S (S <= 6) amplitudes. A
// sub-chunk of 64 is summed by 32 lanes (two amplitudes each, then a fixed
// butterfly), a smaller one by one amplitude per lane; the chunk sum is the
// sequential sum of its sub-chunk sums.
__global__ __launch_bounds__(256) void sub_sum_kernel(const float2 *const *__restrict__ slots,
                                                      uint32_t C, uint32_t S, uint32_t chunks,
                                                      double *__restrict__ csum,
                                                      double *__restrict__ ssum) {
    __shared__ double subs[16];
    const uint32_t c = blockIdx.x, s = blockIdx.y;
    const uint32_t spc = 1u << (C - S), L = 1u << S;
    const float2 *psi = slots[s] + ((uint64_t)c << C);
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *out = ssum + ((uint64_t)s * chunks + c) * spc;
    if (S == 6) {
        // two sub-chunks per wave step: each half-wave covers one with two
        // amplitudes (16 bytes) per lane
        const uint32_t half = lane >> 5, hl = lane & 31;
        for (uint32_t q = wave; 2 * q < spc; q += 4) {
            const uint32_t j = 2 * q + half;
            double v = 0.0;
            if (j < spc) {
                const float4 a = *reinterpret_cast<const float4 *>(psi + (j << 6) + 2 * hl);
                const double x0 = a.x, y0 = a.y, x1 = a.z, y1 = a.w;
                v = fma(x0, x0, y0 * y0) + fma(x1, x1, y1 * y1);
            }
            for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
            if (hl == 0 && j < spc) {
                subs[j] = v;
                out[j] = v;
            }
        }
    } else {
        for (uint32_t j = wave; j < spc; j += 4) {
            double v = 0.0;
            if (lane < L) {
                const float2 a = psi[(j << S) + lane];
                const double x = a.x, y = a.y;
                v = fma(x, x, y * y);
            }
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) {
                subs[j] = v;
                out[j] = v;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (uint32_t j = 0; j < spc; ++j) acc += subs[j];
        csum[(uint64_t)s * chunks + c] = acc;
    }
}

// One thread per (slot, shot). The target u * total is located by a binary
// search over the chunk prefixes, a scan of the chunk's sub-chunk sums and a
// scan of one sub-chunk's amplitudes, the running sum continuing in FP64 from
// the chunk prefix. Where rounding leaves the target past a level's last
// element, that level's last element of non-zero mass is taken, so every
// outcome has non-zero probability.
__global__ __launch_bounds__(256) void draw_kernel(const float2 *const *__restrict__ slots,
                                                   uint32_t n_slots, uint32_t C, uint32_t S,
                                                   uint32_t chunks, const double *__restrict__ csum,
                                                   const double *__restrict__ cpre,
                                                   const double *__restrict__ ssum,
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
    const double *cs = csum + (uint64_t)s * chunks;
    // last chunk with pre[c] <= target, then back over chunks without mass
    uint32_t lo = 0, hi = chunks - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= target) lo = mid;
        else hi = mid - 1;
    }
    while (lo > 0 && cs[lo] == 0.0) --lo;
    const uint32_t spc = 1u << (C - S), L = 1u << S;
    const double *sb = ssum + ((uint64_t)s * chunks + lo) * spc;
    double run = pre[lo], run_last = run;
    int j = -1, last_j = 0;
    for (uint32_t k = 0; k < spc; ++k) {
        const double v = sb[k];
        if (v > 0.0) {
            last_j = (int)k;
            run_last = run;
        }
        if (run + v > target) {
            j = (int)k;
            break;
        }
        run += v;
    }
    if (j < 0) {
        j = last_j;
        run = run_last;
    }
    const float2 *psi = slots[s] + ((uint64_t)lo << C) + ((uint64_t)j << S);
    uint32_t res = 0xFFFFFFFFu, last_i = 0;
    for (uint32_t i = 0; i < L; ++i) {
        const double x = psi[i].x, y = psi[i].y;
        const double pr = fma(x, x, y * y);
        if (pr > 0.0) last_i = i;
        run += pr;
        if (run > target) {
            res = i;
            break;
        }
    }
    if (res == 0xFFFFFFFFu) res = last_i;
    out[gid] = (uint32_t)(((uint64_t)lo << C) + ((uint64_t)j << S) + res);
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
    const uint64_t items = (uint64_t)n_descs * (tiles / red_row_tiles((uint32_t)tiles));
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
                                  uint32_t n_terms, uint32_t rows, uint32_t n_slots,
                                  double *out) {
    if (n_slots == 0) return hipSuccess;
    hipLaunchKernelGGL(expect_finalize_kernel, dim3(n_slots), dim3(256), 0, st, part, coeff,
                       n_terms, rows, out);
    return hipGetLastError();
}

hipError_t launch_sample(hipStream_t st, const float2 *const *slots, uint32_t n_slots,
                         uint32_t n, double *csum, double *cpre, double *ssum, double *total,
                         uint64_t seed, uint64_t task_base, uint32_t shots, uint32_t *out) {
    const uint32_t C = sample_chunk_bits(n), S = sample_sub_bits(n);
    const uint32_t chunks = 1u << (n - C);
    hipLaunchKernelGGL(sub_sum_kernel, dim3(chunks, n_slots), dim3(256), 0, st, slots, C, S, chunks,
                       csum, ssum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(chunk_scan_kernel, dim3(n_slots), dim3(256), 0, st, csum, chunks, cpre,
                       total);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t threads = (uint64_t)n_slots * shots;
    if (threads == 0) return hipSuccess;
    hipLaunchKernelGGL(draw_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, st,
                       slots, n_slots, C, S, chunks, csum, cpre, ssum, total, seed, task_base, shots,
                       out);
    return hipGetLastError();
}

hipError_t launch_measure_sums(hipStream_t st, const float2 *const *slots, const uint32_t *qubit,
                               uint32_t n_slots, uint32_t n, double *part, double *out) {
    if (n_slots == 0) return hipSuccess;
    const uint32_t C = n < 14 ? n : 14;
    const uint32_t chunks = 1u << (n - C);
    hipLaunchKernelGGL(measure_sum_kernel, dim3(chunks, n_slots), dim3(256), 0, st, slots, qubit, C,
                       chunks, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(measure_finalize_kernel, dim3(n_slots), dim3(256), 0, st, part, chunks, out);
    return hipGetLastError();
}

hipError_t launch_joint_masses(hipStream_t st, const float2 *const *slots, const uint64_t *mq,
                               uint32_t n_slots, uint32_t n, uint32_t C, double *csum,
                               uint32_t bin_stride, double *out) {
    if (n_slots == 0) return hipSuccess;
    const uint32_t chunks = 1u << (n - C);
    hipLaunchKernelGGL(chunk_sum_kernel, dim3(chunks, n_slots), dim3(256), 0, st, slots, C, chunks,
                       csum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bin_mass_kernel, dim3(n_slots), dim3(256), 0, st, csum, n - C, mq, bin_stride,
                       out);
    return hipGetLastError();
}

namespace {

// One workgroup per task. A joint cluster's bin masses are staged in LDS;
// each step sums them (and those with the step's bit set) with a fixed
// order (per-thread strided sums, then a fixed tree), decides, and keeps
// the bins that agree with the outcome: bin b moves to b with bit p removed,
// which keeps their order.
constexpr int kDecideThreads = 256;

__device__ __forceinline__ void decide_sums(const double *mass, uint32_t len, uint32_t p, double *red,
                                            double *tot, double *one) {
    const uint32_t t = threadIdx.x;
    double a = 0.0, b1 = 0.0;
    for (uint32_t b = t; b < len; b += kDecideThreads) {
        a += mass[b];
        if ((b >> p) & 1u) b1 += mass[b];
    }
    red[t] = a;
    red[kDecideThreads + t] = b1;
    __syncthreads();
    for (uint32_t h = kDecideThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            red[t] += red[t + h];
            red[kDecideThreads + t] += red[kDecideThreads + t + h];
        }
        __syncthreads();
    }
    *tot = red[0];
    *one = red[kDecideThreads];
    __syncthreads();
}

__global__ __launch_bounds__(kDecideThreads) void meas_decide_kernel(
    const uint32_t *__restrict__ task_first, const uint32_t *__restrict__ task_count,
    const MeasDec *__restrict__ dec, uint32_t n_tasks, int joint, double *__restrict__ sums,
    uint32_t bin_stride, float *__restrict__ dyn, uint8_t *__restrict__ outc, uint32_t *__restrict__ err) {
    __shared__ double buf[2][1u << 12];
    __shared__ double red[2 * kDecideThreads];
    const uint32_t i = blockIdx.x, t = threadIdx.x;
    if (i >= n_tasks) return;
    const uint32_t f0 = task_first[i], k = task_count[i];
    uint32_t bits = 0;     // outcome of measurement j in bit j
    double chosen = 1.0;   // mass of the chosen outcome
    bool zero = false;
    if (!joint) {
        const double S = sums[2 * i], S1 = sums[2 * i + 1];
        if (!(S > 0.0)) {
            zero = true;
        } else {
            const uint32_t b = dec[f0].u < S1 / S ? 1u : 0u;
            bits = b;
            chosen = b ? S1 : S - S1;
        }
    } else {
        uint32_t len = 1u << k;  // k <= 12 (the caller's cluster bound)
        const double *src = sums + (size_t)i * bin_stride;
        for (uint32_t b = t; b < len; b += kDecideThreads) buf[0][b] = src[b];
        __syncthreads();
        int cur = 0;
        double tot, one;
        decide_sums(buf[cur], len, 0, red, &tot, &one);
        if (!(tot > 0.0)) {
            zero = true;
        } else {
            for (uint32_t j = 0; j < k; ++j) {
                const uint32_t p = dec[f0 + j].pos;
                decide_sums(buf[cur], len, p, red, &tot, &one);
                const uint32_t bit = dec[f0 + j].u < one / tot ? 1u : 0u;
                bits |= bit << j;
                const uint32_t lo = (1u << p) - 1u;
                for (uint32_t b = t; b < len; b += kDecideThreads)
                    if (((b >> p) & 1u) == bit) buf[cur ^ 1][((b >> (p + 1)) << p) | (b & lo)] = buf[cur][b];
                __syncthreads();
                cur ^= 1;
                len >>= 1;
            }
            chosen = buf[cur][0];
        }
    }
    if (t != 0) return;
    if (zero) {
        *err = 1u;
        chosen = 1.0;
    }
    const float fac = (float)(1.0 / sqrt(chosen));
    for (uint32_t j = 0; j < k; ++j) {
        const MeasDec &m = dec[f0 + j];
        const uint32_t b = (bits >> j) & 1u;
        const float f = j == 0 ? fac : 1.0f;
        float *e = dyn + 4ull * m.dyn;
        // [[e0, e1], [e2, e3]]: P0 = diag(f, 0), P1 = diag(0, f), X P1 = [[0, f], [0, 0]]
        e[0] = b ? 0.0f : f;
        e[1] = (b && m.reset) ? f : 0.0f;
        e[2] = 0.0f;
        e[3] = (b && !m.reset) ? f : 0.0f;
        outc[m.outc] = (uint8_t)b;
    }
}

__global__ void meas_clear_kernel(uint32_t *err) {
    if (threadIdx.x == 0) *err = 0u;
}

__global__ void zero_words_kernel(uint32_t *p, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

hipError_t launch_meas_decide(hipStream_t st, const uint32_t *task_first, const uint32_t *task_count,
                              const MeasDec *dec, uint32_t n_tasks, int joint, double *sums,
                              uint32_t bin_stride, float *dyn, uint8_t *outc, uint32_t *err) {
    if (n_tasks == 0) return hipSuccess;
    hipLaunchKernelGGL(meas_decide_kernel, dim3(n_tasks), dim3(kDecideThreads), 0, st, task_first, task_count,
                       dec, n_tasks, joint, sums, bin_stride, dyn, outc, err);
    return hipGetLastError();
}

hipError_t launch_meas_clear(hipStream_t st, uint32_t *err) {
    hipLaunchKernelGGL(meas_clear_kernel, dim3(1), dim3(64), 0, st, err);
    return hipGetLastError();
}

hipError_t launch_zero_words(hipStream_t st, uint32_t *p, uint64_t count) {
    if (count == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((count + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_words_kernel, dim3((uint32_t)blocks), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

hipError_t launch_stab_export(hipStream_t st, float2 *psi, uint32_t n, uint64_t x0, uint32_t r,
                              const uint64_t *xs, const uint64_t *zs, const uint32_t *ph,
                              const uint32_t *piv, float norm) {
    const uint64_t total = 1ull << n;
    const uint64_t blocks = std::min<uint64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(stab_export_kernel, dim3((uint32_t)blocks), dim3(256), 0, st, psi, n, x0, r, xs, zs,
                       ph, piv, norm);
    return hipGetLastError();
}

hipError_t kernels_init() { return hipSuccess; }

}  // namespace qw
