// Device helpers and tile operations of libqw, shared by the ahead-of-time
// kernels (qw_kernels.hip) and the pass kernels generated at run time from a
// plan (qw_jit.cpp). This text is compiled by hipRTC as well, so it includes
// nothing and relies only on compiler builtins and the HIP device types.
//
// Register layout of a tile (2^M amplitudes, M >= 10): thread t holds 16
// amplitudes v[0..15]; register k of thread t sits at local index
// tl(t) | roff(k), where roff(k) places the 4 bits of k on the phase's 4
// register bits and tl(t) places the thread index on the other local bits
// (its low 6 bits are the lanes of the 64-wide wavefront).
//
// Every operation below is written with explicit fmaf and separate products,
// and all libqw device code is compiled with FP contraction off, so the
// interpreted and the generated kernels round identically.
#pragma once

#include "qw_desc.h"

namespace qw {

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC_RTC__)
#define QW_CONST __attribute__((address_space(4)))
#define QW_GLOBAL __attribute__((address_space(1)))
#else
#define QW_CONST
#define QW_GLOBAL
#endif

// ------------------------------------------------------------- uniform data
// Descriptors, ops and tables are written by a host-to-device copy before a
// launch and only read during it, so uniform reads may go through the
// constant address space (scalar loads).
template <typename T>
__device__ __forceinline__ T ldu(const T *p) {
    return *(const QW_CONST T *)(p);
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float unif(float v) {
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
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

// Matrix entry i of op record j (wave-uniform scalar load).
__device__ __forceinline__ float opm(const DevOp *ops, uint32_t j, int i) {
    return ldu(&ops[j].m[i]);
}

__device__ __forceinline__ float2 opc(const DevOp *ops, uint32_t j, int i) {
    return make_float2(opm(ops, j, 2 * i), opm(ops, j, 2 * i + 1));
}

template <typename T>
__device__ __forceinline__ const QW_GLOBAL T *gin(const void *p) {
    return (const QW_GLOBAL T *)(p);
}

// OP_URD: the 4 real entries [[e0, e1], [e2, e3]] of op j, read from the
// device address held in the bytes of m[0..1]. An earlier kernel writes
// them (kernel boundaries order the write before these uniform loads).
struct Urd {
    float a, b, c, d;
};
__device__ __forceinline__ Urd urd_entries(const DevOp *ops, uint32_t j) {
    const uint64_t addr = ldu(reinterpret_cast<const uint64_t *>(&ops[j].m[0]));
    const float *e = reinterpret_cast<const float *>(addr);
    return Urd{ldu(e), ldu(e + 1), ldu(e + 2), ldu(e + 3)};
}

template <typename T>
__device__ __forceinline__ QW_GLOBAL T *gout(void *p) {
    return (QW_GLOBAL T *)(p);
}

// ------------------------------------------------------------- arithmetic
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}

// u * x + w * y for complex u, x, w, y
__device__ __forceinline__ float2 cmad2(float2 u, float2 x, float2 w, float2 y) {
    float re = u.x * x.x;
    re = fmaf(-u.y, x.y, re);
    re = fmaf(w.x, y.x, re);
    re = fmaf(-w.y, y.y, re);
    float im = u.x * x.y;
    im = fmaf(u.y, x.x, im);
    im = fmaf(w.x, y.y, im);
    im = fmaf(w.y, y.x, im);
    return make_float2(re, im);
}

// LDS element swizzle: the low 5 bits of the element index are XORed with
// bits 5..9 and 10..13; linear over GF(2), so swz(a ^ b) = swz(a) ^ swz(b).
__host__ __device__ __forceinline__ uint32_t swz(uint32_t l) {
    return l ^ (((l >> 5) ^ (l >> 10)) & 31u);
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

// Workgroup barrier for LDS exchanges only: waits for this wave's LDS
// operations, not for its global loads or stores, so prefetched loads stay
// in flight across exchanges.
__device__ __forceinline__ void lds_barrier() {
    __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Exchange inside one wave (the wave holds the same amplitudes before and
// after it): the wave's own LDS writes must have completed before it reads;
// no other wave touches those addresses, so no workgroup barrier is needed.
__device__ __forceinline__ void lds_wave_sync() {
    __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// ------------------------------------------------------------- lanes
// Value of lane (lane ^ 2^J) of the 64-wide wavefront: DPP quad permutes and
// row mirrors for J < 4, cross-row shuffles for J = 4, 5.
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

// The same exchange for an FP64 value (its two 32-bit halves moved alike).
template <int J>
__device__ __forceinline__ double lane_xor_d(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const float lo = lane_xor<J>(__int_as_float((int)(unsigned)b));
    const float hi = lane_xor<J>(__int_as_float((int)(unsigned)(b >> 32)));
    const unsigned long long r = (unsigned long long)(unsigned)__float_as_int(lo) |
                                 ((unsigned long long)(unsigned)__float_as_int(hi) << 32);
    return __longlong_as_double((long long)r);
}

// ------------------------------------------------------------- buffer I/O
// Global loads and stores use buffer instructions: a resource built in
// scalar registers from a wave-uniform base address plus the lane's 32-bit
// byte offset, so all accesses of a thread share one address register.
// Word 3 is the raw (untyped) setting of CDNA buffer resources.
// Cache policy of the global loads and stores (the buffer instructions'
// auxiliary operand; 2 = non-temporal). A generated kernel defines them
// before including this header: streamed state traffic that no other
// wave reads again is marked non-temporal so it does not displace data that
// is reused (a boundary snapshot read by many tasks). 0 = default policy.
#ifndef QW_LD_AUX
#define QW_LD_AUX 0
#endif
#ifndef QW_ST_AUX
#define QW_ST_AUX 0
#endif

typedef unsigned int qw_v4u __attribute__((ext_vector_type(4)));
typedef unsigned int qw_v2u __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_at(const void *p, uint64_t uni_idx) {
    const char *b = reinterpret_cast<const char *>(p) + uni_idx * 8u;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(b), 0, 0x7fffffff, 0x00020000);
}

__device__ __forceinline__ float4 buf_ld4(const void *p, uint64_t uni_idx, uint32_t lane_bytes) {
    const qw_v4u q = __builtin_amdgcn_raw_buffer_load_b128(rsrc_at(p, uni_idx), lane_bytes, 0, QW_LD_AUX);
    return make_float4(__uint_as_float(q.x), __uint_as_float(q.y), __uint_as_float(q.z),
                       __uint_as_float(q.w));
}

__device__ __forceinline__ float2 buf_ld2(const void *p, uint64_t uni_idx, uint32_t lane_bytes) {
    const qw_v2u q = __builtin_amdgcn_raw_buffer_load_b64(rsrc_at(p, uni_idx), lane_bytes, 0, QW_LD_AUX);
    return make_float2(__uint_as_float(q.x), __uint_as_float(q.y));
}

__device__ __forceinline__ void buf_st4(void *p, uint64_t uni_idx, uint32_t lane_bytes, float2 a,
                                        float2 b) {
    const qw_v4u q = {__float_as_uint(a.x), __float_as_uint(a.y), __float_as_uint(b.x),
                      __float_as_uint(b.y)};
    __builtin_amdgcn_raw_buffer_store_b128(q, rsrc_at(p, uni_idx), lane_bytes, 0, QW_ST_AUX);
}

__device__ __forceinline__ void buf_st2(void *p, uint64_t uni_idx, uint32_t lane_bytes, float2 a) {
    const qw_v2u q = {__float_as_uint(a.x), __float_as_uint(a.y)};
    __builtin_amdgcn_raw_buffer_store_b64(q, rsrc_at(p, uni_idx), lane_bytes, 0, QW_ST_AUX);
}

// Insert a zero bit at each register position r0 < r1 < r2 < r3 of tid: the
// phase's local index of the thread's register 0.
__device__ __forceinline__ uint32_t thread_local_index(uint32_t tid, uint32_t r0, uint32_t r1,
                                                       uint32_t r2, uint32_t r3) {
    uint32_t x = tid;
    x = ((x >> r0) << (r0 + 1)) | (x & ((1u << r0) - 1u));
    x = ((x >> r1) << (r1 + 1)) | (x & ((1u << r1) - 1u));
    x = ((x >> r2) << (r2 + 1)) | (x & ((1u << r2) - 1u));
    x = ((x >> r3) << (r3 + 1)) | (x & ((1u << r3) - 1u));
    return x;
}

// ------------------------------------------------------------- register ops
// S = register slot of the target bit; C = register slot of a control bit.
// Matrix entries are wave-uniform scalars.

// General 2x2 complex matrix [[a, b], [c, d]].
template <int S>
__device__ __forceinline__ void u_r(float2 (&v)[16], float2 a, float2 b, float2 c, float2 d) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k & (1 << S)) continue;
        const float2 x = v[k], y = v[k | (1 << S)];
        v[k] = cmad2(a, x, b, y);
        v[k | (1 << S)] = cmad2(c, x, d, y);
    }
}

// Real 2x2 matrix [[a, b], [c, d]]: 4 FP32 operations per amplitude.
template <int S>
__device__ __forceinline__ void ur_r(float2 (&v)[16], float a, float b, float c, float d) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k & (1 << S)) continue;
        const float2 x = v[k], y = v[k | (1 << S)];
        v[k] = make_float2(fmaf(a, x.x, b * y.x), fmaf(a, x.y, b * y.y));
        v[k | (1 << S)] = make_float2(fmaf(c, x.x, d * y.x), fmaf(c, x.y, d * y.y));
    }
}

// Forms of OP_URT on one pair: 0 = [[1, -t], [t, 1]], 1 = [[1, t], [t, -1]].
template <int F>
__device__ __forceinline__ void urt_pair(float t, float2 &x, float2 &y) {
    const float2 a = x, b = y;
    if constexpr (F == 0) {
        x = make_float2(fmaf(-t, b.x, a.x), fmaf(-t, b.y, a.y));
        y = make_float2(fmaf(t, a.x, b.x), fmaf(t, a.y, b.y));
    } else {
        x = make_float2(fmaf(t, b.x, a.x), fmaf(t, b.y, a.y));
        y = make_float2(fmaf(t, a.x, -b.x), fmaf(t, a.y, -b.y));
    }
}

template <int S, int F>
__device__ __forceinline__ void urt_r(float2 (&v)[16], float t) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k & (1 << S)) continue;
        urt_pair<F>(t, v[k], v[k | (1 << S)]);
    }
}

// Anti-diagonal [[0, p01], [p10, 0]].
template <int S>
__device__ __forceinline__ void perm_r(float2 (&v)[16], float2 p01, float2 p10) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k & (1 << S)) continue;
        const float2 x = v[k], y = v[k | (1 << S)];
        v[k] = cmul(p01, y);
        v[k | (1 << S)] = cmul(p10, x);
    }
}

// CNOT, target slot S, control slot C: a register renaming.
template <int S, int C>
__device__ __forceinline__ void cx_rr(float2 (&v)[16]) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if ((k & (1 << S)) || !(k & (1 << C))) continue;
        const float2 x = v[k];
        v[k] = v[k | (1 << S)];
        v[k | (1 << S)] = x;
    }
}

// CNOT, target slot S, control value c (a thread or global bit).
template <int S>
__device__ __forceinline__ void cx_rb(float2 (&v)[16], bool c) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k & (1 << S)) continue;
        const float2 x = v[k], y = v[k | (1 << S)];
        v[k] = c ? y : x;
        v[k | (1 << S)] = c ? x : y;
    }
}

// diag(d0, d1) on register slot S.
template <int S>
__device__ __forceinline__ void diag_r(float2 (&v)[16], float2 d0, float2 d1) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = cmul((k & (1 << S)) ? d1 : d0, v[k]);
}

// diag(d0, d1) on a thread or global bit of value b.
__device__ __forceinline__ void diag_b(float2 (&v)[16], bool b, float2 d0, float2 d1) {
    const float2 f = b ? d1 : d0;
    #pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = cmul(f, v[k]);
}

__device__ __forceinline__ float2 cneg(float2 a) { return make_float2(-a.x, -a.y); }

// CZ on register slots S and C.
template <int S, int C>
__device__ __forceinline__ void cz_rr(float2 (&v)[16]) {
    #pragma unroll
    for (int k = 0; k < 16; ++k)
        if ((k & (1 << S)) && (k & (1 << C))) v[k] = cneg(v[k]);
}

// CZ on register slot S and a thread or global bit of value c.
template <int S>
__device__ __forceinline__ void cz_rb(float2 (&v)[16], bool c) {
    #pragma unroll
    for (int k = 0; k < 16; ++k)
        if (k & (1 << S)) v[k] = c ? cneg(v[k]) : v[k];
}

// CZ on two thread or global bits whose product is c.
__device__ __forceinline__ void cz_bb(float2 (&v)[16], bool c) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = c ? cneg(v[k]) : v[k];
}

// ------------------------------------------------------------- lane ops
// Target on lane bit J: each lane keeps its own component of the pair and
// reads its partner's amplitude from lane ^ 2^J.

template <int J>
__device__ __forceinline__ void u_l(float2 (&v)[16], float2 a, float2 b, float2 c, float2 d,
                                    uint32_t lane) {
    const bool hi = (lane >> J) & 1u;
    const float2 cs = make_float2(hi ? d.x : a.x, hi ? d.y : a.y);
    const float2 co = make_float2(hi ? c.x : b.x, hi ? c.y : b.y);
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float2 pk = lane_xor2<J>(v[k]);
        v[k] = cmad2(cs, v[k], co, pk);
    }
}

template <int J>
__device__ __forceinline__ void ur_l(float2 (&v)[16], float a, float b, float c, float d,
                                     uint32_t lane) {
    const bool hi = (lane >> J) & 1u;
    const float cs = hi ? d : a, co = hi ? c : b;
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float2 pk = lane_xor2<J>(v[k]);
        v[k] = make_float2(fmaf(cs, v[k].x, co * pk.x), fmaf(cs, v[k].y, co * pk.y));
    }
}

// OP_URT forms on lane bit J: the lane with bit J clear computes the first
// output component, the other the second, with the partner's value from
// lane ^ 2^J; each lane performs the same FMA as urt_pair.
template <int J, int F>
__device__ __forceinline__ void urt_l(float2 (&v)[16], float t, uint32_t lane) {
    const bool hi = (lane >> J) & 1u;
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float2 pk = lane_xor2<J>(v[k]);
        const float2 o = v[k];
        if constexpr (F == 0) {  // x' = x - t y ; y' = y + t x
            const float c = hi ? t : -t;
            v[k] = make_float2(fmaf(c, pk.x, o.x), fmaf(c, pk.y, o.y));
        } else {  // x' = x + t y ; y' = t x - y
            v[k] = make_float2(fmaf(t, pk.x, hi ? -o.x : o.x), fmaf(t, pk.y, hi ? -o.y : o.y));
        }
    }
}

template <int J>
__device__ __forceinline__ void perm_l(float2 (&v)[16], float2 p01, float2 p10, uint32_t lane) {
    const bool hi = (lane >> J) & 1u;
    const float2 co = make_float2(hi ? p10.x : p01.x, hi ? p10.y : p01.y);
    #pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = cmul(co, lane_xor2<J>(v[k]));
}

// CNOT, lane target J, control register slot C.
template <int J, int C>
__device__ __forceinline__ void cx_lr(float2 (&v)[16]) {
    #pragma unroll
    for (int k = 0; k < 16; ++k)
        if (k & (1 << C)) v[k] = lane_xor2<J>(v[k]);
}

// CNOT, lane target J, control value c (a thread or global bit).
template <int J>
__device__ __forceinline__ void cx_lb(float2 (&v)[16], bool c) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float2 pk = lane_xor2<J>(v[k]);
        v[k] = c ? pk : v[k];
    }
}

// ------------------------------------------------------------- diagonal sets
// Per-thread factor of the thread/global members of a diagonal set, folded
// in member order starting from 1.
__device__ __forceinline__ float2 dset_fold(float2 ft, bool bit, float2 d0, float2 d1) {
    return cmul(bit ? d1 : d0, ft);
}

// dset_fold with the member's parity given as a mask (all ones: d1, zero:
// d0); the entry is picked by bit operations, which select exactly the same
// bits (the opaque copy of the mask keeps the compiler from turning them
// back into two-operand selects, which need the entries moved to VGPRs).
__device__ __forceinline__ float2 dset_fold_m(float2 ft, uint32_t m, float2 d0, float2 d1) {
    __asm__ volatile("" : "+v"(m));
    const uint32_t x0 = __float_as_uint(d0.x), y0 = __float_as_uint(d0.y);
    const uint32_t dx = x0 ^ __float_as_uint(d1.x), dy = y0 ^ __float_as_uint(d1.y);
    const float2 d = make_float2(__uint_as_float(x0 ^ (m & dx)), __uint_as_float(y0 ^ (m & dy)));
    return cmul(d, ft);
}

// Parity of the thread and global part of a parity factor's mask.
__device__ __forceinline__ bool pdiag_tg(uint32_t tl, uint64_t base, uint32_t tmask, uint32_t gmask) {
    return ((__popc(tl & tmask) ^ __popcll(base & (uint64_t)gmask)) & 1u) != 0u;
}

// Parity factor with register bits (slots rmask) and thread/global bits of
// parity pt: register k gets d[pt ^ parity(k & rmask)].
__device__ __forceinline__ void pdiag_mixed(float2 (&v)[16], bool pt, float2 d0, float2 d1,
                                            uint32_t rmask) {
    const float2 a = pt ? d1 : d0, b = pt ? d0 : d1;
    #pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = cmul((__popc((uint32_t)k & rmask) & 1u) ? b : a, v[k]);
}

template <int RM>
__device__ __forceinline__ void pdiag_mixed_c(float2 (&v)[16], bool pt, float2 d0, float2 d1) {
    const float2 a = pt ? d1 : d0, b = pt ? d0 : d1;
    #pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = cmul((__builtin_popcount(k & RM) & 1) ? b : a, v[k]);
}

// Apply a diagonal set: table entries T[k] (register-bit part) and/or the
// per-thread factor ft. has_tab / has_ft select the four forms; with both,
// each register gets cmul(cmul(T[k], ft), v[k]).
__device__ __forceinline__ void dset_apply(float2 (&v)[16], const DevOp *tab, bool has_tab,
                                           float2 ft, bool has_ft) {
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        float2 w;
        if (has_tab) {
            const float2 t = make_float2(opm(tab, k >> 2, 2 * (k & 3)), opm(tab, k >> 2, 2 * (k & 3) + 1));
            w = has_ft ? cmul(t, ft) : t;
        } else {
            w = ft;
        }
        v[k] = cmul(w, v[k]);
    }
}

// Apply a diagonal set together with its first mixed member (register slots
// rmask, thread/global parity pt, entries d0, d1): the member's two values
// are folded into two per-thread factors f0 = cmul(pt ? d1 : d0, ft) and
// f1 = cmul(pt ? d0 : d1, ft), and register k gets
// cmul(cmul(T[k], f[parity(k & rmask)]), v[k]) (without a table, the chosen
// factor alone). One complex product per register instead of two.
__device__ __forceinline__ void dset_apply_m(float2 (&v)[16], const DevOp *tab, bool has_tab,
                                             float2 ft, bool pt, float2 d0, float2 d1,
                                             uint32_t rmask) {
    const float2 f0 = cmul(pt ? d1 : d0, ft), f1 = cmul(pt ? d0 : d1, ft);
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float2 f = (__popc((uint32_t)k & rmask) & 1u) ? f1 : f0;
        float2 w;
        if (has_tab) {
            const float2 t = make_float2(opm(tab, k >> 2, 2 * (k & 3)), opm(tab, k >> 2, 2 * (k & 3) + 1));
            w = cmul(t, f);
        } else {
            w = f;
        }
        v[k] = cmul(w, v[k]);
    }
}

// ------------------------------------------------------------- reducer
// Sum over one thread's register pairs of sign_k * Re or Im of
// conj(v[k ^ X]) v[k]; each unordered pair is counted once (the caller
// doubles it). Two FP32 FMAs per pair into one FP32 sum (the sign is
// applied to a factor, which is exact): Re = b.x a.x + b.y a.y and
// Im = b.x a.y - b.y a.x with b = v[k ^ X], a = v[k].
template <int X, bool ODD>
__device__ __forceinline__ float pair_sum(const float2 (&v)[16], uint32_t smask) {
    static_assert(X > 0 && X < 16, "off-diagonal register mask");
    constexpr int lead = (X & 8) ? 8 : (X & 4) ? 4 : (X & 2) ? 2 : 1;
    float acc = 0.0f;
    #pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k & lead) continue;
        const float2 a = v[k], b = v[k ^ X];
        const bool neg = (smask >> k) & 1u;
        const float bx = neg ? -b.x : b.x, by = neg ? -b.y : b.y;
        if constexpr (ODD) {
            acc = fmaf(bx, a.y, acc);
            acc = fmaf(-by, a.x, acc);
        } else {
            acc = fmaf(bx, a.x, acc);
            acc = fmaf(by, a.y, acc);
        }
    }
    return acc;
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
// wave in FP64 (values moved by DPP within rows of 16 lanes, by
// ds_bpermute across them): after the xor 1/2/4 steps lane l holds position
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
        f[i] = mine + lane_xor_d<0>(other);
    }
    double g[2];
    #pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double mine = b1 ? f[2 + i] : f[i];
        const double other = b1 ? f[i] : f[2 + i];
        g[i] = mine + lane_xor_d<1>(other);
    }
    double h;
    {
        const double mine = b2 ? g[1] : g[0];
        const double other = b2 ? g[0] : g[1];
        h = mine + lane_xor_d<2>(other);
    }
    h += lane_xor_d<3>(h);
    h += lane_xor_d<4>(h);
    h += lane_xor_d<5>(h);
    return h;
}

}  // namespace qw
