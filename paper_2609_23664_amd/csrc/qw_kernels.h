// Launch wrappers of the gfx950 kernels (qw_kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "qw_internal.h"


namespace qw {

// Gate pass over n_descs (task, pass) descriptors of one n-qubit layout with
// tile bits m (m < 10: whole-state kernel). remap: XCD-aware tile order.
// use_lds = false is valid only when every descriptor has one phase and no
// PD_NORM_OUT; the kernel then runs without LDS at higher occupancy.
hipError_t launch_pass(hipStream_t st, const PassDesc *d, uint32_t n_descs, uint32_t n,
                       uint32_t m, int remap, bool use_lds);
// scale_out = 1/sqrt(sum norm_part) for descriptors flagged PD_NORM_OUT.
hipError_t launch_norm_finalize(hipStream_t st, const PassDesc *d, uint32_t n_descs,
                                uint32_t tiles);
// Every slot of [base, base + n_slots * 2^n) set to |0...0>.
hipError_t launch_init(hipStream_t st, void *base, uint32_t n, uint32_t n_slots);
// Device-to-device copy of `bytes` (multiple of 16).
hipError_t launch_copy(hipStream_t st, void *dst, const void *src, uint64_t bytes);
// Expectation partials for n_descs (slot, term group) descriptors: one
// workgroup per (descriptor, row of tiles).
hipError_t launch_reduce(hipStream_t st, const ReduceDesc *d, uint32_t n_descs, uint32_t n,
                         uint32_t M);
hipError_t launch_reduce_small(hipStream_t st, const ReduceDescSmall *d, uint32_t n_descs,
                               uint32_t n);
// Per-slot sum over rows (see kRedRowTiles) and terms of the partials.
hipError_t launch_expect_finalize(hipStream_t st, const double *part, const double *coeff,
                                  uint32_t n_terms, uint32_t rows, uint32_t n_slots,
                                  double *out);
// Inverse-CDF sampling of `shots` outcomes for n_slots slots (device array
// of slot pointers). csum/cpre: n_slots * chunks doubles; total: n_slots.
// Measurement sums (FP64, fixed order) of n_slots states: out[2 s] = sum of
// |psi_i|^2, out[2 s + 1] = the same over indices with bit qubit[s] set.
// slots and qubit are device arrays; part holds 2 * n_slots * 2^(n - 14)
// doubles (2 * n_slots for n <= 14).
hipError_t launch_measure_sums(hipStream_t st, const float2 *const *slots, const uint32_t *qubit,
                               uint32_t n_slots, uint32_t n, double *part, double *out);
// Joint measurement masses of n_slots states whose measured qubits are all
// >= C (8 <= C <= 14): out[s * bin_stride + b] = FP64 mass of outcome bin b
// (measured bits of slot s in ascending qubit order), summed in a fixed
// order. mq[s] = measured-qubit mask >> C (device); csum holds
// n_slots * 2^(n - C) doubles.
hipError_t launch_joint_masses(hipStream_t st, const float2 *const *slots, const uint64_t *mq,
                               uint32_t n_slots, uint32_t n, uint32_t C, double *csum,
                               uint32_t bin_stride, double *out);
// Device-side measurement decisions (one thread per task of a decision
// group). Task i's measurements are dec[task_first[i] .. task_first[i] +
// task_count[i]), in gate order. Single measurements (joint = 0) read S and
// S1 from sums[2 i], sums[2 i + 1]; joint clusters read their 2^k outcome-bin
// masses from sums[i * bin_stride ...] (used as work space: halved in place).
// Measurement j takes b = (u < P(1 | earlier outcomes)) in FP64, writes its
// outcome byte to outc[dec.outc] and the 4 FP32 entries of the operator that
// opens the next segment to dyn[4 dec.dyn ...]: the projector on b (the first
// of a task with the factor 1 / sqrt of the chosen mass), times X for a RESET
// with b = 1. A zero state sets *err to 1.
struct MeasDec {
    double u;        // the caller's draw
    uint32_t reset;  // 1: RESET (X on outcome 1), 0: MEASURE
    uint32_t pos;    // joint: bit of this qubit among the bins still open
    uint32_t dyn;    // index of its 4-entry block in dyn
    uint32_t outc;   // index of its outcome byte
};
static_assert(sizeof(MeasDec) == 24, "MeasDec layout");
hipError_t launch_meas_decide(hipStream_t st, const uint32_t *task_first, const uint32_t *task_count,
                              const MeasDec *dec, uint32_t n_tasks, int joint, double *sums,
                              uint32_t bin_stride, float *dyn, uint8_t *outc, uint32_t *err);
// *err = 0 (a kernel, so that it can be recorded in a graph).
hipError_t launch_meas_clear(hipStream_t st, uint32_t *err);
// p[0 .. count) = 0 (a kernel, so that it can be recorded in a graph).
hipError_t launch_zero_words(hipStream_t st, uint32_t *p, uint64_t count);
// Dense export of a stabilizer state into psi (2^n amplitudes): x0, r X-type
// generators (device arrays xs, zs, ph = i-power, piv = pivot qubit), norm =
// 2^{-r/2}. r <= 64.
hipError_t launch_stab_export(hipStream_t st, float2 *psi, uint32_t n, uint64_t x0, uint32_t r,
                              const uint64_t *xs, const uint64_t *zs, const uint32_t *ph,
                              const uint32_t *piv, float norm);
// Sampler: csum [n_slots][chunks] and cpre (same size) chunk sums and
// prefixes, ssum [n_slots][2^(n - sub bits)] sub-chunk sums, total [n_slots].
hipError_t launch_sample(hipStream_t st, const float2 *const *slots, uint32_t n_slots,
                         uint32_t n, double *csum, double *cpre, double *ssum, double *total,
                         uint64_t seed, uint64_t task_base, uint32_t shots, uint32_t *out);
// Bytes of the fixed device scratch of qw_sample_noalloc (qw_noalloc.hip).
constexpr uint64_t kNoAllocScratchBytes = QW_NOALLOC_SCRATCH_BYTES;
// Address of that scratch on `device` (looked up once per device with the
// device current; later calls return the kept address).
hipError_t noalloc_scratch(int device, void **ptr);
// out[i] = base + i * stride for i < count (device array of slot pointers).
hipError_t launch_slot_ptrs(hipStream_t st, const float2 **out, const void *base, uint64_t stride,
                            uint32_t count);
inline uint32_t sample_chunk_bits(uint32_t n) { return n < 10 ? n : 10; }
inline uint32_t sample_sub_bits(uint32_t n) { return n < 6 ? n : 6; }
// One-time kernel attributes (dynamic LDS limits).
hipError_t kernels_init();

// Learned cost model (qw_mlp.hip): forward, backward (gradient of
// L = 1/(2B) sum (y - t)^2 into grad[QW_MLP_PARAMS]) and Adam, all on st.
size_t mlp_workspace_floats(uint32_t batch);
// `rows` (device, may be NULL): batch row b reads input and target row
// rows[b] (a gathered mini-batch) instead of row b.
hipError_t launch_mlp_forward(hipStream_t st, const float *p, const float *x, const uint32_t *rows,
                              uint32_t B, float *ws, float *y);
hipError_t launch_mlp_backward(hipStream_t st, const float *p, const float *x, const float *t,
                               const uint32_t *rows, uint32_t B, float *ws, float *grad);
// Forward pass, then out[0] = 1/(2B) sum (y - t)^2 in FP64 (fixed order).
hipError_t launch_mlp_loss(hipStream_t st, const float *p, const float *x, const float *t,
                           const uint32_t *rows, uint32_t B, float *ws, double *out);
hipError_t launch_mlp_adam(hipStream_t st, float *p, const float *g, float *m, float *v,
                           uint32_t step, float lr, float b1, float b2, float eps);

}  // namespace qw
