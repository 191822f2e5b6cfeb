// Learned planner cost model: a 3-layer perceptron (12 -> 64 -> 64 -> 2,
// ReLU) trained on the GPU with these kernels.
//
// Layout: FP32 master parameters in one array (qw.h, QW_MLP_*):
//   W1[12][64], b1[64], W2[64][64], b2[64], W3[64][2], b3[2]  (row-major,
//   W[k][j] multiplies input k into output j).
// Every GEMM rounds its two inputs to BF16 (round to nearest even) and
// accumulates in FP32 on the matrix cores (v_mfma_f32_16x16x16_bf16);
// biases, ReLU, the loss gradient and Adam are FP32.
//
// MFMA 16x16x16 BF16 operand layout (wave of 64 lanes, lane l, item i<4):
//   A[m][k]: m = l % 16, k = 4 (l / 16) + i
//   B[k][n]: n = l % 16, k = 4 (l / 16) + i
//   D[m][n]: n = l % 16, m = 4 (l / 16) + i
// Reductions over the batch (weight gradients) run in a fixed order (one
// workgroup per output tile walks the batch), so results are
// deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qw_kernels.h"

namespace qw {
namespace {

constexpr int IN = 12, W = 64, OUT = 2;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + IN * W, OFF_W2 = OFF_B1 + W, OFF_B2 = OFF_W2 + W * W,
              OFF_W3 = OFF_B2 + W, OFF_B3 = OFF_W3 + W * OUT, N_PARAMS = OFF_B3 + OUT;
static_assert(N_PARAMS == 5122, "parameter count");

// Workspace per batch row (floats): Z1[64], Z2[64], Y[2], dY[2], dZ2[64], dZ1[64]
constexpr int WS_Z1 = 0, WS_Z2 = 64, WS_Y = 128, WS_DY = 130, WS_DZ2 = 132, WS_DZ1 = 196,
              WS_ROW = 260;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ short bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// One 16x16 output tile of A (M x K) * B (K x N): the wave calls
// a(m, k) and b(k, n) for its operands (zero outside the matrices).
template <class FA, class FB>
__device__ __forceinline__ f32x4 tile_gemm(int K, FA a, FB b) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 av, bv;
        #pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = k0 + 4 * g + i;
            av[i] = bf16_rne(k < K ? a(r, k) : 0.f);
            bv[i] = bf16_rne(k < K ? b(k, r) : 0.f);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    return acc;
}

// Forward pass for 16 rows per wave: Z1, Z2 (pre-activations) and Y.
// Batch row b reads row src_row(rows, b) of the inputs and targets: rows[b]
// when a row list is given (a gathered mini-batch), else b.
__device__ __forceinline__ size_t src_row(const uint32_t *__restrict__ rows, int b) {
    return rows ? (size_t)rows[b] : (size_t)b;
}

__global__ __launch_bounds__(64) void mlp_forward_kernel(const float *__restrict__ p,
                                                         const float *__restrict__ x,
                                                         const uint32_t *__restrict__ rows,
                                                         uint32_t B, float *__restrict__ ws,
                                                         float *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int row0 = blockIdx.x * 16;
    const int n_ = lane & 15, g = lane >> 4;
    auto rowok = [&](int m) { return row0 + m < (int)B; };
    // layer 1: Z1 = X W1 + b1
    for (int t = 0; t < W / 16; ++t) {
        f32x4 acc = tile_gemm(IN,
            [&](int m, int k) { return rowok(m) ? x[src_row(rows, row0 + m) * IN + k] : 0.f; },
            [&](int k, int j) { return p[OFF_W1 + k * W + 16 * t + j]; });
        #pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * g + i, j = 16 * t + n_;
            if (rowok(m)) ws[(size_t)(row0 + m) * WS_ROW + WS_Z1 + j] = acc[i] + p[OFF_B1 + j];
        }
    }
    __syncthreads();
    // layer 2: Z2 = relu(Z1) W2 + b2
    for (int t = 0; t < W / 16; ++t) {
        f32x4 acc = tile_gemm(W,
            [&](int m, int k) {
                return rowok(m) ? fmaxf(ws[(size_t)(row0 + m) * WS_ROW + WS_Z1 + k], 0.f) : 0.f;
            },
            [&](int k, int j) { return p[OFF_W2 + k * W + 16 * t + j]; });
        #pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * g + i, j = 16 * t + n_;
            if (rowok(m)) ws[(size_t)(row0 + m) * WS_ROW + WS_Z2 + j] = acc[i] + p[OFF_B2 + j];
        }
    }
    __syncthreads();
    // layer 3: Y = relu(Z2) W3 + b3
    {
        f32x4 acc = tile_gemm(W,
            [&](int m, int k) {
                return rowok(m) ? fmaxf(ws[(size_t)(row0 + m) * WS_ROW + WS_Z2 + k], 0.f) : 0.f;
            },
            [&](int k, int j) { return j < OUT ? p[OFF_W3 + k * OUT + j] : 0.f; });
        #pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * g + i, j = n_;
            if (rowok(m) && j < OUT) {
                const float v = acc[i] + p[OFF_B3 + j];
                ws[(size_t)(row0 + m) * WS_ROW + WS_Y + j] = v;
                if (y) y[(size_t)(row0 + m) * OUT + j] = v;
            }
        }
    }
}

// Backward through the rows (16 per wave) for L = (1 / 2B) sum (y - t)^2:
// dY = (Y - T) / B, dZ2 = (dY W3^T) * [Z2 > 0], dZ1 = (dZ2 W2^T) * [Z1 > 0].
__global__ __launch_bounds__(64) void mlp_backward_rows_kernel(const float *__restrict__ p,
                                                               const float *__restrict__ tgt,
                                                               const uint32_t *__restrict__ rows,
                                                               uint32_t B, float *__restrict__ ws) {
    const int lane = threadIdx.x & 63;
    const int row0 = blockIdx.x * 16;
    const int n_ = lane & 15, g = lane >> 4;
    auto rowok = [&](int m) { return row0 + m < (int)B; };
    const float invB = 1.0f / (float)B;
    for (int e = lane; e < 16 * OUT; e += 64) {
        const int m = e / OUT, j = e % OUT;
        if (rowok(m)) {
            float *r = ws + (size_t)(row0 + m) * WS_ROW;
            r[WS_DY + j] = (r[WS_Y + j] - tgt[src_row(rows, row0 + m) * OUT + j]) * invB;
        }
    }
    __syncthreads();
    for (int t = 0; t < W / 16; ++t) {
        f32x4 acc = tile_gemm(OUT,
            [&](int m, int k) { return rowok(m) ? ws[(size_t)(row0 + m) * WS_ROW + WS_DY + k] : 0.f; },
            [&](int k, int j) { return p[OFF_W3 + (16 * t + j) * OUT + k]; });
        #pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * g + i, j = 16 * t + n_;
            if (rowok(m)) {
                float *r = ws + (size_t)(row0 + m) * WS_ROW;
                r[WS_DZ2 + j] = r[WS_Z2 + j] > 0.f ? acc[i] : 0.f;
            }
        }
    }
    __syncthreads();
    for (int t = 0; t < W / 16; ++t) {
        f32x4 acc = tile_gemm(W,
            [&](int m, int k) { return rowok(m) ? ws[(size_t)(row0 + m) * WS_ROW + WS_DZ2 + k] : 0.f; },
            [&](int k, int j) { return p[OFF_W2 + (16 * t + j) * W + k]; });
        #pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * g + i, j = 16 * t + n_;
            if (rowok(m)) {
                float *r = ws + (size_t)(row0 + m) * WS_ROW;
                r[WS_DZ1 + j] = r[WS_Z1 + j] > 0.f ? acc[i] : 0.f;
            }
        }
    }
}

// Weight gradients: one workgroup (one wave) per 16x16 tile of dW1, dW2 or
// dW3, reducing over the whole batch in order; bias gradients are column
// sums in FP32, in batch order, by the first lanes of the first tiles.
// Tiles: dW1 1x4 (12 rows padded to 16), dW2 4x4, dW3 4x1 (2 cols padded).
__global__ __launch_bounds__(64) void mlp_backward_weights_kernel(const float *__restrict__ x,
                                                                  const uint32_t *__restrict__ rows,
                                                                  uint32_t B,
                                                                  const float *__restrict__ ws,
                                                                  float *__restrict__ grad) {
    const int lane = threadIdx.x & 63;
    const int n_ = lane & 15, g = lane >> 4;
    int tid = blockIdx.x;
    const int Bi = (int)B;
    if (tid < 4) {  // dW1 = X^T dZ1
        const int t = tid;
        f32x4 acc = tile_gemm(Bi,
            [&](int m, int k) { return m < IN ? x[src_row(rows, k) * IN + m] : 0.f; },
            [&](int k, int j) { return ws[(size_t)k * WS_ROW + WS_DZ1 + 16 * t + j]; });
        #pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * g + i;
            if (m < IN) grad[OFF_W1 + m * W + 16 * t + n_] = acc[i];
        }
        if (lane < 16) {  // db1 columns 16t..16t+15
            float s = 0.f;
            for (int b = 0; b < Bi; ++b) s += ws[(size_t)b * WS_ROW + WS_DZ1 + 16 * t + lane];
            grad[OFF_B1 + 16 * t + lane] = s;
        }
        return;
    }
    tid -= 4;
    if (tid < 16) {  // dW2 = relu(Z1)^T dZ2
        const int tm = tid / 4, tn = tid % 4;
        f32x4 acc = tile_gemm(Bi,
            [&](int m, int k) { return fmaxf(ws[(size_t)k * WS_ROW + WS_Z1 + 16 * tm + m], 0.f); },
            [&](int k, int j) { return ws[(size_t)k * WS_ROW + WS_DZ2 + 16 * tn + j]; });
        #pragma unroll
        for (int i = 0; i < 4; ++i) grad[OFF_W2 + (16 * tm + 4 * g + i) * W + 16 * tn + n_] = acc[i];
        if (tm == 0 && lane < 16) {  // db2
            float s = 0.f;
            for (int b = 0; b < Bi; ++b) s += ws[(size_t)b * WS_ROW + WS_DZ2 + 16 * tn + lane];
            grad[OFF_B2 + 16 * tn + lane] = s;
        }
        return;
    }
    tid -= 16;
    if (tid < 4) {  // dW3 = relu(Z2)^T dY
        const int tm = tid;
        f32x4 acc = tile_gemm(Bi,
            [&](int m, int k) { return fmaxf(ws[(size_t)k * WS_ROW + WS_Z2 + 16 * tm + m], 0.f); },
            [&](int k, int j) { return j < OUT ? ws[(size_t)k * WS_ROW + WS_DY + j] : 0.f; });
        #pragma unroll
        for (int i = 0; i < 4; ++i)
            if (n_ < OUT) grad[OFF_W3 + (16 * tm + 4 * g + i) * OUT + n_] = acc[i];
        if (tm == 0 && lane < OUT) {  // db3
            float s = 0.f;
            for (int b = 0; b < Bi; ++b) s += ws[(size_t)b * WS_ROW + WS_DY + lane];
            grad[OFF_B3 + lane] = s;
        }
    }
}

// Adam (FP32): m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
// p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ __launch_bounds__(256) void mlp_adam_kernel(float *__restrict__ p,
                                                       const float *__restrict__ g,
                                                       float *__restrict__ m, float *__restrict__ v,
                                                       uint32_t n, float lr, float b1, float b2,
                                                       float eps, float c1, float c2) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Loss 1/(2B) sum_b sum_j (Y[b][j] - T[b][j])^2 from the forward pass's Y in
// the workspace, in FP64, by one wave: lane l sums rows l, l + 64, ... in
// order, then the 64 lane sums are added pairwise in a fixed tree.
__global__ __launch_bounds__(64) void mlp_loss_kernel(const float *__restrict__ tgt,
                                                      const uint32_t *__restrict__ rows,
                                                      uint32_t B, const float *__restrict__ ws,
                                                      double *__restrict__ out) {
    __shared__ double part[64];
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int b = lane; b < (int)B; b += 64) {
        for (int j = 0; j < OUT; ++j) {
            const double d = (double)ws[(size_t)b * WS_ROW + WS_Y + j] - (double)tgt[src_row(rows, b) * OUT + j];
            s = fma(d, d, s);
        }
    }
    part[lane] = s;
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
        if (lane < h) part[lane] += part[lane + h];
        __syncthreads();
    }
    if (lane == 0) out[0] = part[0] / (2.0 * (double)B);
}

}  // namespace

size_t mlp_workspace_floats(uint32_t batch) { return (size_t)batch * WS_ROW; }

hipError_t launch_mlp_forward(hipStream_t st, const float *p, const float *x, const uint32_t *rows,
                              uint32_t B, float *ws, float *y) {
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((B + 15) / 16), dim3(64), 0, st, p, x, rows, B, ws, y);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(hipStream_t st, const float *p, const float *x, const float *t,
                               const uint32_t *rows, uint32_t B, float *ws, float *grad) {
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((B + 15) / 16), dim3(64), 0, st, p, x, rows, B, ws,
                       (float *)nullptr);
    hipLaunchKernelGGL(mlp_backward_rows_kernel, dim3((B + 15) / 16), dim3(64), 0, st, p, t, rows, B,
                       ws);
    hipLaunchKernelGGL(mlp_backward_weights_kernel, dim3(24), dim3(64), 0, st, x, rows, B,
                       (const float *)ws, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_loss(hipStream_t st, const float *p, const float *x, const float *t,
                           const uint32_t *rows, uint32_t B, float *ws, double *out) {
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((B + 15) / 16), dim3(64), 0, st, p, x, rows, B, ws,
                       (float *)nullptr);
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(64), 0, st, t, rows, B, (const float *)ws, out);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(hipStream_t st, float *p, const float *g, float *m, float *v,
                           uint32_t step, float lr, float b1, float b2, float eps) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((N_PARAMS + 255) / 256), dim3(256), 0, st, p, g, m, v,
                       (uint32_t)N_PARAMS, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace qw
