/*
 * Oracle statevector simulator -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct complex128 simulator used to check the
 * GPU path. Only the tests, the smoke entry point and the benchmark's CPU
 * baseline may load it; the product library never does, and the two share no
 * source, header or table.
 *
 * What it computes (textbook quantum mechanics; the paper fixes only the
 * reuse rewrite, Sec. I and Fig. 1: run the shared prefix once, keep the
 * exact boundary state, and run each task's suffix from it):
 *   - basis index i = sum_q b_q 2^q (qubit q is bit q), start state e_0;
 *   - gates applied one at a time, in list order, no fusion, no reordering;
 *   - Pauli expectation <P> = Re sum_i conj(psi[i^x]) * i^{#Y} *
 *     (-1)^{popcount(i & z)} * psi[i]  for P given by bit masks (x, z),
 *     Y on the qubits set in both masks;
 *   - Z-basis sampling by inverse CDF with SplitMix64 (Steele, Lea and
 *     Flood, OOPSLA 2014) used as a counter hash.
 *
 * Amplitude loops may run under OpenMP: each amplitude (pair) is updated by
 * one iteration with the same arithmetic whatever the thread count, so the
 * state is bitwise independent of the number of threads. The norm and the
 * CDF are sequential sums. The expectation sum over i is split into a fixed
 * number of consecutive index ranges (64 from 2^12 amplitudes on, else one),
 * each summed in index order, and the range sums are added in range order:
 * the same sum of the same terms whatever the thread count, with its
 * rounding order fixed.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* gate codes of this file (independent of any other numbering) */
enum {
    G_X = 1, G_Y, G_Z, G_H, G_S, G_SDG, G_T, G_TDG,
    G_RX, G_RY, G_RZ, G_P, G_CNOT, G_CZ, G_RENORM
};

void qwo_init_zero(cplx *psi, int n)
{
    uint64_t dim = 1ull << n;
    memset(psi, 0, dim * sizeof(cplx));
    psi[0] = 1.0;
}

/* (psi[i], psi[i + 2^q]) <- [[u00, u01], [u10, u11]] (psi[i], psi[i + 2^q])
 * for every i whose bit q is 0. */
static void apply_matrix_1q(cplx *psi, int n, int q,
                            cplx u00, cplx u01, cplx u10, cplx u11)
{
    uint64_t dim = 1ull << n, bit = 1ull << q;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)dim; ++i) {
        if ((uint64_t)i & bit)
            continue;
        cplx a = psi[i], b = psi[(uint64_t)i | bit];
        psi[i] = u00 * a + u01 * b;
        psi[(uint64_t)i | bit] = u10 * a + u11 * b;
    }
}

static double norm2(const cplx *psi, int n)
{
    uint64_t dim = 1ull << n;
    double s = 0.0;
    for (uint64_t i = 0; i < dim; ++i)
        s += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
    return s;
}

double qwo_norm2(const cplx *psi, int n) { return norm2(psi, n); }

/* Apply one gate. Returns 0, or -1 for an unknown code / bad qubit. */
int qwo_apply_gate(cplx *psi, int n, int code, int q0, int q1, double param)
{
    const double r2 = 1.0 / sqrt(2.0);
    double c = cos(param / 2.0), s = sin(param / 2.0);
    if (code != G_RENORM && (q0 < 0 || q0 >= n))
        return -1;
    if ((code == G_CNOT || code == G_CZ) && (q1 < 0 || q1 >= n || q1 == q0))
        return -1;
    switch (code) {
    case G_X:   apply_matrix_1q(psi, n, q0, 0, 1, 1, 0); break;
    case G_Y:   apply_matrix_1q(psi, n, q0, 0, -I, I, 0); break;
    case G_Z:   apply_matrix_1q(psi, n, q0, 1, 0, 0, -1); break;
    case G_H:   apply_matrix_1q(psi, n, q0, r2, r2, r2, -r2); break;
    case G_S:   apply_matrix_1q(psi, n, q0, 1, 0, 0, I); break;
    case G_SDG: apply_matrix_1q(psi, n, q0, 1, 0, 0, -I); break;
    case G_T:   apply_matrix_1q(psi, n, q0, 1, 0, 0, cexp(I * M_PI / 4.0)); break;
    case G_TDG: apply_matrix_1q(psi, n, q0, 1, 0, 0, cexp(-I * M_PI / 4.0)); break;
    /* RX(t) = [[cos t/2, -i sin t/2], [-i sin t/2, cos t/2]] */
    case G_RX:  apply_matrix_1q(psi, n, q0, c, -I * s, -I * s, c); break;
    /* RY(t) = [[cos t/2, -sin t/2], [sin t/2, cos t/2]] */
    case G_RY:  apply_matrix_1q(psi, n, q0, c, -s, s, c); break;
    /* RZ(t) = diag(e^{-i t/2}, e^{+i t/2}) */
    case G_RZ:  apply_matrix_1q(psi, n, q0, cexp(-I * param / 2.0), 0, 0,
                                cexp(I * param / 2.0)); break;
    /* P(t) = diag(1, e^{i t}) */
    case G_P:   apply_matrix_1q(psi, n, q0, 1, 0, 0, cexp(I * param)); break;
    case G_CNOT: {
        /* |b> -> |b xor (b_c << t)>: swap psi[i], psi[i | 2^t] when bit c of
         * i is 1 and bit t of i is 0. */
        uint64_t dim = 1ull << n, cb = 1ull << q0, tb = 1ull << q1;
        int64_t i;
#pragma omp parallel for schedule(static)
        for (i = 0; i < (int64_t)dim; ++i) {
            if (((uint64_t)i & cb) && !((uint64_t)i & tb)) {
                cplx t = psi[i];
                psi[i] = psi[(uint64_t)i | tb];
                psi[(uint64_t)i | tb] = t;
            }
        }
        break;
    }
    case G_CZ: {
        uint64_t dim = 1ull << n, ab = (1ull << q0) | (1ull << q1);
        int64_t i;
#pragma omp parallel for schedule(static)
        for (i = 0; i < (int64_t)dim; ++i)
            if (((uint64_t)i & ab) == ab)
                psi[i] = -psi[i];
        break;
    }
    case G_RENORM: {
        double s2 = norm2(psi, n);
        double f = 1.0 / sqrt(s2);
        uint64_t dim = 1ull << n;
        int64_t i;
#pragma omp parallel for schedule(static)
        for (i = 0; i < (int64_t)dim; ++i)
            psi[i] *= f;
        break;
    }
    default:
        return -1;
    }
    return 0;
}

/* Apply a list of gates in order. Arrays of length ng. */
int qwo_apply_gates(cplx *psi, int n, int64_t ng, const int32_t *code,
                    const int32_t *q0, const int32_t *q1, const double *param)
{
    for (int64_t g = 0; g < ng; ++g)
        if (qwo_apply_gate(psi, n, code[g], q0[g], q1[g], param[g]) != 0)
            return -1 - (int)g;
    return 0;
}

static int popcount64(uint64_t v) { return __builtin_popcountll(v); }

/* <P> for the Pauli string with masks (x, z). */
double qwo_expect_pauli(const cplx *psi, int n, uint64_t x, uint64_t z)
{
    uint64_t dim = 1ull << n;
    int ny = popcount64(x & z);
    cplx iy = 1.0;
    for (int k = 0; k < ny % 4; ++k)
        iy *= I;
    enum { NR = 64 };
    const int nr = dim >= 4096 ? NR : 1;
    const uint64_t len = dim / (uint64_t)nr;
    cplx part[NR];
    int r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < nr; ++r) {
        cplx acc = 0.0;
        for (uint64_t i = (uint64_t)r * len; i < (uint64_t)(r + 1) * len; ++i) {
            double sign = (popcount64(i & z) & 1) ? -1.0 : 1.0;
            acc += conj(psi[i ^ x]) * iy * sign * psi[i];
        }
        part[r] = acc;
    }
    cplx tot = 0.0;
    for (r = 0; r < nr; ++r)
        tot += part[r];
    return creal(tot);
}

/* SplitMix64 output function applied to state v (one increment, then mix). */
uint64_t qwo_splitmix64(uint64_t v)
{
    uint64_t z = v + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Uniform double in [0, 1) for shot s of task t. */
double qwo_uniform(uint64_t seed, uint64_t t, uint64_t s)
{
    uint64_t h = qwo_splitmix64(seed ^ ((t << 32) + s));
    return (double)(h >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
}

/* Draw `shots` Z-basis outcomes for task t: the smallest i with
 * CDF_i > u * total, CDF_i = sum_{k <= i} |psi_k|^2 (sequential sum). */
int qwo_sample(const cplx *psi, int n, uint64_t seed, uint64_t t,
               uint32_t shots, uint32_t *out)
{
    uint64_t dim = 1ull << n;
    double *cdf = (double *)malloc(dim * sizeof(double));
    if (!cdf)
        return -1;
    double run = 0.0;
    for (uint64_t i = 0; i < dim; ++i) {
        run += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
        cdf[i] = run;
    }
    for (uint32_t s = 0; s < shots; ++s) {
        double target = qwo_uniform(seed, t, s) * run;
        uint64_t lo = 0, hi = dim - 1; /* answer in [lo, hi] */
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > target)
                hi = mid;
            else
                lo = mid + 1;
        }
        out[s] = (uint32_t)lo;
    }
    free(cdf);
    return 0;
}
