// Conservation projection (Sec. 3.3) and the explicit collision update.
//
// For each cell, with the 5 x N^3 integration matrix C whose rows are
// dv^3 (1, v^1, v^2, v^3, |v|^2):
//   b  = C Q~                      (five moment sums, always FP64)
//   l  = (C C^T)^{-1} b            ((C C^T)^{-1} is a per-op constant)
//   Qc = Q~ - C^T l
// One workgroup per cell: each thread loads its strided slice of the cell
// into registers once, accumulates the five sums, the wavefronts reduce them
// with lane shuffles and meet in LDS, and every thread then writes the
// corrected slice from its registers.
#include "bz_internal.h"

namespace bz {
namespace {

struct Cct {
    double inv[25];
};

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

// Threads per cell, R = N^3 / TPB values each.  Up to N = 16 (R = 16) a
// thread keeps its values in registers between the moment sums and the
// correction, so each value is read once; for larger meshes it reads them
// again for the correction (holding them, hipcc also kept every value's
// velocity live across both loops and spilled 100 - 700 bytes per lane).
template <int N>
constexpr int conserve_tpb() {
    return N <= 16 ? 256 : (N <= 24 ? 512 : 1024);
}
template <int N>
constexpr bool conserve_holds() {
    return N <= 16;
}

template <typename Tin, int N>
__global__ __launch_bounds__(conserve_tpb<N>()) void conserve_kernel(const Tin *Qt, double *Qc,
                                                                     double *__restrict__ moments, double dv, Cct cct,
                                                                     const int64_t *__restrict__ off,
                                                                     const int32_t *__restrict__ idx) {
    // Qt and Qc may alias (FP64 in place): each element is read and then
    // written by the same thread.
    constexpr int n3 = N * N * N, TPB = conserve_tpb<N>(), R = n3 / TPB, NW = TPB / kWave;
    static_assert(n3 % TPB == 0, "cells must split evenly over the threads");
    constexpr int c = N / 2;
    const int64_t cell = blockIdx.x;
    const int64_t base = off ? off[cell] : cell * (int64_t)n3;
    const Tin *q = Qt + base;
    constexpr bool hold = conserve_holds<N>();
    constexpr int RH = hold ? R : 1;
    double x[RH];
    if constexpr (hold) {
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = (double)q[r * TPB + threadIdx.x];
    }
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
    auto add = [&](int j, double xr) {
        const double v1 = dv * (j / (N * N) - c), v2 = dv * ((j / N) % N - c), v3 = dv * (j % N - c);
        s0 += xr;
        s1 += xr * v1;
        s2 += xr * v2;
        s3 += xr * v3;
        s4 += xr * (v1 * v1 + v2 * v2 + v3 * v3);
    };
    if constexpr (hold) {
#pragma unroll
        for (int r = 0; r < R; ++r) add(r * TPB + threadIdx.x, x[r]);
    } else {
#pragma unroll 4
        for (int r = 0; r < R; ++r) add(r * TPB + threadIdx.x, (double)q[r * TPB + threadIdx.x]);
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    s3 = wave_sum(s3);
    s4 = wave_sum(s4);
    __shared__ double red[NW][5];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0) {
        red[wave][0] = s0;
        red[wave][1] = s1;
        red[wave][2] = s2;
        red[wave][3] = s3;
        red[wave][4] = s4;
    }
    __syncthreads();
    const double w = dv * dv * dv;
    double b[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        double t = 0.0;
#pragma unroll
        for (int u = 0; u < NW; ++u) t += red[u][a];
        b[a] = w * t;
    }
    double lam[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        double t = 0.0;
#pragma unroll
        for (int e = 0; e < 5; ++e) t += cct.inv[a * 5 + e] * b[e];
        lam[a] = t;
    }
    if (moments && threadIdx.x < 5) {
        // a cell whose sums are not all finite gets the flag value in all
        // five places, so one test of any of them finds it
        bool finite = true;
#pragma unroll
        for (int a = 0; a < 5; ++a) finite = finite && __builtin_isfinite(b[a]);
        moments[(idx ? (int64_t)idx[cell] : cell) * 5 + threadIdx.x] =
            finite ? b[threadIdx.x] : __longlong_as_double((long long)BZ_MOMENTS_NONFINITE_BITS);
    }
    double *out = Qc + base;
    auto put = [&](int j, double xr) {
        const double v1 = dv * (j / (N * N) - c), v2 = dv * ((j / N) % N - c), v3 = dv * (j % N - c);
        out[j] = xr - w * (lam[0] + lam[1] * v1 + lam[2] * v2 + lam[3] * v3 + lam[4] * (v1 * v1 + v2 * v2 + v3 * v3));
    };
    if constexpr (hold) {
#pragma unroll
        for (int r = 0; r < R; ++r) put(r * TPB + threadIdx.x, x[r]);
    } else {
#pragma unroll 4
        for (int r = 0; r < R; ++r) put(r * TPB + threadIdx.x, (double)q[r * TPB + threadIdx.x]);
    }
}

template <typename Tin, int N>
void launch_conserve_n(const bz_op *op, int64_t ncells, const void *Qt, double *Qc, double *moments, hipStream_t s,
                       const Cct &cct, const int64_t *off, const int32_t *idx) {
    hipLaunchKernelGGL((conserve_kernel<Tin, N>), dim3((unsigned)ncells), dim3(conserve_tpb<N>()), 0, s,
                       (const Tin *)Qt, Qc, moments, op->geo.dv, cct, off, idx);
}

__global__ __launch_bounds__(256) void axpy_kernel(int64_t n, double alpha, const double *__restrict__ x,
                                                   double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += alpha * x[i];
}

__global__ __launch_bounds__(256) void axpbz_kernel(int64_t n, const double *__restrict__ x, double a,
                                                    const double *__restrict__ y, double *__restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = x[i] + a * y[i];
}

__global__ __launch_bounds__(256) void heun_finish_kernel(int64_t n, double a, const double *__restrict__ y1,
                                                          const double *__restrict__ y2, double *__restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f[i] += a * (y1[i] + y2[i]);
}

}  // namespace

hipError_t launch_axpbz(int64_t n, const double *x, double a, const double *y, double *z, hipStream_t s) {
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipLaunchKernelGGL(axpbz_kernel, grid, block, 0, s, n, x, a, y, z);
    return hipGetLastError();
}

hipError_t launch_heun_finish(int64_t n, double a, const double *y1, const double *y2, double *f, hipStream_t s) {
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipLaunchKernelGGL(heun_finish_kernel, grid, block, 0, s, n, a, y1, y2, f);
    return hipGetLastError();
}

hipError_t launch_conserve(const bz_op *op, int64_t ncells, const void *Qt, int in_dtype, double *Qc, double *moments,
                           hipStream_t s, const int64_t *off, const int32_t *idx) {
    Cct cct;
    for (int i = 0; i < 25; ++i) cct.inv[i] = op->cct_inv[i];
    const bool f64 = in_dtype == BZ_F64;
    switch (op->N) {
#define BZ_CONS_CASE(NN)                                                                                    \
    case NN:                                                                                                \
        if (f64)                                                                                            \
            launch_conserve_n<double, NN>(op, ncells, Qt, Qc, moments, s, cct, off, idx);                  \
        else                                                                                                \
            launch_conserve_n<float, NN>(op, ncells, Qt, Qc, moments, s, cct, off, idx);                   \
        break;
        BZ_CONS_CASE(8)
        BZ_CONS_CASE(16)
        BZ_CONS_CASE(24)
        BZ_CONS_CASE(32)
        BZ_CONS_CASE(48)
#undef BZ_CONS_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_axpy(int64_t n, double alpha, const double *x, double *y, hipStream_t s) {
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipLaunchKernelGGL(axpy_kernel, grid, block, 0, s, n, alpha, x, y);
    return hipGetLastError();
}

}  // namespace bz
