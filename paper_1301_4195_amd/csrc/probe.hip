// Ceiling probes for the roofline figures of the benchmark (a separate
// library, libbzprobe.so; nothing of the collision path uses it):
//   * vector FMA issue: independent FMA chains in registers, FP64 and FP32
//     (non-packed: the library is built without packed FP32), with all-VGPR
//     operands and with one wave-uniform (SGPR) operand as the convolution's
//     weights are;
//   * memory streams: a read-only pass and a copy over a buffer larger than
//     the 256 MB last-level cache (HBM) and over one that fits in it but not
//     in the 4 MB L2 of each XCD (last-level cache), four loads in flight per
//     thread.
// Each entry point times its kernel with HIP events on the given stream and
// returns milliseconds per launch.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 8;  // independent accumulators per thread

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// a_i <- a_i * x + y, kChains chains, iters rounds: 2 * kChains * iters flops
// per thread.  x, y differ per thread so nothing folds; the sums are stored so
// nothing is dropped.
template <typename T>
__global__ __launch_bounds__(256) void fma_vgpr_kernel(T *out, int iters, T seed) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const T x = (T)1 - (T)(t & 7) * (T)1e-7, y = seed * (T)(t & 15);
    T a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = (T)i;
#pragma unroll 4
    for (int r = 0; r < iters; ++r) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = fma_t(a[i], x, y);
    }
    T s = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i];
    out[t] = s;
}

// the same with the multiplier a kernel argument: a wave-uniform scalar operand
template <typename T>
__global__ __launch_bounds__(256) void fma_sgpr_kernel(T *out, int iters, T x) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const T y = (T)(t & 15) * (T)1e-9;
    T a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = (T)(i + (t & 3));
#pragma unroll 4
    for (int r = 0; r < iters; ++r) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = fma_t(a[i], x, y);
    }
    T s = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i];
    out[t] = s;
}

// read-only stream: every 16-byte vector of buf once per pass (grid-stride,
// four independent loads in flight per thread), summed per thread, one value
// per thread written
__global__ __launch_bounds__(256) void read_kernel(const uint4 *__restrict__ buf, int64_t n16, uint32_t *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t s = 0;
    int64_t i = t;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const uint4 a = buf[i], b = buf[i + stride], c = buf[i + 2 * stride], d = buf[i + 3 * stride];
        s += (a.x ^ a.y ^ a.z ^ a.w) + (b.x ^ b.y ^ b.z ^ b.w) + (c.x ^ c.y ^ c.z ^ c.w) + (d.x ^ d.y ^ d.z ^ d.w);
    }
    for (; i < n16; i += stride) {
        const uint4 v = buf[i];
        s += v.x ^ v.y ^ v.z ^ v.w;
    }
    out[t] = s;
}

__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n16) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = t;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

template <typename K>
int time_launches(K launch, int reps, hipStream_t s, double *ms_per_launch) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -3;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -3;
    }
    launch();  // warm-up
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return -3;
    *ms_per_launch = ms / reps;
    return 0;
}

}  // namespace

extern "C" {

// FMA issue probe.  fp64: 1 FP64 / 0 FP32; sgpr: 1 = wave-uniform multiplier.
// out: device buffer of blocks * 256 values of that type.  Returns 0, or -1
// for bad arguments, -3 for a HIP failure.  flops = 2 * 8 * iters * blocks * 256.
int bzp_fma(int fp64, int sgpr, int blocks, int iters, void *out, int reps, void *stream, double *ms_per_launch) {
    if (blocks < 1 || iters < 1 || reps < 1 || !out || !ms_per_launch) return -1;
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid(blocks), block(256);
    if (fp64) {
        double *o = (double *)out;
        return sgpr ? time_launches([&] { hipLaunchKernelGGL(fma_sgpr_kernel<double>, grid, block, 0, s, o, iters, 0.999999); }, reps, s, ms_per_launch)
                    : time_launches([&] { hipLaunchKernelGGL(fma_vgpr_kernel<double>, grid, block, 0, s, o, iters, 1e-9); }, reps, s, ms_per_launch);
    }
    float *o = (float *)out;
    return sgpr ? time_launches([&] { hipLaunchKernelGGL(fma_sgpr_kernel<float>, grid, block, 0, s, o, iters, 0.999999f); }, reps, s, ms_per_launch)
                : time_launches([&] { hipLaunchKernelGGL(fma_vgpr_kernel<float>, grid, block, 0, s, o, iters, 1e-9f); }, reps, s, ms_per_launch);
}

// Stream probe over nbytes (a multiple of 16) of device memory: copy = 0 reads
// src once per launch (sums into out: blocks * 256 uint32), copy = 1 copies src
// to dst.  Bytes moved per launch: nbytes (read) or 2 * nbytes (copy).
int bzp_stream(int copy, const void *src, void *dst, int64_t nbytes, int blocks, void *out, int reps, void *stream,
               double *ms_per_launch) {
    if (nbytes <= 0 || nbytes % 16 || blocks < 1 || reps < 1 || !src || !ms_per_launch) return -1;
    if ((copy && !dst) || (!copy && !out)) return -1;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n16 = nbytes / 16;
    const dim3 grid(blocks), block(256);
    if (copy)
        return time_launches([&] { hipLaunchKernelGGL(copy_kernel, grid, block, 0, s, (const uint4 *)src, (uint4 *)dst, n16); },
                             reps, s, ms_per_launch);
    return time_launches([&] { hipLaunchKernelGGL(read_kernel, grid, block, 0, s, (const uint4 *)src, n16, (uint32_t *)out); },
                         reps, s, ms_per_launch);
}

}  // extern "C"
