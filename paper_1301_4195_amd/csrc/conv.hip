// Truncated weighted convolution of the collision step (Sec. 3.2):
//   Q^(zeta_k) = sum_{m : k - m + N/2 in [0,N)^3} W[k][m] f^(xi_m) f^(zeta_k - xi_m)
// for a batch of independent cells.  This is the O(N^6) term that dominates
// the run time (Sec. 4.1).
//
// Mapping on CDNA (wave64):
//   * one lane = one cell.  The workspace f^ is [mode][cell], so a wavefront
//     loading one mode for its 64 cells reads one contiguous, coalesced block.
//   * a wavefront owns one row (k1, k2) of outputs, all N values of k3, for 64
//     cells, and sweeps the valid (m1, m2) of that row (optionally one chunk
//     of the m1 range: items with chunk > 0 write separate partial sums that
//     the first inverse-transform pass adds in a fixed order).
//   * for each (m1, m2) the lane loads the two lines u = f^(m1, m2, .) and
//     v = f^(k1-m1+N/2, k2-m2+N/2, .) into registers and forms all 3N^2/4
//     valid (k3, m3) products of the line, so each loaded value is reused
//     ~3N/8 times.
//   * the weights of a line are the same for all 64 cells: they are read with
//     wave-uniform (scalar) loads and fed to the FMAs as scalar operands, so
//     one weight fetch serves 64 cells and the weight stream from memory is
//     cut by the batch size.
#include "bz_internal.h"

namespace bz {
namespace {

template <typename T>
struct C2 {
    T re, im;
};

template <typename T, int N>
__global__ __launch_bounds__(64) void conv_kernel(const C2<T> *__restrict__ fhat, C2<T> *__restrict__ part,
                                                  const T *__restrict__ W, const int64_t *__restrict__ rowoff,
                                                  const ConvItem *__restrict__ items, int64_t cellpad, int S) {
    constexpr int c = N / 2;
    constexpr int P = line_pairs(N);
    const ConvItem it = items[blockIdx.x];
    const int64_t cell = (int64_t)it.group * kWave + threadIdx.x;
    const int k1 = it.row / N, k2 = it.row % N;
    const int lo1 = mlo(N, k1), c1 = mcount(N, k1);
    const int lo2 = mlo(N, k2), c2 = mcount(N, k2);
    const int per = (c1 + S - 1) / S;
    const int a1b = it.chunk * per;
    const int a1e = min(c1, a1b + per);

    // FP64: one running sum per output.  FP32: the terms of each (m1, m2) line
    // are summed into a fresh partial (about 3N/4 terms), and the partials are
    // added to the running sum with Kahan compensation, so the long sum over
    // lines loses no accuracy to FP32 rounding.
    constexpr bool kComp = sizeof(T) == 4;
    T ar[N], ai[N], cr[N], ci[N];
#pragma unroll
    for (int k3 = 0; k3 < N; ++k3) ar[k3] = ai[k3] = cr[k3] = ci[k3] = (T)0;

    const T *wline = W + rowoff[it.row] + (int64_t)a1b * c2 * P;
    for (int a1 = a1b; a1 < a1e; ++a1) {
        const int m1 = lo1 + a1, n1 = k1 - m1 + c;
        for (int a2 = 0; a2 < c2; ++a2) {
            const int m2 = lo2 + a2, n2 = k2 - m2 + c;
            const C2<T> *up = fhat + (int64_t)((m1 * N + m2) * N) * cellpad + cell;
            const C2<T> *vp = fhat + (int64_t)((n1 * N + n2) * N) * cellpad + cell;
            C2<T> u[N], v[N];
#pragma unroll
            for (int t = 0; t < N; ++t) {
                u[t] = up[(int64_t)t * cellpad];
                v[t] = vp[(int64_t)t * cellpad];
            }
            int p = 0;
#pragma unroll
            for (int k3 = 0; k3 < N; ++k3) {
                T sr = (T)0, si = (T)0;
#pragma unroll
                for (int m3 = mlo(N, k3); m3 <= mhi(N, k3); ++m3) {
                    const int n3 = k3 - m3 + c;
                    const T w = wline[p++];
                    const T pr = u[m3].re * v[n3].re - u[m3].im * v[n3].im;
                    const T pi = u[m3].re * v[n3].im + u[m3].im * v[n3].re;
                    if constexpr (kComp) {
                        sr += w * pr;
                        si += w * pi;
                    } else {
                        ar[k3] += w * pr;
                        ai[k3] += w * pi;
                    }
                }
                if constexpr (kComp) {
                    const T yr = sr - cr[k3], yi = si - ci[k3];
                    const T tr = ar[k3] + yr, ti = ai[k3] + yi;
                    cr[k3] = (tr - ar[k3]) - yr;
                    ci[k3] = (ti - ai[k3]) - yi;
                    ar[k3] = tr;
                    ai[k3] = ti;
                }
            }
            wline += P;
        }
    }
    C2<T> *out = part + ((int64_t)it.chunk * N * N * N + (int64_t)it.row * N) * cellpad + cell;
#pragma unroll
    for (int k3 = 0; k3 < N; ++k3) out[(int64_t)k3 * cellpad] = C2<T>{ar[k3], ai[k3]};
}

template <typename T, int N>
hipError_t conv_n(const bz_op *op, int64_t cellpad, int S, const void *fhat, void *part, hipStream_t s) {
    const dim3 grid((unsigned)op->n_items), block(kWave);
    hipLaunchKernelGGL((conv_kernel<T, N>), grid, block, 0, s, (const C2<T> *)fhat, (C2<T> *)part, (const T *)op->W,
                       op->d_rowoff, op->d_items, cellpad, S);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_conv(const bz_op *op, int64_t cellpad, int S, const void *fhat, void *part, hipStream_t s) {
    const bool f64 = op->wdtype == BZ_F64;
    switch (op->N) {
#define BZ_CONV_CASE(NN) \
    case NN:             \
        return f64 ? conv_n<double, NN>(op, cellpad, S, fhat, part, s) : conv_n<float, NN>(op, cellpad, S, fhat, part, s);
        BZ_CONV_CASE(8)
        BZ_CONV_CASE(16)
        BZ_CONV_CASE(24)
        BZ_CONV_CASE(32)
#undef BZ_CONV_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace bz
