// Truncated weighted convolution of the collision step (Sec. 3.2):
//   Q^(zeta_k) = sum_{m : k - m + N/2 in [0,N)^3} W[k][m] f^(xi_m) f^(zeta_k - xi_m)
// for a batch of independent cells.  This is the O(N^6) term that dominates
// the run time (Sec. 4.1).
//
// Mapping on CDNA (wave64):
//   * one lane = one cell.  The workspace f^ is [mode][cell], so a wavefront
//     loading one mode for its 64 cells reads one contiguous, coalesced block.
//   * the pairs m and n = k - m + N/2 carry the same product f^_m f^_n, so each
//     mirrored couple is summed once with the stored weight W[k][m] + W[k][n]:
//     half of the lines (m1, m2) of a row are visited (see half_lines).
//   * a wavefront owns one row (k1, k2) of outputs, all N values of k3, for 64
//     cells, and sweeps the kept lines (m1, m2) of that row (optionally one
//     chunk of the m1 range: items with chunk > 0 write separate partial sums
//     that the first inverse-transform pass adds in a fixed order).
//   * for each line the lane loads u = f^(m1, m2, .) and
//     v = f^(k1-m1+N/2, k2-m2+N/2, .) into registers and forms all 3N^2/4
//     valid (k3, m3) products of the line, so each loaded value is reused
//     ~3N/8 times.
//   * the weights of a line are the same for all 64 cells: one weight fetch
//     serves 64 cells, so the weight stream from memory is cut by the batch
//     size.  They are read with scalar loads into SGPRs, one m3 group ahead
//     of their use, and enter the multiply-adds as scalar operands (no LDS or
//     vector-register traffic for them).
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
    // u(m3) is needed by group m3 only and is loaded kUA groups ahead; v(n3)
    // with n3 < N/2 is first needed by group N/2 - n3 and is loaded kVA groups
    // ahead; v(n3) with n3 >= N/2 is needed from group 0 and is loaded during
    // the previous line, into its register as soon as that line's last use of
    // it has passed (group 3N/2 - 1 - n3).  No line starts by waiting for a
    // whole line of loads.
    constexpr int kUA = 2, kVA = 2;
    const ConvItem it = items[blockIdx.x];
    if (it.row < 0) return;  // padding of the per-XCD schedule
    const int64_t cell = (int64_t)it.group * kWave + threadIdx.x;
    const int k1 = it.row / N, k2 = it.row % N;
    const int lo1 = mlo(N, k1), c1 = mcount(N, k1);
    const int lo2 = mlo(N, k2), c2 = mcount(N, k2);
    // kept half of the mirrored lines (half_a1_end / half_a2_end), m1 range
    // split into S chunks; the chunk's lines are consecutive in (a1, a2) order
    const int h1 = half_a1_end(c1);
    const int per = (h1 + S - 1) / S;
    const int a1b = min(h1, it.chunk * per);
    const int a1e = min(h1, a1b + per);
    const int nlines = a1e <= a1b ? 0
                                  : (a1e - a1b - 1) * c2 + half_a2_end(c1, c2, a1e - 1);

    // FP64: one running sum per output.  FP32: the terms of each (m1, m2) line
    // are summed into a fresh partial (about 3N/4 terms), and the partials are
    // added to the running sum with Kahan compensation, so the long sum over
    // lines loses no accuracy to FP32 rounding.
    constexpr bool kComp = sizeof(T) == 4;
    T ar[N], ai[N], cr[N], ci[N];
#pragma unroll
    for (int k3 = 0; k3 < N; ++k3) ar[k3] = ai[k3] = cr[k3] = ci[k3] = (T)0;

    const int64_t ls = (int64_t)N * cellpad;  // distance between consecutive (m1, m2) lines
    const T *wline = W + rowoff[it.row] + (int64_t)a1b * c2 * P;
    int a1 = a1b, a2 = 0;
    const C2<T> *up = fhat + (int64_t)((lo1 + a1) * N + lo2) * ls + cell;
    const C2<T> *vp = fhat + (int64_t)((k1 - lo1 - a1 + c) * N + (k2 - lo2 + c)) * ls + cell;
    C2<T> u[N], v[N];
    if (nlines > 0) {
#pragma unroll
        for (int t = c; t < N; ++t) v[t] = vp[(int64_t)t * cellpad];
#pragma unroll
        for (int t = 0; t < kUA; ++t) u[t] = up[(int64_t)t * cellpad];
    }
    for (int l = 0; l < nlines; ++l) {
        // the next line of the chunk (the last line names itself: its
        // look-ahead loads are then redundant but stay in bounds)
        int na1 = a1, na2 = a2 + 1;
        if (na2 >= half_a2_end(c1, c2, a1)) {
            na1 = a1 + 1;
            na2 = 0;
        }
        const bool more = l + 1 < nlines;
        const C2<T> *upn = more ? fhat + (int64_t)((lo1 + na1) * N + lo2 + na2) * ls + cell : up;
        const C2<T> *vpn = more ? fhat + (int64_t)((k1 - lo1 - na1 + c) * N + (k2 - lo2 - na2 + c)) * ls + cell : vp;
        __builtin_amdgcn_sched_barrier(0);
        // m3 outer, k3 inner: consecutive multiply-adds go to different
        // outputs, so none waits on the previous one's result.
        T sr[N], si[N];
        if constexpr (kComp) {
#pragma unroll
            for (int k3 = 0; k3 < N; ++k3) sr[k3] = si[k3] = (T)0;
        }
        // weights as scalar operands, loaded one m3 group ahead: wait for
        // the current group, then issue the next group's scalar loads
        const T *__restrict__ wl = wline;
        T wc[N];
#pragma unroll
        for (int i = 0; i < kcount(N, 0); ++i) wc[i] = wl[i];
        int p = 0;
#pragma unroll
        for (int m3 = 0; m3 < N; ++m3) {
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
            T wn[N];
            if (m3 + 1 < N) {
#pragma unroll
                for (int i = 0; i < kcount(N, m3 + 1); ++i) wn[i] = wl[p + kcount(N, m3) + i];
            }
            // vector loads of this group, issued in the order of first use
            if (m3 + kUA < N)
                u[m3 + kUA] = up[(int64_t)(m3 + kUA) * cellpad];
            else
                u[m3 + kUA - N] = upn[(int64_t)(m3 + kUA - N) * cellpad];
            if (m3 == 0) {
                v[c - 1] = vp[(int64_t)(c - 1) * cellpad];
                v[c - 2] = vp[(int64_t)(c - 2) * cellpad];
            } else if (c - 2 - m3 >= 0) {
                v[c - 2 - m3] = vp[(int64_t)(c - 2 - m3) * cellpad];
            }
            if (m3 >= c + 1) v[N + c - m3] = vpn[(int64_t)(N + c - m3) * cellpad];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k3 = klo(N, m3); k3 <= khi(N, m3); ++k3) {
                const int n3 = k3 - m3 + c;
                const T w = wc[k3 - klo(N, m3)];
                const T pr = u[m3].re * v[n3].re - u[m3].im * v[n3].im;
                const T pi = u[m3].re * v[n3].im + u[m3].im * v[n3].re;
                if constexpr (kComp) {
                    sr[k3] += w * pr;
                    si[k3] += w * pi;
                } else {
                    ar[k3] += w * pr;
                    ai[k3] += w * pi;
                }
            }
            p += kcount(N, m3);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < N; ++i) wc[i] = wn[i];
        }
        // v(N/2) is used up to the last group: its next value comes now
        v[c] = vpn[(int64_t)c * cellpad];
        __builtin_amdgcn_sched_barrier(0);
        wline += P;
        up = upn;
        vp = vpn;
        a1 = na1;
        a2 = na2;
        if constexpr (kComp) {
#pragma unroll
            for (int k3 = 0; k3 < N; ++k3) {
                const T yr = sr[k3] - cr[k3], yi = si[k3] - ci[k3];
                const T tr = ar[k3] + yr, ti = ai[k3] + yi;
                cr[k3] = (tr - ar[k3]) - yr;
                ci[k3] = (ti - ai[k3]) - yi;
                ar[k3] = tr;
                ai[k3] = ti;
            }
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
