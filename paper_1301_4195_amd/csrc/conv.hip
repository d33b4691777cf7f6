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
//   * a wavefront owns one row (k1, k2) of outputs for 64 cells -- all N
//     values of k3, or one of KH = 2 or 4 equal k3 ranges (fewer registers,
//     so more wavefronts per SIMD, for KH times the loads per term) -- and
//     sweeps the
//     kept lines (m1, m2) of that row (optionally one chunk of the m1 range:
//     items with chunk > 0 write separate partial sums that the first
//     inverse-transform pass adds in a fixed order).
//   * for each line the lane holds u = f^(m1, m2, .) and
//     v = f^(k1-m1+N/2, k2-m2+N/2, .) in registers and forms every valid
//     (k3, m3) product of its k3 range, so each loaded value is reused up to
//     3N/8 times.  Each value is loaded a fixed number of m3 groups before
//     its first use -- during the previous line when it is needed that
//     early, into a register the previous line no longer reads -- so no line
//     starts by waiting for its loads.
//   * the weights of a line are the same for all 64 cells: one weight fetch
//     serves 64 cells, so the weight stream from memory is cut by the batch
//     size.  They are read with scalar loads into SGPRs, one m3 group ahead
//     of their use, and enter the multiply-adds as scalar operands (no LDS or
//     vector-register traffic for them).
#include "bz_internal.h"

#include <type_traits>

namespace bz {
namespace {

template <typename T>
struct C2 {
    T re, im;
};

// one complex value through a plain or address-space-marked pointer
template <typename T, typename P>
__device__ __forceinline__ C2<T> ld2(P p) {
    return C2<T>{p->re, p->im};
}
template <typename P, typename T>
__device__ __forceinline__ void st2(P p, T re, T im) {
    p->re = re;
    p->im = im;
}

constexpr int kUA = 2;  // u(m3) is loaded this many m3 groups before its use
constexpr int kVA = 2;  // v(n3) likewise, before its first use

// Schedule of one line for the wavefronts that own outputs k3 in
// [H N/KH, (H+1) N/KH).  Group m3 of the line updates the contiguous outputs
// [glo, ghi] (none when glo > ghi) with the weights at woff.. of the line's
// block (m3-major, k3 ascending).  u(m3) is loaded kUA groups ahead (for the
// first kUA groups: in the previous line's last groups).  For each v value it
// records the group whose start issues the load: in the same line (v_same,
// kVA groups ahead of the first use, or at the line start), or, for values
// the first group needs, in the previous line after its last use there
// (v_prev; N = after the previous line's last group).
template <int N, int KH, int H>
struct LinePlan {
    int glo[N], ghi[N], woff[N];
    bool u_used[N];         // u(m3) is read by this k3 range
    int v_same[N], v_prev[N];
    // the same v schedule as lists per issuing group g (g = N: line end)
    int ns[N + 1], s_list[N + 1][N], np[N + 1], p_list[N + 1][N];
    constexpr LinePlan()
        : glo(), ghi(), woff(), u_used(), v_same(), v_prev(), ns(), s_list(), np(), p_list() {
        constexpr int c = N / 2, kb = H * (N / KH), ke = (H + 1) * (N / KH);
        int p = 0;
        for (int m = 0; m < N; ++m) {
            const int lo = klo(N, m), hi = khi(N, m);
            glo[m] = lo > kb ? lo : kb;
            ghi[m] = hi < ke - 1 ? hi : ke - 1;
            woff[m] = p + (glo[m] - lo);
            p += hi - lo + 1;
            u_used[m] = glo[m] <= ghi[m];
        }
        for (int n = 0; n < N; ++n) {
            int first = -1, last = -1;
            for (int m = 0; m < N; ++m) {
                const int k = n + m - c;
                if (k >= glo[m] && k <= ghi[m]) {
                    if (first < 0) first = m;
                    last = m;
                }
            }
            v_same[n] = v_prev[n] = -1;
            if (first < 0) continue;
            if (first > 0)
                v_same[n] = first > kVA ? first - kVA : 0;
            else
                v_prev[n] = last + 1;
        }
        // issue order inside a group: the value needed first goes first
        for (int g = 0; g <= N; ++g) {
            for (int n = N - 1; n >= 0; --n)
                if (v_same[n] == g) s_list[g][ns[g]++] = n;
            for (int n = 0; n < N; ++n)
                if (v_prev[n] == g) p_list[g][np[g]++] = n;
        }
    }
};

// PF, PP, PW: pointer types of f^, the partial sums and the weights (plain
// pointers, or pointers marked as global memory where the compiler could not
// infer it).
template <typename T, int N, int KH, int H, typename PF, typename PP, typename PW>
__device__ __forceinline__ void conv_lines(PF __restrict__ fhat, PP __restrict__ part, int64_t outoff,
                                           PW __restrict__ wline, int k1, int k2, int lo1, int lo2, int c1, int c2,
                                           int a1b, int nlines, int64_t cellpad, int64_t cell) {
    constexpr int c = N / 2;
    constexpr int P = line_pairs(N);
    constexpr int NK = N / KH, kb = H * NK;
    constexpr LinePlan<N, KH, H> pl{};

    // FP64: one running sum per output.  FP32: the terms of each (m1, m2)
    // line (about 3N/4 per output) are summed in FP32 into a fresh partial,
    // and the partial is added to an FP64 running sum -- as many registers as
    // a compensated FP32 sum and half its instructions (convert + add instead
    // of four adds), and the long sum over lines then loses nothing to FP32
    // rounding; the sums that gain and loss cancel in have terms hundreds of
    // times larger than their result.  From N = 32 a partial spans two lines:
    // folding every line there took the two-range variant from three to two
    // wavefronts per SIMD (155 -> 181 VGPRs, 18.1 -> 22.8 ms per 512-cell
    // convolution), and its cells' errors stay near 2e-6 either way.
    constexpr bool kComp = sizeof(T) == 4;
    constexpr int kFold = N >= 32 ? 2 : 1;  // lines per FP32 partial
    using TA = std::conditional_t<kComp, double, T>;  // running-sum type
    TA ar[NK], ai[NK];
    T sr[NK], si[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        ar[j] = ai[j] = (TA)0;
        sr[j] = si[j] = (T)0;
    }

    const int64_t ls = (int64_t)N * cellpad;  // distance between consecutive (m1, m2) lines
    int a1 = a1b, a2 = 0;
    PF up = fhat + (int64_t)((lo1 + a1) * N + lo2) * ls + cell;
    PF vp = fhat + (int64_t)((k1 - lo1 - a1 + c) * N + (k2 - lo2 + c)) * ls + cell;
    C2<T> u[N], v[N];
    if (nlines > 0) {
        // the values the first line needs before its own loads arrive
#pragma unroll
        for (int t = 0; t < kUA; ++t)
            if (pl.u_used[t]) u[t] = ld2<T>(up + ((int64_t)t * cellpad));
#pragma unroll
        for (int g = 0; g <= N; ++g) {
#pragma unroll
            for (int j = 0; j < pl.np[g]; ++j) v[pl.p_list[g][j]] = ld2<T>(vp + ((int64_t)pl.p_list[g][j] * cellpad));
        }
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
        PF upn = more ? fhat + (int64_t)((lo1 + na1) * N + lo2 + na2) * ls + cell : up;
        PF vpn = more ? fhat + (int64_t)((k1 - lo1 - na1 + c) * N + (k2 - lo2 - na2 + c)) * ls + cell : vp;
        __builtin_amdgcn_sched_barrier(0);
        // weights as scalar operands, loaded one m3 group ahead: wait for
        // the current group, then issue the next group's scalar loads
        PW __restrict__ wl = wline;
        T wc[NK];
        if (pl.glo[0] <= pl.ghi[0]) {
#pragma unroll
            for (int i = 0; i <= pl.ghi[0] - pl.glo[0]; ++i) wc[i] = wl[pl.woff[0] + i];
        }
#pragma unroll
        for (int m3 = 0; m3 < N; ++m3) {
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
            T wn[NK];
            if (m3 + 1 < N && pl.glo[m3 + 1] <= pl.ghi[m3 + 1]) {
#pragma unroll
                for (int i = 0; i <= pl.ghi[m3 + 1] - pl.glo[m3 + 1]; ++i) wn[i] = wl[pl.woff[m3 + 1] + i];
            }
            // vector loads of this group: values of this line needed kUA / kVA
            // groups from now, then early values of the next line
            if (m3 + kUA < N) {
                if (pl.u_used[m3 + kUA]) u[m3 + kUA] = ld2<T>(up + ((int64_t)(m3 + kUA) * cellpad));
            }
#pragma unroll
            for (int j = 0; j < pl.ns[m3]; ++j) v[pl.s_list[m3][j]] = ld2<T>(vp + ((int64_t)pl.s_list[m3][j] * cellpad));
            if (m3 + kUA >= N) {
                if (pl.u_used[m3 + kUA - N]) u[m3 + kUA - N] = ld2<T>(upn + ((int64_t)(m3 + kUA - N) * cellpad));
            }
#pragma unroll
            for (int j = 0; j < pl.np[m3]; ++j) v[pl.p_list[m3][j]] = ld2<T>(vpn + ((int64_t)pl.p_list[m3][j] * cellpad));
            __builtin_amdgcn_sched_barrier(0);
            // m3 outer, k3 inner: consecutive multiply-adds go to different
            // outputs, so none waits on the previous one's result.
#pragma unroll
            for (int k3 = pl.glo[m3]; k3 <= pl.ghi[m3]; ++k3) {
                const int n3 = k3 - m3 + c;
                const T w = wc[k3 - pl.glo[m3]];
                const T pr = u[m3].re * v[n3].re - u[m3].im * v[n3].im;
                const T pi = u[m3].re * v[n3].im + u[m3].im * v[n3].re;
                if constexpr (kComp) {
                    sr[k3 - kb] += w * pr;
                    si[k3 - kb] += w * pi;
                } else {
                    ar[k3 - kb] += w * pr;
                    ai[k3 - kb] += w * pi;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < NK; ++i) wc[i] = wn[i];
        }
        // values of the next line whose last use here was the last group
#pragma unroll
        for (int j = 0; j < pl.np[N]; ++j) v[pl.p_list[N][j]] = ld2<T>(vpn + ((int64_t)pl.p_list[N][j] * cellpad));
        __builtin_amdgcn_sched_barrier(0);
        wline += P;
        up = upn;
        vp = vpn;
        a1 = na1;
        a2 = na2;
        if (kComp && (kFold == 1 || (l % kFold) == kFold - 1 || l + 1 == nlines)) {  // fold the partial
#pragma unroll
            for (int j = 0; j < NK; ++j) {
                ar[j] += (double)sr[j];
                ai[j] += (double)si[j];
                sr[j] = si[j] = (T)0;
            }
        }
    }
    PP out = part + outoff + cell;
#pragma unroll
    for (int j = 0; j < NK; ++j) st2(out + (int64_t)(kb + j) * cellpad, (T)ar[j], (T)ai[j]);
}

// One item: output row it.row, m1 chunk it.chunk of S, cells of group
// it.group, k3 range it.half of KH.
template <typename T, int N, int KH, typename PF, typename PP, typename PW, typename PR>
__device__ __forceinline__ void conv_item(PF __restrict__ fhat, PP __restrict__ part, PW __restrict__ W,
                                          PR __restrict__ rowoff, int64_t wbase, const ConvItem &it, int64_t cellpad,
                                          int S) {
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
    const int nlines = a1e <= a1b ? 0 : (a1e - a1b - 1) * c2 + half_a2_end(c1, c2, a1e - 1);
    PW wline = W + (rowoff[it.row] - wbase) + (int64_t)a1b * c2 * line_pairs(N);
    const int64_t outoff = ((int64_t)it.chunk * N * N * N + (int64_t)it.row * N) * cellpad;
#define BZ_LINES(H) \
    conv_lines<T, N, KH, H>(fhat, part, outoff, wline, k1, k2, lo1, lo2, c1, c2, a1b, nlines, cellpad, cell)
    if constexpr (KH == 1) {
        BZ_LINES(0);
    } else if constexpr (KH == 2) {
        if (it.half == 0)
            BZ_LINES(0);
        else
            BZ_LINES(1);
    } else {
        static_assert(KH == 4, "one, two or four k3 ranges");
        if (it.half == 0)
            BZ_LINES(0);
        else if (it.half == 1)
            BZ_LINES(1);
        else if (it.half == 2)
            BZ_LINES(2);
        else
            BZ_LINES(3);
    }
#undef BZ_LINES
}

template <typename T, int N, int KH>
__global__ __launch_bounds__(64) void conv_kernel(const C2<T> *__restrict__ fhat, C2<T> *__restrict__ part,
                                                  const T *__restrict__ W, const int64_t *__restrict__ rowoff,
                                                  int64_t wbase, const ConvItem *__restrict__ items, int64_t cellpad,
                                                  int S) {
    const ConvItem it = items[blockIdx.x];
    if (it.row < 0) return;  // padding of the per-XCD schedule
    conv_item<T, N, KH>(fhat, part, W, rowoff, wbase, it, cellpad, S);
}

// A pointer read from memory is a generic (flat) address to the compiler,
// which then emits flat loads: no scalar loads for the weights, and every
// f^ load counted against the scalar-load counter that the convolution waits
// on.  Pointers of this type are global memory for the compiler.
template <typename X>
using gmem = __attribute__((address_space(1))) X *;
// read-only for the whole launch (weights, row offsets): constant memory,
// which the compiler reads with scalar loads where the address is uniform
template <typename X>
using cmem = __attribute__((address_space(4))) X *;

// A mixed-N batch in one launch: each item runs the variant of its op's N
// (k3 ranges fixed by mix_ranges).  The hardware dispatcher hands the items
// to free wavefront slots in list order, heaviest first within each XCD's
// part, which is the work queue of a persistent kernel without its counter.
template <typename T>
__global__ __launch_bounds__(64) void conv_mixed_kernel(const MixDesc *__restrict__ ops,
                                                        const ConvItem *__restrict__ items) {
    const ConvItem it = items[blockIdx.x];
    if (it.row < 0) return;
    const MixDesc o = ops[it.op];
    const gmem<const C2<T>> fhat = (gmem<const C2<T>>)(const C2<T> *)o.fhat;
    const gmem<C2<T>> part = (gmem<C2<T>>)(C2<T> *)o.part;
    const cmem<const T> W = (cmem<const T>)(const T *)o.W;
    const cmem<const int64_t> rowoff = (cmem<const int64_t>)o.rowoff;
    constexpr bool f64 = sizeof(T) == 8;
    switch (o.N) {
    case 8:
        conv_item<T, 8, mix_ranges(8, f64)>(fhat, part, W, rowoff, 0, it, o.cellpad, o.S);
        break;
    case 16:
        conv_item<T, 16, mix_ranges(16, f64)>(fhat, part, W, rowoff, 0, it, o.cellpad, o.S);
        break;
    case 24:
        conv_item<T, 24, mix_ranges(24, f64)>(fhat, part, W, rowoff, 0, it, o.cellpad, o.S);
        break;
    default:
        conv_item<T, 32, mix_ranges(32, f64)>(fhat, part, W, rowoff, 0, it, o.cellpad, o.S);
        break;
    }
}

template <typename T, int N>
hipError_t conv_n(const bz_op *op, int64_t cellpad, int S, int KH, const void *fhat, void *part, const void *W,
                  int64_t wbase, const ConvItem *items, int64_t nitems, hipStream_t s) {
    const dim3 grid((unsigned)nitems), block(kWave);
    if constexpr (N == 48) {  // only four k3 ranges fit the registers at this mesh
        if (KH != 4) return hipErrorInvalidValue;
        hipLaunchKernelGGL((conv_kernel<T, N, 4>), grid, block, 0, s, (const C2<T> *)fhat, (C2<T> *)part,
                           (const T *)W, op->d_rowoff, wbase, items, cellpad, S);
        return hipGetLastError();
    } else {
        if (KH == 1)
            hipLaunchKernelGGL((conv_kernel<T, N, 1>), grid, block, 0, s, (const C2<T> *)fhat, (C2<T> *)part,
                               (const T *)W, op->d_rowoff, wbase, items, cellpad, S);
        else if (KH == 2)
            hipLaunchKernelGGL((conv_kernel<T, N, 2>), grid, block, 0, s, (const C2<T> *)fhat, (C2<T> *)part,
                               (const T *)W, op->d_rowoff, wbase, items, cellpad, S);
        else
            hipLaunchKernelGGL((conv_kernel<T, N, 4>), grid, block, 0, s, (const C2<T> *)fhat, (C2<T> *)part,
                               (const T *)W, op->d_rowoff, wbase, items, cellpad, S);
        return hipGetLastError();
    }
}

// Trial data for timing the convolution: every real of the workspace set
// from a counter hash to a value in [-1, 1).  Random mantissas draw the same
// power as transformed distributions do; a zeroed workspace runs faster than
// real data and would mislead the choice.
template <typename T>
__global__ __launch_bounds__(256) void fill_trial_kernel(T *x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull;
    h ^= h >> 31;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 29;
    x[i] = (T)((double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0);
}

}  // namespace

hipError_t launch_conv(const bz_op *op, int64_t cellpad, int S, int KH, const void *fhat, void *part,
                       const void *W, int64_t wbase, const ConvItem *items, int64_t nitems, hipStream_t s) {
    if (KH != 1 && KH != 2 && KH != 4) return hipErrorInvalidValue;
    if (nitems <= 0) return hipSuccess;
    const bool f64 = op->wdtype == BZ_F64;
    switch (op->N) {
#define BZ_CONV_CASE(NN)                                                     \
    case NN:                                                                 \
        return f64 ? conv_n<double, NN>(op, cellpad, S, KH, fhat, part, W, wbase, items, nitems, s) \
                   : conv_n<float, NN>(op, cellpad, S, KH, fhat, part, W, wbase, items, nitems, s);
        BZ_CONV_CASE(8)
        BZ_CONV_CASE(16)
        BZ_CONV_CASE(24)
        BZ_CONV_CASE(32)
        BZ_CONV_CASE(48)
#undef BZ_CONV_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_conv_mixed(bool f64, const MixDesc *d_desc, const ConvItem *items, int64_t nitems, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const dim3 grid((unsigned)nitems), block(kWave);
    if (f64)
        hipLaunchKernelGGL(conv_mixed_kernel<double>, grid, block, 0, s, d_desc, items);
    else
        hipLaunchKernelGGL(conv_mixed_kernel<float>, grid, block, 0, s, d_desc, items);
    return hipGetLastError();
}

hipError_t launch_fill_trial(const bz_op *op, void *buf, int64_t nreal, hipStream_t s) {
    const dim3 grid((unsigned)((nreal + 255) / 256)), block(256);
    if (op->wdtype == BZ_F64)
        hipLaunchKernelGGL(fill_trial_kernel<double>, grid, block, 0, s, (double *)buf, nreal);
    else
        hipLaunchKernelGGL(fill_trial_kernel<float>, grid, block, 0, s, (float *)buf, nreal);
    return hipGetLastError();
}

}  // namespace bz
