// Weights computed on the fly (the remedy the Conclusions propose for the
// memory of the six-dimensional weight array): an op of this kind keeps no
// O(N^6) table.  Every convolution recomputes the stored form of the weights
// (one value per mirrored couple, the layout of bz_op::W) one slab of output
// rows at a time into a bounded buffer, which the convolution kernel then
// reads exactly as it reads a stored table.
//
// Only the closed forms (lambda = 0, 1; beta = 1) are evaluated this way.  For
// the pair (k, m) and its mirror n = k - m + N/2 the closed forms depend on
// the integers A = |k - N/2|^2, B = |m - n|^2 (the same for both members of
// the couple) and Cm = |m - N/2|^2 or Cn = |n - N/2|^2:
//   G^ = gain(A, B) - loss(Cm),
// so one gain evaluation serves both weights of a couple, and gain(A, B)
// needs only sin and cos of (pi/2) sqrt(X) at X = A and X = B (the arguments
// y_q, y_p of the closed forms are their sum and difference).  Those, the
// loss term and the B = 0 limit are O(N^2) tables built on the host once per
// op; the per-weight work is table reads, a few multiply-adds and divisions.
#include <algorithm>
#include <cmath>
#include <vector>

#include "bz_internal.h"
#include "ghat_forms.h"

namespace bz {

namespace {

// largest A = |k - N/2|^2 and B = |m - n|^2 of the truncated sum
constexpr int amax(int N) { return 3 * (N / 2) * (N / 2); }
constexpr int bmax(int N) { return 3 * (N - 1) * (N - 1); }

struct FlyView {
    const double *trig;  // [bmax + 1][2]: sin, cos of (pi/2) sqrt(X)
    const double *sq;    // [bmax + 1]: sqrt(X)
    const double *gb0;   // [amax + 1]: G^ gain term at B = 0, times sqrt(2/pi)
    const double *loss;  // [amax + 1]: G^ loss term at Cm = X, times sqrt(2/pi)
    const double *om;    // N per-dimension trapezoid weights, or null: dzeta^3
    const int *pos;      // [3N^2/4]: (m3, k3) of each position of a line, m3 | k3 << 16
    double gscale;       // sqrt(2/pi) r0^{1+lambda} / (dzeta^2 / 2)
    double dz3;
    int lam;
};

FlyView view_of(const bz_op *op) {
    const int N = op->N, xb = bmax(N) + 1, xa = amax(N) + 1;
    FlyView v;
    v.trig = op->d_fly;
    v.sq = v.trig + 2 * xb;
    v.gb0 = v.sq + xb;
    v.loss = v.gb0 + xa;
    v.om = op->fly_has_omega ? v.loss + xa : nullptr;
    v.pos = op->d_fly_pos;
    const double r0 = op->L, dz = kPi / op->L;
    v.gscale = std::sqrt(2.0 / kPi) * (op->lambda == 0.0 ? r0 : r0 * r0) / (0.5 * dz * dz);
    v.dz3 = dz * dz * dz;
    v.lam = (int)op->lambda;
    return v;
}

// Stored weight of the couple (m, n = k - m + N/2) of output k, m on the kept
// line: omega_m G^(m) + omega_n G^(n), or omega_m G^(m) alone on a
// self-mirrored line.
template <int N>
__device__ __forceinline__ double fly_weight(const FlyView &t, int k1, int k2, int k3, int m1, int m2, int m3, bool self) {
    constexpr int c = N / 2;
    const int ka = k1 - c, kb = k2 - c, kc = k3 - c;
    const int A = ka * ka + kb * kb + kc * kc;
    if (A == 0) return 0.0;  // G(u, 0) = 0
    const int n1 = k1 - m1 + c, n2 = k2 - m2 + c, n3 = k3 - m3 + c;
    const int d1 = m1 - n1, d2 = m2 - n2, d3 = m3 - n3;
    const int B = d1 * d1 + d2 * d2 + d3 * d3;
    double g;
    if (B == 0) {
        g = t.gb0[A];
    } else {
        const double sA = t.sq[A], sB = t.sq[B];
        const double sa = t.trig[2 * A], ca = t.trig[2 * A + 1];
        const double sb = t.trig[2 * B], cb = t.trig[2 * B + 1];
        const double yq = 0.5 * kPi * (sA + sB);
        const double yp = 0.5 * kPi * (double)(A - B) / (sA + sB);
        const double sinq = sa * cb + ca * sb, cosq = ca * cb - sa * sb;
        const double sinp = sa * cb - ca * sb, cosp = ca * cb + sa * sb;
        double tp, tq;
        if (t.lam == 0) {  // sinc(y_p) - sinc(y_q)
            tq = sinq / yq;
            tp = fabs(yp) < 1.0 ? sinc_series(yp) : sinp / yp;
        } else {  // X~(y_p) - X~(y_q)
            tq = (yq * sinq + cosq - 1.0) / (yq * yq);
            tp = fabs(yp) < 1.0 ? xtilde_series(yp) : (yp * sinp + cosp - 1.0) / (yp * yp);
        }
        g = t.gscale * (tp - tq) / (sA * sB);
    }
    const int e1 = m1 - c, e2 = m2 - c, e3 = m3 - c;
    const int Cm = e1 * e1 + e2 * e2 + e3 * e3;
    const double om = t.om ? t.om[m1] * t.om[m2] * t.om[m3] : t.dz3;
    double w = om * (g - t.loss[Cm]);
    if (!self) {
        const int f1 = n1 - c, f2 = n2 - c, f3 = n3 - c;
        const int Cn = f1 * f1 + f2 * f2 + f3 * f3;
        const double on = t.om ? t.om[n1] * t.om[n2] * t.om[n3] : t.dz3;
        w += on * (g - t.loss[Cn]);
    }
    return w;
}

// One slab: rows row0 + blockIdx.y, each row's packed weights (kept lines in
// (a1, a2) order, 3N^2/4 positions per line) written to out[rowoff[row] -
// wbase + pos].  A workgroup covers kFlyPer x 256 consecutive positions of its
// row, each thread kFlyPer of them 256 apart (stores stay coalesced; fewer,
// longer waves than one position per thread).
constexpr int kFlyPer = 4;

template <typename TW, int N>
__global__ __launch_bounds__(256) void fly_weights_kernel(TW *__restrict__ out, const int64_t *__restrict__ rowoff,
                                                         int64_t wbase, int row0, FlyView t) {
    constexpr int P = line_pairs(N);
    const int row = row0 + blockIdx.y;
    const int k1 = row / N, k2 = row % N;
    const int c1 = mcount(N, k1), c2 = mcount(N, k2);
    const int lo1 = mlo(N, k1), lo2 = mlo(N, k2);
    const int len = half_lines(c1, c2) * P;
    TW *o = out + (rowoff[row] - wbase);
#pragma unroll
    for (int r = 0; r < kFlyPer; ++r) {
        const int pos = (blockIdx.x * kFlyPer + r) * 256 + threadIdx.x;
        if (pos >= len) return;
        const int q = pos / P, p = pos % P;
        const int a1 = q / c2, a2 = q % c2;
        const int mk = t.pos[p];
        const int m3 = mk & 0xffff, k3 = mk >> 16;
        o[pos] = (TW)fly_weight<N>(t, k1, k2, k3, lo1 + a1, lo2 + a2, m3, self_mirror(c1, c2, a1, a2));
    }
}

// bz_weights_gather for an op without a table: the same evaluation for the
// kept member of each requested couple, rounded to the op's weight type as a
// slab would store it.
template <typename TW, int N>
__global__ __launch_bounds__(256) void fly_gather_kernel(int64_t npairs, const int32_t *__restrict__ kl,
                                                        const int32_t *__restrict__ ml, double *__restrict__ out,
                                                        FlyView t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npairs) return;
    constexpr int c = N / 2, N3 = N * N * N;
    const int k = kl[i], m = ml[i];
    if (k < 0 || m < 0 || k >= N3 || m >= N3) {
        out[i] = 0.0;
        return;
    }
    const int k1 = k / (N * N), k2 = (k / N) % N, k3 = k % N;
    int m1 = m / (N * N), m2 = (m / N) % N, m3 = m % N;
    const int n1 = k1 - m1 + c, n2 = k2 - m2 + c, n3 = k3 - m3 + c;
    if (n1 < 0 || n1 >= N || n2 < 0 || n2 >= N || n3 < 0 || n3 >= N) {
        out[i] = 0.0;
        return;
    }
    const int c1 = mcount(N, k1), c2 = mcount(N, k2);
    int a1 = m1 - mlo(N, k1), a2 = m2 - mlo(N, k2);
    if (a1 >= half_a1_end(c1) || a2 >= half_a2_end(c1, c2, a1)) {  // the kept member is n
        a1 = c1 - 1 - a1;
        a2 = c2 - 1 - a2;
        m1 = n1;
        m2 = n2;
        m3 = n3;
    }
    out[i] = (double)(TW)fly_weight<N>(t, k1, k2, k3, m1, m2, m3, self_mirror(c1, c2, a1, a2));
}

}  // namespace

int64_t fly_table_doubles(int N, bool omega) { return 3 * (int64_t)(bmax(N) + 1) + 2 * (amax(N) + 1) + (omega ? N : 0); }

// Host tables of an op whose weights are computed on the fly (see FlyView).
void fly_tables(int N, double L, int lam, const double *omega1d, std::vector<double> &d, std::vector<int> &pos) {
    const int xb = bmax(N) + 1, xa = amax(N) + 1;
    d.assign(fly_table_doubles(N, omega1d != nullptr), 0.0);
    double *trig = d.data(), *sq = trig + 2 * xb, *gb0 = sq + xb, *loss = gb0 + xa;
    for (int x = 0; x < xb; ++x) {
        const double s = std::sqrt((double)x), y = 0.5 * kPi * s;
        trig[2 * x] = std::sin(y);
        trig[2 * x + 1] = std::cos(y);
        sq[x] = s;
    }
    const double r0 = L, sc = std::sqrt(2.0 / kPi);
    const double r3l = lam == 0 ? r0 * r0 * r0 : r0 * r0 * r0 * r0;  // r0^{3 + lambda}
    for (int x = 0; x < xa; ++x) {
        const double s = std::sqrt((double)x);
        gb0[x] = sc * r3l * (lam == 0 ? g0(0.5 * kPi * s) : g1(0.5 * kPi * s));
        loss[x] = sc * r3l * (lam == 0 ? g0(kPi * s) : g1(kPi * s));
    }
    if (omega1d)
        for (int i = 0; i < N; ++i) loss[xa + i] = omega1d[i];
    pos.clear();
    for (int m3 = 0; m3 < N; ++m3)
        for (int k3 = klo(N, m3); k3 <= khi(N, m3); ++k3) pos.push_back(m3 | (k3 << 16));
}

hipError_t launch_fly_weights(const bz_op *op, int row0, int row1, void *out, hipStream_t s) {
    const int N = op->N;
    int64_t longest = 0;
    for (int r = row0; r < row1; ++r)
        longest = std::max<int64_t>(longest, (int64_t)half_lines(mcount(N, r / N), mcount(N, r % N)));
    longest *= line_pairs(N);
    const dim3 grid((unsigned)((longest + 256 * kFlyPer - 1) / (256 * kFlyPer)), (unsigned)(row1 - row0)), block(256);
    const FlyView t = view_of(op);
    const int64_t wbase = op->h_rowoff[row0];
    const bool f64 = op->wdtype == BZ_F64;
    switch (N) {
#define BZ_FLY_CASE(NN)                                                                                         \
    case NN:                                                                                                    \
        if (f64)                                                                                                \
            hipLaunchKernelGGL((fly_weights_kernel<double, NN>), grid, block, 0, s, (double *)out, op->d_rowoff, \
                               wbase, row0, t);                                                                 \
        else                                                                                                    \
            hipLaunchKernelGGL((fly_weights_kernel<float, NN>), grid, block, 0, s, (float *)out, op->d_rowoff,  \
                               wbase, row0, t);                                                                 \
        return hipGetLastError();
        BZ_FLY_CASE(8)
        BZ_FLY_CASE(16)
        BZ_FLY_CASE(24)
        BZ_FLY_CASE(32)
        BZ_FLY_CASE(48)
#undef BZ_FLY_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fly_gather(const bz_op *op, int64_t npairs, const int32_t *k, const int32_t *m, double *out,
                             hipStream_t s) {
    const dim3 grid((unsigned)((npairs + 255) / 256)), block(256);
    const FlyView t = view_of(op);
    const bool f64 = op->wdtype == BZ_F64;
    switch (op->N) {
#define BZ_FLYG_CASE(NN)                                                                                      \
    case NN:                                                                                                  \
        if (f64)                                                                                              \
            hipLaunchKernelGGL((fly_gather_kernel<double, NN>), grid, block, 0, s, npairs, k, m, out, t);     \
        else                                                                                                  \
            hipLaunchKernelGGL((fly_gather_kernel<float, NN>), grid, block, 0, s, npairs, k, m, out, t);      \
        return hipGetLastError();
        BZ_FLYG_CASE(8)
        BZ_FLYG_CASE(16)
        BZ_FLYG_CASE(24)
        BZ_FLYG_CASE(32)
        BZ_FLYG_CASE(48)
#undef BZ_FLYG_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace bz
