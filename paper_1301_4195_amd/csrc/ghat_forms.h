// Closed-form pieces of the weights G^ (Sec. 2.2, the closed forms that
// follow eq. GHat_calc) for the kernels |u|^0 and |u|^1, shared by the stored
// precompute and by the weights computed on the fly.  Each function switches
// to its Taylor series below |y| = 1, where the closed form cancels.
//   X~(y) = (y sin y + cos y - 1)/y^2
//   g0(y) = (sin y - y cos y)/y^3
//   g1(y) = ((2 - y^2) cos y + 2 y sin y - 2)/y^4
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace bz {

constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }

// Series coefficients, fixed at compile time (a factorial evaluated on the
// device would be a recursive call per term).
struct Coefs {
    double v[13];
};
constexpr Coefs xtilde_coefs() {  // index n = 1..11
    Coefs r{};
    for (int n = 1; n <= 11; ++n) r.v[n] = ((n & 1) ? 1.0 : -1.0) * (2 * n - 1) / fact(2 * n);
    return r;
}
constexpr Coefs sinc_coefs() {  // index n = 0..10
    Coefs r{};
    for (int n = 0; n <= 10; ++n) r.v[n] = ((n & 1) ? -1.0 : 1.0) / fact(2 * n + 1);
    return r;
}
constexpr Coefs g0_coefs() {  // index k = 1..11
    Coefs r{};
    for (int k = 1; k <= 11; ++k) r.v[k] = ((k & 1) ? 1.0 : -1.0) * (2 * k) / fact(2 * k + 1);
    return r;
}
constexpr Coefs g1_coefs() {  // index j = 2..12
    Coefs r{};
    for (int j = 2; j <= 12; ++j) r.v[j] = ((j & 1) ? -1.0 : 1.0) * 2.0 * (2 * j - 1) * (j - 1) / fact(2 * j);
    return r;
}

// X~(y) = sum_{n>=1} (-1)^{n-1} (2n-1) y^{2n-2} / (2n)!, for |y| < 1
__host__ __device__ inline double xtilde_series(double y) {
    constexpr Coefs k = xtilde_coefs();
    const double y2 = y * y;
    double acc = 0.0;
#pragma unroll
    for (int n = 11; n >= 1; --n) acc = acc * y2 + k.v[n];
    return acc;
}

// sin(y)/y = sum_{n>=0} (-1)^n y^{2n} / (2n+1)!, for |y| < 1
__host__ __device__ inline double sinc_series(double y) {
    constexpr Coefs k = sinc_coefs();
    const double y2 = y * y;
    double acc = 0.0;
#pragma unroll
    for (int n = 10; n >= 0; --n) acc = acc * y2 + k.v[n];
    return acc;
}

__host__ __device__ inline double xtilde(double y) {
    if (fabs(y) < 1.0) return xtilde_series(y);
    return (y * sin(y) + cos(y) - 1.0) / (y * y);
}

__host__ __device__ inline double sinc(double y) { return y == 0.0 ? 1.0 : sin(y) / y; }

// g0(y) = sum_{k>=1} (-1)^{k+1} 2k y^{2k-2} / (2k+1)!
__host__ __device__ inline double g0(double y) {
    if (y < 1.0) {
        constexpr Coefs c = g0_coefs();
        const double y2 = y * y;
        double acc = 0.0;
#pragma unroll
        for (int k = 11; k >= 1; --k) acc = acc * y2 + c.v[k];
        return acc;
    }
    return (sin(y) - y * cos(y)) / (y * y * y);
}

// g1(y) = sum_{j>=2} (-1)^j 2 (2j-1)(j-1) y^{2j-4} / (2j)!
__host__ __device__ inline double g1(double y) {
    if (y < 1.0) {
        constexpr Coefs c = g1_coefs();
        const double y2 = y * y;
        double acc = 0.0;
#pragma unroll
        for (int j = 12; j >= 2; --j) acc = acc * y2 + c.v[j];
        return acc;
    }
    const double y2 = y * y;
    return ((2.0 - y2) * cos(y) + 2.0 * y * sin(y) - 2.0) / (y2 * y2);
}

}  // namespace bz
