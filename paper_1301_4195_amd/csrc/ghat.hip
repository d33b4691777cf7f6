// Precompute of the convolution weights W[k][m] = omega_m G^(xi_m, zeta_k)
// (Sec. 2.2, eq. GHat_calc and its closed forms for lambda = 0, 1), FP64.
// Other exponents (Sec. 2.2, last paragraph) integrate the radial integral
// of eq. GHat_calc numerically: see GhatQuad below.
//
// With r0 = L and dzeta = pi/L every trig argument is independent of L:
//   y_q = r0 (|zeta|/2 + |xi - zeta/2|) = (pi/2)(sqrt A + sqrt B)
//   y_p = r0 (|zeta|/2 - |xi - zeta/2|) = (pi/2)(A - B)/(sqrt A + sqrt B)
//   y_s = r0 |xi| = pi sqrt Cm,    y_a = r0 |zeta|/2 = (pi/2) sqrt A
// for the integers A = |k - N/2|^2, B = |2m - k - N/2|^2, Cm = |m - N/2|^2,
// which also decide the limiting branches exactly.  Writing
//   sinc(y) = sin y / y,
//   X~(y) = (y sin y + cos y - 1)/y^2,
//   g0(y) = (sin y - y cos y)/y^3,
//   g1(y) = ((2 - y^2) cos y + 2 y sin y - 2)/y^4,
// the closed forms become, with 2ab = (dzeta^2/2) sqrt(A B):
//   lambda = 0:  G^ = sqrt(2/pi) ( r0   [sinc(y_p) - sinc(y_q)]/(2ab) - r0^3 g0(y_s) )
//   lambda = 1:  G^ = sqrt(2/pi) ( r0^2 [X~(y_p)  - X~(y_q)] /(2ab) - r0^4 g1(y_s) )
// B = 0 replaces the first term by r0^{3+lambda} g_lambda(y_a) (the gain
// integrand loses its second sinc), and A = 0 gives G^ = 0 (G(u, 0) = 0).
// Near zero each function is evaluated from its Taylor series.
#include <cmath>
#include <vector>

#include "bz_internal.h"
#include "ghat_forms.h"

namespace bz {
namespace {

// Radial integral of eq. GHat_calc for an exponent without a closed form,
//   G^ = sqrt(2/pi) int_0^{r0} r^{lambda+2} [sinc(a r) sinc(b r) - sinc(s r)] dr,
// a = |zeta|/2, b = |xi - zeta/2|, s = |xi|, by n-point Gauss-Jacobi
// quadrature for the weight r^{lambda+2} on [0, r0]: with r = r0 (1 + x)/2
// the integral is (r0/2)^{lambda+3} int_{-1}^{1} (1 + x)^{lambda+2} g dx, and
// the rule with weight (1 + x)^{lambda+2} integrates the smooth remainder g
// to spectral accuracy.  r[j] are the mapped nodes, w[j] the rule's weights
// times sqrt(2/pi) (r0/2)^{lambda+3}.
struct GhatQuad {
    const double *r = nullptr;
    const double *w = nullptr;
    int n = 0;
};

__device__ double ghat_quad(double a, double b, double s, const GhatQuad &q) {
    double acc = 0.0;
    for (int j = 0; j < q.n; ++j) {
        const double r = q.r[j];
        acc += q.w[j] * (sinc(a * r) * sinc(b * r) - sinc(s * r));
    }
    return acc;
}

// lam = 0 or 1: closed forms; lam < 0: the quadrature q, with the inelastic
// lengths beta |zeta|/2 and |xi - beta zeta/2| when beta != 1.
__device__ double ghat_value(int N, double L, int lam, double beta, const GhatQuad &q, int k1, int k2, int k3,
                             int m1, int m2, int m3) {
    const int c = N / 2;
    const int ka = k1 - c, kb = k2 - c, kc = k3 - c;
    const int ba = 2 * m1 - k1 - c, bb = 2 * m2 - k2 - c, bc = 2 * m3 - k3 - c;
    const int ma = m1 - c, mb = m2 - c, mc = m3 - c;
    const int A = ka * ka + kb * kb + kc * kc;
    const int B = ba * ba + bb * bb + bc * bc;
    const int Cm = ma * ma + mb * mb + mc * mc;
    if (A == 0) return 0.0;
    const double r0 = L, dz = kPi / L;
    const double sA = sqrt((double)A), sB = sqrt((double)B);
    if (lam < 0) {
        if (beta == 1.0) return ghat_quad(0.5 * dz * sA, 0.5 * dz * sB, dz * sqrt((double)Cm), q);
        const double d1 = ma - 0.5 * beta * ka, d2 = mb - 0.5 * beta * kb, d3 = mc - 0.5 * beta * kc;
        return ghat_quad(0.5 * beta * dz * sA, dz * sqrt(d1 * d1 + d2 * d2 + d3 * d3), dz * sqrt((double)Cm), q);
    }
    const double ys = kPi * sqrt((double)Cm);
    double gain, loss;
    if (lam == 0) {
        loss = r0 * r0 * r0 * g0(ys);
        if (B == 0) {
            gain = r0 * r0 * r0 * g0(0.5 * kPi * sA);
        } else {
            const double yq = 0.5 * kPi * (sA + sB);
            const double yp = 0.5 * kPi * (double)(A - B) / (sA + sB);
            gain = r0 * (sinc(yp) - sinc(yq)) / (0.5 * dz * dz * sA * sB);
        }
    } else {
        loss = r0 * r0 * r0 * r0 * g1(ys);
        if (B == 0) {
            gain = r0 * r0 * r0 * r0 * g1(0.5 * kPi * sA);
        } else {
            const double yq = 0.5 * kPi * (sA + sB);
            const double yp = 0.5 * kPi * (double)(A - B) / (sA + sB);
            gain = r0 * r0 * (xtilde(yp) - xtilde(yq)) / (0.5 * dz * dz * sA * sB);
        }
    }
    return sqrt(2.0 / kPi) * (gain - loss);
}

// position of (k3, m3) inside the packed 1-D line: m3-major, k3 ascending
__device__ __host__ inline int line_pos(int N, int k3, int m3) {
    int p = 0;
    for (int t = 0; t < m3; ++t) p += kcount(N, t);
    return p + (k3 - klo(N, m3));
}

template <typename TW>
__global__ __launch_bounds__(256) void build_weights_kernel(TW *__restrict__ W, const int64_t *__restrict__ rowoff,
                                                            const double *__restrict__ omega1d, int N, double L,
                                                            int lam, double beta, GhatQuad q) {
    // blockIdx.x = (row * N + a1) * N + a2; only the kept half of the lines
    // (see half_lines) is stored, each weight summed with its mirror's.
    const int a2 = blockIdx.x % N;
    const int a1 = (blockIdx.x / N) % N;
    const int row = blockIdx.x / (N * N);
    const int k1 = row / N, k2 = row % N;
    const int c1 = mcount(N, k1), c2 = mcount(N, k2);
    if (a1 >= half_a1_end(c1) || a2 >= half_a2_end(c1, c2, a1)) return;
    const int c = N / 2;
    const int m1 = mlo(N, k1) + a1, m2 = mlo(N, k2) + a2;
    const int n1 = k1 - m1 + c, n2 = k2 - m2 + c;
    const bool self = self_mirror(c1, c2, a1, a2);
    const int P = line_pairs(N);
    TW *out = W + rowoff[row] + ((int64_t)a1 * c2 + a2) * P;
    const double dz = kPi / L;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        int m3 = 0, base = 0;
        while (base + kcount(N, m3) <= p) {
            base += kcount(N, m3);
            ++m3;
        }
        const int k3 = klo(N, m3) + (p - base);
        const int n3 = k3 - m3 + c;
        const double om = omega1d ? omega1d[m1] * omega1d[m2] * omega1d[m3] : dz * dz * dz;
        double w = om * ghat_value(N, L, lam, beta, q, k1, k2, k3, m1, m2, m3);
        if (!self) {
            const double on = omega1d ? omega1d[n1] * omega1d[n2] * omega1d[n3] : dz * dz * dz;
            w += on * ghat_value(N, L, lam, beta, q, k1, k2, k3, n1, n2, n3);
        }
        out[p] = (TW)w;
    }
}

template <typename TW>
__global__ __launch_bounds__(256) void gather_weights_kernel(const TW *__restrict__ W, const int64_t *__restrict__ rowoff,
                                                             int N, int64_t npairs, const int32_t *__restrict__ kl,
                                                             const int32_t *__restrict__ ml, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npairs) return;
    const int k = kl[i], m = ml[i];
    const int k1 = k / (N * N), k2 = (k / N) % N, k3 = k % N;
    const int m1 = m / (N * N), m2 = (m / N) % N, m3 = m % N;
    const int c = N / 2;
    const int n1 = k1 - m1 + c, n2 = k2 - m2 + c, n3 = k3 - m3 + c;
    if (k < 0 || m < 0 || k >= N * N * N || m >= N * N * N || n1 < 0 || n1 >= N || n2 < 0 || n2 >= N || n3 < 0 ||
        n3 >= N) {
        out[i] = 0.0;
        return;
    }
    const int row = k1 * N + k2;
    const int c1 = mcount(N, k1), c2 = mcount(N, k2);
    int a1 = m1 - mlo(N, k1), a2 = m2 - mlo(N, k2), q3 = m3;
    if (a1 >= half_a1_end(c1) || a2 >= half_a2_end(c1, c2, a1)) {  // stored on the mirrored line
        a1 = c1 - 1 - a1;
        a2 = c2 - 1 - a2;
        q3 = n3;
    }
    const int64_t idx = rowoff[row] + ((int64_t)a1 * c2 + a2) * line_pairs(N) + line_pos(N, k3, q3);
    out[i] = (double)W[idx];
}

}  // namespace

// Gauss-Jacobi rule for the weight (1 + x)^beta on [-1, 1] (beta > -1), by
// the Golub-Welsch method: the nodes are the eigenvalues of the symmetric
// tridiagonal Jacobi matrix of the orthogonal polynomials' three-term
// recurrence, and each weight is mu0 times the squared first component of
// the normalised eigenvector (mu0 = int (1 + x)^beta dx = 2^{beta+1}/(beta+1)).
// The eigenproblem is solved by the implicit QL algorithm for symmetric
// tridiagonal matrices with Wilkinson-type shifts (Bowdler, Martin, Reinsch
// and Wilkinson, "The QR and QL algorithms for symmetric matrices", Numer.
// Math. 11, 1968 -- the tql2 procedure of the Handbook for Automatic
// Computation, vol. II), carrying only the first row of the eigenvector matrix.
bool gauss_jacobi(int n, double beta, std::vector<double> &x, std::vector<double> &w) {
    const double al = 0.0, be = beta, ab = al + be;
    std::vector<double> d(n), e(n, 0.0), z(n, 0.0);
    for (int j = 0; j < n; ++j) {
        const double t = 2.0 * j + ab;
        d[j] = (j == 0) ? (be - al) / (ab + 2.0) : (be * be - al * al) / (t * (t + 2.0));
    }
    for (int j = 1; j < n; ++j) {
        const double t = 2.0 * j + ab;
        const double bj = 4.0 * j * (j + al) * (j + be) * (j + ab) / (t * t * (t + 1.0) * (t - 1.0));
        e[j - 1] = std::sqrt(bj);  // e[j-1] couples rows j-1 and j
    }
    z[0] = 1.0;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0;; ++iter) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) + dd == dd) break;  // negligible at working precision
            }
            if (m == l) break;
            if (iter == 60) return false;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double sn = 1.0, cs = 1.0, p = 0.0;
            int i = m - 1;
            for (; i >= l; --i) {
                double f = sn * e[i], b = cs * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    break;
                }
                sn = f / r;
                cs = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * sn + 2.0 * cs * b;
                p = sn * r;
                d[i + 1] = g + p;
                g = cs * r - b;
                f = z[i + 1];
                z[i + 1] = sn * z[i] + cs * f;
                z[i] = cs * z[i] - sn * f;
            }
            if (r == 0.0 && i >= l) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    const double mu0 = std::pow(2.0, be + 1.0) / (be + 1.0);
    x.assign(d.begin(), d.end());
    w.resize(n);
    for (int j = 0; j < n; ++j) w[j] = mu0 * z[j] * z[j];
    return true;
}

hipError_t launch_build_weights(bz_op *op, const double *d_omega1d, const double *d_quad, int nquad,
                                hipStream_t s) {
    const int N = op->N;
    const dim3 grid((unsigned)(N * N * N * N)), block(256);
    // closed forms for lambda = 0, 1; the quadrature (nodes d_quad[0, n),
    // weights d_quad[n, 2n)) otherwise
    const int lam = nquad > 0 ? -1 : (int)op->lambda;
    GhatQuad q;
    if (nquad > 0) {
        q.r = d_quad;
        q.w = d_quad + nquad;
        q.n = nquad;
    }
    if (op->wdtype == BZ_F64)
        hipLaunchKernelGGL(build_weights_kernel<double>, grid, block, 0, s, (double *)op->W, op->d_rowoff, d_omega1d,
                           N, op->L, lam, op->beta, q);
    else
        hipLaunchKernelGGL(build_weights_kernel<float>, grid, block, 0, s, (float *)op->W, op->d_rowoff, d_omega1d, N,
                           op->L, lam, op->beta, q);
    return hipGetLastError();
}

hipError_t launch_gather_weights(const bz_op *op, int64_t npairs, const int32_t *k, const int32_t *m, double *out,
                                 hipStream_t s) {
    const dim3 grid((unsigned)((npairs + 255) / 256)), block(256);
    if (op->wdtype == BZ_F64)
        hipLaunchKernelGGL(gather_weights_kernel<double>, grid, block, 0, s, (const double *)op->W, op->d_rowoff,
                           op->N, npairs, k, m, out);
    else
        hipLaunchKernelGGL(gather_weights_kernel<float>, grid, block, 0, s, (const float *)op->W, op->d_rowoff, op->N,
                           npairs, k, m, out);
    return hipGetLastError();
}

}  // namespace bz
