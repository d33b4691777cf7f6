// 1-D finite-volume transport df/dt + v_1 df/dx = 0 (Sec. 3.4), FP64.
//
// Cells g = 2..M+1 are interior, g = 0, 1 and M+2, M+3 are ghosts (two on each
// side, as in the paper's ghost-cell exchange).  One stage maps fin -> fout:
//   ghosts   zeroth-order extrapolation of the adjacent interior cell; ghost
//            widths equal the adjacent interior width
//   slopes   s_g = minmod((f_{g+1}-f_g)/(x_{g+1}-x_g), (f_g-f_{g-1})/(x_g-x_{g-1}),
//                         (f_{g+1}-f_{g-1})/(x_{g+1}-x_{g-1}))      eq. (minmod)
//   fluxes   F_{g+1/2} = v1 (f_g + dx_g s_g / 2)          v1 >= 0
//                      = v1 (f_{g+1} - dx_{g+1} s_{g+1}/2) v1 <  0   eq. (upwind)
//   walls    on a diffuse wall the incoming half of the boundary-face flux is
//            v1 sigma_w M_w(v), M_w = (2 pi T_w)^{-3/2} e^{-|v - V_w|^2/(2 T_w)},
//            with sigma_w chosen so that the discrete net mass flux through the
//            face is zero (eq. BC); a no-flux boundary drops the incoming half
//   update   fout_g = fin_g - dt/dx_g (F_{g+1/2} - F_{g-1/2})          eq. (transport)
// and a Heun step is f <- (f + S(S(f)))/2.  One thread per (cell, velocity):
// consecutive threads take consecutive velocities of one cell, so the loads of
// the five cells of the stencil are coalesced.
#include "bz_internal.h"

namespace bz {
namespace {

struct WallP {
    int kind;
    double Tw, V0, V1, V2;
};

__device__ __forceinline__ double minmod3(double a, double b, double c) {
    if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
    if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
    return 0.0;
}

// geometry of cell g (ghosts included) from the M+1 faces
struct Geo1 {
    const double *xf;
    int64_t M;
    __device__ double dx(int64_t g) const {
        if (g < 2) g = 2;
        if (g > M + 1) g = M + 1;
        return xf[g - 1] - xf[g - 2];
    }
    __device__ double xc(int64_t g) const {
        if (g < 2) return 0.5 * (xf[0] + xf[1]) - (double)(2 - g) * dx(2);
        if (g > M + 1) return 0.5 * (xf[M - 1] + xf[M]) + (double)(g - M - 1) * dx(M + 1);
        return 0.5 * (xf[g - 2] + xf[g - 1]);
    }
};

__global__ __launch_bounds__(256) void ghost_fill_kernel(double *f, int64_t M, int64_t n3) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n3) return;
    const double a = f[2 * n3 + v], b = f[(M + 1) * n3 + v];
    f[v] = a;
    f[n3 + v] = a;
    f[(M + 2) * n3 + v] = b;
    f[(M + 3) * n3 + v] = b;
}

__device__ __forceinline__ double maxwell_w(const WallP &w, double v1, double v2, double v3) {
    const double d1 = v1 - w.V0, d2 = v2 - w.V1, d3 = v3 - w.V2;
    const double t = 2.0 * kPi * w.Tw;
    return exp(-(d1 * d1 + d2 * d2 + d3 * d3) / (2.0 * w.Tw)) / (t * sqrt(t));
}

// sigma_w for both walls: block 0 = left face, block 1 = right face.
__global__ __launch_bounds__(256) void wall_sigma_kernel(const double *__restrict__ f, const double *__restrict__ xf,
                                                         int64_t M, int N, double dv, WallP left, WallP right,
                                                         double *__restrict__ sig) {
    const int side = blockIdx.x;
    const WallP w = side == 0 ? left : right;
    if (w.kind != BZ_WALL_DIFFUSE) {
        if (threadIdx.x == 0) sig[side] = 0.0;
        return;
    }
    const Geo1 geo{xf, M};
    const int64_t n3 = (int64_t)N * N * N;
    const double nrm = side == 0 ? 1.0 : -1.0;
    const int64_t gi = side == 0 ? 2 : M + 1;
    const double xm = geo.xc(gi - 1), x0 = geo.xc(gi), xp = geo.xc(gi + 1), dxi = geo.dx(gi);
    const int c = N / 2;
    double out = 0.0, inc = 0.0;
    for (int64_t v = threadIdx.x; v < n3; v += blockDim.x) {
        const double v1 = dv * ((int)(v / (N * N)) - c), v2 = dv * ((int)((v / N) % N) - c), v3 = dv * ((int)(v % N) - c);
        const double vn = nrm * v1;
        if (vn < 0.0) {
            const double fm = f[(gi - 1) * n3 + v], f0 = f[gi * n3 + v], fp = f[(gi + 1) * n3 + v];
            const double s = minmod3((fp - f0) / (xp - x0), (f0 - fm) / (x0 - xm), (fp - fm) / (xp - xm));
            out += -vn * (f0 - nrm * 0.5 * dxi * s);
        } else if (vn > 0.0) {
            inc += vn * maxwell_w(w, v1, v2, v3);
        }
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = out;
    red[1][threadIdx.x] = inc;
    __syncthreads();
    for (int h = blockDim.x / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) sig[side] = red[1][0] > 0.0 ? red[0][0] / red[1][0] : 0.0;
}

// flux through the face between cells g and g+1 (g = 1 .. M+1)
__device__ __forceinline__ double face_flux(const double *__restrict__ f, const Geo1 &geo, int64_t g, int64_t v,
                                            int64_t n3, double v1, double v2, double v3, int64_t M,
                                            const WallP &left, const WallP &right, const double *__restrict__ sig) {
    const bool lface = (g == 1), rface = (g == M + 1);
    if (lface && v1 > 0.0 && left.kind != BZ_WALL_EXTRAPOLATE)
        return left.kind == BZ_WALL_NOFLUX ? 0.0 : v1 * sig[0] * maxwell_w(left, v1, v2, v3);
    if (rface && v1 < 0.0 && right.kind != BZ_WALL_EXTRAPOLATE)
        return right.kind == BZ_WALL_NOFLUX ? 0.0 : v1 * sig[1] * maxwell_w(right, v1, v2, v3);
    const int64_t d = v1 >= 0.0 ? g : g + 1;  // donor cell
    const double fm = f[(d - 1) * n3 + v], f0 = f[d * n3 + v], fp = f[(d + 1) * n3 + v];
    const double xm = geo.xc(d - 1), x0 = geo.xc(d), xp = geo.xc(d + 1);
    const double s = minmod3((fp - f0) / (xp - x0), (f0 - fm) / (x0 - xm), (fp - fm) / (xp - xm));
    const double half = 0.5 * geo.dx(d) * s;
    return v1 * (v1 >= 0.0 ? f0 + half : f0 - half);
}

__global__ __launch_bounds__(256) void transport_update_kernel(const double *__restrict__ fin, double *__restrict__ fout,
                                                               const double *__restrict__ xf, int64_t M, int N,
                                                               double dv, double dt, WallP left, WallP right,
                                                               const double *__restrict__ sig) {
    const int64_t n3 = (int64_t)N * N * N;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * n3) return;
    const int64_t g = t / n3 + 2, v = t % n3;
    const int c = N / 2;
    const double v1 = dv * ((int)(v / (N * N)) - c), v2 = dv * ((int)((v / N) % N) - c), v3 = dv * ((int)(v % N) - c);
    const Geo1 geo{xf, M};
    const double Fp = face_flux(fin, geo, g, v, n3, v1, v2, v3, M, left, right, sig);
    const double Fm = face_flux(fin, geo, g - 1, v, n3, v1, v2, v3, M, left, right, sig);
    fout[g * n3 + v] = fin[g * n3 + v] - dt / geo.dx(g) * (Fp - Fm);
}

__global__ __launch_bounds__(256) void heun_combine_kernel(double *__restrict__ f, const double *__restrict__ f2,
                                                           int64_t M, int64_t n3) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * n3) return;
    const int64_t i = 2 * n3 + t;
    f[i] = 0.5 * (f[i] + f2[i]);
}

}  // namespace

hipError_t launch_transport_step(bz_op *op, int64_t M, double *f, const double *x_faces, double dt,
                                 const bz_wall &left, const bz_wall &right, hipStream_t s) {
    const int N = op->N;
    const int64_t n3 = (int64_t)N * N * N;
    const int64_t tot = (M + 4) * n3;
    double *f1 = op->d_tr_work, *f2 = op->d_tr_work + tot, *sig = op->d_tr_work + 2 * tot;
    const WallP wl{left.kind, left.Tw, left.Vw[0], left.Vw[1], left.Vw[2]};
    const WallP wr{right.kind, right.Tw, right.Vw[0], right.Vw[1], right.Vw[2]};
    const dim3 b(256), gg((unsigned)((n3 + 255) / 256)), gu((unsigned)((M * n3 + 255) / 256));
    const double dv = op->geo.dv;
    const double *stage_in[2] = {f, f1};
    double *stage_out[2] = {f1, f2};
    for (int st = 0; st < 2; ++st) {
        double *fin = const_cast<double *>(stage_in[st]);
        hipLaunchKernelGGL(ghost_fill_kernel, gg, b, 0, s, fin, M, n3);
        hipLaunchKernelGGL(wall_sigma_kernel, dim3(2), b, 0, s, fin, x_faces, M, N, dv, wl, wr, sig);
        hipLaunchKernelGGL(transport_update_kernel, gu, b, 0, s, fin, stage_out[st], x_faces, M, N, dv, dt, wl, wr,
                           sig);
    }
    hipLaunchKernelGGL(heun_combine_kernel, gu, b, 0, s, f, f2, M, n3);
    hipLaunchKernelGGL(ghost_fill_kernel, gg, b, 0, s, f, M, n3);
    return hipGetLastError();
}

}  // namespace bz
