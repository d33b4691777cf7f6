// Forward and inverse 3-D transforms of the collision step (Sec. 3.2):
//   f^_k = (2pi)^{-3/2} dv^3 (-1)^{k1+k2+k3} DFT[(-1)^{j1+j2+j3} f]_k
//   Q~_j = Re (2pi)^{-3/2} dzeta^3 (-1)^{j1+j2+j3} IDFT[(-1)^{k1+k2+k3} Q^]_j
// which is the trapezoid rule for e^{-+i zeta_k . v_j} on the centred meshes
// of Sec. 3.1 (zeta_k v_j = (2pi/N)(k - N/2)(j - N/2); the extra factor
// e^{-+i pi N/2} per dimension is 1 because N is a multiple of 4).
//
// Each transform is three passes, one per axis -- for N <= 24 the two axes
// that touch the caller's layout are fused into one pass through LDS (see
// fwd_plane).  A thread owns one 1-D line of one cell and does its N-point FFT
// in registers (radix-2 decimation in frequency, with one radix-3 stage when
// N = 24).  Consecutive threads own the
// same line of consecutive cells, so every load and store of the
// [mode][cell] workspace is coalesced across the wavefront; the first forward
// and last inverse pass convert from/to the caller's [cell][mode] layout.
//
// Precision: the FP32 path's forward transform reads FP32 f, computes in FP64
// and rounds each f^ value to FP32 once, at its last store (its passes hand
// FP64 intermediates to each other).  FP64 vector instructions issue at up
// to half the rate of non-packed FP32 ones, but these passes are bound by
// memory and latency, so the wider arithmetic costs only the intermediate's
// bytes; a radix-2 FP32 transform would spread rounding noise of the size of
// the line's largest values over every mode, which the convolution then
// multiplies by the largest f^ values.  The inverse transform of the FP32
// path stays FP32: its error relative to ||Q^|| is that of the transform
// itself (Parseval), a few units in the last place.
#include "bz_internal.h"

namespace bz {
namespace {

template <typename T>
struct C2 {
    T re, im;
};

constexpr int bitrev(int x, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
    return r;
}
constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Position in the register array at which frequency k ends up after fft_line.
template <int N>
constexpr int out_pos(int k) {
    constexpr int R3 = (N % 3 == 0) ? 3 : 1;
    constexpr int M = N / R3;
    return (k % R3) * M + bitrev(k / R3, ilog2(M));
}

// x <- x * e^{DIR 2 pi i t / N}, with exact factors for t in {0, N/4, N/2, 3N/4}.
template <typename T, int N, int DIR>
__device__ __forceinline__ void twiddle(T &xr, T &xi, int t, const T *__restrict__ tw) {
    t %= N;
    if (t == 0) return;
    if (4 * t == N) {  // DIR i
        const T r = xr;
        xr = -DIR * xi;
        xi = DIR * r;
        return;
    }
    if (2 * t == N) {
        xr = -xr;
        xi = -xi;
        return;
    }
    if (4 * t == 3 * N) {  // -DIR i
        const T r = xr;
        xr = DIR * xi;
        xi = -DIR * r;
        return;
    }
    const T c = tw[t], s = DIR * tw[N + t];
    const T r = xr * c - xi * s;
    xi = xr * s + xi * c;
    xr = r;
}

// In-register FFT of one line: X_k = sum_j x_j e^{DIR 2 pi i j k / N}, output
// frequency k at register out_pos<N>(k).
template <typename T, int N, int DIR>
__device__ __forceinline__ void fft_line(T (&xr)[N], T (&xi)[N], const T *__restrict__ tw) {
    constexpr int R3 = (N % 3 == 0) ? 3 : 1;
    constexpr int M = N / R3;
    if constexpr (R3 == 3) {
        const T h = (T)0.86602540378443864676;  // sqrt(3)/2
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const T ar = xr[j], ai = xi[j];
            const T br = xr[j + M], bi = xi[j + M];
            const T cr = xr[j + 2 * M], ci = xi[j + 2 * M];
            const T tr = br + cr, ti = bi + ci;
            const T dr = br - cr, di = bi - ci;
            const T sr = ar - (T)0.5 * tr, si = ai - (T)0.5 * ti;
            // DIR i (sqrt3/2)(b - c)
            const T ur = -DIR * h * di, ui = DIR * h * dr;
            xr[j] = ar + tr;
            xi[j] = ai + ti;
            T y1r = sr + ur, y1i = si + ui, y2r = sr - ur, y2i = si - ui;
            twiddle<T, N, DIR>(y1r, y1i, j, tw);
            twiddle<T, N, DIR>(y2r, y2i, 2 * j, tw);
            xr[j + M] = y1r;
            xi[j + M] = y1i;
            xr[j + 2 * M] = y2r;
            xi[j + 2 * M] = y2i;
        }
    }
#pragma unroll
    for (int h = M / 2; h >= 1; h /= 2) {
#pragma unroll
        for (int blk = 0; blk < N; blk += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const T ar = xr[blk + j], ai = xi[blk + j];
                const T br = xr[blk + j + h], bi = xi[blk + j + h];
                xr[blk + j] = ar + br;
                xi[blk + j] = ai + bi;
                T dr = ar - br, di = ai - bi;
                twiddle<T, N, DIR>(dr, di, j * (N / (2 * h)), tw);
                xr[blk + j + h] = dr;
                xi[blk + j + h] = di;
            }
        }
    }
}

// ---------------------------------------------------------------- forward
// pass 1: axis 3, real input [cell][N^3] (type TI) -> work[(line*N + k3)][cell]
// (type T, the arithmetic's)
template <typename TI, typename T, int N>
__global__ __launch_bounds__(256) void fwd_axis3(const TI *__restrict__ f, C2<T> *__restrict__ work,
                                                 const T *__restrict__ tw, int64_t ncells, int64_t cellpad,
                                                 int64_t cw, const int64_t *__restrict__ off) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cell = tid % cellpad;
    const int64_t line = tid / cellpad;  // j1 * N + j2
    if (line >= N * N || cell >= cw) return;
    T xr[N], xi[N];
    if (cell < ncells) {
        const TI *src = f + (off ? off[cell] : cell * (int64_t)(N * N * N)) + line * N;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const T x = (T)src[j];
            xr[j] = (j & 1) ? -x : x;
            xi[j] = (T)0;
        }
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j) xr[j] = xi[j] = (T)0;
    }
    fft_line<T, N, -1>(xr, xi, tw);
    C2<T> *dst = work + (line * N) * cellpad + cell;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int p = out_pos<N>(k);
        const T s = (k & 1) ? (T)-1 : (T)1;
        dst[(int64_t)k * cellpad] = C2<T>{s * xr[p], s * xi[p]};
    }
}

// pass over axis 2 (stride N modes) or axis 1 (stride N^2 modes) of the
// [mode][cell] workspace; DIR -1 forward, +1 inverse; optional scale and
// summation of S partial buffers (inverse, axis 1 only).  Reads TIN, computes
// in T, writes TOUT.
template <typename TIN, typename T, typename TOUT, int N, int AXIS, int DIR>
__global__ __launch_bounds__(256) void mid_pass(const C2<TIN> *in, int S, int64_t part_stride, C2<TOUT> *out,
                                                const T *__restrict__ tw, int64_t cellpad, int64_t cw, T scale) {
    // `in` may equal `out` (in-place pass, TIN = TOUT): every element of a
    // line is read before the line is written, and lines of different threads
    // are disjoint.
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cell = tid % cellpad;
    const int64_t line = tid / cellpad;
    if (line >= N * N || cell >= cw) return;
    int64_t base, stride;
    if (AXIS == 2) {  // line = (i1, i3)
        base = (line / N) * N * N + (line % N);
        stride = N;
    } else {  // AXIS == 1, line = (i2, i3)
        base = line;
        stride = N * N;
    }
    T xr[N], xi[N];
    // partial sum s of all N points at once (N independent loads per round
    // trip), added in the order s = 0, 1, ..., S - 1 for every point
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const C2<TIN> z = in[(base + j * stride) * cellpad + cell];
        xr[j] = (T)z.re;
        xi[j] = (T)z.im;
    }
    for (int s = 1; s < S; ++s) {
        C2<TIN> w[N];
#pragma unroll
        for (int j = 0; j < N; ++j) w[j] = in[(base + j * stride) * cellpad + cell + s * part_stride];
        __builtin_amdgcn_sched_barrier(0);  // all N loads before the first add
#pragma unroll
        for (int j = 0; j < N; ++j) {
            xr[j] += (T)w[j].re;
            xi[j] += (T)w[j].im;
        }
    }
#pragma unroll
    for (int j = 1; j < N; j += 2) {
        xr[j] = -xr[j];
        xi[j] = -xi[j];
    }
    fft_line<T, N, DIR>(xr, xi, tw);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int p = out_pos<N>(k);
        const T s = (k & 1) ? -scale : scale;
        out[(base + k * stride) * cellpad + cell] = C2<TOUT>{(TOUT)(s * xr[p]), (TOUT)(s * xi[p])};
    }
}

// ---------------------------------------------------------------- inverse
// last pass: axis 3 of work[(line*N + k3)][cell] -> real Qt[cell][line*N + j3]
template <typename T, int N>
__global__ __launch_bounds__(256) void inv_axis3(const C2<T> *__restrict__ work, T *__restrict__ Qt,
                                                 const T *__restrict__ tw, int64_t ncells, int64_t cellpad, T scale,
                                                 const int64_t *__restrict__ off) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cell = tid % cellpad;
    const int64_t line = tid / cellpad;
    if (line >= N * N || cell >= ncells) return;
    T xr[N], xi[N];
    const C2<T> *src = work + (line * N) * cellpad + cell;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const C2<T> z = src[(int64_t)k * cellpad];
        xr[k] = (k & 1) ? -z.re : z.re;
        xi[k] = (k & 1) ? -z.im : z.im;
    }
    fft_line<T, N, +1>(xr, xi, tw);
    T *dst = Qt + (off ? off[cell] : cell * (int64_t)(N * N * N)) + line * N;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int p = out_pos<N>(j);
        dst[j] = ((j & 1) ? -scale : scale) * xr[p];
    }
}

// ------------------------------------------------- fused axis-3 + axis-2
// One workgroup takes plane j1 of CB consecutive cells through LDS: the
// caller's [cell][j1][j2][j3] plane (N^2 contiguous reals per cell) is read
// coalesced, transformed along j3 and then j2 in LDS (one line per thread per
// axis), and written to the [mode][cell] workspace as runs of CB cells per
// mode.  The inverse kernel does the reverse (axis 2, axis 3, real part,
// scale, caller layout).  Each LDS line, and each cell's plane, is padded by
// one element so that the threads of a wavefront reading point j of their
// lines, or mode q of their cells, hit distinct banks.
template <typename T, int N>
struct PlaneShape {
    // cells per workgroup: small blocks give more, shorter workgroups per CU
    // whose load, LDS and store phases overlap (FP64 N = 16: 8 -> 4 cells
    // took the 256-cell step from 298 to 290 us); FP32 N = 16 measured best
    // at 16
    static constexpr int CB = sizeof(T) == 8 ? (N <= 16 ? (N <= 8 ? 8 : 4) : 4) : (N <= 8 ? 8 : (N <= 16 ? 16 : 8));
    static constexpr int LINES = CB * N;  // lines per axis = threads
    static constexpr int LD = N + 1;      // padded line length
    static constexpr int CS = N * LD + 1; // padded plane length (cell stride)
    static constexpr int THREADS = LINES;
    static_assert(kWave % CB == 0, "cell blocks must tile the 64-cell padding");
    static_assert(THREADS <= 256, "one line per thread");
};

// Element offset of each of the block's CB cells in the caller's [cell][mode]
// buffer (-1 for padding cells beyond ncells), read once into LDS so that the
// loads and stores of the plane need no per-element offset lookups (a lookup
// per element would wait for its offset, and with it for every load or store
// issued before).  Visible to the block after its next __syncthreads.
template <int N, int CB>
__device__ __forceinline__ void plane_cell_bases(int64_t (&cbase)[CB], int64_t cell0, int64_t ncells,
                                                 const int64_t *__restrict__ off, int t) {
    if (t < CB) {
        const int64_t cell = cell0 + t;
        cbase[t] = cell < ncells ? (off ? off[cell] : cell * (int64_t)N * N * N) : -1;
    }
}

template <typename T, int N, int DIR>
__device__ __forceinline__ void lds_line_fft(C2<T> *lds, int base, int step, const T *__restrict__ tw, T outscale) {
    T xr[N], xi[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const C2<T> z = lds[base + j * step];
        xr[j] = (j & 1) ? -z.re : z.re;
        xi[j] = (j & 1) ? -z.im : z.im;
    }
    fft_line<T, N, DIR>(xr, xi, tw);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int p = out_pos<N>(k);
        const T sgn = (k & 1) ? -outscale : outscale;
        lds[base + k * step] = C2<T>{sgn * xr[p], sgn * xi[p]};
    }
}

template <typename TI, typename T, int N>
__global__ __launch_bounds__((PlaneShape<T, N>::THREADS)) void fwd_plane(const TI *__restrict__ f, C2<T> *__restrict__ work,
                                                                       const T *__restrict__ tw, int64_t ncells,
                                                                       int64_t cellpad, const int64_t *__restrict__ off) {
    using PS = PlaneShape<T, N>;
    constexpr int CB = PS::CB, LD = PS::LD, CS = PS::CS, NP = N * N;
    __shared__ C2<T> lds[CB * CS];
    const int j1 = blockIdx.x % N;
    const int64_t cell0 = (int64_t)(blockIdx.x / N) * CB;
    const int t = threadIdx.x;
    __shared__ int64_t cbase[CB];
    plane_cell_bases<N>(cbase, cell0, ncells, off, t);
    __syncthreads();
    // load: element pair e = (cell c, positions q, q + 1; q = j2 N + j3 even)
    // of the block's planes, two reals per load (every plane starts at an
    // even element offset: N is even).  All N/2 loads of a thread are issued
    // before the first is used (one round trip instead of one per load); a
    // padding cell reads from the buffer's first N^3 values (in bounds for
    // any buffer that holds a cell) and keeps zeros.
    constexpr int LI = CB * NP / 2 / PS::THREADS;
    static_assert(LI * PS::THREADS == CB * NP / 2, "whole rounds of loads");
    C2<TI> x[LI];
#pragma unroll
    for (int i = 0; i < LI; ++i) {
        const int e = t + i * PS::THREADS;
        const int c = e / (NP / 2), q = 2 * (e % (NP / 2));
        const int64_t b = cbase[c];
        x[i] = *reinterpret_cast<const C2<TI> *>(f + (b < 0 ? 0 : b) + (int64_t)j1 * NP + q);
        if (b < 0) x[i] = C2<TI>{(TI)0, (TI)0};
    }
#pragma unroll
    for (int i = 0; i < LI; ++i) {
        const int e = t + i * PS::THREADS;
        const int c = e / (NP / 2), q = 2 * (e % (NP / 2));
        lds[c * CS + (q / N) * LD + q % N] = C2<T>{(T)x[i].re, (T)0};
        lds[c * CS + (q / N) * LD + q % N + 1] = C2<T>{(T)x[i].im, (T)0};
    }
    __syncthreads();
    // axis 3: line (c, j2) = t, points contiguous
    lds_line_fft<T, N, -1>(lds, (t / N) * CS + (t % N) * LD, 1, tw, (T)1);
    __syncthreads();
    // axis 2: line (c, k3) = t, points one padded line apart
    lds_line_fft<T, N, -1>(lds, (t / N) * CS + t % N, LD, tw, (T)1);
    __syncthreads();
    // store: mode (j1, k2, k3) of cell c -> work[mode][cell], runs of CB cells
#pragma unroll
    for (int i = 0; i < CB * NP / PS::THREADS; ++i) {
        const int e = t + i * PS::THREADS;
        const int c = e % CB, q = e / CB;
        work[((int64_t)j1 * NP + q) * cellpad + cell0 + c] = lds[c * CS + (q / N) * LD + q % N];
    }
}

template <typename T, int N>
__global__ __launch_bounds__((PlaneShape<T, N>::THREADS)) void inv_plane(const C2<T> *__restrict__ work, T *__restrict__ Qt,
                                                                       const T *__restrict__ tw, int64_t ncells,
                                                                       int64_t cellpad, T scale,
                                                                       const int64_t *__restrict__ off) {
    using PS = PlaneShape<T, N>;
    constexpr int CB = PS::CB, LD = PS::LD, CS = PS::CS, NP = N * N;
    __shared__ C2<T> lds[CB * CS];
    const int j1 = blockIdx.x % N;
    const int64_t cell0 = (int64_t)(blockIdx.x / N) * CB;
    const int t = threadIdx.x;
    __shared__ int64_t cbase[CB];
    plane_cell_bases<N>(cbase, cell0, ncells, off, t);
    // all N loads of a thread in flight before the first LDS write
    constexpr int LI = CB * NP / PS::THREADS;
    static_assert(LI * PS::THREADS == CB * NP, "whole rounds of loads");
    C2<T> x[LI];
#pragma unroll
    for (int i = 0; i < LI; ++i) {
        const int e = t + i * PS::THREADS;
        x[i] = work[((int64_t)j1 * NP + e / CB) * cellpad + cell0 + e % CB];
    }
#pragma unroll
    for (int i = 0; i < LI; ++i) {
        const int e = t + i * PS::THREADS;
        const int c = e % CB, q = e / CB;
        lds[c * CS + (q / N) * LD + q % N] = x[i];
    }
    __syncthreads();
    // axis 2: line (c, k3) = t
    lds_line_fft<T, N, +1>(lds, (t / N) * CS + t % N, LD, tw, (T)1);
    __syncthreads();
    // axis 3: line (c, j2) = t, with the transform's scale
    lds_line_fft<T, N, +1>(lds, (t / N) * CS + (t % N) * LD, 1, tw, scale);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CB * NP / 2 / PS::THREADS; ++i) {  // two reals per store, as in fwd_plane
        const int e = t + i * PS::THREADS;
        const int c = e / (NP / 2), q = 2 * (e % (NP / 2));
        const int64_t b = cbase[c];
        if (b >= 0)
            *reinterpret_cast<C2<T> *>(Qt + b + (int64_t)j1 * NP + q) =
                C2<T>{lds[c * CS + (q / N) * LD + q % N].re, lds[c * CS + (q / N) * LD + q % N + 1].re};
    }
}

// ------------------------------------------------------- whole cells
// For a single cell at N <= 16 the plain (unbatched) path transforms the whole
// cell in one workgroup of N^2 threads: the N^3 values sit in LDS (lines
// padded by one element, planes by one more) and the three axes are done
// there one after the other, the same line transforms (phases, radix passes,
// signs and scale) as the plane and middle passes, so results are identical.
// The workspace then holds the one cell unpadded (cell stride 1), so f^ and
// the partial sums are contiguous.  One launch per direction instead of two.
// Workgroup b of a batch runs on XCD b mod 8.  The cells that share a cache
// line of the [mode][cell] workspace (G of them: 8 FP64 or 16 FP32 complex
// values) go to the same XCD, so their scattered writes and reads meet in one
// L2: XCD x takes the line groups g = x, x + 8, ... in turn.  ncells rounded
// up to a multiple of 8 G (the workspace's 64-cell padding is one); with one
// cell, cell 0.
template <int G>
__device__ __forceinline__ int64_t cell_of_block(int64_t b) {
    const int64_t x = b % kXcds, i = b / kXcds;
    return G * (x + kXcds * (i / G)) + i % G;
}

template <int N>
struct CellShape {
    static constexpr int LD = N + 1;       // padded line
    static constexpr int PS = N * LD + 1;  // padded plane
    static constexpr int SIZE = N * PS;
    static constexpr int THREADS = N * N;  // one line per thread per axis (N values per thread)
};

// forward: real f of cell blockIdx.x (TI) -> f^ (TO) at fhat[q * cellpad + cell],
// computed in T
template <typename TI, typename T, typename TO, int N>
__global__ __launch_bounds__(N * N) void fwd_cell(const TI *__restrict__ f, C2<TO> *__restrict__ fhat,
                                                 const T *__restrict__ tw, int64_t ncells, int64_t cellpad, T scale) {
    using CS = CellShape<N>;
    __shared__ C2<T> lds[CS::SIZE];
    const int64_t cell = cellpad == 1 ? 0 : cell_of_block<128 / sizeof(C2<TO>)>(blockIdx.x);
    if (cell >= ncells) return;  // padding cells: their lanes of the convolution are never read back
    const int t = threadIdx.x;
    const TI *src = f + cell * (int64_t)(N * N * N);
    // all N loads of a thread in flight at once (q = (j1 N + j2) N + j3, coalesced)
    TI x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = src[t + i * CS::THREADS];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int q = t + i * CS::THREADS;
        lds[(q / (N * N)) * CS::PS + ((q / N) % N) * CS::LD + q % N] = C2<T>{(T)x[i], (T)0};
    }
    __syncthreads();
    const int a = t / N, b = t % N;
    lds_line_fft<T, N, -1>(lds, a * CS::PS + b * CS::LD, 1, tw, (T)1);  // axis 3: line (j1, j2)
    __syncthreads();
    lds_line_fft<T, N, -1>(lds, a * CS::PS + b, CS::LD, tw, (T)1);      // axis 2: line (j1, k3)
    __syncthreads();
    lds_line_fft<T, N, -1>(lds, a * CS::LD + b, CS::PS, tw, scale);     // axis 1: line (k2, k3)
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int q = t + i * CS::THREADS;
        const C2<T> z = lds[(q / (N * N)) * CS::PS + ((q / N) % N) * CS::LD + q % N];
        fhat[q * cellpad + cell] = C2<TO>{(TO)z.re, (TO)z.im};
    }
}

// inverse: the S partial sums of cell blockIdx.x (added in the order s = 0 ..
// S - 1) -> real Q~ (caller layout)
template <typename T, int N>
__global__ __launch_bounds__(N * N) void inv_cell(const C2<T> *__restrict__ part, int S, int64_t part_stride,
                                                 T *__restrict__ Qt, const T *__restrict__ tw, int64_t ncells,
                                                 int64_t cellpad, T scale) {
    using CS = CellShape<N>;
    __shared__ C2<T> lds[CS::SIZE];
    const int64_t cell = cellpad == 1 ? 0 : cell_of_block<128 / sizeof(C2<T>)>(blockIdx.x);
    if (cell >= ncells) return;
    const int t = threadIdx.x;
    // all N values of a thread per partial in flight at once, partials added
    // in the order s = 0, 1, ..., S - 1
    C2<T> z[N];
#pragma unroll
    for (int i = 0; i < N; ++i) z[i] = part[(t + i * CS::THREADS) * cellpad + cell];
    for (int s = 1; s < S; ++s) {
        C2<T> w[N];
#pragma unroll
        for (int i = 0; i < N; ++i) w[i] = part[(t + i * CS::THREADS) * cellpad + cell + s * part_stride];
        __builtin_amdgcn_sched_barrier(0);  // all N loads before the first add
#pragma unroll
        for (int i = 0; i < N; ++i) {
            z[i].re += w[i].re;
            z[i].im += w[i].im;
        }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int q = t + i * CS::THREADS;
        lds[(q / (N * N)) * CS::PS + ((q / N) % N) * CS::LD + q % N] = z[i];
    }
    __syncthreads();
    const int a = t / N, b = t % N;
    lds_line_fft<T, N, +1>(lds, a * CS::LD + b, CS::PS, tw, (T)1);      // axis 1: line (k2, k3)
    __syncthreads();
    lds_line_fft<T, N, +1>(lds, a * CS::PS + b, CS::LD, tw, (T)1);      // axis 2: line (j1, k3)
    __syncthreads();
    lds_line_fft<T, N, +1>(lds, a * CS::PS + b * CS::LD, 1, tw, scale);  // axis 3: line (j1, j2)
    __syncthreads();
    T *dst = Qt + cell * (int64_t)(N * N * N);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int q = t + i * CS::THREADS;
        dst[q] = lds[(q / (N * N)) * CS::PS + ((q / N) % N) * CS::LD + q % N].re;
    }
}

// Cells a pass works on: the whole padded group (64-cell multiples keep every
// wavefront on one line, coalesced), or for a batch under one group only its
// cells -- the padding's transforms are never read (no pass mixes cells, and
// only real cells reach Qt), and a single cell would otherwise pay for 64.
// The threads keep the padded layout (a thread per line and padded cell,
// the padding's threads return at once), so a few cells' lines still spread
// over many workgroups.
int64_t cells_worked(int64_t ncells, int64_t cellpad) { return ncells < kWave ? ncells : cellpad; }

// For N <= 24 the first pass writes tmp (a buffer of fhat's size that is free
// during the forward transform) and the second reads it into fhat: measured
// 7 us instead of 13 us for the second pass of 256 N = 16 cells than in
// place.  At N = 32 the FP64 passes stay in place on fhat: one array of
// 268 MB (512 FP64 cells) instead of two keeps more of it in the 256 MB
// last-level cache (out of place the middle passes took 110 and 129 us
// instead of 91 and 89).  The FP32 path (T = float) computes in FP64 (TW):
// its intermediates are FP64 in tmp, which then holds at least twice fhat's
// FP32 size, and only the last pass writes FP32 f^ into fhat.
template <typename T, int N>
hipError_t forward_n(const bz_op *op, int64_t ncells, int64_t cellpad, const void *f, void *fhat, void *tmp,
                     const int64_t *off, hipStream_t s) {
    using TW = double;
    const TW *tw = op->d_tw64;
    const int64_t cw = cells_worked(ncells, cellpad);
    const int64_t threads = (int64_t)N * N * cellpad;
    const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
    C2<T> *w = (C2<T> *)fhat;
    C2<TW> *t = (C2<TW> *)tmp;
    const TW scale = (TW)op->geo.fwd_scale;
    if constexpr (N <= 24) {  // axes 3 and 2 in one pass through LDS
        using PS = PlaneShape<TW, N>;
        hipLaunchKernelGGL((fwd_plane<T, TW, N>), dim3((unsigned)(N * ((cw + PS::CB - 1) / PS::CB))),
                           dim3(PS::THREADS), 0, s, (const T *)f, t, tw, ncells, cellpad, off);
        hipLaunchKernelGGL((mid_pass<TW, TW, T, N, 1, -1>), grid, block, 0, s, t, 1, (int64_t)0, w, tw, cellpad, cw,
                           scale);
    } else if constexpr (sizeof(T) == sizeof(TW)) {  // in place on fhat
        C2<TW> *x = (C2<TW> *)fhat;
        hipLaunchKernelGGL((fwd_axis3<T, TW, N>), grid, block, 0, s, (const T *)f, x, tw, ncells, cellpad, cw, off);
        hipLaunchKernelGGL((mid_pass<TW, TW, TW, N, 2, -1>), grid, block, 0, s, x, 1, (int64_t)0, x, tw, cellpad, cw,
                           (TW)1);
        hipLaunchKernelGGL((mid_pass<TW, TW, TW, N, 1, -1>), grid, block, 0, s, x, 1, (int64_t)0, x, tw, cellpad, cw,
                           scale);
    } else {  // FP64 intermediates in tmp, FP32 f^ in fhat
        hipLaunchKernelGGL((fwd_axis3<T, TW, N>), grid, block, 0, s, (const T *)f, t, tw, ncells, cellpad, cw, off);
        hipLaunchKernelGGL((mid_pass<TW, TW, TW, N, 2, -1>), grid, block, 0, s, t, 1, (int64_t)0, t, tw, cellpad, cw,
                           (TW)1);
        hipLaunchKernelGGL((mid_pass<TW, TW, T, N, 1, -1>), grid, block, 0, s, t, 1, (int64_t)0, w, tw, cellpad, cw,
                           scale);
    }
    return hipGetLastError();
}

template <typename T, int N>
hipError_t inverse_n(const bz_op *op, int64_t ncells, int64_t cellpad, int S, void *part, void *work, void *Qt,
                     const T *tw, const int64_t *off, hipStream_t s) {
    const int64_t cw = cells_worked(ncells, cellpad);
    const int64_t threads = (int64_t)N * N * cellpad;
    const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
    const int64_t pstride = (int64_t)N * N * N * cellpad;
    C2<T> *w = (C2<T> *)work;
    hipLaunchKernelGGL((mid_pass<T, T, T, N, 1, +1>), grid, block, 0, s, (const C2<T> *)part, S, pstride, w, tw,
                       cellpad, cw, (T)1);
    if constexpr (N <= 24) {  // axes 2 and 3 in one pass through LDS
        using PS = PlaneShape<T, N>;
        hipLaunchKernelGGL((inv_plane<T, N>), dim3((unsigned)(N * ((cw + PS::CB - 1) / PS::CB))), dim3(PS::THREADS),
                           0, s, (const C2<T> *)w, (T *)Qt, tw, ncells, cellpad, (T)op->geo.inv_scale, off);
    } else {
        hipLaunchKernelGGL((mid_pass<T, T, T, N, 2, +1>), grid, block, 0, s, w, 1, (int64_t)0, w, tw, cellpad, cw,
                           (T)1);
        hipLaunchKernelGGL((inv_axis3<T, N>), grid, block, 0, s, w, (T *)Qt, tw, ncells, cellpad,
                           (T)op->geo.inv_scale, off);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_forward(const bz_op *op, int64_t ncells, int64_t cellpad, const void *f, void *fhat, void *tmp,
                          const int64_t *off, hipStream_t s) {
    const bool f64 = op->wdtype == BZ_F64;
    switch (op->N) {
#define BZ_FWD_CASE(NN)                                                                        \
    case NN:                                                                                   \
        return f64 ? forward_n<double, NN>(op, ncells, cellpad, f, fhat, tmp, off, s) \
                   : forward_n<float, NN>(op, ncells, cellpad, f, fhat, tmp, off, s);
        BZ_FWD_CASE(8)
        BZ_FWD_CASE(16)
        BZ_FWD_CASE(24)
        BZ_FWD_CASE(32)
        BZ_FWD_CASE(48)
#undef BZ_FWD_CASE
    }
    return hipErrorInvalidValue;
}

bool cell_transforms_ok(const bz_op *op, int64_t cellpad) {
    const int64_t per_xcd = 8 * (op->wdtype == BZ_F64 ? 8 : 16);  // XCDs x cells per cache line
    return op->N <= 16 && (cellpad == 1 || cellpad % per_xcd == 0);
}

hipError_t launch_forward_cells(const bz_op *op, int64_t ncells, int64_t cellpad, const void *f, void *fhat,
                                hipStream_t s) {
    if (!cell_transforms_ok(op, cellpad) || ncells < 1 || ncells > cellpad) return hipErrorInvalidValue;
    const double scale = op->geo.fwd_scale;
    const dim3 grid((unsigned)(cellpad == 1 ? 1 : cellpad)), block((unsigned)(op->N * op->N));
    const bool f64 = op->wdtype == BZ_F64;
    switch (op->N) {
#define BZ_FWDC_CASE(NN)                                                                                         \
    case NN:                                                                                                     \
        if (f64)                                                                                                 \
            hipLaunchKernelGGL((fwd_cell<double, double, double, NN>), grid, block, 0, s, (const double *)f,    \
                               (C2<double> *)fhat, op->d_tw64, ncells, cellpad, scale);                                  \
        else                                                                                                     \
            hipLaunchKernelGGL((fwd_cell<float, double, float, NN>), grid, block, 0, s, (const float *)f,       \
                               (C2<float> *)fhat, op->d_tw64, ncells, cellpad, scale);                                   \
        return hipGetLastError();
        BZ_FWDC_CASE(8)
        BZ_FWDC_CASE(16)
#undef BZ_FWDC_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_inverse_cells(const bz_op *op, int64_t ncells, int64_t cellpad, int S, const void *part,
                                void *Qt, hipStream_t s) {
    if (!cell_transforms_ok(op, cellpad) || ncells < 1 || ncells > cellpad) return hipErrorInvalidValue;
    const int64_t pstride = (int64_t)op->N * op->N * op->N * cellpad;
    const dim3 grid((unsigned)(cellpad == 1 ? 1 : cellpad)), block((unsigned)(op->N * op->N));
    const bool f64 = op->wdtype == BZ_F64;
    switch (op->N) {
#define BZ_INVC_CASE(NN)                                                                                          \
    case NN:                                                                                                      \
        if (f64)                                                                                                  \
            hipLaunchKernelGGL((inv_cell<double, NN>), grid, block, 0, s, (const C2<double> *)part, S, pstride,   \
                               (double *)Qt, op->d_tw64, ncells, cellpad, op->geo.inv_scale);                             \
        else                                                                                                      \
            hipLaunchKernelGGL((inv_cell<float, NN>), grid, block, 0, s, (const C2<float> *)part, S, pstride,     \
                               (float *)Qt, op->d_tw32, ncells, cellpad, (float)op->geo.inv_scale);                       \
        return hipGetLastError();
        BZ_INVC_CASE(8)
        BZ_INVC_CASE(16)
#undef BZ_INVC_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_inverse(const bz_op *op, int64_t ncells, int64_t cellpad, int S, void *part, void *Qt,
                          const int64_t *off, hipStream_t s, void *work) {
    const bool f64 = op->wdtype == BZ_F64;
    if (!work) work = op->d_fhat;  // the forward transform is dead once the convolution has run
    switch (op->N) {
#define BZ_INV_CASE(NN)                                                                            \
    case NN:                                                                                       \
        return f64 ? inverse_n<double, NN>(op, ncells, cellpad, S, part, work, Qt, op->d_tw64, off, s) \
                   : inverse_n<float, NN>(op, ncells, cellpad, S, part, work, Qt, op->d_tw32, off, s);
        BZ_INV_CASE(8)
        BZ_INV_CASE(16)
        BZ_INV_CASE(24)
        BZ_INV_CASE(32)
        BZ_INV_CASE(48)
#undef BZ_INV_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace bz
