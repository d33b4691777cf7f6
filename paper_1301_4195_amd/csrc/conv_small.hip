// Truncated weighted convolution of the collision step (Sec. 3.2) for small
// batches -- one cell up to one group of 64 cells:
//   Q^(zeta_k) = sum_{m : k - m + N/2 in [0,N)^3} W[k][m] f^(xi_m) f^(zeta_k - xi_m)
// With few cells each weight serves a few multiply-adds (10 flops per stored
// FP64 weight and cell: 1.25 flop per byte), so the sum -- the O(N^6) term of
// Sec. 4.1 -- is bound by the stream of weights from memory, and the mapping
// of conv.hip (one lane per cell, weights as scalar operands) would leave
// most lanes idle and wait on one scalar load per m3 group.  Here:
//   * a workgroup of kSmallWaves (4 or 8) wavefronts owns one item (output row
//     (k1, k2), one of S chunks of its m1 range, one block of CB cells); its
//     wavefronts take every kSmallWaves-th kept line (m1, m2) of the chunk.
//   * lane = (k3, j): output k3 = lane mod N, m3 residue j = lane / N, with
//     R = 64 / N residues, so a lane visits m3 = j, j + R, ... of each line.
//     A line's weights are read by all lanes at once, m3 by m3: R runs of
//     consecutive k3 of the m3-major line block per load (coalesced); a lane
//     applies each weight it loads to all CB cells of the block.
//   * the line's f^ values u(m3) and v(n3) of the block's cells are staged
//     in the wavefront's own part of LDS (no barrier: LDS operations of one
//     wavefront complete in issue order).  The next line's values and the
//     next batch of weights are loaded while the current batch is summed.
//   * the mirrored couples of the batched kernel are kept: half of the lines,
//     weight W[k][m] + W[k][n] (the same packed table).
//   * at the end the lanes' sums of equal k3 (R residues, kSmallWaves
//     wavefronts) are added in a fixed order, so results are reproducible.
// FP32 sums fold each line's partial into an FP64 running sum, as the
// batched kernel does.
#include "bz_internal.h"

#include <type_traits>

namespace bz {
namespace {

template <typename T>
struct C2 {
    T re, im;
};

// wavefronts per workgroup (one item): eight for blocks of one or two cells
// (shorter chains of lines per wavefront), four for larger blocks (whose
// sums would fill more LDS at the end)
template <int CB>
constexpr int kSmallWaves = CB <= 2 ? 8 : 4;

// Offset of the m3 block of a line's packed weights: sum of kcount(N, t) for
// t < m.  kcount(t) = t + N/2 for t <= N/2 and N + N/2 - t for t >= N/2.
__host__ __device__ constexpr int line_woff(int N, int m) {
    const int c = N / 2;
    if (m <= c) return m * (m - 1) / 2 + m * c;
    const int at_c = c * (c - 1) / 2 + c * c;
    return at_c + (m - c) * (N + c) - (m - c) * (c + m - 1) / 2;
}

constexpr bool woff_matches(int N) {
    int p = 0;
    for (int m = 0; m < N; ++m) {
        if (line_woff(N, m) != p) return false;
        p += kcount(N, m);
    }
    return p == line_pairs(N) && line_woff(N, N) == p;
}
static_assert(woff_matches(8) && woff_matches(16) && woff_matches(24) && woff_matches(32) && woff_matches(48),
              "closed form of the line block offsets");

template <typename T, int N, int CB>
__global__ __launch_bounds__(64 * kSmallWaves<CB>) void conv_small_kernel(
    const C2<T> *__restrict__ fhat, C2<T> *__restrict__ part, const T *__restrict__ W,
    const int64_t *__restrict__ rowoff, int64_t wbase, int row0, int S, int nblk, int64_t ncells, int64_t cellpad) {
    constexpr int c = N / 2;
    constexpr int P = line_pairs(N);
    constexpr int R = 64 / N;             // m3 residues (lanes per output k3)
    static_assert(R >= 1 && N % R == 0, "whole m3 residue classes");
    constexpr int IT = N / R;             // m3 values per lane and line
    constexpr int KB = IT <= 8 ? IT : (IT % 8 == 0 ? 8 : 6);  // of which one batch of loads is in flight
    static_assert(IT % KB == 0, "whole batches");
    constexpr int NU = N * CB;            // staged u values (then as many v values)
    constexpr int NV = (2 * NU + 63) / 64;  // staged values per lane
    constexpr int kRed = 64 * CB;
    constexpr int kLds = 2 * NU > kRed ? 2 * NU : kRed;
    constexpr bool kComp = sizeof(T) == 4;
    using TA = std::conditional_t<kComp, double, T>;  // running-sum type
    // the staging area, reused at the end for the lanes' running sums
    constexpr int kWaveBytes = (int)(kLds * sizeof(C2<T>) > kRed * sizeof(C2<TA>) ? kLds * sizeof(C2<T>)
                                                                                    : kRed * sizeof(C2<TA>));
    __shared__ __align__(16) unsigned char lds_raw[kSmallWaves<CB>][kWaveBytes];

    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
    const int blk = blockIdx.x % nblk;
    const int chunk = (blockIdx.x / nblk) % S;
    const int row = row0 + blockIdx.x / (nblk * S);
    const int k1 = row / N, k2 = row % N;
    const int lo1 = mlo(N, k1), c1 = mcount(N, k1);
    const int lo2 = mlo(N, k2), c2 = mcount(N, k2);
    // the chunk's kept lines, consecutive in (a1, a2) order (as in conv.hip)
    const int h1 = half_a1_end(c1);
    const int per = (h1 + S - 1) / S;
    const int a1b = min(h1, chunk * per);
    const int a1e = min(h1, a1b + per);
    const int nlines = a1e <= a1b ? 0 : (a1e - a1b - 1) * c2 + half_a2_end(c1, c2, a1e - 1);
    const T *__restrict__ wrow = W + (rowoff[row] - wbase) + (int64_t)a1b * c2 * P;
    const int64_t cell0 = (int64_t)blk * CB;

    const int k3 = lane % N, j = lane / N;
    const bool active = j < R;  // lanes past R N idle (N = 24, 48)
    C2<T> *st = reinterpret_cast<C2<T> *>(lds_raw[wv]);

    TA ar[CB], ai[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b) ar[b] = ai[b] = (TA)0;

    // the line's u and v values of the block's cells: value e is u(e / CB)
    // for e < NU, else v((e - NU) / CB), of cell e mod CB; staged cell-major
    // (u of cell b at b N + m3, v at NU + b N + n3) so that lanes of
    // consecutive n3 read consecutive LDS words
    auto load_values = [&](C2<T> (&sv)[NV], int l) {
        const int a1 = a1b + l / c2, a2 = l % c2;
        const int64_t ub = ((int64_t)(lo1 + a1) * N + (lo2 + a2)) * N;
        const int64_t vb = ((int64_t)(k1 - lo1 - a1 + c) * N + (k2 - lo2 - a2 + c)) * N;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const int e = lane + 64 * q;
            if (e < 2 * NU) {
                const int r = e < NU ? e : e - NU;
                const int64_t mode = (e < NU ? ub : vb) + r / CB;
                sv[q] = fhat[mode * cellpad + cell0 + r % CB];
            }
        }
    };
    // weights of m3 batch ib of line l (0 where the pair is outside the sum)
    auto load_weights = [&](T (&w)[KB], int l, int ib) {
        const T *__restrict__ wl = wrow + (int64_t)l * P;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            const int m3 = j + R * (ib * KB + i), n3 = k3 - m3 + c;
            const bool valid = active && n3 >= 0 && n3 < N;
            // in the line's block for every lane (index 0 where invalid)
            const T x = wl[valid ? line_woff(N, m3) + k3 - klo(N, m3) : 0];
            w[i] = valid ? x : (T)0;
        }
    };
    constexpr int NB = IT / KB;  // weight batches per line
    // software pipeline: the next line's values and the next batch's
    // weights are in flight while the current batch is summed
    const int nmine = nlines > wv ? (nlines - wv + kSmallWaves<CB> - 1) / kSmallWaves<CB> : 0;
    C2<T> svn[NV];
    T wn[KB];
    if (nmine > 0) {
        load_values(svn, wv);
        load_weights(wn, wv, 0);
    }
    for (int t = 0; t < nmine; ++t) {
        const int l = wv + kSmallWaves<CB> * t;
        const bool more = t + 1 < nmine;
        // the previous line's reads of the staging area were issued before
        // these writes, and this line's reads are issued after them
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const int e = lane + 64 * q;
            if (e < 2 * NU) {
                const int r = e < NU ? e : e - NU;
                st[(e < NU ? 0 : NU) + (r % CB) * N + r / CB] = svn[q];
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (more) load_values(svn, l + kSmallWaves<CB>);
        T sr[CB], si[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) sr[b] = si[b] = (T)0;
#pragma unroll 1
        for (int ib = 0; ib < NB; ++ib) {
            T w[KB];
#pragma unroll
            for (int i = 0; i < KB; ++i) w[i] = wn[i];
            if (ib + 1 < NB)
                load_weights(wn, l, ib + 1);
            else if (more)
                load_weights(wn, l + kSmallWaves<CB>, 0);
#pragma unroll
            for (int i = 0; i < KB; ++i) {
                const int m3 = j + R * (ib * KB + i), n3 = k3 - m3 + c;
                const bool valid = active && n3 >= 0 && n3 < N;
                const int mu = valid ? m3 : 0, nv = valid ? n3 : 0;  // in bounds; the weight is 0 then
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    const C2<T> u = st[b * N + mu], v = st[NU + b * N + nv];
                    const T pr = u.re * v.re - u.im * v.im;
                    const T pi = u.re * v.im + u.im * v.re;
                    if constexpr (kComp) {
                        sr[b] += w[i] * pr;
                        si[b] += w[i] * pi;
                    } else {
                        ar[b] += w[i] * pr;
                        ai[b] += w[i] * pi;
                    }
                }
            }
        }
        if constexpr (kComp) {  // fold the line's partial
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                ar[b] += (double)sr[b];
                ai[b] += (double)si[b];
            }
        }
    }
    // sums of equal k3: residues j, then wavefronts, in a fixed order, in the
    // running sums' precision
    __syncthreads();
#pragma unroll
    for (int b = 0; b < CB; ++b) reinterpret_cast<C2<TA> *>(lds_raw[wv])[lane * CB + b] = C2<TA>{ar[b], ai[b]};
    __syncthreads();
    for (int t = threadIdx.x; t < N * CB; t += 64 * kSmallWaves<CB>) {
        const int kk = t / CB, b = t % CB;
        TA sr = (TA)0, si = (TA)0;
        for (int w = 0; w < kSmallWaves<CB>; ++w)
            for (int jj = 0; jj < R; ++jj) {
                const C2<TA> x = reinterpret_cast<const C2<TA> *>(lds_raw[w])[(jj * N + kk) * CB + b];
                sr += x.re;
                si += x.im;
            }
        const int64_t cell = cell0 + b;
        if (cell < ncells)
            part[((int64_t)chunk * N * N * N + (int64_t)row * N + kk) * cellpad + cell] = C2<T>{(T)sr, (T)si};
    }
}

// ------------------------------------------------------------ one cell
// The same sum for a single cell (the plain per-cell path, N <= 16, cell
// stride 1 in the workspace), shaped so that all of a workgroup's weight
// loads are in flight at once: with one cell the packed table is read once
// and used for one multiply-add each, so the kernel is a stream of the table
// and its time is how long the loads wait.  A workgroup owns one item (output
// row, m1 chunk); thread (g, h) of its G x P/2 threads takes the two
// consecutive line positions 2h, 2h + 1 (fixed (m3, k3) pairs) of every G-th
// kept line of the chunk, g first, and issues the 16-byte (FP64) or 8-byte
// (FP32) weight loads of all of them together.  The chunk's u
// and v lines are staged in LDS first.  Each thread keeps the two sums of its
// two positions (FP64; FP32 terms are added in FP64); at the end the sums of
// equal k3 are added in a fixed order: positions ascending per line group,
// then the groups.
template <int N>
struct CellPlan {
    static constexpr int P = line_pairs(N);
    int m3[P], k3[P];    // pair at line position q
    int nq[N];           // positions with output k3, ascending
    int q[N][N];
    constexpr CellPlan() : m3(), k3(), nq(), q() {
        int p = 0;
        for (int m = 0; m < N; ++m)
            for (int k = klo(N, m); k <= khi(N, m); ++k) {
                m3[p] = m;
                k3[p] = k;
                q[k][nq[k]++] = p;
                ++p;
            }
    }
};

template <int N>
constexpr int kCellGroups = N <= 8 ? 16 : 4;  // line groups per workgroup
template <int N>
constexpr int kCellThreads = kCellGroups<N> * line_pairs(N) / 2;
constexpr int kCellMinChunks = 2;  // sizes the LDS stage of a chunk's lines
// kept lines of one chunk, at most: a row keeps at most N/2 values of a1
// (half of up to N), a chunk at most ceil((N/2) / S) of them, each with up to
// N lines (m2); S >= kCellMinChunks
template <int N>
constexpr int kCellMaxLines = ((N / 2 + kCellMinChunks - 1) / kCellMinChunks) * N;

template <typename T, int N>
__global__ __launch_bounds__(kCellThreads<N>) void conv_cell_kernel(const C2<T> *__restrict__ fhat,
                                                                    C2<T> *__restrict__ part, const T *__restrict__ W,
                                                                    const int64_t *__restrict__ rowoff, int64_t wbase,
                                                                    int row0, int S) {
    constexpr int c = N / 2;
    constexpr int P = line_pairs(N);
    constexpr int HP = P / 2;
    constexpr int G = kCellGroups<N>;
    constexpr int ML = kCellMaxLines<N>;
    constexpr int NB = (ML + G - 1) / G;  // lines per thread, at most
    constexpr CellPlan<N> cp{};
    using TA = double;  // sums (FP32 terms added in FP64)
    struct alignas(2 * sizeof(T)) Pair {
        T a, b;
    };
    // staged values per thread, and the stage: line l of the chunk holds u
    // at [l][0, N) and v at [l][N, 2N); lines past ML only take the repeated
    // values of threads beyond the chunk's lines
    constexpr int SI = (2 * ML * N + kCellThreads<N> - 1) / kCellThreads<N>;
    constexpr int MLP = (SI * kCellThreads<N> + 2 * N - 1) / (2 * N);
    __shared__ C2<T> sx[MLP][2 * N];
    __shared__ C2<TA> red[G][P];
    __shared__ C2<TA> red2[N][G];

    const int t = threadIdx.x, g = t / HP, h = t % HP;
    const int chunk = blockIdx.x % S;
    const int row = row0 + blockIdx.x / S;
    const int k1 = row / N, k2 = row % N;
    const int lo1 = mlo(N, k1), c1 = mcount(N, k1);
    const int lo2 = mlo(N, k2), c2 = mcount(N, k2);
    const int h1 = half_a1_end(c1);
    const int per = (h1 + S - 1) / S;
    const int a1b = min(h1, chunk * per);
    const int a1e = min(h1, a1b + per);
    const int nl = a1e <= a1b ? 0 : (a1e - a1b - 1) * c2 + half_a2_end(c1, c2, a1e - 1);
    // nl <= ML by construction (S >= kCellMinChunks); were it not, no line is
    // read and the item's sums come out NaN instead of touching LDS beyond
    // the stage
    const bool fits = nl <= ML;
    const int nlines = fits ? nl : 0;
    const T *__restrict__ wrow = W + (rowoff[row] - wbase) + (int64_t)a1b * c2 * P;

    // the thread's two line positions (table reads issued with the loads below)
    const int qa = 2 * h, qb = 2 * h + 1;
    const int ma = cp.m3[qa], ka = cp.k3[qa], mb = cp.m3[qb], kb = cp.k3[qb];
    // every weight of the thread's lines in flight, then the chunk's u and v
    // lines (all of a thread's loads issued before the first LDS write): the
    // loads of the whole item make one round trip
    Pair wb[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int l = g + G * i;
        if (l < nlines) wb[i] = *reinterpret_cast<const Pair *>(wrow + (int64_t)l * P + 2 * h);
    }
    // a thread past the chunk's 2 N nlines values loads the last one again
    // and stores it to an unused place: loads and stores without a branch,
    // so that the compiler keeps every load ahead of the first store
    const int ne = 2 * nlines * N;
    C2<T> st[SI];
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        const int e = min(t + i * kCellThreads<N>, max(ne - 1, 0));
        const int l = e / (2 * N), r = e % (2 * N);
        const int a1 = a1b + l / c2, a2 = l % c2;
        st[i] = fhat[r < N ? ((lo1 + a1) * N + (lo2 + a2)) * N + r
                           : ((k1 - lo1 - a1 + c) * N + (k2 - lo2 - a2 + c)) * N + (r - N)];
    }
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        const int e = t + i * kCellThreads<N>;
        sx[e / (2 * N)][e % (2 * N)] = st[i];
    }
    __syncthreads();

    TA ar = 0, ai = 0, br = 0, bi = 0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int l = g + G * i;
        if (l < nlines) {
            const C2<T> u = sx[l][ma], v = sx[l][N + ka - ma + c];
            const T pr = u.re * v.re - u.im * v.im, pi = u.re * v.im + u.im * v.re;
            ar += (TA)(wb[i].a * pr);
            ai += (TA)(wb[i].a * pi);
            const C2<T> ub = sx[l][mb], vb = sx[l][N + kb - mb + c];
            const T qr = ub.re * vb.re - ub.im * vb.im, qi = ub.re * vb.im + ub.im * vb.re;
            br += (TA)(wb[i].b * qr);
            bi += (TA)(wb[i].b * qi);
        }
    }
    // sums of equal k3, in a fixed order
    red[g][qa] = C2<TA>{ar, ai};
    red[g][qb] = C2<TA>{br, bi};
    __syncthreads();
    if (t < N * G) {
        const int k = t / G, gg = t % G;
        TA sr = 0, si = 0;
        for (int j = 0; j < cp.nq[k]; ++j) {
            const C2<TA> x = red[gg][cp.q[k][j]];
            sr += x.re;
            si += x.im;
        }
        red2[k][gg] = C2<TA>{sr, si};
    }
    __syncthreads();
    if (t < N) {
        TA sr = fits ? 0 : __builtin_nan(""), si = sr;
        for (int gg = 0; gg < G; ++gg) {
            sr += red2[t][gg].re;
            si += red2[t][gg].im;
        }
        part[(int64_t)chunk * N * N * N + (int64_t)row * N + t] = C2<T>{(T)sr, (T)si};
    }
}

template <typename T, int N, int CB>
hipError_t launch_cb(const void *fhat, void *part, const void *W, const int64_t *rowoff, int64_t wbase, int row0,
                     int nrows, int S, int nblk, int64_t ncells, int64_t cellpad, hipStream_t s) {
    const dim3 grid((unsigned)((int64_t)nrows * S * nblk)), block(64 * kSmallWaves<CB>);
    hipLaunchKernelGGL((conv_small_kernel<T, N, CB>), grid, block, 0, s, (const C2<T> *)fhat, (C2<T> *)part,
                       (const T *)W, rowoff, wbase, row0, S, nblk, ncells, cellpad);
    return hipGetLastError();
}

template <typename T, int N>
hipError_t launch_n(int CB, const void *fhat, void *part, const void *W, const int64_t *rowoff, int64_t wbase,
                    int row0, int nrows, int S, int nblk, int64_t ncells, int64_t cellpad, hipStream_t s) {
    switch (CB) {
    case 1: return launch_cb<T, N, 1>(fhat, part, W, rowoff, wbase, row0, nrows, S, nblk, ncells, cellpad, s);
    case 2: return launch_cb<T, N, 2>(fhat, part, W, rowoff, wbase, row0, nrows, S, nblk, ncells, cellpad, s);
    case 4:
        if constexpr (N <= 32)
            return launch_cb<T, N, 4>(fhat, part, W, rowoff, wbase, row0, nrows, S, nblk, ncells, cellpad, s);
        break;
    case 8:
        if constexpr (N <= 16)
            return launch_cb<T, N, 8>(fhat, part, W, rowoff, wbase, row0, nrows, S, nblk, ncells, cellpad, s);
        break;
    }
    return hipErrorInvalidValue;
}

}  // namespace

int small_cells_per_block(int N, int64_t ncells) {
    const int cap = N <= 16 ? 8 : (N <= 32 ? 4 : 2);
    int cb = 1;
    while (cb < cap && cb < ncells) cb *= 2;
    return cb;
}

// three chunks for one block of cells (measured best at N = 16, 24, 32 in
// FP64 and FP32: 3 x N^2 workgroups of 4-8 wavefronts), fewer as blocks add
// workgroups (more chunks add partial sums for the inverse transform to read)
int small_default_chunks(int N, int64_t ncells) {
    if (ncells == 1 && cell_conv_ok(N, 2)) return 2;  // the one-cell kernel: 12.9 us at 2, 13.9 at 3, 16.2 at 5 (N = 16)
    const int64_t nblk = (ncells + small_cells_per_block(N, ncells) - 1) / small_cells_per_block(N, ncells);
    return (int)std::max<int64_t>(1, std::min<int64_t>((3 + nblk - 1) / nblk, max_chunks(N)));
}

// measured crossover with the batched kernel: about 32 cells up to N = 16,
// about 16 above (where each block of cells re-reads a larger table)
bool small_by_default(int N, int64_t ncells) { return ncells <= (N <= 16 ? 32 : 16); }

bool cell_conv_ok(int N, int S) { return (N == 8 || N == 16) && S >= kCellMinChunks && S <= max_chunks(N); }

hipError_t launch_conv_cell(const bz_op *op, int S, const void *fhat, void *part, const void *W, int64_t wbase,
                            int row0, int row1, hipStream_t s) {
    if (!cell_conv_ok(op->N, S) || row1 <= row0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((row1 - row0) * S));
    const bool f64 = op->wdtype == BZ_F64;
    switch (op->N) {
#define BZ_CELL_CASE(NN)                                                                                           \
    case NN:                                                                                                       \
        if (f64)                                                                                                   \
            hipLaunchKernelGGL((conv_cell_kernel<double, NN>), grid, dim3(kCellThreads<NN>), 0, s,                 \
                               (const C2<double> *)fhat, (C2<double> *)part, (const double *)W, op->d_rowoff,      \
                               wbase, row0, S);                                                                    \
        else                                                                                                       \
            hipLaunchKernelGGL((conv_cell_kernel<float, NN>), grid, dim3(kCellThreads<NN>), 0, s,                  \
                               (const C2<float> *)fhat, (C2<float> *)part, (const float *)W, op->d_rowoff, wbase,  \
                               row0, S);                                                                           \
        return hipGetLastError();
        BZ_CELL_CASE(8)
        BZ_CELL_CASE(16)
#undef BZ_CELL_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_conv_small(const bz_op *op, int64_t ncells, int64_t cellpad, int S, const void *fhat, void *part,
                             const void *W, int64_t wbase, int row0, int row1, hipStream_t s) {
    if (ncells < 1 || ncells > kSmallMaxCells || cellpad < ncells || row1 <= row0) return hipErrorInvalidValue;
    const int N = op->N;
    const int CB = small_cells_per_block(N, ncells);
    const int nblk = (int)((ncells + CB - 1) / CB);
    const bool f64 = op->wdtype == BZ_F64;
    switch (N) {
#define BZ_SMALL_CASE(NN)                                                                                     \
    case NN:                                                                                                  \
        return f64 ? launch_n<double, NN>(CB, fhat, part, W, op->d_rowoff, wbase, row0, row1 - row0, S, nblk, \
                                          ncells, cellpad, s)                                                 \
                   : launch_n<float, NN>(CB, fhat, part, W, op->d_rowoff, wbase, row0, row1 - row0, S, nblk,  \
                                         ncells, cellpad, s);
        BZ_SMALL_CASE(8)
        BZ_SMALL_CASE(16)
        BZ_SMALL_CASE(24)
        BZ_SMALL_CASE(32)
        BZ_SMALL_CASE(48)
#undef BZ_SMALL_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace bz
