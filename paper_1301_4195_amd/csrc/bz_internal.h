// Internal declarations of the gfx950 collision-operator library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/bz.h"

namespace bz {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kWave = 64;  // CDNA wavefront width: one lane per cell in the convolution
constexpr int kXcds = 8;   // XCDs of the chip: workgroup b of a launch runs on XCD b mod 8

// Meshes the kernels are compiled for, and the k3 range counts each allows
// (at N = 48 only four ranges keep the convolution's registers in bounds).
constexpr bool mesh_ok(int N) { return N == 8 || N == 16 || N == 24 || N == 32 || N == 48; }
constexpr bool ranges_ok(int N, int KH) { return N == 48 ? KH == 4 : (KH == 1 || KH == 2 || KH == 4); }

// Valid m-range of one coordinate for output index k: the truncated sum keeps
// m with 0 <= k - m + N/2 <= N-1 (and 0 <= m <= N-1).
__host__ __device__ constexpr int mlo(int N, int k) { return k - N / 2 + 1 > 0 ? k - N / 2 + 1 : 0; }
__host__ __device__ constexpr int mhi(int N, int k) { return k + N / 2 < N - 1 ? k + N / 2 : N - 1; }
__host__ __device__ constexpr int mcount(int N, int k) { return mhi(N, k) - mlo(N, k) + 1; }
// The same set seen from m: outputs k with 0 <= k - m + N/2 <= N-1.
__host__ __device__ constexpr int klo(int N, int m) { return m - N / 2 > 0 ? m - N / 2 : 0; }
__host__ __device__ constexpr int khi(int N, int m) { return m + N / 2 - 1 < N - 1 ? m + N / 2 - 1 : N - 1; }
__host__ __device__ constexpr int kcount(int N, int m) { return khi(N, m) - klo(N, m) + 1; }
// pairs (k3, m3) of one 1-D line: 3N^2/4.  Weights of a line are stored
// m3-major (k3 ascending inside), so that consecutive multiply-adds of the
// convolution update different outputs and do not wait on each other.
__host__ __device__ constexpr int line_pairs(int N) { return 3 * N * N / 4; }

// Mirror symmetry of the truncated sum.  For an output k the pairs (m, n) with
// n = k - m + N/2 come in mirrored couples (m, n) and (n, m) carrying the same
// product f^_m f^_n, so the sum is taken once per couple with the weight
// W[k][m] + W[k][n].  In a row (k1, k2) the line (m1, m2) = (lo1 + a1,
// lo2 + a2) mirrors to (a1, a2) -> (c1 - 1 - a1, c2 - 1 - a2); the kept half
// is a1 < c1/2 with every a2, plus, when c1 is odd, the middle a1 = (c1-1)/2
// with a2 <= (c2-1)/2.  If c2 is also odd the last of these is its own mirror
// (u = v) and keeps the plain weights.
__host__ __device__ constexpr int half_a1_end(int c1) { return (c1 + 1) / 2; }  // a1 in [0, this)
__host__ __device__ constexpr int half_a2_end(int c1, int c2, int a1) {
    return ((c1 & 1) && a1 == c1 / 2) ? (c2 + 1) / 2 : c2;
}
__host__ __device__ constexpr int half_lines(int c1, int c2) { return (c1 / 2) * c2 + ((c1 & 1) ? (c2 + 1) / 2 : 0); }
__host__ __device__ constexpr bool self_mirror(int c1, int c2, int a1, int a2) {
    return (c1 & 1) && (c2 & 1) && a1 == c1 / 2 && a2 == c2 / 2;
}

// Scale factors of the transform pair (Sec. 2.2 with the meshes of Sec. 3.1).
struct Geometry {
    int N;
    double L, dv, dz;
    double fwd_scale;  // (2 pi)^{-3/2} dv^3
    double inv_scale;  // (2 pi)^{-3/2} dzeta^3
};

// One launch of the convolution processes items (row, m1-chunk, cell group,
// k3 range).
struct ConvItem {
    int row;    // k1 * N + k2
    int chunk;  // m1 chunk index in [0, S)
    int group;  // cell group (64 cells); row < 0 marks an empty item
    int half;   // which of the KH equal k3 ranges of the row (0 when KH = 1)
    int op;     // which op of a mixed launch (0 otherwise)
};

// A mixed-N batch runs its convolution as one launch over the items of all
// its ops (at most kMaxMix), each op's rows split into a fixed number of k3
// ranges, chosen so that no variant needs more registers than three
// wavefronts per SIMD allow (the launch's register count is the largest of
// the variants it contains).
constexpr int kMaxMix = 8;
__host__ __device__ constexpr int mix_ranges(int N, bool f64) { return N <= 16 ? 1 : (f64 ? 4 : 2); }

// one op's share of a mixed launch
struct MixPart {
    int N;
    int64_t cellpad;
    int S, KH;
};

// what the mixed kernel reads of each op (an array in device memory, so
// that the kernel's per-item lookup is a scalar load)
struct MixDesc {
    const void *fhat;
    void *part;
    const void *W;
    const int64_t *rowoff;
    int64_t cellpad;
    int S, N;
};

}  // namespace bz

struct bz_op {
    int device = 0;
    int N = 0;
    double L = 0, lambda = 0;
    double beta = 1.0;  // (1 + e)/2 for restitution coefficient e; 1 = elastic
    int wdtype = BZ_F64;
    bz::Geometry geo{};
    // weights, packed per row (k1,k2): for each kept line (m1, m2) of the
    // mirror-halved set (see half_lines) the 3N^2/4 (k3, m3) pairs of the line
    // in the order m3-major, k3 ascending; each value is the couple's summed
    // weight W[k][m] + W[k][k - m + N/2] (plain W on a self-mirrored line)
    // (an op whose weights are computed on the fly holds one slab of this
    // layout here instead, see the fly_* fields)
    void *W = nullptr;
    int64_t w_count = 0;
    int64_t *d_rowoff = nullptr;  // [N*N] first packed index of each row
    std::vector<int64_t> h_rowoff;
    // FFT twiddles cos/sin(2 pi t / N), t = 0..N-1, in both precisions
    // The convolution runs one launch per row range [slab_rows[j],
    // slab_rows[j+1]) (for a stored table: windows of consecutive rows, a
    // single one below 512 MiB of weights).  Weights computed on the fly:
    // small tables (fly.hip) in d_fly / d_fly_pos, range j's weights
    // recomputed into W before its launch; W then holds the longest range
    // (w_slab entries).
    bool fly = false;
    bool fly_has_omega = false;
    double *d_fly = nullptr;
    int *d_fly_pos = nullptr;
    std::vector<int> slab_rows;
    int64_t w_slab = 0;
    // with two or more slabs: a second slab buffer and stream, so that slab
    // j + 1's weights are computed while slab j is convolved
    void *W2 = nullptr;
    hipStream_t slab_side = nullptr;
    hipEvent_t ev_slab_fork = nullptr, ev_slab_join = nullptr;
    double *d_tw64 = nullptr;
    float *d_tw32 = nullptr;
    // conservation: (C C^T)^{-1}, 5x5 row-major, FP64
    double cct_inv[25] = {0};
    // workspace
    int64_t cap_cells = 0;       // cells the workspace holds (multiple of 64)
    int S = 1;                   // m1 chunks (partial sums) for cap_cells
    void *d_fhat = nullptr;      // [N^3][cellpad] complex
    void *d_part = nullptr;      // [S][N^3][cellpad] complex
    bz::ConvItem *d_items = nullptr;  // slab j's items at [slab_items[j], slab_items[j+1])
    int64_t n_items = 0;
    std::vector<int64_t> slab_items;
    // item list of a mixed launch led by this op (the first op of a ragged
    // call), for the key (N, padded cells, chunks) of each op in order
    std::vector<int64_t> mix_key;
    bz::ConvItem *d_mix_items = nullptr;
    int64_t n_mix_items = 0, mix_cap = 0;
    std::vector<bz::MixDesc> h_mix_desc;
    bz::MixDesc *d_mix_desc = nullptr;
    // bz_autotune_ragged's choice for the layout mix_key had when it ran:
    // 1 = one launch, 0 = per-op launches on forked streams
    std::vector<int64_t> rag_mode_key;
    int rag_mode = 1;
    int64_t sched_cells = -1;    // cellpad the item list was built for
    int sched_S = 0;
    int sched_KH = 1;            // k3 ranges per row in the item list (0: small-batch form)
    int64_t sched_n = 0;         // cells of the small-batch form's schedule
    // (cellpad, (chunks, k3 ranges)) chosen by bz_autotune
    std::vector<std::pair<int64_t, std::pair<int, int>>> tuned;
    double *d_tr_work = nullptr; // transport stage buffers
    int64_t tr_cells = 0;
    // ragged batches: this op's cells in the packed buffers
    std::vector<int64_t> h_rag_off;
    std::vector<int32_t> h_rag_idx;
    int64_t *d_rag_off = nullptr;
    int32_t *d_rag_idx = nullptr;
    int64_t rag_cap = 0;
    hipStream_t side = nullptr;  // stream of this op's share of a ragged batch
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    double *d_step_work = nullptr; // Strang step: Q~ / second stage, first stage, f*  (3 x cells x N^3)
    int64_t step_cells = 0;
    int64_t bytes_held = 0;
    // measurement hooks (bz_timing_*): a pool of event pairs around the convolution
    bool timing = false;
    std::vector<hipEvent_t> ev_start, ev_stop;
    size_t ev_used = 0;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
};

namespace bz {

// Work split of the convolution: S chunks of each row's m1 range, KH equal
// ranges of each row's k3 outputs.  KH = 0 selects the small-batch form
// (conv_small.hip; at most kSmallMaxCells cells), whose items are (row, m1
// chunk, block of cells).
struct Split {
    int S, KH;
};
constexpr int kSmallMaxCells = 64;  // the small-batch form takes at most one cell group

// schedule.hip
int max_chunks(int N);                                    // shortest kept m1 range of any row
// tuned choice for this batch size (by its cellpad), else the default
Split choose_split(const bz_op *op, int64_t cellpad, int64_t ncells);
int range_pairs(int N, int KH, int h);                    // (k3, m3) pairs of a line in k3 range h
// items of the output rows [row0, row1)
std::vector<ConvItem> make_items(int N, int64_t cellpad, int S, int KH, int row0, int row1);
// items of every op of a mixed launch (all rows), item.op = index into parts
std::vector<ConvItem> make_mixed_items(const std::vector<MixPart> &parts);
// row boundaries of slabs of at most max_elems packed weights each (rows in
// order, every slab at least one row); empty if one row alone is longer
std::vector<int> slab_bounds(const std::vector<int64_t> &rowoff, int64_t total, int64_t max_elems);
// windows of a stored table: slabs merged until each has >= min_rows rows
std::vector<int> window_bounds(const std::vector<int64_t> &rowoff, int64_t total, int64_t max_elems, int min_rows);
// rows a launch needs so that its items fill the chip (see kFillItems)
int fill_rows(int64_t cellpad, int S, int KH);

// api.hip helpers shared with the no-allocation entry point
int check_device(const bz_op *op);
bool pair_aligned(const void *p, int dtype);
int64_t round_cells(int64_t n);

// error plumbing
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
#define BZ_HIP(call)                                         \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return ::bz::hip_fail(e_, #call); \
    } while (0)

// weights (ghat.hip)
// d_quad: nquad mapped nodes then nquad weights of the radial quadrature
// (nquad = 0: closed forms for lambda = 0, 1)
hipError_t launch_build_weights(bz_op *op, const double *d_omega1d, const double *d_quad, int nquad,
                                hipStream_t s);
// Gauss-Jacobi nodes and weights for the weight (1 + x)^beta on [-1, 1]
bool gauss_jacobi(int n, double beta, std::vector<double> &x, std::vector<double> &w);
hipError_t launch_gather_weights(const bz_op *op, int64_t npairs, const int32_t *k, const int32_t *m,
                                 double *out, hipStream_t s);
// weights computed on the fly (fly.hip): table sizes and contents for an op,
// the slab of rows [row0, row1) into `out` (a slab buffer), and the gather of
// single weights
int64_t fly_table_doubles(int N, bool omega);
void fly_tables(int N, double L, int lam, const double *omega1d, std::vector<double> &d, std::vector<int> &pos);
hipError_t launch_fly_weights(const bz_op *op, int row0, int row1, void *out, hipStream_t s);
hipError_t launch_fly_gather(const bz_op *op, int64_t npairs, const int32_t *k, const int32_t *m, double *out,
                             hipStream_t s);

// transforms (fft.hip)
// off (nullable): element offset of each cell in f / Qt (packed ragged
// layout); null means cell c starts at c N^3.
// tmp: a buffer of at least fhat's size, free during the transform
hipError_t launch_forward(const bz_op *op, int64_t ncells, int64_t cellpad, const void *f, void *fhat, void *tmp,
                          const int64_t *off, hipStream_t s);
// work (nullable): a buffer of fhat's size for the intermediate (default: the
// op's f^ workspace, dead once the convolution has run)
hipError_t launch_inverse(const bz_op *op, int64_t ncells, int64_t cellpad, int S, void *part, void *Qt,
                          const int64_t *off, hipStream_t s, void *work = nullptr);

// whole-cell transforms (one workgroup per cell, N <= 16): cell c of f
// ([cell][N^3]) to f^ at fhat[q * cellpad + c], and the S partial sums (part +
// s N^3 cellpad) back to Qt[c][N^3]; cellpad = 1 for a single cell, else a
// multiple of 8 x the cells of one cache line
bool cell_transforms_ok(const bz_op *op, int64_t cellpad);
hipError_t launch_forward_cells(const bz_op *op, int64_t ncells, int64_t cellpad, const void *f, void *fhat,
                                hipStream_t s);
hipError_t launch_inverse_cells(const bz_op *op, int64_t ncells, int64_t cellpad, int S, const void *part,
                                void *Qt, hipStream_t s);

// small-batch convolution (conv_small.hip): cells per block (CB) and default
// chunk count for a batch size, and the launch over rows [row0, row1) of W
// (weights of row r at W + rowoff[r] - wbase)
int small_cells_per_block(int N, int64_t ncells);
int small_default_chunks(int N, int64_t ncells);
bool small_by_default(int N, int64_t ncells);  // the default form for this batch size
hipError_t launch_conv_small(const bz_op *op, int64_t ncells, int64_t cellpad, int S, const void *fhat, void *part,
                             const void *W, int64_t wbase, int row0, int row1, hipStream_t s);
// the same sum for one cell on the unpadded workspace (cell stride 1), every
// workgroup's weight loads in flight at once (N = 8, 16)
bool cell_conv_ok(int N, int S);
hipError_t launch_conv_cell(const bz_op *op, int S, const void *fhat, void *part, const void *W, int64_t wbase,
                            int row0, int row1, hipStream_t s);

// convolution (conv.hip)
// items [0, nitems) of `items`, reading the packed weights of row r at
// W + rowoff[r] - wbase
hipError_t launch_conv(const bz_op *op, int64_t cellpad, int S, int KH, const void *fhat, void *part,
                       const void *W, int64_t wbase, const ConvItem *items, int64_t nitems, hipStream_t s);
// one launch over the items of several ops (ops[item.op]), each with its own
// workspace, full weight table and split (S = ops[j]->sched_S, KH =
// mix_ranges); every op's table must be stored (not computed on the fly)
hipError_t launch_conv_mixed(bool f64, const MixDesc *d_desc, const ConvItem *items, int64_t nitems, hipStream_t s);
// pseudo-random trial values (in [-1, 1)) for `nreal` reals of buf, for timing
hipError_t launch_fill_trial(const bz_op *op, void *buf, int64_t nreal, hipStream_t s);

// conservation and updates (conserve.hip)
// off (nullable) as for the transforms; idx (nullable): row of moments for
// each cell
hipError_t launch_conserve(const bz_op *op, int64_t ncells, const void *Qt, int in_dtype, double *Qc,
                           double *moments, hipStream_t s, const int64_t *off = nullptr,
                           const int32_t *idx = nullptr);
hipError_t launch_axpy(int64_t n, double alpha, const double *x, double *y, hipStream_t s);
// z = x + a y
hipError_t launch_axpbz(int64_t n, const double *x, double a, const double *y, double *z, hipStream_t s);
// f += a (y1 + y2)
hipError_t launch_heun_finish(int64_t n, double a, const double *y1, const double *y2, double *f, hipStream_t s);

// transport (transport.hip)
hipError_t launch_transport_step(bz_op *op, int64_t ncells, double *f, const double *x_faces, double dt,
                                 const bz_wall &left, const bz_wall &right, hipStream_t s);

}  // namespace bz
