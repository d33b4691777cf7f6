// C ABI of the collision-operator library: argument checking, op lifetime,
// workspace management and the launch sequence of each entry point.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bz_internal.h"

struct bz_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace bz {

namespace {
thread_local std::string g_err = "no error";
int64_t g_mem_cap = 0;  // 0 = unlimited
// default slab of weights computed on the fly: the size of the chip's
// last-level (Infinity) cache, so a slab just written is read back from it,
// or 1/16 of the table where that is larger (at N = 48 256 MiB slabs hold
// ~28 output rows, too few for one launch to fill the chip: FP64, 128 cells,
// 439 cell-evals/s at 256 MiB against 878 at 1 GiB and 1041 stored)
constexpr int64_t kDefaultSlabBytes = (int64_t)256 << 20;
constexpr int kDefaultSlabFraction = 16;
// A stored table above this size is convolved in launches over consecutive
// row ranges of at most this many bytes of weights: all XCDs then stream the
// same rows at the same time and share them in the last-level cache, instead
// of each XCD reading the whole table for its own cell groups (measured at
// N = 32: 10 % faster in FP64; one range for N <= 24).  A window also keeps
// enough rows for its launch to fill the chip at the batch's size
// (fill_rows), so small batches get fewer, larger windows.
constexpr int64_t kStoredWindowBytes = (int64_t)512 << 20;

hipError_t dmalloc(void **p, size_t bytes) { return hipMalloc(p, bytes); }
}  // namespace

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? BZ_ENOMEM : BZ_EHIP;
}

int check_device(const bz_op *op) {
    int dev = -1;
    BZ_HIP(hipGetDevice(&dev));
    if (dev != op->device) return fail(BZ_EINVAL, "op was created on another device than the current one");
    return BZ_OK;
}

// cell counts are padded to whole wavefronts of cells in the workspace
int64_t round_cells(int64_t n) { return (n + kWave - 1) / kWave * kWave; }

// The transforms move the caller's reals two at a time.
bool pair_aligned(const void *p, int dtype) {
    return ((uintptr_t)p % (2 * (dtype == BZ_F64 ? sizeof(double) : sizeof(float)))) == 0;
}

namespace {

size_t elem_bytes(int dtype) { return dtype == BZ_F64 ? sizeof(double) : sizeof(float); }

// (C C^T)^{-1} by Gauss-Jordan with partial pivoting; C rows dv^3 (1, v, |v|^2).
// nrows = 5: mass, momentum and energy; nrows = 4: mass and momentum only
// (the inverse of the leading 4 x 4 block, zero in row and column 4, so the
// projection leaves the energy moment alone).
void cct_inverse(int N, double dv, int nrows, double out[25]) {
    const int c = N / 2;
    double S0 = 0, S2 = 0, S4 = 0, S1 = 0, S3 = 0;  // 1-D moment sums of the mesh
    for (int j = 0; j < N; ++j) {
        const double v = dv * (j - c);
        S0 += 1.0;
        S1 += v;
        S2 += v * v;
        S3 += v * v * v;
        S4 += v * v * v * v;
    }
    // 3-D sums over the product mesh
    double A[5][10] = {};
    const double w2 = std::pow(dv, 6);
    // rows: phi_0 = 1, phi_i = v_i, phi_4 = |v|^2
    // sum 1 = S0^3; sum v_i = S1 S0^2; sum v_i v_j = S2 S0^2 (i=j) or S1^2 S0 (i!=j);
    // sum v_i |v|^2 = S3 S0^2 + 2 S1 S2 S0; sum |v|^2 = 3 S2 S0^2;
    // sum |v|^4 = 3 S4 S0^2 + 6 S2^2 S0
    A[0][0] = S0 * S0 * S0;
    for (int i = 1; i <= 3; ++i) A[0][i] = A[i][0] = S1 * S0 * S0;
    A[0][4] = A[4][0] = 3 * S2 * S0 * S0;
    for (int i = 1; i <= 3; ++i)
        for (int j = 1; j <= 3; ++j) A[i][j] = (i == j) ? S2 * S0 * S0 : S1 * S1 * S0;
    for (int i = 1; i <= 3; ++i) A[i][4] = A[4][i] = S3 * S0 * S0 + 2 * S1 * S2 * S0;
    A[4][4] = 3 * S4 * S0 * S0 + 6 * S2 * S2 * S0;
    const int n = nrows;
    for (int i = 0; i < 5; ++i) {
        for (int j = 0; j < 5; ++j) A[i][j] *= w2;
        for (int j = 0; j < 5; ++j) A[i][5 + j] = (i == j) ? 1.0 : 0.0;
    }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
        if (piv != col)
            for (int j = 0; j < 10; ++j) std::swap(A[piv][j], A[col][j]);
        const double d = A[col][col];
        for (int j = 0; j < 10; ++j) A[col][j] /= d;
        for (int r = 0; r < n; ++r)
            if (r != col) {
                const double m = A[r][col];
                for (int j = 0; j < 10; ++j) A[r][j] -= m * A[col][j];
            }
    }
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) out[i * 5 + j] = (i < n && j < n) ? A[i][5 + j] : 0.0;
}


void free_workspace(bz_op *op) {
    if (op->d_fhat) (void)hipFree(op->d_fhat);
    if (op->d_part) (void)hipFree(op->d_part);
    if (op->d_items) (void)hipFree(op->d_items);
    op->d_fhat = op->d_part = nullptr;
    op->d_items = nullptr;
    op->cap_cells = 0;
    op->n_items = 0;
    op->slab_items.clear();
    op->sched_cells = -1;
}

// device bytes of the op's weights (the table, or the slab buffer and the
// on-the-fly tables) and of its other create-time tables
int64_t table_bytes(const bz_op *op) {
    const int64_t w = op->fly ? op->w_slab * (op->slab_rows.size() > 2 ? 2 : 1) * (int64_t)elem_bytes(op->wdtype) +
                                    fly_table_doubles(op->N, op->fly_has_omega) * (int64_t)sizeof(double) +
                                    (int64_t)line_pairs(op->N) * (int64_t)sizeof(int)
                              : op->w_count * (int64_t)elem_bytes(op->wdtype);
    return w + (int64_t)op->N * op->N * (int64_t)sizeof(int64_t) +
           (int64_t)op->N * 2 * (int64_t)(sizeof(double) + sizeof(float));
}

// force.S > 0 overrides the work split (autotuning trials).
int ensure_workspace(bz_op *op, int64_t ncells, Split force = {0, 0}) {
    const int64_t cellpad = round_cells(std::max<int64_t>(ncells, 1));
    const Split sp = force.S > 0 ? force : choose_split(op, cellpad, ncells);
    const int S = sp.S;
    const bool small = sp.KH == 0;
    const int64_t n3 = (int64_t)op->N * op->N * op->N;
    const size_t cb = 2 * elem_bytes(op->wdtype);
    if (cellpad > op->cap_cells || S > op->S) {
        const int64_t newcap = std::max(cellpad, op->cap_cells);
        const int newS = std::max(S, op->S);
        // the partial sums also hold the forward transform's intermediate,
        // which is FP64 for both paths: two FP32 chunks' worth at least
        const int pchunks = std::max(newS, op->wdtype == BZ_F32 ? 2 : 1);
        const int64_t need = n3 * newcap * (int64_t)cb * (1 + pchunks);
        const int64_t trb = op->tr_cells ? (2 * (op->tr_cells + 4) * n3 + 2) * (int64_t)sizeof(double) : 0;
        if (g_mem_cap > 0 && table_bytes(op) + need + trb > g_mem_cap)
            return fail(BZ_ENOMEM, "workspace would exceed the memory cap set by bz_set_memory_cap");
        BZ_HIP(hipDeviceSynchronize());  // earlier launches may still read the old workspace
        free_workspace(op);
        void *a = nullptr, *b = nullptr;
        hipError_t e = dmalloc(&a, n3 * newcap * cb);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace f^)");
        e = dmalloc(&b, n3 * newcap * cb * pchunks);
        if (e != hipSuccess) {
            (void)hipFree(a);
            return hip_fail(e, "hipMalloc(workspace partial sums)");
        }
        op->d_fhat = a;
        op->d_part = b;
        op->cap_cells = newcap;
        op->S = newS;
    }
    if (small) {
        // no item list: the launch derives its items from the grid.  A
        // stored table is one launch (a plain stream of weights); the slabs
        // of an on-the-fly op stay as they are.
        if (!op->fly) op->slab_rows = {0, op->N * op->N};
        op->slab_items.assign(op->slab_rows.size(), 0);
        op->sched_cells = cellpad;
        op->sched_S = S;
        op->sched_KH = 0;
        op->sched_n = ncells;
        return BZ_OK;
    }
    if (op->sched_cells != cellpad || op->sched_S != S || op->sched_KH != sp.KH) {
        BZ_HIP(hipDeviceSynchronize());  // earlier launches may still read the old item list
        // stored table: windows of at most kStoredWindowBytes of weights, each
        // with enough rows to fill the chip at this batch size
        if (!op->fly)
            op->slab_rows = window_bounds(op->h_rowoff, op->w_count,
                                          kStoredWindowBytes / (int64_t)elem_bytes(op->wdtype),
                                          fill_rows(cellpad, S, sp.KH));
        // one list per slab or window of rows
        std::vector<ConvItem> items;
        std::vector<int64_t> starts{0};
        for (size_t j = 0; j + 1 < op->slab_rows.size(); ++j) {
            const std::vector<ConvItem> sl = make_items(op->N, cellpad, S, sp.KH, op->slab_rows[j], op->slab_rows[j + 1]);
            items.insert(items.end(), sl.begin(), sl.end());
            starts.push_back((int64_t)items.size());
        }
        if ((int64_t)items.size() > op->n_items || !op->d_items) {
            if (op->d_items) (void)hipFree(op->d_items);
            op->d_items = nullptr;
            void *p = nullptr;
            // sized for the largest item list this op can need at this capacity
            const int64_t maxn = ((int64_t)op->N * op->N * (op->N / 2 + 1) * 2 * (op->cap_cells / kWave) +
                                  kXcds * (int64_t)op->slab_rows.size()) * 2;
            hipError_t e = dmalloc(&p, sizeof(ConvItem) * std::max<int64_t>(maxn, items.size()));
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(item list)");
            op->d_items = (ConvItem *)p;
        }
        BZ_HIP(hipMemcpy(op->d_items, items.data(), sizeof(ConvItem) * items.size(), hipMemcpyHostToDevice));
        op->n_items = (int64_t)items.size();
        op->slab_items = starts;
        op->sched_cells = cellpad;
        op->sched_S = S;
        op->sched_KH = sp.KH;
    }
    return BZ_OK;
}

// Wait for the recorded event pairs and fold their durations into the totals.
int drain_timing(bz_op *op) {
    for (size_t i = 0; i < op->ev_used; ++i) {
        BZ_HIP(hipEventSynchronize(op->ev_stop[i]));
        float ms = 0.0f;
        BZ_HIP(hipEventElapsedTime(&ms, op->ev_start[i], op->ev_stop[i]));
        op->timed_ms += ms;
        ++op->timed_launches;
    }
    op->ev_used = 0;
    return BZ_OK;
}

int check_walls(const bz_wall *left, const bz_wall *right) {
    for (const bz_wall *w : {left, right}) {
        if (w->kind != BZ_WALL_DIFFUSE && w->kind != BZ_WALL_EXTRAPOLATE && w->kind != BZ_WALL_NOFLUX)
            return fail(BZ_EINVAL, "unknown wall kind");
        if (w->kind == BZ_WALL_DIFFUSE && (!(w->Tw > 0.0) || !std::isfinite(w->Tw)))
            return fail(BZ_EINVAL, "diffuse wall needs a finite Tw > 0");
        if (w->kind == BZ_WALL_DIFFUSE && w->Vw[0] != 0.0)
            return fail(BZ_EINVAL, "a wall moves tangentially only: Vw[0] must be 0");
        for (int i = 0; i < 3; ++i)
            if (!std::isfinite(w->Vw[i])) return fail(BZ_EINVAL, "wall velocity must be finite");
    }
    return BZ_OK;
}

// Grow a device buffer of `count` doubles held in (*buf, *have); waits for the
// device before freeing an old buffer that queued work may still use.
int grow_buffer(bz_op *op, double **buf, int64_t *have, int64_t cells, int64_t count, const char *what) {
    if (*buf && cells <= *have) return BZ_OK;
    const int64_t need = count * (int64_t)sizeof(double);
    if (g_mem_cap > 0 && table_bytes(op) + need > g_mem_cap)
        return fail(BZ_ENOMEM, std::string(what) + " would exceed the memory cap");
    if (*buf) {
        BZ_HIP(hipDeviceSynchronize());
        (void)hipFree(*buf);
    }
    *buf = nullptr;
    *have = 0;
    hipError_t e = hipMalloc((void **)buf, need);
    if (e != hipSuccess) return hip_fail(e, what);
    *have = cells;
    return BZ_OK;
}

int ensure_transport(bz_op *op, int64_t ncells) {
    const int64_t n3 = (int64_t)op->N * op->N * op->N;
    return grow_buffer(op, &op->d_tr_work, &op->tr_cells, ncells, 2 * (ncells + 4) * n3 + 2,
                       "hipMalloc(transport workspace)");
}

// The convolution of the prepared workspace: one launch per row range of
// the op (see bz_op::slab_rows) over that range's items; for an op without a
// stored table each launch is preceded by the recomputation of the range's
// weights into the slab buffer.
hipError_t enqueue_conv(bz_op *op, int64_t cellpad, int S, int KH, hipStream_t s) {
    const size_t n = op->slab_rows.size() - 1;
    // two slab buffers on two streams: even slabs in W on s, odd slabs in W2
    // on slab_side, so one slab's weights are computed while the other slab
    // is convolved (a buffer is rewritten only after its stream's previous
    // convolution; the launches write disjoint rows of the partial sums)
    const bool two = op->fly && n >= 2 && op->W2;
    hipError_t e = hipSuccess;
    if (two) {
        if ((e = hipEventRecord(op->ev_slab_fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(op->slab_side, op->ev_slab_fork, 0)) != hipSuccess) return e;
    }
    for (size_t j = 0; j < n; ++j) {
        const int r0 = op->slab_rows[j], r1 = op->slab_rows[j + 1];
        const bool odd = two && (j & 1);
        void *buf = odd ? op->W2 : op->W;
        hipStream_t st = odd ? op->slab_side : s;
        if (op->fly && (e = launch_fly_weights(op, r0, r1, buf, st)) != hipSuccess) return e;
        const int64_t wbase = op->fly ? op->h_rowoff[r0] : 0;
        if (KH == 0 && cellpad == 1 && cell_conv_ok(op->N, S))  // one cell, unpadded workspace
            e = launch_conv_cell(op, S, op->d_fhat, op->d_part, buf, wbase, r0, r1, st);
        else if (KH == 0)
            e = launch_conv_small(op, op->sched_n, cellpad, S, op->d_fhat, op->d_part, buf, wbase, r0, r1, st);
        else
            e = launch_conv(op, cellpad, S, KH, op->d_fhat, op->d_part, buf, wbase, op->d_items + op->slab_items[j],
                            op->slab_items[j + 1] - op->slab_items[j], st);
        if (e != hipSuccess) return e;
    }
    if (two) {
        if ((e = hipEventRecord(op->ev_slab_join, op->slab_side)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, op->ev_slab_join, 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// forward FFT, convolution, inverse FFT; the workspace must be prepared
int enqueue_collision(bz_op *op, int64_t ncells, const void *f, void *Qt, hipStream_t s,
                      const int64_t *off = nullptr) {
    // one cell with the small-batch convolution (the plain per-cell path) at
    // N <= 16: whole-cell transforms and the workspace unpadded (cell stride
    // 1); batches at N = 8: whole-cell transforms on the padded workspace
    // (collision_eval, 1024 cells: FP32 45.4 -> 41.4 us, FP64 61.7 -> 53.6
    // us).  N = 16 batches keep the plane and middle passes (256 cells, five
    // chunks: FP64 277 us against 289 us, FP32 175 us against 182 us; the
    // whole-cell inverse reads each cell's partial sums 16 bytes per cache
    // line)
    // From N = 32 one cell takes the passes on the unpadded workspace too
    // (each pass thread owns one line; the plane passes of N <= 24 need a
    // block of cells): the convolution then reads each line of f^ as
    // contiguous values instead of one 16-byte value per 64-cell row.
    const bool one_cell = ncells == 1 && !off && op->sched_KH == 0;
    const bool one = one_cell && cell_transforms_ok(op, 1);
    const int64_t cellpad = one || (one_cell && op->N >= 32) ? 1 : round_cells(ncells);
    const bool batch_cells = op->N == 8;
    const bool cells = one || (batch_cells && !off && cell_transforms_ok(op, cellpad));
    // FP32 batches at N = 16 take the whole-cell forward transform with the
    // passes' inverse (its FP64 intermediates stay in LDS instead of a
    // round trip through the workspace: 256 cells 173.5 -> 170 us, 1024
    // cells 555 -> 549 us; FP64 at 256 cells no faster)
    const bool fwd_cells =
        cells || (op->N == 16 && op->wdtype == BZ_F32 && !off && cell_transforms_ok(op, cellpad));
    const int S = op->sched_S;
    if (fwd_cells)
        BZ_HIP(launch_forward_cells(op, ncells, cellpad, f, op->d_fhat, s));
    else
        BZ_HIP(launch_forward(op, ncells, cellpad, f, op->d_fhat, op->d_part, off, s));
    if (op->timing) {
        if (op->ev_used == op->ev_start.size()) {
            int rc = drain_timing(op);
            if (rc) return rc;
        }
        BZ_HIP(hipEventRecord(op->ev_start[op->ev_used], s));
    }
    BZ_HIP(enqueue_conv(op, cellpad, S, op->sched_KH, s));
    if (op->timing) BZ_HIP(hipEventRecord(op->ev_stop[op->ev_used++], s));
    if (cells)
        BZ_HIP(launch_inverse_cells(op, ncells, cellpad, S, op->d_part, Qt, s));
    else
        BZ_HIP(launch_inverse(op, ncells, cellpad, S, op->d_part, Qt, off, s));
    return BZ_OK;
}


int check_step_args(bz_op *op, int64_t ncells, double *f, const double *x_faces, double dt, double eps,
                    const bz_wall *left, const bz_wall *right) {
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    if (op->wdtype != BZ_F64) return fail(BZ_EINVAL, "the time step needs an FP64 op");
    if (ncells < 1 || ncells > ((int64_t)1 << 26)) return fail(BZ_EINVAL, "ncells out of range");
    if (!f || !x_faces || !left || !right) return fail(BZ_EINVAL, "null argument");
    if (!pair_aligned(f, BZ_F64)) return fail(BZ_EINVAL, "f must be aligned to 16 bytes");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(BZ_EINVAL, "dt must be finite and > 0");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(BZ_EINVAL, "eps must be finite and > 0");
    int rc = check_walls(left, right);
    if (rc) return rc;
    return check_device(op);
}

// every allocation and schedule change a step needs, done before enqueueing
int prepare_step(bz_op *op, int64_t ncells) {
    const int64_t n3 = (int64_t)op->N * op->N * op->N;
    int rc = ensure_workspace(op, ncells);
    if (rc) return rc;
    rc = ensure_transport(op, ncells);
    if (rc) return rc;
    return grow_buffer(op, &op->d_step_work, &op->step_cells, ncells, 3 * ncells * n3, "hipMalloc(step workspace)");
}

// transport dt/2, collision dt (Heun on P_N Q~), transport dt/2; launches only
int enqueue_strang(bz_op *op, int64_t M, double *f, const double *xf, double dt, double eps, const bz_wall &left,
                   const bz_wall &right, hipStream_t s) {
    const int64_t n3 = (int64_t)op->N * op->N * op->N, n = M * n3;
    double *fi = f + 2 * n3;  // interior cells
    double *q2 = op->d_step_work, *q1 = q2 + n, *fs = q1 + n;
    BZ_HIP(launch_transport_step(op, M, f, xf, 0.5 * dt, left, right, s));
    int rc = enqueue_collision(op, M, fi, q1, s);
    if (rc) return rc;
    BZ_HIP(launch_conserve(op, M, q1, BZ_F64, q1, nullptr, s));
    BZ_HIP(launch_axpbz(n, fi, dt / eps, q1, fs, s));
    rc = enqueue_collision(op, M, fs, q2, s);
    if (rc) return rc;
    BZ_HIP(launch_conserve(op, M, q2, BZ_F64, q2, nullptr, s));
    BZ_HIP(launch_heun_finish(n, 0.5 * dt / eps, q1, q2, fi, s));
    BZ_HIP(launch_transport_step(op, M, f, xf, 0.5 * dt, left, right, s));
    return BZ_OK;
}

// Split a ragged batch by op: upload each op's element offsets and cell
// indices (only when they differ from the previous call), and make sure its
// workspace holds its share.  On success counts[j] is op j's cell count.
int prepare_ragged(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                   const int64_t *offset_of_cell, int dtype, std::vector<int64_t> &counts) {
    if (!ops || nops < 1 || nops > 64) return fail(BZ_EINVAL, "need 1..64 ops");
    if (ncells < 0 || ncells > ((int64_t)1 << 26)) return fail(BZ_EINVAL, "ncells out of range");
    if (ncells > 0 && (!op_of_cell || !offset_of_cell)) return fail(BZ_EINVAL, "index arrays are NULL");
    for (int j = 0; j < nops; ++j) {
        if (!ops[j]) return fail(BZ_EINVAL, "an op is NULL");
        if (dtype >= 0 && ops[j]->wdtype != dtype) return fail(BZ_EINVAL, "an op's weight dtype differs from dtype");
        for (int i = 0; i < j; ++i)
            if (ops[i] == ops[j]) return fail(BZ_EINVAL, "ops must be distinct");
        int rc = check_device(ops[j]);
        if (rc) return rc;
    }
    std::vector<std::vector<int64_t>> off(nops);
    std::vector<std::vector<int32_t>> idx(nops);
    for (int64_t c = 0; c < ncells; ++c) {
        const int j = op_of_cell[c];
        if (j < 0 || j >= nops) return fail(BZ_EINVAL, "op_of_cell out of range");
        if (offset_of_cell[c] < 0) return fail(BZ_EINVAL, "negative cell offset");
        if (offset_of_cell[c] % 2) return fail(BZ_EINVAL, "cell offsets must be even (cells start on pairs of values)");
        off[j].push_back(offset_of_cell[c]);
        idx[j].push_back((int32_t)c);
    }
    counts.assign(nops, 0);
    for (int j = 0; j < nops; ++j) {
        bz_op *op = ops[j];
        counts[j] = (int64_t)off[j].size();
        if (counts[j] == 0) continue;
        int rc = ensure_workspace(op, counts[j]);
        if (rc) return rc;
        if (off[j] != op->h_rag_off || idx[j] != op->h_rag_idx) {
            BZ_HIP(hipDeviceSynchronize());  // queued work may still read the old lists
            if (counts[j] > op->rag_cap) {
                if (op->d_rag_off) (void)hipFree(op->d_rag_off);
                if (op->d_rag_idx) (void)hipFree(op->d_rag_idx);
                op->d_rag_off = nullptr;
                op->d_rag_idx = nullptr;
                op->rag_cap = 0;
                BZ_HIP(hipMalloc((void **)&op->d_rag_off, sizeof(int64_t) * counts[j]));
                BZ_HIP(hipMalloc((void **)&op->d_rag_idx, sizeof(int32_t) * counts[j]));
                op->rag_cap = counts[j];
            }
            BZ_HIP(hipMemcpy(op->d_rag_off, off[j].data(), sizeof(int64_t) * counts[j], hipMemcpyHostToDevice));
            BZ_HIP(hipMemcpy(op->d_rag_idx, idx[j].data(), sizeof(int32_t) * counts[j], hipMemcpyHostToDevice));
            op->h_rag_off = std::move(off[j]);
            op->h_rag_idx = std::move(idx[j]);
        }
        if (!op->side) {
            BZ_HIP(hipStreamCreateWithFlags(&op->side, hipStreamNonBlocking));
            BZ_HIP(hipEventCreateWithFlags(&op->ev_fork, hipEventDisableTiming));
            BZ_HIP(hipEventCreateWithFlags(&op->ev_join, hipEventDisableTiming));
        }
    }
    return BZ_OK;
}

// Item list and op table of a mixed launch (kept by ops[0]), rebuilt when
// the ops, their batch sizes or splits, or their workspaces change.
int prepare_mixed(bz_op *const *ops, int nops, const std::vector<int64_t> &counts) {
    bz_op *lead = ops[0];
    std::vector<int64_t> key;
    std::vector<MixPart> parts;
    std::vector<MixDesc> desc;
    for (int j = 0; j < nops; ++j) {
        const bz_op *op = ops[j];
        const int64_t cellpad = counts[j] > 0 ? round_cells(counts[j]) : 0;
        const bool f64 = op->wdtype == BZ_F64;
        key.insert(key.end(), {(int64_t)(uintptr_t)op, op->N, op->wdtype, cellpad, op->sched_S});
        parts.push_back({op->N, cellpad, op->sched_S, mix_ranges(op->N, f64)});
        desc.push_back({op->d_fhat, op->d_part, op->W, op->d_rowoff, cellpad, op->sched_S, op->N});
    }
    if (key != lead->mix_key) {
        BZ_HIP(hipDeviceSynchronize());  // queued launches may still read the old list
        const std::vector<ConvItem> items = make_mixed_items(parts);
        if ((int64_t)items.size() > lead->mix_cap) {
            if (lead->d_mix_items) (void)hipFree(lead->d_mix_items);
            lead->d_mix_items = nullptr;
            lead->mix_cap = 0;
            BZ_HIP(hipMalloc((void **)&lead->d_mix_items, sizeof(ConvItem) * items.size()));
            lead->mix_cap = (int64_t)items.size();
        }
        BZ_HIP(hipMemcpy(lead->d_mix_items, items.data(), sizeof(ConvItem) * items.size(), hipMemcpyHostToDevice));
        lead->n_mix_items = (int64_t)items.size();
        lead->mix_key = key;
    }
    bool same = desc.size() == lead->h_mix_desc.size();
    for (size_t j = 0; same && j < desc.size(); ++j)
        same = std::memcmp(&desc[j], &lead->h_mix_desc[j], sizeof(MixDesc)) == 0;
    if (!same) {
        BZ_HIP(hipDeviceSynchronize());
        if (!lead->d_mix_desc) BZ_HIP(hipMalloc((void **)&lead->d_mix_desc, sizeof(MixDesc) * kMaxMix));
        BZ_HIP(hipMemcpy(lead->d_mix_desc, desc.data(), sizeof(MixDesc) * desc.size(), hipMemcpyHostToDevice));
        lead->h_mix_desc = desc;
    }
    return BZ_OK;
}

// Validate, then build an op: the stored weight table, or (slab_bytes >= 0)
// the tables for weights computed on the fly in slabs of at most slab_bytes.
int create_op(int N, double L, double lambda, double beta, int weight_dtype, const double *omega1d,
              int64_t slab_bytes, bz_op **out) {
    if (!out) return fail(BZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mesh_ok(N)) return fail(BZ_EINVAL, "N must be 8, 16, 24, 32 or 48");
    if (!(L > 0.0) || !std::isfinite(L)) return fail(BZ_EINVAL, "L must be finite and > 0");
    if (!std::isfinite(lambda)) return fail(BZ_EINVAL, "lambda must be finite");
    if (!(lambda > -3.0 && lambda <= 2.0))
        return fail(BZ_EUNSUPPORTED, "lambda must lie in (-3, 2] (the radial integral diverges at lambda <= -3)");
    if (!(beta >= 0.5 && beta <= 1.0))
        return fail(BZ_EINVAL, "beta = (1 + e)/2 must lie in [0.5, 1] (restitution coefficient e in [0, 1])");
    if (weight_dtype != BZ_F64 && weight_dtype != BZ_F32) return fail(BZ_EINVAL, "weight_dtype must be BZ_F64 or BZ_F32");
    if (omega1d)
        for (int i = 0; i < N; ++i)
            if (!std::isfinite(omega1d[i])) return fail(BZ_EINVAL, "omega1d holds a non-finite weight");

    int device = -1;
    BZ_HIP(hipGetDevice(&device));
    bz_op *op = new (std::nothrow) bz_op();
    if (!op) return fail(BZ_ENOMEM, "host allocation failed");
    op->device = device;
    op->N = N;
    op->L = L;
    op->lambda = lambda;
    op->beta = beta;
    op->wdtype = weight_dtype;
    op->geo.N = N;
    op->geo.L = L;
    op->geo.dv = 2.0 * L / N;
    op->geo.dz = kPi / L;
    op->geo.fwd_scale = std::pow(2.0 * kPi, -1.5) * std::pow(op->geo.dv, 3);
    op->geo.inv_scale = std::pow(2.0 * kPi, -1.5) * std::pow(op->geo.dz, 3);

    // packed row offsets
    op->h_rowoff.resize((size_t)N * N);
    int64_t acc = 0;
    for (int r = 0; r < N * N; ++r) {
        op->h_rowoff[r] = acc;
        acc += (int64_t)half_lines(mcount(N, r / N), mcount(N, r % N)) * line_pairs(N);
    }
    op->w_count = acc;
    const bool fly = slab_bytes >= 0;
    op->fly = fly;
    op->fly_has_omega = fly && omega1d;
    if (fly) {
        op->slab_rows = slab_bounds(op->h_rowoff, acc, slab_bytes / (int64_t)elem_bytes(weight_dtype));
        if (op->slab_rows.empty()) {
            delete op;
            return fail(BZ_EINVAL, "slab_bytes is below the weights of one output row");
        }
        for (size_t j = 0; j + 1 < op->slab_rows.size(); ++j) {
            const int r0 = op->slab_rows[j], r1 = op->slab_rows[j + 1];
            const int64_t end = r1 < N * N ? op->h_rowoff[r1] : acc;
            op->w_slab = std::max(op->w_slab, end - op->h_rowoff[r0]);
        }
    } else {  // windows follow the batch (ensure_workspace); one until the first
        op->slab_rows = {0, N * N};
    }
    if (g_mem_cap > 0 && table_bytes(op) > g_mem_cap) {
        delete op;
        return fail(BZ_ENOMEM, "weight table would exceed the memory cap set by bz_set_memory_cap");
    }

    auto cleanup = [&](int code) {
        bz_op_destroy(op);
        return code;
    };
    hipError_t e = hipMalloc(&op->W, (size_t)(fly ? op->w_slab : op->w_count) * elem_bytes(weight_dtype));
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipMalloc(weights)"));
    if (fly && op->slab_rows.size() > 2) {  // second slab buffer and its stream
        if ((e = hipMalloc(&op->W2, (size_t)op->w_slab * elem_bytes(weight_dtype))) != hipSuccess ||
            (e = hipStreamCreateWithFlags(&op->slab_side, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&op->ev_slab_fork, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&op->ev_slab_join, hipEventDisableTiming)) != hipSuccess)
            return cleanup(hip_fail(e, "second slab buffer"));
    }
    e = hipMalloc((void **)&op->d_rowoff, sizeof(int64_t) * N * N);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipMalloc(row offsets)"));
    e = hipMalloc((void **)&op->d_tw64, sizeof(double) * 2 * N);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipMalloc(twiddles)"));
    e = hipMalloc((void **)&op->d_tw32, sizeof(float) * 2 * N);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipMalloc(twiddles)"));
    std::vector<double> tw(2 * N);
    std::vector<float> tw32(2 * N);
    for (int t = 0; t < N; ++t) {
        tw[t] = std::cos(2.0 * kPi * t / N);
        tw[N + t] = std::sin(2.0 * kPi * t / N);
    }
    for (int t = 0; t < 2 * N; ++t) tw32[t] = (float)tw[t];
    if (fly) {  // small tables only; the weights are computed by every convolution
        std::vector<double> ft;
        std::vector<int> pos;
        fly_tables(N, L, (int)lambda, omega1d, ft, pos);
        if ((e = hipMalloc((void **)&op->d_fly, sizeof(double) * ft.size())) != hipSuccess ||
            (e = hipMalloc((void **)&op->d_fly_pos, sizeof(int) * pos.size())) != hipSuccess ||
            (e = hipMemcpy(op->d_fly, ft.data(), sizeof(double) * ft.size(), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(op->d_fly_pos, pos.data(), sizeof(int) * pos.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return cleanup(hip_fail(e, "on-the-fly weight tables"));
    }
    double *d_om = nullptr;
    if ((e = hipMemcpy(op->d_rowoff, op->h_rowoff.data(), sizeof(int64_t) * N * N, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(op->d_tw64, tw.data(), sizeof(double) * 2 * N, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(op->d_tw32, tw32.data(), sizeof(float) * 2 * N, hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(hip_fail(e, "hipMemcpy(tables)"));
    if (omega1d && !fly) {
        if ((e = hipMalloc((void **)&d_om, sizeof(double) * N)) != hipSuccess)
            return cleanup(hip_fail(e, "hipMalloc(omega1d)"));
        if ((e = hipMemcpy(d_om, omega1d, sizeof(double) * N, hipMemcpyHostToDevice)) != hipSuccess) {
            (void)hipFree(d_om);
            return cleanup(hip_fail(e, "hipMemcpy(omega1d)"));
        }
    }
    // exponents without a closed form, and inelastic collisions: Gauss-Jacobi
    // rule for the radial
    // integral, resolving its fastest oscillation (about 2.7 N radians over
    // [-1, 1]) with a wide margin
    double *d_q = nullptr;
    int nq = 0;
    if ((lambda != 0.0 && lambda != 1.0) || beta != 1.0) {
        nq = 3 * N + 32;
        std::vector<double> x, w;
        if (!gauss_jacobi(nq, lambda + 2.0, x, w)) {
            if (d_om) (void)hipFree(d_om);
            return cleanup(fail(BZ_EINVAL, "Gauss-Jacobi eigenvalue iteration did not converge"));
        }
        const double r0 = L, scale = std::sqrt(2.0 / kPi) * std::pow(0.5 * r0, lambda + 3.0);
        std::vector<double> q(2 * nq);
        for (int j = 0; j < nq; ++j) {
            q[j] = 0.5 * r0 * (1.0 + x[j]);
            q[nq + j] = scale * w[j];
        }
        if ((e = hipMalloc((void **)&d_q, sizeof(double) * 2 * nq)) != hipSuccess ||
            (e = hipMemcpy(d_q, q.data(), sizeof(double) * 2 * nq, hipMemcpyHostToDevice)) != hipSuccess) {
            if (d_q) (void)hipFree(d_q);
            if (d_om) (void)hipFree(d_om);
            return cleanup(hip_fail(e, "quadrature table"));
        }
    }
    e = fly ? hipSuccess : launch_build_weights(op, d_om, d_q, nq, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (d_om) (void)hipFree(d_om);
    if (d_q) (void)hipFree(d_q);
    if (e != hipSuccess) return cleanup(hip_fail(e, "weight precompute"));
    cct_inverse(N, op->geo.dv, beta == 1.0 ? 5 : 4, op->cct_inv);
    op->bytes_held = table_bytes(op);
    *out = op;
    return BZ_OK;
}

}  // namespace
}  // namespace bz

using namespace bz;

extern "C" {

const char *bz_last_error(void) { return g_err.c_str(); }

int bz_set_memory_cap(int64_t bytes) {
    if (bytes < 0) return fail(BZ_EINVAL, "memory cap must be >= 0");
    g_mem_cap = bytes;
    return BZ_OK;
}

int bz_op_create(int N, double L, double lambda, int weight_dtype, const double *omega1d, bz_op **out) {
    return create_op(N, L, lambda, 1.0, weight_dtype, omega1d, -1, out);
}

int bz_op_create_inelastic(int N, double L, double lambda, double beta, int weight_dtype, const double *omega1d,
                           bz_op **out) {
    return create_op(N, L, lambda, beta, weight_dtype, omega1d, -1, out);
}

int bz_op_create_onthefly(int N, double L, double lambda, int weight_dtype, const double *omega1d,
                          int64_t slab_bytes, bz_op **out) {
    if (!out) return fail(BZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (std::isfinite(lambda) && lambda > -3.0 && lambda <= 2.0 && lambda != 0.0 && lambda != 1.0)
        return fail(BZ_EUNSUPPORTED, "weights on the fly need a closed form: lambda 0 or 1");
    if (slab_bytes < 0) return fail(BZ_EINVAL, "slab_bytes must be >= 0");
    if (slab_bytes == 0 && mesh_ok(N) && (weight_dtype == BZ_F64 || weight_dtype == BZ_F32)) {
        int64_t total = 0;
        for (int r = 0; r < N * N; ++r)
            total += (int64_t)half_lines(mcount(N, r / N), mcount(N, r % N)) * line_pairs(N);
        slab_bytes = std::max(kDefaultSlabBytes, total * (int64_t)elem_bytes(weight_dtype) / kDefaultSlabFraction);
    }
    return create_op(N, L, lambda, 1.0, weight_dtype, omega1d, slab_bytes == 0 ? kDefaultSlabBytes : slab_bytes, out);
}

int bz_op_table_bytes(const bz_op *op, int64_t *bytes) {
    if (!op || !bytes) return fail(BZ_EINVAL, "null argument");
    *bytes = table_bytes(op);
    return BZ_OK;
}

int bz_op_destroy(bz_op *op) {
    if (!op) return BZ_OK;
    free_workspace(op);
    if (op->W) (void)hipFree(op->W);
    if (op->W2) (void)hipFree(op->W2);
    if (op->slab_side) (void)hipStreamDestroy(op->slab_side);
    if (op->ev_slab_fork) (void)hipEventDestroy(op->ev_slab_fork);
    if (op->ev_slab_join) (void)hipEventDestroy(op->ev_slab_join);
    if (op->d_fly) (void)hipFree(op->d_fly);
    if (op->d_fly_pos) (void)hipFree(op->d_fly_pos);
    if (op->d_mix_items) (void)hipFree(op->d_mix_items);
    if (op->d_mix_desc) (void)hipFree(op->d_mix_desc);
    if (op->d_rowoff) (void)hipFree(op->d_rowoff);
    if (op->d_tw64) (void)hipFree(op->d_tw64);
    if (op->d_tw32) (void)hipFree(op->d_tw32);
    if (op->d_tr_work) (void)hipFree(op->d_tr_work);
    if (op->d_step_work) (void)hipFree(op->d_step_work);
    if (op->d_rag_off) (void)hipFree(op->d_rag_off);
    if (op->d_rag_idx) (void)hipFree(op->d_rag_idx);
    if (op->side) (void)hipStreamDestroy(op->side);
    if (op->ev_fork) (void)hipEventDestroy(op->ev_fork);
    if (op->ev_join) (void)hipEventDestroy(op->ev_join);
    for (hipEvent_t e : op->ev_start) (void)hipEventDestroy(e);
    for (hipEvent_t e : op->ev_stop) (void)hipEventDestroy(e);
    delete op;
    return BZ_OK;
}

int bz_op_n(const bz_op *op) {
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    return op->N;
}

int bz_op_reserve(bz_op *op, int64_t ncells) {
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    if (ncells < 0) return fail(BZ_EINVAL, "ncells must be >= 0");
    int rc = check_device(op);
    if (rc) return rc;
    rc = ensure_workspace(op, ncells);
    if (rc) return rc;
    BZ_HIP(hipDeviceSynchronize());
    return BZ_OK;
}

int bz_get_split(const bz_op *op, int64_t ncells, int *chunks, int *ranges) {
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    if (ncells < 1) return fail(BZ_EINVAL, "ncells must be >= 1");
    const Split sp = choose_split(op, round_cells(ncells), ncells);
    if (chunks) *chunks = sp.S;
    if (ranges) *ranges = sp.KH;
    return BZ_OK;
}

int bz_set_split(bz_op *op, int64_t ncells, int chunks, int ranges) {
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    if (ncells < 1) return fail(BZ_EINVAL, "ncells must be >= 1");
    if (ncells > (int64_t)1 << 26) return fail(BZ_EINVAL, "ncells too large");
    if (chunks < 1 || chunks > max_chunks(op->N))
        return fail(BZ_EINVAL, "chunks must be in [1, " + std::to_string(max_chunks(op->N)) + "] for this N");
    if (ranges == 0 && ncells > kSmallMaxCells)
        return fail(BZ_EINVAL, "ranges = 0 (small-batch form) takes at most " + std::to_string(kSmallMaxCells) +
                                   " cells");
    if (ranges != 0 && !ranges_ok(op->N, ranges))
        return fail(BZ_EINVAL, "ranges must be 0 (small-batch form), 1, 2 or 4 (4 at N = 48)");
    int rc = check_device(op);
    if (rc) return rc;
    const int64_t cellpad = round_cells(ncells);
    op->tuned.erase(std::remove_if(op->tuned.begin(), op->tuned.end(),
                                   [&](const std::pair<int64_t, std::pair<int, int>> &t) { return t.first == cellpad; }),
                    op->tuned.end());
    op->tuned.emplace_back(cellpad, std::make_pair(chunks, ranges));
    rc = ensure_workspace(op, ncells);
    if (rc) return rc;
    BZ_HIP(hipDeviceSynchronize());
    return BZ_OK;
}

int bz_autotune(bz_op *op, int64_t ncells, int *chosen_chunks, int *chosen_ranges, double *best_ms, void *stream) {
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    if (ncells < 1) return fail(BZ_EINVAL, "ncells must be >= 1");
    if (ncells > (int64_t)1 << 26) return fail(BZ_EINVAL, "ncells too large");
    int rc = check_device(op);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int64_t cellpad = round_cells(ncells);
    // forget an earlier choice for this batch size while the trials run
    op->tuned.erase(std::remove_if(op->tuned.begin(), op->tuned.end(),
                                   [&](const std::pair<int64_t, std::pair<int, int>> &t) { return t.first == cellpad; }),
                    op->tuned.end());
    const int smax = max_chunks(op->N);
    const int64_t n3 = (int64_t)op->N * op->N * op->N;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BZ_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    Split best{0, 0};
    double best_t = 0.0;
    int sfit = smax;  // chunk counts above this do not fit the memory cap
    for (int KH : {0, 1, 2, 4}) {  // 0: the small-batch form
        if (KH == 0 ? ncells > kSmallMaxCells : !ranges_ok(op->N, KH)) continue;
        for (int S = 1; S <= std::min(sfit, 8); ++S) {
            rc = ensure_workspace(op, ncells, Split{S, KH});
            if (rc == BZ_ENOMEM && best.S > 0) {  // keep to the splits that fit
                rc = BZ_OK;
                sfit = S - 1;
                break;
            }
            if (rc) break;
            // pseudo-random finite values: the time depends on the data only
            // through the chip's power draw, which random mantissas match
            // each trial: the convolution and the inverse transform, whose
            // first pass adds the S partial sums (its output goes to the
            // partial-sum buffer, already read by then)
            he = launch_fill_trial(op, op->d_fhat, n3 * cellpad * 2, s);
            if (he == hipSuccess) he = enqueue_conv(op, cellpad, S, KH, s);
            if (he == hipSuccess) he = launch_inverse(op, ncells, cellpad, S, op->d_part, op->d_part, nullptr, s);
            double t = 1e30;
            for (int rep = 0; rep < 3 && he == hipSuccess; ++rep) {
                he = launch_fill_trial(op, op->d_fhat, n3 * cellpad * 2, s);  // the inverse overwrote it
                if (he == hipSuccess) he = hipEventRecord(e0, s);
                if (he == hipSuccess) he = enqueue_conv(op, cellpad, S, KH, s);
                if (he == hipSuccess)
                    he = launch_inverse(op, ncells, cellpad, S, op->d_part, op->d_part, nullptr, s);
                if (he == hipSuccess) he = hipEventRecord(e1, s);
                if (he == hipSuccess) he = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
                t = std::min(t, (double)ms);
                if (t > 20.0) break;  // long launches: one timing is enough
            }
            if (he != hipSuccess) {
                rc = hip_fail(he, "autotune trial");
                break;
            }
            if (best.S == 0 || t < best_t) {
                best = {S, KH};
                best_t = t;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    op->tuned.emplace_back(cellpad, std::make_pair(best.S, best.KH));
    rc = ensure_workspace(op, ncells);
    if (rc) return rc;
    if (chosen_chunks) *chosen_chunks = best.S;
    if (chosen_ranges) *chosen_ranges = best.KH;
    if (best_ms) *best_ms = best_t;
    return BZ_OK;
}

int collision_eval(bz_op *op, int64_t ncells, const void *f, void *Qt, int dtype, void *stream) {
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    if (ncells < 0) return fail(BZ_EINVAL, "ncells must be >= 0");
    if (dtype != BZ_F64 && dtype != BZ_F32) return fail(BZ_EINVAL, "dtype must be BZ_F64 or BZ_F32");
    if (dtype != op->wdtype) return fail(BZ_EINVAL, "dtype differs from the op's weight dtype");
    if (ncells == 0) return BZ_OK;
    if (!f || !Qt) return fail(BZ_EINVAL, "f or Qt is NULL");
    if (f == Qt) return fail(BZ_EINVAL, "Qt must not alias f");
    if (!pair_aligned(f, dtype) || !pair_aligned(Qt, dtype))
        return fail(BZ_EINVAL, "f and Qt must be aligned to two values (16 bytes FP64, 8 bytes FP32)");
    if (ncells > (int64_t)1 << 26) return fail(BZ_EINVAL, "ncells too large");
    int rc = check_device(op);
    if (rc) return rc;
    rc = ensure_workspace(op, ncells);
    if (rc) return rc;
    return enqueue_collision(op, ncells, f, Qt, (hipStream_t)stream);
}

int bz_timing_enable(bz_op *op, int on) {
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    int rc = check_device(op);
    if (rc) return rc;
    if (on && op->ev_start.empty()) {
        constexpr int kPool = 256;
        for (int i = 0; i < kPool; ++i) {
            hipEvent_t a, b;
            BZ_HIP(hipEventCreate(&a));
            op->ev_start.push_back(a);
            BZ_HIP(hipEventCreate(&b));
            op->ev_stop.push_back(b);
        }
    }
    if (!on) {
        rc = drain_timing(op);
        if (rc) return rc;
    }
    op->timing = on != 0;
    op->timed_ms = 0.0;
    op->timed_launches = 0;
    return BZ_OK;
}

int bz_timing_read(bz_op *op, double *conv_ms, int64_t *launches) {
    if (!op || !conv_ms || !launches) return fail(BZ_EINVAL, "null argument");
    int rc = check_device(op);
    if (rc) return rc;
    rc = drain_timing(op);
    if (rc) return rc;
    *conv_ms = op->timed_ms;
    *launches = op->timed_launches;
    op->timed_ms = 0.0;
    op->timed_launches = 0;
    return BZ_OK;
}

int conserve(const bz_op *op, int64_t ncells, const void *Qt, int in_dtype, double *Qc, double *moments_out,
             void *stream) {
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    if (ncells < 0) return fail(BZ_EINVAL, "ncells must be >= 0");
    if (in_dtype != BZ_F64 && in_dtype != BZ_F32) return fail(BZ_EINVAL, "in_dtype must be BZ_F64 or BZ_F32");
    if (ncells == 0) return BZ_OK;
    if (!Qt || !Qc) return fail(BZ_EINVAL, "Qt or Qc is NULL");
    if (in_dtype == BZ_F32 && (const void *)Qc == Qt) return fail(BZ_EINVAL, "Qc may alias Qt only for FP64 input");
    if (ncells > 0x7fffffff) return fail(BZ_EINVAL, "ncells too large");
    int rc = check_device(op);
    if (rc) return rc;
    BZ_HIP(launch_conserve(op, ncells, Qt, in_dtype, Qc, moments_out, (hipStream_t)stream));
    return BZ_OK;
}

int bz_axpy(int64_t n, double alpha, const double *x, double *y, void *stream) {
    if (n < 0) return fail(BZ_EINVAL, "n must be >= 0");
    if (n == 0) return BZ_OK;
    if (!x || !y) return fail(BZ_EINVAL, "x or y is NULL");
    if (!std::isfinite(alpha)) return fail(BZ_EINVAL, "alpha must be finite");
    BZ_HIP(launch_axpy(n, alpha, x, y, (hipStream_t)stream));
    return BZ_OK;
}

int transport_step(bz_op *op, int64_t ncells, double *f, const double *x_faces, double dt, const bz_wall *left,
                   const bz_wall *right, void *stream) {
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    if (ncells < 1) return fail(BZ_EINVAL, "ncells must be >= 1");
    if (!f || !x_faces || !left || !right) return fail(BZ_EINVAL, "null argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(BZ_EINVAL, "dt must be finite and > 0");
    int rc = check_walls(left, right);
    if (rc) return rc;
    rc = check_device(op);
    if (rc) return rc;
    rc = ensure_transport(op, ncells);
    if (rc) return rc;
    BZ_HIP(launch_transport_step(op, ncells, f, x_faces, dt, *left, *right, (hipStream_t)stream));
    return BZ_OK;
}

}  // extern "C"

namespace bz {
namespace {
// Fork: the side stream of every op with cells waits for the work queued on
// s so far (all fork events are recorded before any wait, so they mark the
// same point and the ops' work then runs concurrently).  Join: s waits for
// every side stream.
hipError_t fork_sides(bz_op *const *ops, int nops, const std::vector<int64_t> &counts, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int j = 0; j < nops && e == hipSuccess; ++j)
        if (counts[j] > 0) e = hipEventRecord(ops[j]->ev_fork, s);
    for (int j = 0; j < nops && e == hipSuccess; ++j)
        if (counts[j] > 0) e = hipStreamWaitEvent(ops[j]->side, ops[j]->ev_fork, 0);
    return e;
}
hipError_t join_sides(bz_op *const *ops, int nops, const std::vector<int64_t> &counts, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int j = 0; j < nops && e == hipSuccess; ++j)
        if (counts[j] > 0) e = hipEventRecord(ops[j]->ev_join, ops[j]->side);
    for (int j = 0; j < nops && e == hipSuccess; ++j)
        if (counts[j] > 0) e = hipStreamWaitEvent(s, ops[j]->ev_join, 0);
    return e;
}

bool ragged_fusable(bz_op *const *ops, int nops) {
    bool ok = nops <= kMaxMix;
    for (int j = 0; j < nops; ++j) ok = ok && !ops[j]->fly && ops[j]->N <= 32;
    return ok;
}

// Validate a ragged collision call, prepare the ops' workspaces and index
// lists (may allocate and synchronise), and choose the convolution form:
// form 1 = one launch for every op (needs at most kMaxMix ops with stored
// tables), 0 = per-op launches, -1 = the choice bz_autotune_ragged or
// bz_set_ragged_form made for this layout (one launch by default).
int plan_ragged(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                const int64_t *offset_of_cell, const void *f, const void *Qt, int dtype, int form,
                std::vector<int64_t> &counts, bool *fuse) {
    if (dtype != BZ_F64 && dtype != BZ_F32) return fail(BZ_EINVAL, "dtype must be BZ_F64 or BZ_F32");
    if (form < -1 || form > 1) return fail(BZ_EINVAL, "form must be -1, 0 or 1");
    if (ncells > 0 && (!f || !Qt)) return fail(BZ_EINVAL, "f or Qt is NULL");
    if (ncells > 0 && f == Qt) return fail(BZ_EINVAL, "Qt must not alias f");
    if (ncells > 0 && (!pair_aligned(f, dtype) || !pair_aligned(Qt, dtype)))
        return fail(BZ_EINVAL, "f and Qt must be aligned to two values (16 bytes FP64, 8 bytes FP32)");
    int rc = prepare_ragged(ops, nops, ncells, op_of_cell, offset_of_cell, dtype, counts);
    if (rc || ncells == 0) return rc;
    const bool can = ragged_fusable(ops, nops);
    if (form == 1 && !can)
        return fail(BZ_EINVAL, "one launch needs at most 8 ops, all with stored tables and N <= 32");
    bool fu = can && form != 0;
    if (fu) {
        rc = prepare_mixed(ops, nops, counts);
        if (rc) return rc;
        if (form == -1) fu = ops[0]->rag_mode == 1 || ops[0]->rag_mode_key != ops[0]->mix_key;
    }
    *fuse = fu;
    return BZ_OK;
}

// The ragged collision evaluation on stream s (plan_ragged first).
int enqueue_ragged(bz_op *const *ops, int nops, const std::vector<int64_t> &counts, const void *f, void *Qt,
                   int dtype, bool fuse, hipStream_t s) {
    if (fuse) {
        // transforms per op, then the convolution of every op in one launch
        // forward transforms concurrently on the ops' streams
        BZ_HIP(fork_sides(ops, nops, counts, s));
        for (int j = 0; j < nops; ++j)
            if (counts[j] > 0)
                BZ_HIP(launch_forward(ops[j], counts[j], round_cells(counts[j]), f, ops[j]->d_fhat, ops[j]->d_part,
                                      ops[j]->d_rag_off, ops[j]->side));
        BZ_HIP(join_sides(ops, nops, counts, s));
        BZ_HIP(launch_conv_mixed(dtype == BZ_F64, ops[0]->d_mix_desc, ops[0]->d_mix_items, ops[0]->n_mix_items, s));
        // inverse transforms likewise
        BZ_HIP(fork_sides(ops, nops, counts, s));
        for (int j = 0; j < nops; ++j)
            if (counts[j] > 0)
                BZ_HIP(launch_inverse(ops[j], counts[j], round_cells(counts[j]), ops[j]->sched_S, ops[j]->d_part, Qt,
                                      ops[j]->d_rag_off, ops[j]->side));
        BZ_HIP(join_sides(ops, nops, counts, s));
        return BZ_OK;
    }
    // more than kMaxMix ops, an op with weights on the fly (one slab buffer
    // each), or per-op launches chosen for this layout: fork one stream per
    // op from s, run the ops' shares concurrently, join back
    BZ_HIP(fork_sides(ops, nops, counts, s));
    for (int j = 0; j < nops; ++j) {
        if (counts[j] == 0) continue;
        const int rc = enqueue_collision(ops[j], counts[j], f, Qt, ops[j]->side, ops[j]->d_rag_off);
        if (rc) return rc;
    }
    BZ_HIP(join_sides(ops, nops, counts, s));
    return BZ_OK;
}

// The projection of a ragged batch on stream s (prepare_ragged first).
int enqueue_conserve_ragged(bz_op *const *ops, int nops, const std::vector<int64_t> &counts, const void *Qt,
                            int in_dtype, double *Qc, double *moments_out, hipStream_t s) {
    for (int j = 0; j < nops; ++j)
        if (counts[j] > 0)
            BZ_HIP(launch_conserve(ops[j], counts[j], Qt, in_dtype, Qc, moments_out, s, ops[j]->d_rag_off,
                                   ops[j]->d_rag_idx));
    return BZ_OK;
}
}  // namespace
}  // namespace bz

extern "C" {

int collision_eval_ragged(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                          const int64_t *offset_of_cell, const void *f, void *Qt, int dtype, void *stream) {
    using namespace bz;
    std::vector<int64_t> counts;
    bool fuse = false;
    int rc = plan_ragged(ops, nops, ncells, op_of_cell, offset_of_cell, f, Qt, dtype, -1, counts, &fuse);
    if (rc || ncells == 0) return rc;
    return enqueue_ragged(ops, nops, counts, f, Qt, dtype, fuse, (hipStream_t)stream);
}

int bz_autotune_ragged(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                       const int64_t *offset_of_cell, int dtype, int *one_launch, double *ms_one, double *ms_per_op,
                       void *stream) {
    if (dtype != BZ_F64 && dtype != BZ_F32) return fail(BZ_EINVAL, "dtype must be BZ_F64 or BZ_F32");
    if (ncells < 1) return fail(BZ_EINVAL, "ncells must be >= 1");
    std::vector<int64_t> counts;
    int rc = prepare_ragged(ops, nops, ncells, op_of_cell, offset_of_cell, dtype, counts);
    if (rc) return rc;
    bool fusable = nops <= kMaxMix;
    for (int j = 0; j < nops; ++j) fusable = fusable && !ops[j]->fly && ops[j]->N <= 32;
    if (!fusable) {  // only the per-op form exists for this set of ops
        if (one_launch) *one_launch = 0;
        if (ms_one) *ms_one = -1.0;
        if (ms_per_op) *ms_per_op = -1.0;
        return BZ_OK;
    }
    rc = prepare_mixed(ops, nops, counts);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    for (int j = 0; j < nops; ++j)
        if (counts[j] > 0) {
            const int64_t n3 = (int64_t)ops[j]->N * ops[j]->N * ops[j]->N;
            BZ_HIP(launch_fill_trial(ops[j], ops[j]->d_fhat, n3 * round_cells(counts[j]) * 2, s));
        }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BZ_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    double best[2] = {1e30, 1e30};
    // mode 1: the one launch; mode 0: each op's own convolution on its stream
    for (int rep = 0; rep < 4 && he == hipSuccess; ++rep)
        for (int mode = 1; mode >= 0 && he == hipSuccess; --mode) {
            he = hipEventRecord(e0, s);
            if (mode == 1) {
                if (he == hipSuccess)
                    he = launch_conv_mixed(dtype == BZ_F64, ops[0]->d_mix_desc, ops[0]->d_mix_items,
                                           ops[0]->n_mix_items, s);
            } else {
                if (he == hipSuccess) he = fork_sides(ops, nops, counts, s);
                for (int j = 0; j < nops && he == hipSuccess; ++j)
                    if (counts[j] > 0)
                        he = enqueue_conv(ops[j], round_cells(counts[j]), ops[j]->sched_S, ops[j]->sched_KH,
                                          ops[j]->side);
                if (he == hipSuccess) he = join_sides(ops, nops, counts, s);
            }
            if (he == hipSuccess) he = hipEventRecord(e1, s);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) best[mode] = std::min(best[mode], (double)ms);  // the first round warms up
        }
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (he != hipSuccess) return hip_fail(he, "ragged autotune trial");
    ops[0]->rag_mode = best[1] <= best[0] ? 1 : 0;
    ops[0]->rag_mode_key = ops[0]->mix_key;
    if (one_launch) *one_launch = ops[0]->rag_mode;
    if (ms_one) *ms_one = best[1];
    if (ms_per_op) *ms_per_op = best[0];
    return BZ_OK;
}

int conserve_ragged(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                    const int64_t *offset_of_cell, const void *Qt, int in_dtype, double *Qc, double *moments_out,
                    void *stream) {
    if (in_dtype != BZ_F64 && in_dtype != BZ_F32) return fail(BZ_EINVAL, "in_dtype must be BZ_F64 or BZ_F32");
    if (ncells > 0 && (!Qt || !Qc)) return fail(BZ_EINVAL, "Qt or Qc is NULL");
    if (in_dtype == BZ_F32 && (const void *)Qc == Qt) return fail(BZ_EINVAL, "Qc may alias Qt only for FP64 input");
    std::vector<int64_t> counts;
    int rc = prepare_ragged(ops, nops, ncells, op_of_cell, offset_of_cell, -1, counts);
    if (rc || ncells == 0) return rc;
    return enqueue_conserve_ragged(ops, nops, counts, Qt, in_dtype, Qc, moments_out, (hipStream_t)stream);
}

int bz_set_ragged_form(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                       const int64_t *offset_of_cell, int dtype, int one_launch) {
    using namespace bz;
    if (one_launch != 0 && one_launch != 1) return fail(BZ_EINVAL, "one_launch must be 0 or 1");
    if (ncells < 1) return fail(BZ_EINVAL, "ncells must be >= 1");
    std::vector<int64_t> counts;
    int rc = prepare_ragged(ops, nops, ncells, op_of_cell, offset_of_cell, dtype, counts);
    if (rc) return rc;
    if (!ragged_fusable(ops, nops)) {
        if (one_launch) return fail(BZ_EINVAL, "one launch needs at most 8 ops, all with stored tables and N <= 32");
        return BZ_OK;  // per-op launches are the only form for these ops
    }
    rc = prepare_mixed(ops, nops, counts);
    if (rc) return rc;
    ops[0]->rag_mode = one_launch;
    ops[0]->rag_mode_key = ops[0]->mix_key;
    return BZ_OK;
}

int bz_graph_capture_ragged(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                            const int64_t *offset_of_cell, const void *f, void *Qt, int dtype, double *Qc,
                            double *moments_out, int form, bz_graph **out) {
    using namespace bz;
    if (!out) return fail(BZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (ncells < 1) return fail(BZ_EINVAL, "ncells must be >= 1");
    if (!Qc) return fail(BZ_EINVAL, "Qc is NULL");
    if (dtype == BZ_F32 && (const void *)Qc == Qt) return fail(BZ_EINVAL, "Qc may alias Qt only for FP64 input");
    std::vector<int64_t> counts;
    bool fuse = false;
    int rc = plan_ragged(ops, nops, ncells, op_of_cell, offset_of_cell, f, Qt, dtype, form, counts, &fuse);
    if (rc) return rc;
    BZ_HIP(hipDeviceSynchronize());
    hipStream_t cs = nullptr;
    BZ_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    rc = enqueue_ragged(ops, nops, counts, f, Qt, dtype, fuse, cs);
    if (rc == BZ_OK) rc = enqueue_conserve_ragged(ops, nops, counts, Qt, dtype, Qc, moments_out, cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    bz_graph *g = new (std::nothrow) bz_graph{graph, exec};
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return fail(BZ_ENOMEM, "host allocation failed");
    }
    *out = g;
    return BZ_OK;
}

int bz_strang_step(bz_op *op, int64_t ncells, double *f, const double *x_faces, double dt, double eps,
                   const bz_wall *left, const bz_wall *right, void *stream) {
    int rc = check_step_args(op, ncells, f, x_faces, dt, eps, left, right);
    if (rc) return rc;
    rc = prepare_step(op, ncells);
    if (rc) return rc;
    return enqueue_strang(op, ncells, f, x_faces, dt, eps, *left, *right, (hipStream_t)stream);
}

int bz_graph_capture_strang(bz_op *op, int64_t ncells, double *f, const double *x_faces, double dt, double eps,
                            const bz_wall *left, const bz_wall *right, int nsteps, bz_graph **out) {
    if (!out) return fail(BZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (nsteps < 1) return fail(BZ_EINVAL, "nsteps must be >= 1");
    int rc = check_step_args(op, ncells, f, x_faces, dt, eps, left, right);
    if (rc) return rc;
    rc = prepare_step(op, ncells);
    if (rc) return rc;
    BZ_HIP(hipDeviceSynchronize());
    hipStream_t cs = nullptr;
    BZ_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    for (int i = 0; i < nsteps && rc == BZ_OK; ++i) rc = enqueue_strang(op, ncells, f, x_faces, dt, eps, *left, *right, cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    bz_graph *g = new (std::nothrow) bz_graph{graph, exec};
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return fail(BZ_ENOMEM, "host allocation failed");
    }
    *out = g;
    return BZ_OK;
}

int bz_graph_launch(bz_graph *g, void *stream) {
    if (!g) return fail(BZ_EINVAL, "graph is NULL");
    BZ_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return BZ_OK;
}

int bz_graph_destroy(bz_graph *g) {
    if (!g) return BZ_OK;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
    return BZ_OK;
}

int bz_plan_items(int N, int64_t ncells, int chunks, int ranges, int row0, int row1, int32_t *out, int64_t cap,
                  int64_t *count) {
    if (!mesh_ok(N)) return fail(BZ_EINVAL, "N must be 8, 16, 24, 32 or 48");
    if (ncells < 1 || ncells > ((int64_t)1 << 26)) return fail(BZ_EINVAL, "ncells out of range");
    if (chunks < 1 || chunks > max_chunks(N)) return fail(BZ_EINVAL, "chunks out of range");
    if (!ranges_ok(N, ranges)) return fail(BZ_EINVAL, "ranges must be 1, 2 or 4 (4 at N = 48)");
    if (row0 < 0 || row1 > N * N || row0 >= row1) return fail(BZ_EINVAL, "row range out of bounds");
    if (!count) return fail(BZ_EINVAL, "count is NULL");
    const std::vector<ConvItem> items = make_items(N, round_cells(ncells), chunks, ranges, row0, row1);
    *count = (int64_t)items.size();
    if (!out) return BZ_OK;
    if (cap < (int64_t)items.size()) return fail(BZ_EINVAL, "out holds fewer than *count items");
    for (size_t i = 0; i < items.size(); ++i) {
        const ConvItem &it = items[i];
        const int32_t v[5] = {it.row, it.chunk, it.group, it.half, it.op};
        std::memcpy(out + 5 * i, v, sizeof(v));
    }
    return BZ_OK;
}

int bz_plan_mixed_items(int nops, const int32_t *N, const int64_t *ncells, const int32_t *chunks, int f64,
                        int32_t *out, int64_t cap, int64_t *count) {
    if (nops < 1 || nops > kMaxMix || !N || !ncells || !chunks || !count) return fail(BZ_EINVAL, "bad arguments");
    std::vector<MixPart> parts;
    for (int j = 0; j < nops; ++j) {
        if (N[j] != 8 && N[j] != 16 && N[j] != 24 && N[j] != 32)
            return fail(BZ_EINVAL, "a mixed launch takes N = 8, 16, 24 or 32");
        if (ncells[j] < 0 || ncells[j] > ((int64_t)1 << 26)) return fail(BZ_EINVAL, "ncells out of range");
        if (chunks[j] < 1 || chunks[j] > max_chunks(N[j])) return fail(BZ_EINVAL, "chunks out of range");
        parts.push_back({N[j], ncells[j] > 0 ? round_cells(ncells[j]) : 0, chunks[j], mix_ranges(N[j], f64 != 0)});
    }
    const std::vector<ConvItem> items = make_mixed_items(parts);
    *count = (int64_t)items.size();
    if (!out) return BZ_OK;
    if (cap < (int64_t)items.size()) return fail(BZ_EINVAL, "out holds fewer than *count items");
    for (size_t i = 0; i < items.size(); ++i) {
        const ConvItem &it = items[i];
        const int32_t v[5] = {it.row, it.chunk, it.group, it.half, it.op};
        std::memcpy(out + 5 * i, v, sizeof(v));
    }
    return BZ_OK;
}

int bz_plan_windows(int N, int weight_dtype, int64_t max_bytes, int min_rows, int32_t *bounds, int cap, int *count) {
    if (!mesh_ok(N)) return fail(BZ_EINVAL, "N must be 8, 16, 24, 32 or 48");
    if (weight_dtype != BZ_F64 && weight_dtype != BZ_F32) return fail(BZ_EINVAL, "weight_dtype must be BZ_F64 or BZ_F32");
    if (max_bytes < 1 || !count) return fail(BZ_EINVAL, "bad arguments");
    std::vector<int64_t> rowoff((size_t)N * N);
    int64_t acc = 0;
    for (int r = 0; r < N * N; ++r) {
        rowoff[r] = acc;
        acc += (int64_t)half_lines(mcount(N, r / N), mcount(N, r % N)) * line_pairs(N);
    }
    if (min_rows < 1) return fail(BZ_EINVAL, "min_rows must be >= 1");
    const std::vector<int> b = window_bounds(rowoff, acc, max_bytes / (int64_t)elem_bytes(weight_dtype), min_rows);
    if (b.empty()) return fail(BZ_EINVAL, "max_bytes is below the weights of one output row");
    *count = (int)b.size();
    if (!bounds) return BZ_OK;
    if (cap < (int)b.size()) return fail(BZ_EINVAL, "bounds holds fewer than *count entries");
    for (size_t i = 0; i < b.size(); ++i) bounds[i] = b[i];
    return BZ_OK;
}

int bz_plan_small_batch(int N, int64_t ncells, int *cells_per_block, int *blocks, int *default_chunks,
                        int *is_default) {
    if (!mesh_ok(N)) return fail(BZ_EINVAL, "N must be 8, 16, 24, 32 or 48");
    if (ncells < 1 || ncells > kSmallMaxCells)
        return fail(BZ_EINVAL, "the small-batch form takes 1 to " + std::to_string(kSmallMaxCells) + " cells");
    const int cb = small_cells_per_block(N, ncells);
    if (cells_per_block) *cells_per_block = cb;
    if (blocks) *blocks = (int)((ncells + cb - 1) / cb);
    if (default_chunks) *default_chunks = small_default_chunks(N, ncells);
    if (is_default) *is_default = small_by_default(N, ncells) ? 1 : 0;
    return BZ_OK;
}

int bz_weights_gather(const bz_op *op, int64_t npairs, const int32_t *k_lin, const int32_t *m_lin, double *out,
                      void *stream) {
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    if (npairs < 0) return fail(BZ_EINVAL, "npairs must be >= 0");
    if (npairs == 0) return BZ_OK;
    if (!k_lin || !m_lin || !out) return fail(BZ_EINVAL, "null argument");
    int rc = check_device(op);
    if (rc) return rc;
    if (op->fly)
        BZ_HIP(launch_fly_gather(op, npairs, k_lin, m_lin, out, (hipStream_t)stream));
    else
        BZ_HIP(launch_gather_weights(op, npairs, k_lin, m_lin, out, (hipStream_t)stream));
    return BZ_OK;
}

}  // extern "C"
