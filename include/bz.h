/*
 * bz.h -- C ABI of the MI355X (gfx950) library for the conservative spectral
 * Boltzmann collision operator (Gamba-Tharkabhushanam method as extended in
 * Haack, arXiv:1301.4195).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every call returns an int: BZ_OK (0) or a negative BZ_E* code.  On error a
 *   thread-local message is available from bz_last_error().  Arguments are
 *   validated before anything is enqueued; no C++ exception crosses the ABI.
 * - Distribution arrays are caller-owned DEVICE buffers laid out as
 *   [ncells][N][N][N], row-major, j3 fastest, where grid point j carries the
 *   velocity v_j = dv (j - N/2), dv = 2L/N, on the cube [-L, L]^3
 *   (Sec. 3.1, eq. meshpoints).  The library never allocates or frees caller
 *   buffers.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *   compute calls are enqueue-only and asynchronous on that stream; the caller
 *   synchronises.  A bz_op must not be used by two streams at once (its
 *   workspace is shared).
 * - NaN/Inf inputs are not rejected (checking would cost a pass); they
 *   propagate to the outputs, and conserve() flags the cells whose moment
 *   sums are not finite in moments_out (BZ_MOMENTS_NONFINITE_BITS).
 * - A bz_op lives on the device that was current when it was created; calls
 *   must be made with that device current.
 */
#ifndef BZ_H
#define BZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BZ_OK 0
#define BZ_EINVAL (-1)      /* bad argument (null pointer, bad size/N/L/lambda/dtype) */
#define BZ_ENOMEM (-2)      /* device allocation failed or above the op's memory cap  */
#define BZ_EHIP (-3)        /* a HIP runtime call or kernel launch failed             */
#define BZ_EUNSUPPORTED (-4) /* valid request the library does not implement           */

/* number types */
#define BZ_F64 0
#define BZ_F32 1

/* wall kinds for transport_step */
#define BZ_WALL_DIFFUSE 0     /* diffuse Maxwell wall, Sec. 2.1 eq. (BC)              */
#define BZ_WALL_EXTRAPOLATE 1 /* zeroth-order extrapolation ghost cells (outflow)     */
#define BZ_WALL_NOFLUX 2      /* incoming characteristics carry no flux (Sec. 3.4)    */

typedef struct bz_op bz_op;

typedef struct bz_wall {
    int kind;     /* BZ_WALL_* */
    double Tw;    /* wall temperature (diffuse only), > 0 */
    double Vw[3]; /* wall velocity; the normal component Vw[0] must be 0 */
} bz_wall;

/*
 * bz_op_create -- precompute everything that depends only on (N, L, lambda):
 * the trapezoid-weighted convolution weights
 *     W[k][m] = omega_m * G^(xi_m, zeta_k)
 * (Sec. 2.2 eq. GHat_calc: its closed forms for lambda = 0 (Maxwell
 * molecules) and lambda = 1 (hard spheres); for any other exponent the
 * radial integral itself by Gauss-Jacobi quadrature, as the last paragraph
 * of Sec. 2.2 prescribes; isotropic b = 1/(4 pi), beta = 1, cutoff r0 = L),
 * stored only for the pairs the truncated sum of Sec. 3.2 visits, mirrored
 * couples combined, computed in FP64 on the device and stored in
 * `weight_dtype` (BZ_F64 or BZ_F32; collision_eval's dtype must match it);
 * plus the conservation matrix data of Sec. 3.3 ((C C^T)^{-1}, FP64).
 *   N         velocity points per dimension: 8, 16, 24, 32 or 48
 *   L         half-width of the velocity cube, > 0
 *   lambda    exponent of the kernel |u|^lambda, in (-3, 2]: variable hard
 *             (0 < lambda < 1), hard-sphere-like and soft (lambda < 0)
 *             potentials (outside: BZ_EUNSUPPORTED)
 *   omega1d   NULL for the uniform trapezoid weight dzeta^3, or N per-dimension
 *             host weights (omega_m = w[m1] w[m2] w[m3]); read during the call
 *   out       receives the op; the library owns all of its device memory
 * Synchronous.  Errors: BZ_EINVAL, BZ_EUNSUPPORTED, BZ_ENOMEM, BZ_EHIP.
 */
int bz_op_create(int N, double L, double lambda, int weight_dtype, const double *omega1d,
                 bz_op **out);

/*
 * bz_op_create_inelastic -- bz_op_create for inelastic collisions: the law
 * v' = v + (beta/2)(|u| sigma - u) of the weak form (Sec. 2.2, eqs. G_eqn and
 * GHat_calc with beta), beta = (1 + e)/2 for the restitution coefficient e,
 * and the conservation constraint set of Sec. 3.3 without energy, which
 * inelastic collisions do not preserve: conserve() then projects onto zero
 * mass and momentum only.  The weights come from the radial integral by
 * Gauss-Jacobi quadrature (no closed form applies for beta < 1).
 *   beta   in [0.5, 1]; 1 is exactly bz_op_create
 * Other arguments and errors as bz_op_create (BZ_EINVAL for beta outside).
 */
int bz_op_create_inelastic(int N, double L, double lambda, double beta, int weight_dtype, const double *omega1d,
                           bz_op **out);

/*
 * bz_op_create_onthefly -- bz_op_create without the stored weight table: the
 * weights are computed on the fly, as the Conclusions propose for meshes whose
 * six-dimensional weight array would not fit in memory.  The op keeps small
 * O(N^2) tables (sin and cos of (pi/2) sqrt(X) for the integer squared
 * lengths X of the closed forms, the loss term and the B = 0 limit) and one
 * slab buffer of at most `slab_bytes` -- two when the weights take more than
 * one slab, so that one slab's weights are computed (on a second stream of
 * the op's) while the other is convolved; every convolution (collision_eval,
 * the Strang step, ragged batches, bz_autotune's trials) recomputes the
 * weights of the output rows one slab at a time into that buffer and runs the
 * convolution of those rows on it.  Results equal bz_op_create's up to the
 * rounding of the weights (same closed forms, evaluated through the
 * angle-sum identities); the weights do not depend on the slab size, nor do
 * the results.
 *   lambda      0 or 1 (the closed forms of Sec. 2.2); any other exponent of
 *               (-3, 2] gives BZ_EUNSUPPORTED
 *   slab_bytes  upper bound of the slab buffer in bytes; 0 = the larger of
 *               256 MiB (the chip's last-level cache) and 1/16 of the table
 *               (1.3 GB at N = 48 FP64); below one output row's weights
 *               (for N = 32 FP64 about 3.5 MB) gives BZ_EINVAL.  Larger
 *               slabs mean fewer, fuller convolution launches.
 * Other arguments and errors as bz_op_create.
 */
int bz_op_create_onthefly(int N, double L, double lambda, int weight_dtype, const double *omega1d,
                          int64_t slab_bytes, bz_op **out);

/*
 * bz_op_table_bytes -- device bytes the op holds for its weights (the stored
 * table, or the on-the-fly tables and slab buffer) and its other create-time
 * tables; the per-batch workspace is not included.  Host only.
 * Errors: BZ_EINVAL (NULL argument).
 */
int bz_op_table_bytes(const bz_op *op, int64_t *bytes);

/* Free an op and its device tables.  NULL is accepted.  Synchronous. */
int bz_op_destroy(bz_op *op);

/* Velocity points per dimension of an op (or BZ_EINVAL for NULL). */
int bz_op_n(const bz_op *op);

/*
 * bz_op_reserve -- grow the op's workspace (transformed distributions and
 * partial sums) for batches of up to `ncells` cells now, so that later calls
 * with ncells <= this value allocate nothing (required before capturing them
 * into a HIP graph).  Synchronous.  Errors: BZ_EINVAL, BZ_ENOMEM, BZ_EHIP.
 */
int bz_op_reserve(bz_op *op, int64_t ncells);

/*
 * bz_autotune -- choose the convolution's work split for batches of `ncells`
 * cells (the batching of the method's sum over the kept m lines, Sec. 3.2 and
 * Sec. 4.1, into launch items).  Each item is one output row (k1, k2) x one
 * of S chunks of the row's m1 range x one of KH equal ranges of the row's k3
 * outputs x 64 cells.  For ncells <= 64 there is also the small-batch form
 * (KH reported as 0): items of one output row x one m1 chunk x a block of up
 * to 8 cells (4 at N = 24, 32; 2 at N = 48), whose lanes run over the (k3,
 * m3) pairs of a line so that the weights stream from memory coalesced and
 * each serves the whole block -- the memory-bound form for few cells.  The
 * trials S in {1, 2, 3, 4, 6, 8} (up to the shortest m1 range) and KH in
 * {0 (ncells <= 64), 1, 2, 4} (4 only at N = 48) are each timed on the op's own workspace filled
 * with pseudo-random values (the convolution and the inverse transform, whose
 * first pass adds the S partial sums, three times on `stream`, fastest kept;
 * the workspace's earlier contents are lost), and the fastest split is used by every
 * later call of this op with a batch of the same padded size (ncells rounded
 * up to a multiple of 64).  Results of later calls differ from untuned ones
 * only in rounding (summation order, and multiply-add contraction, which the
 * compiled variants for different k3 range counts do differently).  Synchronous; grows the workspace for the largest
 * trial that fits the memory cap.  `chosen_chunks` (S), `chosen_ranges` (KH)
 * and `best_ms` (that time) are nullable outputs.  Must not be called
 * while another call of this op is queued or being captured.
 * Errors: BZ_EINVAL (NULL op, ncells < 1), BZ_ENOMEM, BZ_EHIP.
 */
int bz_autotune(bz_op *op, int64_t ncells, int *chosen_chunks, int *chosen_ranges, double *best_ms, void *stream);

/*
 * bz_set_split -- fix the convolution's work split for batches of `ncells`
 * cells (same padded size rule as bz_autotune): `chunks` chunks of each
 * row's m1 range (1 .. (N/2 + 2)/2) and `ranges` equal k3 ranges per row
 * (1, 2 or 4; at N = 48 only 4), or ranges = 0: the small-batch form
 * (bz_autotune) with `chunks` chunks, for ncells <= 64 only.  Replaces an autotuned choice; later calls of this op with that
 * batch size use it, so their results are bitwise repeatable across runs.
 * Synchronous; grows the workspace.  Errors: BZ_EINVAL, BZ_ENOMEM, BZ_EHIP.
 */
int bz_set_split(bz_op *op, int64_t ncells, int chunks, int ranges);

/*
 * bz_get_split -- the work split (m1 chunks, k3 ranges) this op uses for
 * batches of `ncells` cells: the bz_set_split / bz_autotune choice for that
 * padded size, else the default: the small-batch form (ranges 0) for up to
 * 32 cells at N <= 16 and up to 16 cells above, with 3 chunks for one block
 * of cells and fewer for more blocks; otherwise 4 chunks, capped at (N/2 + 2)/2,
 * and 2 ranges at N = 32, 4 at N = 48, else 1.  Host only, no device work.
 * Errors: BZ_EINVAL (NULL op, ncells < 1).
 */
int bz_get_split(const bz_op *op, int64_t ncells, int *chunks, int *ranges);

/*
 * bz_set_memory_cap -- upper bound (bytes) on device memory any single op may
 * hold (weights + workspace); 0 = unlimited (default).  Requests above the cap
 * fail with BZ_ENOMEM.  Process-wide.
 */
int bz_set_memory_cap(int64_t bytes);

/*
 * collision_eval -- the unprojected collision operator Q~ for a batch of
 * independent cells (Sec. 3.2):
 *   f^(zeta_k) = (2pi)^{-3/2} dv^3 sum_j f_j e^{-i zeta_k . v_j}   (FFT)
 *   Q^(zeta_k) = sum_{m : k-m+N/2 in grid} W[k][m] f^(xi_m) f^(zeta_k - xi_m)
 *   Q~_j       = Re (2pi)^{-3/2} dzeta^3 sum_k Q^(zeta_k) e^{+i zeta_k . v_j}
 *   f       device [ncells][N][N][N] of `dtype` (input, unchanged)
 *   Qt      device [ncells][N][N][N] of `dtype` (output, may not alias f)
 *   (f and Qt aligned to two values: 16 bytes FP64, 8 bytes FP32)
 *   dtype   BZ_F64 (FP64 transforms and sums) or BZ_F32 (FP32 weights, f^
 *           and products; the forward transform computed in FP64 and f^
 *           rounded to FP32 once; each line's FP32 partial sum added to an
 *           FP64 running sum; FP32 inverse transform); must equal the op's
 *           weight_dtype
 * ncells = 0 is a no-op.  May grow the workspace (see bz_op_reserve).
 * Errors: BZ_EINVAL, BZ_ENOMEM, BZ_EHIP.
 */
int collision_eval(bz_op *op, int64_t ncells, const void *f, void *Qt, int dtype, void *stream);

/*
 * collision_eval_noalloc -- collision_eval for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): the same Q~, with no hipMalloc, hipFree or allocating
 * library call.  Its workspace (f^, the partial sums, the transforms'
 * intermediates) is a library-owned device array of 64 MiB per GPU
 * (BZ_NOALLOC_SCRATCH_BYTES), held from the first call on that GPU until the
 * process ends.  The convolution is the small-batch form (one cell up to 64),
 * with the op's split for this batch size when it is that form and fits, else
 * fewer m1 chunks (then results differ from collision_eval only in summation
 * order).
 *   ncells  1..64; f, Qt, dtype as for collision_eval (caller-owned)
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (other streams, other threads) race and give wrong results.  No part
 * of the array needs clearing between calls: a call reads only what it wrote.
 * Errors: BZ_EINVAL (as collision_eval; ncells > 64; a batch whose workspace
 * exceeds the array even with one chunk, e.g. N = 48), BZ_EHIP.
 */
#define BZ_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
#define BZ_NOALLOC_MAX_CELLS 64
int collision_eval_noalloc(bz_op *op, int64_t ncells, const void *f, void *Qt, int dtype, void *stream);

/*
 * conserve -- the conservation projection of Sec. 3.3 in FP64:
 *   b = C Q~ (rows dv^3 (1, v^1, v^2, v^3, |v|^2)),
 *   Qc = Q~ - C^T (C C^T)^{-1} b
 * (for an op from bz_op_create_inelastic with beta < 1: the first four rows
 * only -- mass and momentum; moments_out still receives all five sums)
 *   Qt           device [ncells][N^3] of in_dtype (BZ_F64 or BZ_F32)
 *   Qc           device [ncells][N^3] FP64 (may alias Qt when in_dtype = BZ_F64)
 *   moments_out  device [ncells][5] FP64 receiving b (pre-projection), or NULL;
 *                for a cell whose five sums are not all finite (NaN or Inf
 *                in its Q~) all five places hold the quiet NaN whose bit
 *                pattern is BZ_MOMENTS_NONFINITE_BITS, the per-cell
 *                non-finite flag (its Qc is then not finite either)
 * Errors: BZ_EINVAL, BZ_EHIP.
 */
#define BZ_MOMENTS_NONFINITE_BITS 0x7FF80000000BADF1ull
int conserve(const bz_op *op, int64_t ncells, const void *Qt, int in_dtype, double *Qc,
             double *moments_out, void *stream);

/*
 * bz_axpy -- y <- y + alpha x over n FP64 values (device pointers): the
 * explicit time update f <- f + (dt/eps) Qc of the semi-discrete collision
 * problem df/dt = P_N Q~ (Sec. 3.3), and the stages of the Runge-Kutta
 * integrators of Sec. 3.1.  Errors: BZ_EINVAL, BZ_EHIP.
 */
int bz_axpy(int64_t n, double alpha, const double *x, double *y, void *stream);

/*
 * transport_step -- one Heun (two-stage, second-order) step of the 1-D
 * transport sub-problem df/dt + v_1 df/dx = 0 (Sec. 3.4): finite volumes on
 * non-uniform cells, upwind fluxes with minmod-limited slopes (eqs. transport,
 * upwind, minmod), ghost cells by extrapolation, and boundary faces given by
 * `left` / `right` (diffuse wall of Sec. 2.1 eq. (BC) with sigma_w set by zero
 * net mass flux, extrapolation, or no inflow).
 *   f        device FP64 [ncells + 4][N^3]: two ghost cells at each end, interior
 *            cells at 2..ncells+1; updated in place, ghosts rewritten
 *   x_faces  device FP64 [ncells + 1], strictly increasing cell faces
 *   dt       time step (> 0)
 * Errors: BZ_EINVAL, BZ_ENOMEM, BZ_EHIP.
 */
int transport_step(bz_op *op, int64_t ncells, double *f, const double *x_faces, double dt,
                   const bz_wall *left, const bz_wall *right, void *stream);

/*
 * collision_eval_ragged -- collision_eval for a batch whose cells use
 * different velocity meshes (one op per N).  Cell c uses ops[op_of_cell[c]]
 * and occupies the elements [offset_of_cell[c], offset_of_cell[c] + N_c^3) of
 * the packed device buffers f and Qt (same layout per cell as collision_eval).
 *   ops          nops ops, all with weight dtype `dtype`, distinct objects
 *   op_of_cell   HOST int32 [ncells], values in [0, nops)
 *   offset_of_cell HOST int64 [ncells], element offsets (even, >= 0; cells
 *                must not overlap -- not checked); f and Qt aligned to two
 *                values, as for collision_eval
 * The cells of each op are gathered into that op's own batch (offset lists are
 * uploaded to the op, synchronously, only when they change).  With at most 8
 * ops, all with stored weight tables and N <= 32, the transforms run per op and the
 * convolution of every op is ONE launch over all their items on `stream`
 * (each op's rows in 1 k3 range up to N = 16, above that in 4 (FP64) or 2
 * (FP32); its m1 chunks as bz_get_split gives for its cell count), so every
 * cell's result equals collision_eval of its op at that split bit for bit.
 * Otherwise (more ops, an op computing its weights on the fly, N = 48, or
 * bz_autotune_ragged found them faster for this layout) the per-op pipelines
 * run concurrently on forked streams joined back to `stream`.
 * The item list of the one-launch form is kept by ops[0] and rebuilt,
 * synchronously, when the ops, their batch sizes or their splits change.
 * Errors: BZ_EINVAL, BZ_ENOMEM, BZ_EHIP.
 */
int collision_eval_ragged(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                          const int64_t *offset_of_cell, const void *f, void *Qt, int dtype, void *stream);

/*
 * bz_autotune_ragged -- choose, for this ragged layout (same arguments as
 * collision_eval_ragged, without the data), between the one-launch
 * convolution and the per-op launches on forked streams: both are timed on
 * the ops' workspaces filled with pseudo-random values (one warm-up round,
 * best of three; the workspaces' contents are lost), and later
 * collision_eval_ragged calls with the same ops, batch sizes and splits use
 * the faster.  Run bz_autotune on the ops first if their splits are to be
 * tuned: a later split change returns the layout to the default (one launch).
 * When only the per-op form applies (more than 8 ops, or an op with weights
 * on the fly) nothing is timed and the times are -1.  Outputs (nullable):
 * one_launch (1 or 0), ms_one and ms_per_op (convolution time of each form).
 * Synchronous.  Errors: BZ_EINVAL, BZ_ENOMEM, BZ_EHIP.
 */
int bz_autotune_ragged(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                       const int64_t *offset_of_cell, int dtype, int *one_launch, double *ms_one, double *ms_per_op,
                       void *stream);

/*
 * conserve_ragged -- conserve() for the packed ragged layout of
 * collision_eval_ragged (same host index arrays).  Qc is a packed FP64 buffer
 * with the same element offsets; moments_out (device [ncells][5] or NULL) is
 * indexed by cell.  Errors: BZ_EINVAL, BZ_ENOMEM, BZ_EHIP.
 */
int conserve_ragged(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                    const int64_t *offset_of_cell, const void *Qt, int in_dtype, double *Qc, double *moments_out,
                    void *stream);

/*
 * bz_strang_step -- one time step of df/dt + v_1 df/dx = Q(f, f)/eps (eq. BTE
 * in one space dimension) by Strang splitting of the transport and collision
 * sub-problems (Sec. 3.1): transport over dt/2, collision over dt, transport
 * over dt/2, each advanced with Heun's second-order Runge-Kutta method.  The
 * collision stages apply the projected operator P_N Q~ (collision_eval +
 * conserve) to every interior cell:
 *     f* = f + (dt/eps) P_N Q~(f),   f <- f + (dt/(2 eps)) (P_N Q~(f) + P_N Q~(f*)).
 *   op        an FP64 op (weights BZ_F64)
 *   f         device FP64 [ncells + 4][N^3] with two ghost cells at each end,
 *             updated in place; aligned to 16 bytes
 *   x_faces   device FP64 [ncells + 1]; dt > 0, eps > 0
 *   left/right  boundary kinds as for transport_step
 * Stage buffers live in the op's workspace (grown on the first call).  After
 * one call with a given ncells the step allocates nothing and never
 * synchronises the host, so it may be captured into a HIP graph.
 * Errors: BZ_EINVAL, BZ_ENOMEM, BZ_EHIP.
 */
int bz_strang_step(bz_op *op, int64_t ncells, double *f, const double *x_faces, double dt, double eps,
                   const bz_wall *left, const bz_wall *right, void *stream);

/*
 * HIP-graph capture of nsteps consecutive bz_strang_step calls: the library
 * grows every workspace first, captures the kernels on a private stream and
 * instantiates the graph.  bz_graph_launch replays it on `stream` (the
 * pointers and scalars captured are fixed); bz_graph_destroy frees it.
 * Errors: BZ_EINVAL, BZ_ENOMEM, BZ_EHIP.
 */
typedef struct bz_graph bz_graph;
int bz_graph_capture_strang(bz_op *op, int64_t ncells, double *f, const double *x_faces, double dt, double eps,
                            const bz_wall *left, const bz_wall *right, int nsteps, bz_graph **out);

/*
 * bz_set_ragged_form -- pin the convolution form of later
 * collision_eval_ragged calls with this layout (same arguments as
 * collision_eval_ragged, without the data): one_launch = 1 the one launch
 * over every op's items, 0 the per-op launches on forked streams (what
 * bz_autotune_ragged would otherwise choose by timing).  Both give each cell
 * its op's collision_eval result at the split that form uses.  One launch is
 * refused (BZ_EINVAL) where it does not apply (more than 8 ops, an op with
 * weights on the fly, N = 48).  Synchronous.  Errors: BZ_EINVAL, BZ_ENOMEM,
 * BZ_EHIP.
 */
int bz_set_ragged_form(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                       const int64_t *offset_of_cell, int dtype, int one_launch);

/*
 * bz_graph_capture_ragged -- HIP-graph capture of one step of a mixed-N
 * batch (Sec. 3.2 operator for every cell, then the Sec. 3.3 projection):
 * collision_eval_ragged into Qt followed by conserve_ragged into Qc (and
 * moments_out, nullable), with the arguments of those two calls.  form: 1 one
 * convolution launch, 0 per-op launches, -1 the form collision_eval_ragged
 * would use for this layout.  The library prepares every workspace and index
 * list first (synchronously), captures the kernels -- the per-op streams
 * forked from and joined back to a private capture stream -- and instantiates
 * the graph; bz_graph_launch replays it (pointers fixed at capture; f may be
 * refilled between replays).  Errors: BZ_EINVAL, BZ_ENOMEM, BZ_EHIP.
 */
int bz_graph_capture_ragged(bz_op *const *ops, int nops, int64_t ncells, const int32_t *op_of_cell,
                            const int64_t *offset_of_cell, const void *f, void *Qt, int dtype, double *Qc,
                            double *moments_out, int form, bz_graph **out);
int bz_graph_launch(bz_graph *g, void *stream);
int bz_graph_destroy(bz_graph *g);

/*
 * bz_weights_gather -- read back stored weights (as FP64) for `npairs` linear
 * indices k = (k1 N + k2) N + k3 and m likewise (device int32 arrays).  The
 * truncated sum visits the pairs m and n = k - m + N/2 with the same product
 * f^_m f^_n, and the library stores one weight per such couple:
 *     W[k][m] + W[k][n]   when (m1, m2) != (n1, n2),
 *     W[k][m]             when (m1, m2) == (n1, n2) (a self-mirrored line),
 * with W[k][m] = omega_m G^(xi_m, zeta_k).  Pairs outside the truncation box
 * give 0.  For testing the precompute against an independent evaluation.
 * Errors: BZ_EINVAL, BZ_EHIP.
 */
int bz_weights_gather(const bz_op *op, int64_t npairs, const int32_t *k_lin,
                      const int32_t *m_lin, double *out, void *stream);

/*
 * Work-plan inspection (host only: no device work, usable without a GPU).
 *
 * bz_plan_items -- the convolution item list one launch processes for the
 * output rows [row0, row1) of a batch of `ncells` cells with `chunks` m1
 * chunks and `ranges` k3 ranges (the batching of the sum of Sec. 3.2 into
 * launch items): 5 int32 per item (row k1*N+k2, chunk, 64-cell group, k3
 * range, op 0), in launch order; rows of -1 pad the list to whole rounds of
 * the chip's 8 XCDs (workgroup i runs on XCD i mod 8).  *count receives the
 * number of items; with out == NULL nothing else is written.
 * bz_plan_mixed_items -- the same for the one-launch convolution of a
 * ragged batch: op j has mesh N[j], ncells[j] cells (0 allowed) and
 * chunks[j] chunks; the item's last field is j.  f64 selects the k3 range
 * counts of the FP64 variants.
 * bz_plan_windows -- the row ranges of an op's convolution launches: the
 * weights split at `max_bytes` (the slabs of an on-the-fly op with
 * slab_bytes = max_bytes, min_rows = 1), then merged until every range has at
 * least `min_rows` rows (a stored table uses max_bytes = 512 MiB and the rows
 * that give one launch 8192 items at its batch size and split):
 * *count boundaries 0 = b0 < b1 < ... = N*N, launch j covering rows
 * [b_j, b_{j+1}).
 * bz_plan_small_batch -- the small-batch convolution's plan for `ncells`
 * (1..64) cells (bz_autotune): cells per block (1, 2, 4 or 8; at most 4 at
 * N = 24, 32 and 2 at N = 48), the number of blocks (each re-reads the whole
 * weight table), the default m1 chunk count, and whether the form is the
 * default for this batch size (nonzero) or only selectable.  Outputs are
 * nullable.
 * Errors: BZ_EINVAL.
 */
int bz_plan_items(int N, int64_t ncells, int chunks, int ranges, int row0, int row1, int32_t *out, int64_t cap,
                  int64_t *count);
int bz_plan_mixed_items(int nops, const int32_t *N, const int64_t *ncells, const int32_t *chunks, int f64,
                        int32_t *out, int64_t cap, int64_t *count);
int bz_plan_windows(int N, int weight_dtype, int64_t max_bytes, int min_rows, int32_t *bounds, int cap, int *count);
int bz_plan_small_batch(int N, int64_t ncells, int *cells_per_block, int *blocks, int *default_chunks,
                        int *is_default);

/*
 * bz_timing_enable / bz_timing_read -- measurement hooks.  While enabled,
 * collision_eval brackets its convolution kernel (the O(N^6) weighted sum of
 * Sec. 3.2, the dominant kernel of the method) with a HIP event pair on the
 * caller's stream.  bz_timing_read waits for the recorded events, returns the
 * summed kernel time in milliseconds and the number of launches since the last
 * read (or since enabling), and resets both.  Enabling preallocates events;
 * timing adds two event records per call.  Errors: BZ_EINVAL, BZ_EHIP.
 */
int bz_timing_enable(bz_op *op, int on);
int bz_timing_read(bz_op *op, double *conv_ms, int64_t *launches);

/* Thread-local message describing the last non-zero status (never NULL). */
const char *bz_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BZ_H */
