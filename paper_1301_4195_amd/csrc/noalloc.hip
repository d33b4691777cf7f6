// collision_eval without allocation: the workspace of one evaluation (f^, the
// m1-chunk partial sums, the transforms' intermediates) lives in a file-scope
// device array instead of the op's hipMalloc'ed workspace, so the call makes
// no allocating call at all.  The convolution is the small-batch form
// (conv_small.hip), whose items come from the grid, so no item list is needed
// either.  Each GPU holds its own copy of the array, at its own address: the
// address is taken once per device with hipGetSymbolAddress (with that device
// current) and only that pointer is handed to kernels -- in host code the
// array's name stands for a host-side shadow, not device memory.
#include "bz_internal.h"

#include <algorithm>
#include <mutex>

namespace bz {
namespace {

constexpr int64_t kScratchBytes = BZ_NOALLOC_SCRATCH_BYTES;
static_assert(BZ_NOALLOC_MAX_CELLS == kSmallMaxCells, "the small-batch form takes at most one cell group");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of this device's copy of `scratch` (the current device).
int scratch_ptr(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(BZ_EINVAL, "device index beyond the no-allocation table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(BZ_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BZ_OK;
}

}  // namespace
}  // namespace bz

extern "C" {

int collision_eval_noalloc(bz_op *op, int64_t ncells, const void *f, void *Qt, int dtype, void *stream) {
    using namespace bz;
    if (!op) return fail(BZ_EINVAL, "op is NULL");
    if (ncells < 0) return fail(BZ_EINVAL, "ncells must be >= 0");
    if (dtype != BZ_F64 && dtype != BZ_F32) return fail(BZ_EINVAL, "dtype must be BZ_F64 or BZ_F32");
    if (dtype != op->wdtype) return fail(BZ_EINVAL, "dtype differs from the op's weight dtype");
    if (ncells == 0) return BZ_OK;
    if (ncells > BZ_NOALLOC_MAX_CELLS) return fail(BZ_EINVAL, "collision_eval_noalloc takes at most 64 cells");
    if (!f || !Qt) return fail(BZ_EINVAL, "f or Qt is NULL");
    if (f == Qt) return fail(BZ_EINVAL, "Qt must not alias f");
    if (!pair_aligned(f, dtype) || !pair_aligned(Qt, dtype))
        return fail(BZ_EINVAL, "f and Qt must be aligned to two values (16 bytes FP64, 8 bytes FP32)");
    int rc = check_device(op);
    if (rc) return rc;
    // workspace layout in the array: f^ [N^3][cellpad] complex, then the
    // partial sums [S][N^3][cellpad] complex (at least two FP32 chunks: the
    // FP32 forward transform keeps its FP64 intermediate there)
    const int N = op->N;
    const int64_t cellpad = round_cells(ncells);
    const int64_t buf = (int64_t)N * N * N * cellpad * 2 * (dtype == BZ_F64 ? 8 : 4);
    const Split sp = choose_split(op, cellpad, ncells);
    int S = sp.KH == 0 ? sp.S : small_default_chunks(N, ncells);
    const int pmin = dtype == BZ_F32 ? 2 : 1;
    while (S > 1 && buf * (1 + std::max(S, pmin)) > kScratchBytes) --S;
    if (buf * (1 + std::max(S, pmin)) > kScratchBytes)
        return fail(BZ_EINVAL, "this batch's workspace exceeds the 64 MiB no-allocation array");
    int dev = -1;
    BZ_HIP(hipGetDevice(&dev));
    void *base = nullptr;
    rc = scratch_ptr(dev, &base);
    if (rc) return rc;
    void *fhat = base;
    void *part = (unsigned char *)base + buf;
    hipStream_t s = (hipStream_t)stream;
    BZ_HIP(launch_forward(op, ncells, cellpad, f, fhat, part, nullptr, s));
    if (op->fly) {  // each slab's weights into the op's own slab buffer, then its rows
        for (size_t j = 0; j + 1 < op->slab_rows.size(); ++j) {
            const int r0 = op->slab_rows[j], r1 = op->slab_rows[j + 1];
            BZ_HIP(launch_fly_weights(op, r0, r1, op->W, s));
            BZ_HIP(launch_conv_small(op, ncells, cellpad, S, fhat, part, op->W, op->h_rowoff[r0], r0, r1, s));
        }
    } else {
        BZ_HIP(launch_conv_small(op, ncells, cellpad, S, fhat, part, op->W, 0, 0, N * N, s));
    }
    BZ_HIP(launch_inverse(op, ncells, cellpad, S, part, Qt, nullptr, s, fhat));
    return BZ_OK;
}

}  // extern "C"
