"""Python binding of the gfx950 conservative spectral collision-operator library.

Thin ctypes marshalling over the C ABI declared in ``include/bz.h``: every step
of the computation runs in the HIP kernels of ``libbz.so``; PyTorch is used only
for device memory and streams.  Importing the package does not touch the GPU;
the first call loads ``libbz.so`` and raises ``BzLibraryMissing`` if it has not
been built (``python -m paper_1301_4195_amd.build``) -- there is no fallback.

Entry points (same names as the C ABI; EXPORTS lists them all):
  bz_op_create, bz_op_create_inelastic, bz_op_create_onthefly,
  bz_op_table_bytes, bz_op_destroy, bz_op_reserve,
  bz_autotune, bz_set_split, bz_get_split, bz_set_memory_cap,
  collision_eval, collision_eval_noalloc, collision_eval_ragged, bz_autotune_ragged, conserve,
  conserve_ragged, bz_axpy,
  transport_step, bz_strang_step, bz_graph_capture_strang, bz_graph_launch,
  bz_graph_destroy, bz_weights_gather, bz_plan_items, bz_plan_mixed_items,
  bz_plan_windows, bz_plan_small_batch, bz_timing_enable, bz_timing_read,
  bz_set_ragged_form, bz_graph_capture_ragged, bz_last_error
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbz.so")

BZ_OK, BZ_EINVAL, BZ_ENOMEM, BZ_EHIP, BZ_EUNSUPPORTED = 0, -1, -2, -3, -4
BZ_F64, BZ_F32 = 0, 1
BZ_WALL_DIFFUSE, BZ_WALL_EXTRAPOLATE, BZ_WALL_NOFLUX = 0, 1, 2
# bit pattern conserve() writes to all five moments of a cell whose sums are not finite
BZ_MOMENTS_NONFINITE_BITS = 0x7FF80000000BADF1

EXPORTS = (
    "bz_op_create", "bz_op_create_inelastic", "bz_op_create_onthefly", "bz_op_table_bytes", "bz_op_destroy", "bz_op_n", "bz_op_reserve", "bz_autotune", "bz_set_split", "bz_get_split", "bz_set_memory_cap",
    "collision_eval", "collision_eval_noalloc", "conserve", "bz_axpy", "transport_step", "bz_weights_gather", "bz_plan_items", "bz_plan_mixed_items", "bz_plan_windows",
    "bz_plan_small_batch",
    "bz_timing_enable", "bz_timing_read", "bz_strang_step", "bz_graph_capture_strang",
    "bz_graph_launch", "bz_graph_destroy", "collision_eval_ragged", "bz_autotune_ragged", "conserve_ragged",
    "bz_set_ragged_form", "bz_graph_capture_ragged", "bz_last_error",
)


class BzLibraryMissing(RuntimeError):
    pass


class BzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bz error {code}: {msg}")
        self.code = code


class bz_wall(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("Tw", ctypes.c_double), ("Vw", ctypes.c_double * 3)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64


def load():
    """Load libbz.so (once).  Fails loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BzLibraryMissing(f"{LIB_PATH} not found: build it with `python -m paper_1301_4195_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.bz_op_create.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_vp)]
    lib.bz_op_create_inelastic.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_vp)]
    lib.bz_op_create_onthefly.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_double), _i64, ctypes.POINTER(_vp)]
    lib.bz_op_table_bytes.argtypes = [_vp, ctypes.POINTER(_i64)]
    lib.bz_op_destroy.argtypes = [_vp]
    lib.bz_op_n.argtypes = [_vp]
    lib.bz_op_reserve.argtypes = [_vp, _i64]
    lib.bz_set_split.argtypes = [_vp, _i64, ctypes.c_int, ctypes.c_int]
    lib.bz_get_split.argtypes = [_vp, _i64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.bz_autotune.argtypes = [_vp, _i64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_double), _vp]
    lib.bz_set_memory_cap.argtypes = [_i64]
    lib.collision_eval.argtypes = [_vp, _i64, _vp, _vp, ctypes.c_int, _vp]
    lib.collision_eval_noalloc.argtypes = [_vp, _i64, _vp, _vp, ctypes.c_int, _vp]
    lib.conserve.argtypes = [_vp, _i64, _vp, ctypes.c_int, _vp, _vp, _vp]
    lib.bz_axpy.argtypes = [_i64, ctypes.c_double, _vp, _vp, _vp]
    lib.transport_step.argtypes = [_vp, _i64, _vp, _vp, ctypes.c_double, ctypes.POINTER(bz_wall),
                                   ctypes.POINTER(bz_wall), _vp]
    lib.bz_weights_gather.argtypes = [_vp, _i64, _vp, _vp, _vp, _vp]
    lib.bz_plan_items.argtypes = [ctypes.c_int, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp,
                                  _i64, ctypes.POINTER(_i64)]
    lib.bz_plan_mixed_items.argtypes = [ctypes.c_int, _vp, _vp, _vp, ctypes.c_int, _vp, _i64, ctypes.POINTER(_i64)]
    lib.bz_plan_windows.argtypes = [ctypes.c_int, ctypes.c_int, _i64, ctypes.c_int, _vp, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int)]
    ip = ctypes.POINTER(ctypes.c_int)
    lib.bz_plan_small_batch.argtypes = [ctypes.c_int, _i64, ip, ip, ip, ip]
    lib.bz_timing_enable.argtypes = [_vp, ctypes.c_int]
    lib.bz_timing_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]
    wp = ctypes.POINTER(bz_wall)
    lib.bz_strang_step.argtypes = [_vp, _i64, _vp, _vp, ctypes.c_double, ctypes.c_double, wp, wp, _vp]
    lib.bz_graph_capture_strang.argtypes = [_vp, _i64, _vp, _vp, ctypes.c_double, ctypes.c_double, wp, wp,
                                            ctypes.c_int, ctypes.POINTER(_vp)]
    lib.bz_graph_launch.argtypes = [_vp, _vp]
    lib.bz_graph_destroy.argtypes = [_vp]
    lib.bz_autotune_ragged.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _i64, _vp, _vp, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double), _vp]
    lib.collision_eval_ragged.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _i64, _vp, _vp, _vp, _vp,
                                          ctypes.c_int, _vp]
    lib.conserve_ragged.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _i64, _vp, _vp, _vp, ctypes.c_int, _vp,
                                    _vp, _vp]
    lib.bz_set_ragged_form.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _i64, _vp, _vp, ctypes.c_int, ctypes.c_int]
    lib.bz_graph_capture_ragged.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _i64, _vp, _vp, _vp, _vp,
                                            ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.POINTER(_vp)]
    lib.bz_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "bz_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def bz_last_error() -> str:
    return load().bz_last_error().decode()


def _check(rc: int):
    if rc != BZ_OK:
        raise BzError(rc, bz_last_error())


def _ptr(x):
    """Device/host address of a torch tensor, an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dtype_code(t) -> int:
    import torch

    if t.dtype == torch.float64:
        return BZ_F64
    if t.dtype == torch.float32:
        return BZ_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _need(t, numel: int, what: str):
    if not t.is_cuda or not t.is_contiguous() or t.numel() < numel:
        raise ValueError(f"{what} must be a contiguous device tensor with at least {numel} elements")


class Op:
    """Owns a bz_op handle (weights and workspace for one (N, L, lambda, dtype))."""

    def __init__(self, handle: int, N: int, L: float, lam: float, dtype: int):
        self.handle = handle
        self.N, self.L, self.lam, self.dtype = N, L, lam, dtype

    def destroy(self):
        if self.handle:
            _check(load().bz_op_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def bz_op_create(N: int, L: float, lam: float, weight_dtype: int = BZ_F64, omega1d=None) -> Op:
    lib = load()
    h = _vp()
    om = None
    if omega1d is not None:
        om = (ctypes.c_double * N)(*[float(x) for x in omega1d])
    _check(lib.bz_op_create(int(N), float(L), float(lam), int(weight_dtype), om, ctypes.byref(h)))
    return Op(h.value, int(N), float(L), float(lam), int(weight_dtype))


def bz_op_create_inelastic(N: int, L: float, lam: float, beta: float, weight_dtype: int = BZ_F64,
                           omega1d=None) -> Op:
    """Op for inelastic collisions, beta = (1 + e)/2 in [0.5, 1]; its
    projection conserves mass and momentum only."""
    lib = load()
    h = _vp()
    om = None
    if omega1d is not None:
        om = (ctypes.c_double * N)(*[float(x) for x in omega1d])
    _check(lib.bz_op_create_inelastic(int(N), float(L), float(lam), float(beta), int(weight_dtype), om,
                                      ctypes.byref(h)))
    return Op(h.value, int(N), float(L), float(lam), int(weight_dtype))


def bz_op_create_onthefly(N: int, L: float, lam: float, weight_dtype: int = BZ_F64, omega1d=None,
                          slab_bytes: int = 0) -> Op:
    """Op without a stored weight table (lambda 0 or 1): every convolution
    recomputes the weights one slab of output rows at a time into a buffer of
    at most `slab_bytes` (0: the larger of 256 MiB and 1/16 of the table)."""
    lib = load()
    h = _vp()
    om = None
    if omega1d is not None:
        om = (ctypes.c_double * N)(*[float(x) for x in omega1d])
    _check(lib.bz_op_create_onthefly(int(N), float(L), float(lam), int(weight_dtype), om, int(slab_bytes),
                                     ctypes.byref(h)))
    return Op(h.value, int(N), float(L), float(lam), int(weight_dtype))


def bz_op_table_bytes(op: Op) -> int:
    """Device bytes of the op's weights (table, or on-the-fly tables and slab
    buffer) and other create-time tables."""
    b = _i64()
    _check(load().bz_op_table_bytes(op.handle, ctypes.byref(b)))
    return int(b.value)


def bz_op_destroy(op: Op):
    op.destroy()


def bz_op_reserve(op: Op, ncells: int):
    _check(load().bz_op_reserve(op.handle, int(ncells)))


def bz_autotune(op: Op, ncells: int, stream=None):
    """Pick the convolution's work split for batches of `ncells` cells by
    timing the candidates on the device; returns (m1 chunks, k3 ranges,
    ms per launch).  k3 ranges 0 is the small-batch form (at most 64 cells)."""
    S = ctypes.c_int()
    KH = ctypes.c_int()
    ms = ctypes.c_double()
    _check(load().bz_autotune(op.handle, int(ncells), ctypes.byref(S), ctypes.byref(KH), ctypes.byref(ms),
                              _stream(stream)))
    return S.value, KH.value, ms.value


def bz_set_split(op: Op, ncells: int, chunks: int, ranges: int = 1):
    """Fix the convolution's work split (m1 chunks, k3 ranges) for batches of
    `ncells` cells; ranges = 0 selects the small-batch form (at most 64
    cells)."""
    _check(load().bz_set_split(op.handle, int(ncells), int(chunks), int(ranges)))


def bz_get_split(op: Op, ncells: int):
    """(m1 chunks, k3 ranges) the op uses for batches of `ncells` cells (k3
    ranges 0: the small-batch form)."""
    S = ctypes.c_int()
    KH = ctypes.c_int()
    _check(load().bz_get_split(op.handle, int(ncells), ctypes.byref(S), ctypes.byref(KH)))
    return S.value, KH.value


def bz_set_memory_cap(nbytes: int):
    _check(load().bz_set_memory_cap(int(nbytes)))


def collision_eval(op: Op, ncells: int, f, Qt, dtype: int | None = None, stream=None):
    """Q~ (unprojected) for `ncells` cells: f, Qt device tensors [ncells, N, N, N]."""
    n3 = op.N ** 3
    if ncells > 0:
        _need(f, ncells * n3, "f")
        _need(Qt, ncells * n3, "Qt")
    dt = _dtype_code(f) if dtype is None else int(dtype)
    _check(load().collision_eval(op.handle, int(ncells), _ptr(f), _ptr(Qt), dt, _stream(stream)))


NOALLOC_MAX_CELLS = 64


def collision_eval_noalloc(op: Op, ncells: int, f, Qt, dtype: int | None = None, stream=None):
    """collision_eval with no device allocation (at most 64 cells; the
    library's fixed 64 MiB array per GPU as workspace; overlapping calls on
    one GPU race)."""
    n3 = op.N ** 3
    if ncells > 0:
        _need(f, ncells * n3, "f")
        _need(Qt, ncells * n3, "Qt")
    dt = _dtype_code(f) if dtype is None else int(dtype)
    _check(load().collision_eval_noalloc(op.handle, int(ncells), _ptr(f), _ptr(Qt), dt, _stream(stream)))


def conserve(op: Op, ncells: int, Qt, Qc, moments=None, in_dtype: int | None = None, stream=None):
    """FP64 conservation projection: Qc = Q~ - C^T (C C^T)^{-1} C Q~."""
    n3 = op.N ** 3
    if ncells > 0:
        _need(Qt, ncells * n3, "Qt")
        _need(Qc, ncells * n3, "Qc")
        if moments is not None:
            _need(moments, ncells * 5, "moments")
    dt = _dtype_code(Qt) if in_dtype is None else int(in_dtype)
    _check(load().conserve(op.handle, int(ncells), _ptr(Qt), dt, _ptr(Qc), _ptr(moments), _stream(stream)))


def bz_axpy(alpha: float, x, y, stream=None):
    """y += alpha x (FP64 device tensors)."""
    if x.numel() != y.numel():
        raise ValueError("x and y differ in size")
    _check(load().bz_axpy(int(x.numel()), float(alpha), _ptr(x), _ptr(y), _stream(stream)))


def _wall(w) -> bz_wall:
    kind, Tw, Vw = w
    return bz_wall(int(kind), float(Tw), (ctypes.c_double * 3)(*[float(v) for v in Vw]))


def transport_step(op: Op, ncells: int, f, x_faces, dt: float,
                   left=(BZ_WALL_DIFFUSE, 1.0, (0.0, 0.0, 0.0)),
                   right=(BZ_WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0)), stream=None):
    """One Heun step of 1-D FV transport in place: f [ncells + 4, N, N, N] FP64."""
    _need(f, (ncells + 4) * op.N ** 3, "f")
    _need(x_faces, ncells + 1, "x_faces")
    lw, rw = _wall(left), _wall(right)
    _check(load().transport_step(op.handle, int(ncells), _ptr(f), _ptr(x_faces), float(dt),
                                 ctypes.byref(lw), ctypes.byref(rw), _stream(stream)))


def bz_weights_gather(op: Op, k_lin, m_lin, out, stream=None):
    """out[i] = W[k_lin[i]][m_lin[i]] as FP64 (device int32 / float64 tensors)."""
    n = int(k_lin.numel())
    _check(load().bz_weights_gather(op.handle, n, _ptr(k_lin), _ptr(m_lin), _ptr(out), _stream(stream)))


def bz_plan_items(N: int, ncells: int, chunks: int, ranges: int = 1, row0: int = 0, row1: int | None = None):
    """Convolution items of one launch (host only): int32 array [count, 5] of
    (row, chunk, group, k3 range, op), rows of -1 padding, in launch order."""
    import numpy as np

    lib = load()
    row1 = N * N if row1 is None else row1
    n = _i64()
    _check(lib.bz_plan_items(int(N), int(ncells), int(chunks), int(ranges), int(row0), int(row1), None, 0,
                             ctypes.byref(n)))
    out = np.zeros((n.value, 5), dtype=np.int32)
    _check(lib.bz_plan_items(int(N), int(ncells), int(chunks), int(ranges), int(row0), int(row1), out.ctypes.data,
                             n.value, ctypes.byref(n)))
    return out


def bz_plan_mixed_items(Ns, ncells, chunks, f64: bool):
    """Items of the one-launch convolution of a ragged batch (host only)."""
    import numpy as np

    lib = load()
    a = np.ascontiguousarray(Ns, dtype=np.int32)
    b = np.ascontiguousarray(ncells, dtype=np.int64)
    c = np.ascontiguousarray(chunks, dtype=np.int32)
    n = _i64()
    _check(lib.bz_plan_mixed_items(len(a), a.ctypes.data, b.ctypes.data, c.ctypes.data, int(bool(f64)), None, 0,
                                   ctypes.byref(n)))
    out = np.zeros((n.value, 5), dtype=np.int32)
    _check(lib.bz_plan_mixed_items(len(a), a.ctypes.data, b.ctypes.data, c.ctypes.data, int(bool(f64)),
                                   out.ctypes.data, n.value, ctypes.byref(n)))
    return out


def bz_plan_windows(N: int, weight_dtype: int, max_bytes: int, min_rows: int = 1):
    """Row boundaries of the convolution launches for weights split at
    max_bytes and merged to at least min_rows rows per launch (host only)."""
    import numpy as np

    lib = load()
    n = ctypes.c_int()
    _check(lib.bz_plan_windows(int(N), int(weight_dtype), int(max_bytes), int(min_rows), None, 0, ctypes.byref(n)))
    out = np.zeros(n.value, dtype=np.int32)
    _check(lib.bz_plan_windows(int(N), int(weight_dtype), int(max_bytes), int(min_rows), out.ctypes.data, n.value,
                               ctypes.byref(n)))
    return out


def bz_plan_small_batch(N: int, ncells: int):
    """(cells per block, blocks, default m1 chunks, is the default form) of
    the small-batch convolution for `ncells` cells (host only)."""
    lib = load()
    cb, nb, ch, dflt = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib.bz_plan_small_batch(int(N), int(ncells), ctypes.byref(cb), ctypes.byref(nb), ctypes.byref(ch),
                                   ctypes.byref(dflt)))
    return cb.value, nb.value, ch.value, bool(dflt.value)


def bz_timing_enable(op: Op, on: bool = True):
    """Bracket every convolution launch of collision_eval with HIP events."""
    _check(load().bz_timing_enable(op.handle, 1 if on else 0))


def bz_timing_read(op: Op):
    """(summed convolution kernel time in ms, launches) since the last read."""
    ms = ctypes.c_double()
    n = _i64()
    _check(load().bz_timing_read(op.handle, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def bz_strang_step(op: Op, ncells: int, f, x_faces, dt: float, eps: float,
                   left=(BZ_WALL_DIFFUSE, 1.0, (0.0, 0.0, 0.0)),
                   right=(BZ_WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0)), stream=None):
    """One Strang step (transport dt/2, Heun collision dt, transport dt/2) in place:
    f [ncells + 4, N, N, N] FP64 with ghosts."""
    _need(f, (ncells + 4) * op.N ** 3, "f")
    _need(x_faces, ncells + 1, "x_faces")
    lw, rw = _wall(left), _wall(right)
    _check(load().bz_strang_step(op.handle, int(ncells), _ptr(f), _ptr(x_faces), float(dt), float(eps),
                                 ctypes.byref(lw), ctypes.byref(rw), _stream(stream)))


class Graph:
    """An instantiated HIP graph: captured Strang steps, or one step of a ragged batch."""

    def __init__(self, handle: int):
        self.handle = handle

    def launch(self, stream=None):
        _check(load().bz_graph_launch(self.handle, _stream(stream)))

    def destroy(self):
        if self.handle:
            _check(load().bz_graph_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def bz_graph_capture_strang(op: Op, ncells: int, f, x_faces, dt: float, eps: float, nsteps: int,
                            left=(BZ_WALL_DIFFUSE, 1.0, (0.0, 0.0, 0.0)),
                            right=(BZ_WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))) -> Graph:
    """Capture `nsteps` Strang steps on f (fixed pointers) into a HIP graph."""
    _need(f, (ncells + 4) * op.N ** 3, "f")
    _need(x_faces, ncells + 1, "x_faces")
    lw, rw = _wall(left), _wall(right)
    h = _vp()
    _check(load().bz_graph_capture_strang(op.handle, int(ncells), _ptr(f), _ptr(x_faces), float(dt), float(eps),
                                          ctypes.byref(lw), ctypes.byref(rw), int(nsteps), ctypes.byref(h)))
    return Graph(h.value)


def _ops_array(ops):
    arr = (_vp * len(ops))(*[o.handle for o in ops])
    return arr


def collision_eval_ragged(ops, op_of_cell, offset_of_cell, f, Qt, dtype: int, stream=None):
    """Mixed-N batch: cell c uses ops[op_of_cell[c]] and starts at element
    offset_of_cell[c] of the packed device buffers f and Qt (host index arrays)."""
    import numpy as np

    oc = np.ascontiguousarray(op_of_cell, dtype=np.int32)
    of = np.ascontiguousarray(offset_of_cell, dtype=np.int64)
    if oc.shape != of.shape:
        raise ValueError("op_of_cell and offset_of_cell differ in length")
    _check(load().collision_eval_ragged(_ops_array(ops), len(ops), int(oc.size), oc.ctypes.data, of.ctypes.data,
                                        _ptr(f), _ptr(Qt), int(dtype), _stream(stream)))


def bz_autotune_ragged(ops, op_of_cell, offset_of_cell, dtype: int, stream=None):
    """Time the one-launch and the per-op convolution of this ragged layout and
    keep the faster; returns (one_launch 1/0, ms one launch, ms per-op)."""
    import numpy as np

    oc = np.ascontiguousarray(op_of_cell, dtype=np.int32)
    of = np.ascontiguousarray(offset_of_cell, dtype=np.int64)
    if oc.shape != of.shape:
        raise ValueError("op_of_cell and offset_of_cell differ in length")
    one, t1, t0 = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    _check(load().bz_autotune_ragged(_ops_array(ops), len(ops), int(oc.size), oc.ctypes.data, of.ctypes.data,
                                     int(dtype), ctypes.byref(one), ctypes.byref(t1), ctypes.byref(t0),
                                     _stream(stream)))
    return one.value, t1.value, t0.value


def _ragged_index(op_of_cell, offset_of_cell):
    import numpy as np

    oc = np.ascontiguousarray(op_of_cell, dtype=np.int32)
    of = np.ascontiguousarray(offset_of_cell, dtype=np.int64)
    if oc.shape != of.shape:
        raise ValueError("op_of_cell and offset_of_cell differ in length")
    return oc, of


def bz_set_ragged_form(ops, op_of_cell, offset_of_cell, dtype: int, one_launch: int):
    """Pin the convolution form (1 one launch, 0 per-op launches) of this ragged layout."""
    oc, of = _ragged_index(op_of_cell, offset_of_cell)
    _check(load().bz_set_ragged_form(_ops_array(ops), len(ops), int(oc.size), oc.ctypes.data, of.ctypes.data,
                                     int(dtype), int(one_launch)))


def bz_graph_capture_ragged(ops, op_of_cell, offset_of_cell, f, Qt, Qc, dtype: int, moments=None,
                            form: int = -1) -> Graph:
    """Capture collision_eval_ragged + conserve_ragged of this layout into a
    HIP graph (form 1 one launch, 0 per-op launches, -1 the layout's choice)."""
    oc, of = _ragged_index(op_of_cell, offset_of_cell)
    h = _vp()
    _check(load().bz_graph_capture_ragged(_ops_array(ops), len(ops), int(oc.size), oc.ctypes.data, of.ctypes.data,
                                          _ptr(f), _ptr(Qt), int(dtype), _ptr(Qc), _ptr(moments), int(form),
                                          ctypes.byref(h)))
    return Graph(h.value)


def conserve_ragged(ops, op_of_cell, offset_of_cell, Qt, Qc, moments=None, in_dtype: int | None = None,
                    stream=None):
    """FP64 projection of a packed mixed-N batch (same layout as collision_eval_ragged)."""
    import numpy as np

    oc = np.ascontiguousarray(op_of_cell, dtype=np.int32)
    of = np.ascontiguousarray(offset_of_cell, dtype=np.int64)
    dt = _dtype_code(Qt) if in_dtype is None else int(in_dtype)
    _check(load().conserve_ragged(_ops_array(ops), len(ops), int(oc.size), oc.ctypes.data, of.ctypes.data,
                                  _ptr(Qt), dt, _ptr(Qc), _ptr(moments), _stream(stream)))
