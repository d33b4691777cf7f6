"""collision_eval_noalloc: the collision evaluation for callers that cannot
allocate device memory, against collision_eval (the same Q~: FP64 within
1e-12 relative L2 per cell, bit for bit where both use the same small-batch
split; FP32 within the stated bound) on two calls in a row, the second with a
smaller batch, and against the oracle on sampled cells."""
import sys

import numpy as np
import pytest

import synth
from tests.gpu_util import f32_check, f32_report, rel_l2_per_cell, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bz():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1301_4195_amd as bz

    bz.load()  # raises if libbz.so is missing: no fallback
    return bz


def _note(msg):
    print(msg, file=sys.stderr, flush=True)


def _eval(bz, op, f, dtype, noalloc):
    import torch

    td = torch.float64 if dtype == bz.BZ_F64 else torch.float32
    fd = to_dev(f, td)
    qt = torch.full_like(fd, float("nan"))
    (bz.collision_eval_noalloc if noalloc else bz.collision_eval)(op, f.shape[0], fd, qt)
    return to_host(qt).astype(np.float64)


# (N, dtype, first batch, second smaller batch, bitwise): bitwise where both
# entry points use the small-batch form at the same split (the default up to
# 32 cells at N <= 16 and 16 above, when the chunks fit the array)
CASES = [(16, "f64", 29, 7, True), (8, "f64", 64, 1, False), (24, "f64", 16, 3, True), (32, "f64", 5, 2, False),
         (16, "f32", 64, 33, False), (24, "f32", 13, 2, True)]


@pytest.mark.parametrize("N,dt,n1,n2,bitwise", CASES)
def test_noalloc_matches_collision_eval(bz, orc, N, dt, n1, n2, bitwise):
    L = 6.0
    code = bz.BZ_F64 if dt == "f64" else bz.BZ_F32
    f1 = synth.two_maxwellian(N, L, n1, synth.seed_for(700 + N))
    f2 = synth.two_maxwellian(N, L, n2, synth.seed_for(800 + N))
    _note(f"noalloc N={N} {dt}: {n1} then {n2} cells")
    with bz.bz_op_create(N, L, 1, code) as op:
        a1 = _eval(bz, op, f1, code, True)
        a2 = _eval(bz, op, f2, code, True)
        b1 = _eval(bz, op, f1, code, False)
        b2 = _eval(bz, op, f2, code, False)
    for a, b, f in ((a1, b1, f1), (a2, b2, f2)):
        assert np.all(np.isfinite(a))
        if bitwise:
            assert np.array_equal(a, b)
        if dt == "f64":
            assert rel_l2_per_cell(a, b).max() <= 1e-12
            s = [0, f.shape[0] - 1]
            assert rel_l2_per_cell(a[s], orc.collision(N, L, 1, f[s])).max() <= 1e-12
        else:  # each FP32 result within the stated bound of the oracle (two
            # FP32 sums in different orders may differ by twice that)
            s = list(range(0, f.shape[0], max(1, f.shape[0] // 16)))
            err, floor, ok = f32_check(orc, N, L, 1, f[s], a[s])
            assert ok.all(), f32_report(err, floor, ok, s)


def test_noalloc_on_the_fly_op(bz, orc):
    """An op whose weights are computed on the fly (three slabs, recomputed
    into the op's own slab buffer before each slab's rows)."""
    N, L = 16, 6.0
    f = synth.two_maxwellian(N, L, 5, synth.seed_for(720))
    with bz.bz_op_create_onthefly(N, L, 1, bz.BZ_F64, slab_bytes=10 << 20) as op:
        a = _eval(bz, op, f, bz.BZ_F64, True)
        b = _eval(bz, op, f, bz.BZ_F64, False)
    assert rel_l2_per_cell(a, b).max() <= 1e-12
    assert rel_l2_per_cell(a, orc.collision(N, L, 1, f)).max() <= 1e-12


def test_noalloc_allocates_nothing_and_rejects_what_does_not_fit(bz):
    """After the first call on the device (which loads the array), further
    calls of other sizes leave the device's free memory unchanged; more than
    64 cells, and a mesh whose one-chunk workspace exceeds the array, are
    rejected before any device work."""
    import torch

    N, L = 16, 6.0
    f = to_dev(synth.two_maxwellian(N, L, 64, synth.seed_for(730)))
    qt = torch.empty_like(f)
    with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
        bz.collision_eval_noalloc(op, 3, f, qt)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for n in (64, 1, 17, 40):
            bz.collision_eval_noalloc(op, n, f, qt)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        with pytest.raises(bz.BzError):
            bz.collision_eval_noalloc(op, 65, torch.empty(65 * N ** 3, dtype=torch.float64, device="cuda"),
                                      torch.empty(65 * N ** 3, dtype=torch.float64, device="cuda"))
    with bz.bz_op_create_onthefly(48, L, 1, bz.BZ_F64, slab_bytes=64 << 20) as op48:
        x = torch.zeros(48 ** 3, dtype=torch.float64, device="cuda")
        with pytest.raises(bz.BzError):
            bz.collision_eval_noalloc(op48, 1, x, torch.empty_like(x))
