"""Weights computed on the fly (the memory remedy of the paper's Conclusions):
an op without the stored O(N^6) table recomputes the weights, one slab of
output rows at a time, inside every convolution.  Same bars as the stored
path against the FP64 oracle (1e-12 relative L2 per cell in FP64, 1e-5 in
FP32); the slab size changes nothing, bit for bit.
"""
import math
import sys

import numpy as np
import pytest

import synth
from tests.gpu_util import f32_check, f32_report, rel_l2_per_cell, to_dev, to_host

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


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


def _collide(bz, op, f, dtype):
    import torch

    td = torch.float64 if dtype == bz.BZ_F64 else torch.float32
    fd = to_dev(f, td)
    qt = torch.empty_like(fd)
    bz.collision_eval(op, f.shape[0], fd, qt)
    return to_host(qt).astype(np.float64)


def _row_lengths(N):
    """Stored weights of each output row (k1, k2): kept half of the mirrored
    lines (m1, m2) times the 3N^2/4 (k3, m3) pairs of a line."""
    def count(k):
        return min(k + N // 2, N - 1) - max(k - N // 2 + 1, 0) + 1

    out = []
    for k1 in range(N):
        for k2 in range(N):
            c1, c2 = count(k1), count(k2)
            out.append(((c1 // 2) * c2 + ((c2 + 1) // 2 if c1 % 2 else 0)) * 3 * N * N // 4)
    return np.array(out)


@pytest.mark.parametrize("N", [8, 16, 24, 32])
@pytest.mark.parametrize("lam", [0, 1])
def test_onthefly_weights_match_oracle(bz, orc, N, lam):
    """The weights as the on-the-fly evaluation forms them (gathered through
    the same device function), against the oracle's closed forms, at random
    pairs and at every limiting branch (A = 0, B = 0, p = 0, Cm = 0)."""
    import torch

    _note(f"on-the-fly weights N={N} lam={lam}")
    L = 6.0
    c = N // 2
    rng = np.random.default_rng(300 + N + lam)
    ks, ms = [], []
    while len(ks) < 400:
        k = rng.integers(0, N, 3)
        m = rng.integers(0, N, 3)
        if np.all((k - m + c >= 0) & (k - m + c < N)):
            ks.append(k)
            ms.append(m)
    ks += [np.array([c, c, c]), np.array([c + 2, c, c - 2]), np.array([c + 2, c, c]), np.array([c + 3, c - 1, c + 1])]
    ms += [np.array([c + 1, c, c]), np.array([c + 1, c, c - 1]), np.array([c + 1, c + 1, c]), np.array([c, c, c])]
    ks.append(np.array([0, c, c]))  # outside the truncation box -> 0
    ms.append(np.array([N - 1, c, c]))
    lin = lambda a: (a[0] * N + a[1]) * N + a[2]
    kl = np.array([lin(k) for k in ks], dtype=np.int32)
    ml = np.array([lin(m) for m in ms], dtype=np.int32)
    dz3 = (math.pi / L) ** 3

    def stored(k, m):
        n = np.asarray(k) - np.asarray(m) + c
        w = dz3 * orc.ghat(N, L, lam, k, m)
        if not (n[0] == m[0] and n[1] == m[1]):
            w += dz3 * orc.ghat(N, L, lam, k, n)
        return w

    ref = np.array([stored(k, m) for k, m in zip(ks, ms)])
    ref[-1] = 0.0
    scale = np.abs(ref).max()
    for wd, tol in ((bz.BZ_F64, 1e-13), (bz.BZ_F32, 1e-7)):
        with bz.bz_op_create_onthefly(N, L, lam, wd) as op:
            out = torch.empty(len(kl), dtype=torch.float64, device="cuda")
            bz.bz_weights_gather(op, to_dev(kl), to_dev(ml), out)
            got = to_host(out)
        err = np.abs(got - ref)
        ok = bool(np.all(err <= tol * np.maximum(np.abs(ref), 1e-3 * scale)))
        assert ok, (wd, float(err.max()), int(np.argmax(err)))
        assert got[-1] == 0.0 and got[len(ks) - 5] == 0.0


@pytest.mark.parametrize("N,ncells,lam,nslab,sample", [
    (8, 3, 0, 3, [0, 1, 2]),
    (16, 70, 1, 5, [0, 37, 69]),
    (24, 67, 1, 4, [66]),
    (32, 65, 1, 6, [64]),
    (32, 1, 1, 6, [0]),  # one cell: the unpadded workspace, slabs on two streams
])
def test_onthefly_collision_matches_oracle_and_stored(bz, orc, N, ncells, lam, nslab, sample):
    """Q~ of an on-the-fly op, its weights recomputed in about `nslab` slabs:
    sampled cells against the oracle (1e-12), every cell against the stored
    table's op (the same sums; only the weights' last bits differ), and bit
    for bit equal to a one-slab on-the-fly op."""
    _note(f"on-the-fly collision N={N} ncells={ncells} lam={lam} slabs~{nslab}")
    L = 6.0
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(400 + N))
    rows = _row_lengths(N)
    slab = int(max(rows.max(), -(-rows.sum() // nslab))) * 8
    with bz.bz_op_create_onthefly(N, L, lam, bz.BZ_F64, slab_bytes=slab) as op:
        many = _collide(bz, op, f, bz.BZ_F64)
    with bz.bz_op_create_onthefly(N, L, lam, bz.BZ_F64, slab_bytes=int(rows.sum()) * 8) as op:
        one = _collide(bz, op, f, bz.BZ_F64)
    with bz.bz_op_create(N, L, lam, bz.BZ_F64) as op:
        stored = _collide(bz, op, f, bz.BZ_F64)
    assert np.array_equal(many, one)
    assert rel_l2_per_cell(many, stored).max() <= 1e-13
    ref = orc.collision(N, L, lam, f[sample])
    err = rel_l2_per_cell(many[sample], ref)
    assert err.max() <= F64_TOL, err.max()


def test_onthefly_f32_within_bound(bz, orc):
    """FP32 path (weights computed in FP64 and rounded to FP32, FP32 f^ and
    products, FP64 line sums) of an on-the-fly op, three slabs, every cell
    within the FP32 bound of the FP64 oracle on the same input."""
    _note("on-the-fly f32 N=16")
    N, L, ncells = 16, 6.0, 40
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(450))
    rows = _row_lengths(N)
    with bz.bz_op_create_onthefly(N, L, 1, bz.BZ_F32, slab_bytes=int(-(-rows.sum() // 3)) * 4) as op:
        got = _collide(bz, op, f, bz.BZ_F32)
    err, floor, ok = f32_check(orc, N, L, 1, f, got)
    _note("  " + f32_report(err, floor, ok))
    assert ok.all(), f32_report(err, floor, ok)


def test_onthefly_nonuniform_trapezoid_weights(bz):
    """Per-dimension trapezoid weights (end points halved) enter the
    on-the-fly weights as they enter the stored table."""
    N, L = 8, 6.0
    dz = math.pi / L
    om = [dz] * N
    om[0] = om[-1] = 0.5 * dz
    f = synth.two_maxwellian(N, L, 5, synth.seed_for(460))
    with bz.bz_op_create_onthefly(N, L, 1, bz.BZ_F64, omega1d=om, slab_bytes=200000) as op:
        fly = _collide(bz, op, f, bz.BZ_F64)
    with bz.bz_op_create(N, L, 1, bz.BZ_F64, omega1d=om) as op:
        stored = _collide(bz, op, f, bz.BZ_F64)
    with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
        uniform = _collide(bz, op, f, bz.BZ_F64)
    assert rel_l2_per_cell(fly, stored).max() <= 1e-13
    assert rel_l2_per_cell(uniform, stored).min() > 1e-6  # the weights do matter


def test_onthefly_memory_and_errors(bz):
    """The op holds a slab, not the table; slab and exponent limits are
    reported as errors."""
    N, L = 16, 6.0
    total = int(_row_lengths(N).sum()) * 8
    with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
        held_stored = bz.bz_op_table_bytes(op)
    with bz.bz_op_create_onthefly(N, L, 1, bz.BZ_F64, slab_bytes=total // 8) as op:
        held_fly = bz.bz_op_table_bytes(op)
    assert held_stored >= total
    assert held_fly <= 2 * (total // 8) + 200000  # two slab buffers (eight slabs)
    for lam, slab, code in ((0.5, 0, bz.BZ_EUNSUPPORTED), (1, 1000, bz.BZ_EINVAL), (1, -1, bz.BZ_EINVAL)):
        with pytest.raises(bz.BzError) as e:
            bz.bz_op_create_onthefly(N, L, lam, bz.BZ_F64, slab_bytes=slab)
        assert e.value.code == code


def test_onthefly_autotune_and_graph_replay(bz):
    """The work-split trials and the captured Strang step run the slab
    sequence too: results after autotuning stay within rounding of the stored
    op's, and a graph of two steps replays bit for bit like the eager steps."""
    N, L, M, lam, eps = 8, 8.0, 24, 1, 0.1
    xf = synth.boundary_layer_faces(M, X=4.0)
    f0 = synth.boundary_layer_state(N, L, M)
    left = (bz.BZ_WALL_DIFFUSE, 2.0, (0.0, 0.0, 0.0))
    right = (bz.BZ_WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))
    dt = 0.5 * np.diff(xf).min() / L
    f = synth.two_maxwellian(N, L, 100, synth.seed_for(470))
    with bz.bz_op_create(N, L, lam, bz.BZ_F64) as op:
        stored = _collide(bz, op, f, bz.BZ_F64)
    with bz.bz_op_create_onthefly(N, L, lam, bz.BZ_F64, slab_bytes=100000) as op:
        S, KH, ms = bz.bz_autotune(op, 100)
        assert ms > 0.0
        fly = _collide(bz, op, f, bz.BZ_F64)
        assert rel_l2_per_cell(fly, stored).max() <= 1e-13
        xd = to_dev(xf)
        fd = to_dev(f0)
        eager = []
        for _ in range(2):
            bz.bz_strang_step(op, M, fd, xd, dt, eps, left, right)
        eager = to_host(fd).copy()
        gd = to_dev(f0)
        with bz.bz_graph_capture_strang(op, M, gd, xd, dt, eps, 2, left, right) as g:
            g.launch()
            first = to_host(gd).copy()
    assert np.array_equal(first, eager)
