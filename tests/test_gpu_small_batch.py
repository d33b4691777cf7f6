"""The small-batch convolution (one cell up to one group of 64 cells; the
default up to 32 cells at N <= 16, 16 above): lanes over (k3, m3 residue)
with the weights read as a coalesced stream and applied to a block of
cells.  Same bars as the batched
kernel against the FP64 oracle (1e-12 relative L2 per cell in FP64, the
stated FP32 bound), agreement with the batched kernel within rounding, block
boundaries inside a batch, weights computed on the fly in slabs (bit for bit
independent of the slab size), and a captured Strang step.
"""
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


@pytest.mark.parametrize("N,ncells,lam,sample", [
    (8, 1, 0, [0]),
    (8, 11, 1, list(range(11))),
    (16, 1, 1, [0]),
    (16, 13, 1, list(range(13))),  # two blocks of 8 cells, the second ragged
    (24, 3, 1, [0, 2]),
    (32, 1, 1, [0]),
    (32, 6, 1, [5]),               # two blocks of 4 cells
])
def test_small_batch_matches_oracle(bz, orc, N, ncells, lam, sample):
    """The default form for these batch sizes is the small-batch one; its
    result matches the oracle on the sampled cells."""
    _note(f"small batch N={N} ncells={ncells} lam={lam}")
    L = 6.0
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(500 + N + ncells))
    with bz.bz_op_create(N, L, lam, bz.BZ_F64) as op:
        assert bz.bz_get_split(op, ncells)[1] == 0
        got = _collide(bz, op, f, bz.BZ_F64)
        again = _collide(bz, op, f, bz.BZ_F64)
    assert np.array_equal(got, again)
    ref = orc.collision(N, L, lam, f[sample])
    err = rel_l2_per_cell(got[sample], ref)
    assert err.max() <= F64_TOL, err.max()


@pytest.mark.parametrize("N,ncells,chunks", [(16, 40, [1, 3, 5]), (16, 64, [2]), (24, 9, [1, 7]), (32, 17, [1, 9]),
                                             (8, 64, [3])])
def test_small_form_agrees_with_batched_form(bz, N, ncells, chunks):
    """Forced with bz_set_split (ranges = 0), the small-batch form at every
    chunk count gives the batched kernel's result within rounding, up to a
    full group of 64 cells."""
    _note(f"small vs batched N={N} ncells={ncells} chunks={chunks}")
    L = 6.0
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(520 + N))
    with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
        bz.bz_set_split(op, ncells, 2, 2 if N >= 32 else 1)
        batched = _collide(bz, op, f, bz.BZ_F64)
        for S in chunks:
            bz.bz_set_split(op, ncells, S, 0)
            assert bz.bz_get_split(op, ncells) == (S, 0)
            small = _collide(bz, op, f, bz.BZ_F64)
            assert rel_l2_per_cell(small, batched).max() <= 1e-13, S


@pytest.mark.parametrize("N,ncells", [(16, 7), (32, 3), (32, 1)])
def test_small_batch_f32_within_bound(bz, orc, N, ncells):
    """FP32 weights, f^ and products (each line's partial folded into an
    FP64 sum), every cell within the stated FP32 bound (one cell at N = 32:
    the passes and the convolution on the unpadded workspace)."""
    _note(f"small batch f32 N={N} ncells={ncells}")
    L = 6.0
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(540 + N))
    with bz.bz_op_create(N, L, 1, bz.BZ_F32) as op:
        assert bz.bz_get_split(op, ncells)[1] == 0
        got = _collide(bz, op, f, bz.BZ_F32)
    sample = list(range(ncells)) if N <= 16 else [ncells - 1]
    err, floor, ok = f32_check(orc, N, L, 1, f[sample], got[sample])
    _note("  " + f32_report(err, floor, ok, sample))
    assert ok.all(), f32_report(err, floor, ok, sample)


def _lines_per_row(N):
    def count(k):
        return min(k + N // 2, N - 1) - max(k - N // 2 + 1, 0) + 1

    out = []
    for k1 in range(N):
        for k2 in range(N):
            c1, c2 = count(k1), count(k2)
            out.append(((c1 // 2) * c2 + ((c2 + 1) // 2 if c1 % 2 else 0)) * 3 * N * N // 4)
    return np.array(out)


def test_small_batch_weights_on_the_fly(bz):
    """An on-the-fly op in about five slabs (two buffers on two streams) runs
    the small-batch form slab by slab: bit for bit equal to one slab, and
    within rounding of the stored table's op."""
    N, L, n = 32, 6.0, 5
    f = synth.two_maxwellian(N, L, n, synth.seed_for(560))
    rows = _lines_per_row(N)
    with bz.bz_op_create_onthefly(N, L, 1, bz.BZ_F64, slab_bytes=int(-(-rows.sum() // 5)) * 8) as op:
        assert bz.bz_get_split(op, n)[1] == 0
        many = _collide(bz, op, f, bz.BZ_F64)
    with bz.bz_op_create_onthefly(N, L, 1, bz.BZ_F64, slab_bytes=int(rows.sum()) * 8) as op:
        one = _collide(bz, op, f, bz.BZ_F64)
    with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
        stored = _collide(bz, op, f, bz.BZ_F64)
    assert np.array_equal(many, one)
    assert rel_l2_per_cell(many, stored).max() <= 1e-13


def test_small_batch_autotune_and_graph_replay(bz, orc):
    """Ten cells of the boundary layer: bz_autotune chooses among both forms,
    and a captured graph of two Strang steps replays like the eager steps
    (bit for bit) and matches the oracle's composition of the same steps."""
    import torch

    N, L, M, lam, eps = 8, 8.0, 10, 1, 0.1
    xf = synth.boundary_layer_faces(M, X=1.0)
    f0 = synth.boundary_layer_state(N, L, M)
    left = (bz.BZ_WALL_DIFFUSE, 2.0, (0.0, 0.0, 0.0))
    right = (bz.BZ_WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))
    dt = 0.5 * float(np.diff(xf).min()) / L
    with bz.bz_op_create(N, L, lam, bz.BZ_F64) as op:
        S, KH, ms = bz.bz_autotune(op, M)
        assert KH in (0, 1, 2, 4) and ms > 0.0
        _note(f"small batch graph: autotuned split ({S}, {KH})")
        xd = to_dev(xf)
        fd = to_dev(f0)
        for _ in range(2):
            bz.bz_strang_step(op, M, fd, xd, dt, eps, left, right)
        eager = to_host(fd).copy()
        gd = to_dev(f0)
        with bz.bz_graph_capture_strang(op, M, gd, xd, dt, eps, 2, left, right) as g:
            g.launch()
            first = to_host(gd).copy()
            gd.copy_(torch.from_numpy(f0).to(gd.device))
            g.launch()
            second = to_host(gd).copy()
    assert np.array_equal(first, eager) and np.array_equal(second, eager)
    ref = f0.copy()
    for _ in range(2):
        ref = orc.transport_step(N, L, ref, xf, 0.5 * dt, left=left, right=right)
        fi = ref[2:-2]
        q1, _ = orc.project(N, L, orc.collision(N, L, lam, fi))
        fs = fi + dt / eps * q1
        q2, _ = orc.project(N, L, orc.collision(N, L, lam, fs))
        ref = ref.copy()
        ref[2:-2] = fi + 0.5 * dt / eps * (q1 + q2)
        ref = orc.transport_step(N, L, ref, xf, 0.5 * dt, left=left, right=right)
    err = np.abs(first - ref).max() / np.abs(ref).max()
    assert err <= 1e-12, err


def test_small_batch_in_a_ragged_batch(bz, orc):
    """A packed batch of eight cells on four meshes (one op computing its
    weights on the fly, so the ragged call runs each mesh's cells on that
    mesh's op): every mesh takes the small-batch form, and each cell equals
    its op's own collision_eval bit for bit; one cell per mesh against the
    oracle."""
    import torch

    L = 6.0
    Ns = [8, 16, 24, 32]
    counts = [3, 2, 1, 2]
    order = [0, 1, 3, 0, 2, 1, 3, 0]  # op of each packed cell, interleaved
    fs_by = {j: synth.two_maxwellian(Ns[j], L, counts[j], synth.seed_for(580 + j)) for j in range(4)}
    taken = {j: 0 for j in range(4)}
    cells = []
    for j in order:
        cells.append((j, taken[j]))
        taken[j] += 1
    op_of = np.array([j for j, _ in cells], dtype=np.int32)
    sizes = np.array([Ns[j] ** 3 for j in op_of], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.concatenate([fs_by[j][t].ravel() for j, t in cells])
    ops = [bz.bz_op_create(8, L, 1, bz.BZ_F64), bz.bz_op_create_onthefly(16, L, 1, bz.BZ_F64),
           bz.bz_op_create(24, L, 1, bz.BZ_F64), bz.bz_op_create(32, L, 1, bz.BZ_F64)]
    try:
        for j in range(4):
            assert bz.bz_get_split(ops[j], counts[j])[1] == 0
        fd = to_dev(flat)
        qd = torch.empty_like(fd)
        bz.collision_eval_ragged(ops, op_of, offs, fd, qd, bz.BZ_F64)
        got = to_host(qd)
        for j in range(4):
            dense = _collide(bz, ops[j], fs_by[j], bz.BZ_F64)
            for i, (jj, t) in enumerate(cells):
                if jj == j:
                    assert np.array_equal(got[offs[i]:offs[i] + Ns[j] ** 3], dense[t].ravel()), (Ns[j], i)
            ref = orc.collision(Ns[j], L, 1, fs_by[j][-1:])
            assert rel_l2_per_cell(dense[-1:], ref).max() <= F64_TOL, Ns[j]
    finally:
        for o in ops:
            o.destroy()


@pytest.mark.parametrize("N", [8, 16])
def test_one_cell_kernel_every_split(bz, orc, N):
    """One cell per call at N <= 16 runs the one-cell convolution (every
    workgroup's weight loads in flight together, unpadded workspace) at 2 or
    more m1 chunks and the small-batch kernel at one: every split, FP64 and
    FP32, against the oracle."""
    import torch

    L = 6.0
    f = synth.two_maxwellian(N, L, 1, synth.seed_for(560 + N))
    ref = orc.collision(N, L, 1, f)
    for dt in (bz.BZ_F64, bz.BZ_F32):
        with bz.bz_op_create(N, L, 1, dt) as op:
            S_max = (N // 2 + 2) // 2
            for S in range(1, S_max + 1):
                _note(f"one cell N={N} dtype={dt} chunks={S}")
                bz.bz_set_split(op, 1, S, 0)
                got = _collide(bz, op, f, dt)
                if dt == bz.BZ_F64:
                    assert rel_l2_per_cell(got, ref).max() <= 1e-12, S
                else:
                    err, floor, ok = f32_check(orc, N, L, 1, f, got)
                    assert ok.all(), (S, f32_report(err, floor, ok))
