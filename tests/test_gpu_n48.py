"""The 48-point mesh (N^3 = 110 592 modes per cell; stored FP64 weights
20.6 GB, on the fly two slab buffers of 1/16 of that): parity of one sampled cell with the FP64
oracle (which takes about a minute per cell at this mesh), every cell of a
two-group ragged batch equal between the stored table and the weights
computed on the fly, and the properties that hold at any size (the
unprojected mass vanishes; the projection conserves mass, momentum and
energy)."""
import sys

import numpy as np
import pytest

import synth
from tests.gpu_util import f32_check, f32_report, rel_l2_per_cell, to_dev, to_host

pytestmark = pytest.mark.gpu

N, L, LAM, NCELLS = 48, 6.0, 1, 65
F64_TOL = 1e-12


@pytest.fixture(scope="module")
def bz():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1301_4195_amd as bz

    bz.load()  # raises if libbz.so is missing: no fallback
    return bz


@pytest.fixture(scope="module")
def batch():
    return synth.two_maxwellian(N, L, NCELLS, synth.seed_for(480))


@pytest.fixture(scope="module")
def ref_cell(orc, batch):
    """The oracle's Q~ of the last cell (the ragged tail group)."""
    print("oracle N=48, one cell", file=sys.stderr, flush=True)
    return orc.collision(N, L, LAM, batch[-1:])


def _run(bz, op, f, dtype):
    import torch

    td = torch.float64 if dtype == bz.BZ_F64 else torch.float32
    fd = to_dev(f, td)
    qt = torch.empty_like(fd)
    qc = torch.empty(fd.shape, dtype=torch.float64, device="cuda")
    mom = torch.empty((f.shape[0], 5), dtype=torch.float64, device="cuda")
    bz.collision_eval(op, f.shape[0], fd, qt)
    bz.conserve(op, f.shape[0], qt, qc, mom)
    return to_host(qt).astype(np.float64), to_host(qc), to_host(mom)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_n48_stored_and_on_the_fly(bz, orc, batch, ref_cell, dtype):
    code = bz.BZ_F64 if dtype == "f64" else bz.BZ_F32
    print(f"N=48 {dtype}: stored table", file=sys.stderr, flush=True)
    with bz.bz_op_create(N, L, LAM, code) as op:
        assert bz.bz_get_split(op, NCELLS)[1] == 4
        held = bz.bz_op_table_bytes(op)
        qt, qc, mom = _run(bz, op, batch, code)
    print(f"N=48 {dtype}: weights on the fly", file=sys.stderr, flush=True)
    with bz.bz_op_create_onthefly(N, L, LAM, code) as op:
        assert bz.bz_op_table_bytes(op) <= held // 7  # two default slabs of 1/16 of the table
        qt2, _, _ = _run(bz, op, batch, code)
    # the same sums over weights that differ only in their last bits
    assert rel_l2_per_cell(qt2, qt).max() <= (1e-13 if dtype == "f64" else 1e-6)
    # one cell against the oracle
    if dtype == "f64":
        err = rel_l2_per_cell(qt[-1:], ref_cell)
        print(f"  rel L2 vs oracle {err.max():.2e}", file=sys.stderr, flush=True)
        assert err.max() <= F64_TOL
    else:
        print("oracle N=48, one cell, FP32 input", file=sys.stderr, flush=True)
        err, floor, ok = f32_check(orc, N, L, LAM, batch[-1:], qt[-1:])
        print("  FP32 " + f32_report(err, floor, ok), file=sys.stderr, flush=True)
        assert ok.all(), f32_report(err, floor, ok)
    # properties at any size: the unprojected mass vanishes (G^(., 0) = 0),
    # and the projected operator conserves mass, momentum and energy
    dv = 2 * L / N
    mass = qt.reshape(NCELLS, -1).sum(axis=1) * dv ** 3
    scale = np.abs(qt).reshape(NCELLS, -1).sum(axis=1) * dv ** 3
    assert np.all(np.abs(mass) <= (1e-12 if dtype == "f64" else 1e-5) * scale)
    v = synth.velocity_points(N, L)
    v1, v2, v3 = np.meshgrid(v, v, v, indexing="ij")
    C = dv ** 3 * np.stack([np.ones_like(v1), v1, v2, v3, v1 * v1 + v2 * v2 + v3 * v3]).reshape(5, -1)
    cons = np.abs(qc.reshape(NCELLS, -1) @ C.T).max()
    assert cons <= 1e-13 * np.abs(C).max() * np.abs(qc).reshape(NCELLS, -1).sum(axis=1).max()
    assert np.abs(mom[:, 0]).max() <= (1e-12 if dtype == "f64" else 1e-5) * scale.max()


def test_n48_small_batch_form(bz, batch, ref_cell):
    """Three cells (blocks of two at this mesh): the small-batch form, the
    default for so few cells, against the batched kernel and the oracle's
    cell, and with the weights computed on the fly in slabs."""
    f = batch[-3:]
    print("N=48 f64: small-batch form, three cells", file=sys.stderr, flush=True)
    with bz.bz_op_create(N, L, LAM, bz.BZ_F64) as op:
        assert bz.bz_get_split(op, 3)[1] == 0
        small, _, _ = _run(bz, op, f, bz.BZ_F64)
        bz.bz_set_split(op, 3, 4, 4)
        batched, _, _ = _run(bz, op, f, bz.BZ_F64)
    assert rel_l2_per_cell(small, batched).max() <= 1e-13
    err = rel_l2_per_cell(small[-1:], ref_cell)
    print(f"  rel L2 vs oracle {err.max():.2e}", file=sys.stderr, flush=True)
    assert err.max() <= F64_TOL
    with bz.bz_op_create_onthefly(N, L, LAM, bz.BZ_F64) as op:
        fly, _, _ = _run(bz, op, f, bz.BZ_F64)
    assert rel_l2_per_cell(fly, small).max() <= 1e-13
