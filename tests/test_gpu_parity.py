"""Parity of the gfx950 library (through its C ABI) with the FP64 CPU oracle.

Bars: FP64 path within 1e-12 relative L2 per cell; FP32 path (FP32 weights
and f^, FP32 products, FP64 line sums) within 1e-5 relative L2 per cell
against the oracle on the same FP32 input (twice the FP32 storage floor on
the rare cells whose floor alone exceeds half of that, see
tests.gpu_util.f32_check); the FP64 projection within 1e-12.  Inputs are the seeded synthetic batches of
``synth``.
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


# ----------------------------------------------------------------- weights
@pytest.mark.parametrize("N", [8, 16, 24, 32])
@pytest.mark.parametrize("lam", [0, 1, 0.5, -1.5])
def test_weights_match_oracle(bz, orc, N, lam):
    _check_weights(bz, orc, N, lam, 1.0)


@pytest.mark.parametrize("N,lam,beta", [(8, 0, 0.8), (16, 1, 0.8), (16, 0.5, 0.55)])
def test_inelastic_weights_match_oracle(bz, orc, N, lam, beta):
    _check_weights(bz, orc, N, lam, beta)


def _check_weights(bz, orc, N, lam, beta):
    import torch

    _note(f"weights N={N} lam={lam} beta={beta}")
    L = 6.0
    c = N // 2
    rng = np.random.default_rng(int(100 + N + lam) if lam in (0, 1) else int(200 + N + 10 * lam))
    ks, ms = [], []
    # random valid pairs plus every limiting branch of the closed form
    while len(ks) < 400:
        k = rng.integers(0, N, 3)
        m = rng.integers(0, N, 3)
        if np.all((k - m + c >= 0) & (k - m + c < N)):
            ks.append(k)
            ms.append(m)
    ks += [np.array([c, c, c]), np.array([c + 2, c, c - 2]), np.array([c + 2, c, c]), np.array([c + 3, c - 1, c + 1])]
    ms += [np.array([c + 1, c, c]), np.array([c + 1, c, c - 1]), np.array([c + 1, c + 1, c]), np.array([c, c, c])]
    ks.append(np.array([0, c, c]))  # an invalid pair: n1 = c - N + 1 < 0 -> 0
    ms.append(np.array([N - 1, c, c]))
    lin = lambda a: (a[0] * N + a[1]) * N + a[2]
    kl = np.array([lin(k) for k in ks], dtype=np.int32)
    ml = np.array([lin(m) for m in ms], dtype=np.int32)
    dz3 = (math.pi / L) ** 3

    def stored(k, m):
        # one weight per mirrored couple (m, n = k - m + N/2): summed unless the
        # couple lies on one line (m1, m2) == (n1, n2)
        n = np.asarray(k) - np.asarray(m) + c
        w = dz3 * orc.ghat(N, L, lam, k, m, beta=beta)
        if not (n[0] == m[0] and n[1] == m[1]):
            w += dz3 * orc.ghat(N, L, lam, k, n, beta=beta)
        return w

    ref = np.array([stored(k, m) for k, m in zip(ks, ms)])
    ref[-1] = 0.0
    for wd, tol in ((bz.BZ_F64, 1e-13), (bz.BZ_F32, 1e-7)):
        with bz.bz_op_create_inelastic(N, L, lam, beta, wd) as op:
            out = torch.empty(len(kl), dtype=torch.float64, device="cuda")
            bz.bz_weights_gather(op, to_dev(kl), to_dev(ml), out)
            got = to_host(out)
        scale = np.abs(ref).max()
        err = np.abs(got - ref)
        # two independent quadratures (non-integer lambda) agree to ~1e-16 of
        # the weight scale, so small weights are compared at that level
        floor = 1e-3 if lam in (0, 1) and beta == 1.0 else 1e-2
        ok = bool(np.all(err <= tol * np.maximum(np.abs(ref), floor * scale)))
        assert ok, (wd, float(err.max()), int(np.argmax(err)))
        assert got[-1] == 0.0 and got[len(ks) - 5] == 0.0  # invalid pair, zeta = 0 row


# ------------------------------------------------------------ collision FP64
@pytest.mark.parametrize("N,ncells,lam", [(8, 1, 0), (8, 3, 1), (16, 70, 1), (16, 5, 0), (8, 67, 0.5), (16, 20, 0.5),
                                          (16, 3, -1.5)])
def test_collision_f64_matches_oracle(bz, orc, N, ncells, lam):
    _note(f"collision f64 N={N} ncells={ncells} lam={lam}")
    L = 6.0
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(10 + N + ncells))
    ref = orc.collision(N, L, lam, f)
    with bz.bz_op_create(N, L, lam, bz.BZ_F64) as op:
        got = _collide(bz, op, f, bz.BZ_F64)
    err = rel_l2_per_cell(got, ref)
    assert err.max() <= F64_TOL, err.max()


@pytest.mark.parametrize("N,ncells,lam", [(8, 67, 1), (16, 20, 0)])
def test_inelastic_collision_and_projection(bz, orc, N, ncells, lam):
    """Inelastic collisions (beta = 0.8): Q~ as the oracle's, the projection
    keeps mass and momentum only (C_4 Q_c = 0) and matches the oracle's
    four-row projection; the energy moment is reported unprojected."""
    import torch

    _note(f"inelastic N={N} ncells={ncells} lam={lam}")
    L, beta = 6.0, 0.8
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(60 + N))
    qt_ref = orc.collision(N, L, lam, f, beta=beta)
    qc_ref, mom_ref = orc.project(N, L, qt_ref, energy=False)
    with bz.bz_op_create_inelastic(N, L, lam, beta, bz.BZ_F64) as op:
        fd = to_dev(f, torch.float64)
        qt = torch.empty_like(fd)
        bz.collision_eval(op, ncells, fd, qt)
        qc = torch.empty_like(fd)
        mom = torch.empty((ncells, 5), dtype=torch.float64, device="cuda")
        bz.conserve(op, ncells, qt, qc, mom)
        qt_h, qc_h, mom_h = to_host(qt), to_host(qc), to_host(mom)
    assert rel_l2_per_cell(qt_h, qt_ref).max() <= F64_TOL
    assert rel_l2_per_cell(qc_h, qc_ref).max() <= F64_TOL
    assert np.abs(mom_h - mom_ref).max() <= 1e-12 * np.abs(mom_ref).max()
    dv = 2 * L / N
    v = synth.velocity_points(N, L)
    v1, v2, v3 = np.meshgrid(v, v, v, indexing="ij")
    C4 = dv ** 3 * np.stack([np.ones_like(v1), v1, v2, v3]).reshape(4, -1)
    cons = np.abs(qc_h.reshape(ncells, -1) @ C4.T).max()
    assert cons <= 1e-13 * np.abs(C4).max() * np.abs(qt_h).reshape(ncells, -1).sum(axis=1).max()
    # energy is not conserved: the projected energy moment is the operator's cooling
    assert np.all(mom_h[:, 4] < 0.0)


def test_collision_f64_full_workload_n16(bz, orc):
    """Hard spheres, N = 16, 256 two-Maxwellian cells (the benchmark's batch),
    every cell against the oracle."""
    _note("collision f64 hs_n16_256")
    w = synth.WORKLOADS["hs_n16_256"]
    f = synth.two_maxwellian(w["N"], w["L"], w["ncells"], synth.seed_for(w["index"]))
    ref = orc.collision(w["N"], w["L"], w["lam"], f)
    with bz.bz_op_create(w["N"], w["L"], w["lam"], bz.BZ_F64) as op:
        got = _collide(bz, op, f, bz.BZ_F64)
    err = rel_l2_per_cell(got, ref)
    assert err.max() <= F64_TOL, err.max()


@pytest.mark.parametrize("N,ncells,sample", [(24, 67, [0, 33, 66]), (32, 65, [0, 64])])
def test_collision_f64_large_n_sampled(bz, orc, N, ncells, sample):
    """Larger meshes: the whole batch on the GPU (two cell groups, ragged tail),
    sampled cells on the oracle."""
    _note(f"collision f64 N={N} ncells={ncells}")
    L = 6.0
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(20 + N))
    with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
        got = _collide(bz, op, f, bz.BZ_F64)
    ref = orc.collision(N, L, 1, f[sample])
    err = rel_l2_per_cell(got[sample], ref)
    assert err.max() <= F64_TOL, err.max()


def test_collision_deterministic_and_batch_independent(bz):
    """Bitwise identical on repeat, and a cell's result does not depend on the
    rest of the batch (one cell alone vs inside 130 cells)."""
    N, L = 16, 6.0
    f = synth.two_maxwellian(N, L, 130, 77)
    with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
        a = _collide(bz, op, f, bz.BZ_F64)
        b = _collide(bz, op, f, bz.BZ_F64)
        one = _collide(bz, op, f[129:130], bz.BZ_F64)
    assert np.array_equal(a, b)
    assert rel_l2_per_cell(one, a[129:130]).max() <= F64_TOL


@pytest.mark.parametrize("N,ncells,splits,sample", [
    (8, 70, [(1, 2), (3, 2), (3, 1), (2, 4)], list(range(70))),
    (16, 70, [(1, 2), (5, 2), (5, 1), (2, 1), (3, 4)], list(range(70))),
    (24, 67, [(2, 2), (7, 1), (1, 2), (4, 4)], [0, 66]),
    (32, 65, [(3, 2), (9, 2), (9, 1), (1, 4)], [0, 64]),
])
def test_every_split_matches_oracle(bz, orc, N, ncells, splits, sample):
    """Every work split (m1 chunks x k3 ranges), forced with bz_set_split,
    gives the oracle's result on the sampled cells and agrees with the other
    splits on every cell (FP64 bar)."""
    L, lam = 6.0, 1
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(50 + N))
    ref = orc.collision(N, L, lam, f[sample])
    outs = []
    with bz.bz_op_create(N, L, lam, bz.BZ_F64) as op:
        for S, KH in splits:
            _note(f"split N={N} ncells={ncells} chunks={S} ranges={KH}")
            bz.bz_set_split(op, ncells, S, KH)
            outs.append(_collide(bz, op, f, bz.BZ_F64))
            assert rel_l2_per_cell(outs[-1][sample], ref).max() <= F64_TOL, (S, KH)
    for o in outs[1:]:
        assert rel_l2_per_cell(o, outs[0]).max() <= F64_TOL


def test_set_split_rejects_bad_values(bz):
    with bz.bz_op_create(16, 6.0, 1, bz.BZ_F64) as op:
        for n, S, KH in ((64, 0, 1), (64, 6, 1), (64, 1, 3), (64, 1, 8), (65, 1, 0), (64, 6, 0)):
            with pytest.raises(bz.BzError):
                bz.bz_set_split(op, n, S, KH)
        bz.bz_set_split(op, 64, 1, 0)  # the small-batch form takes up to 64 cells


# ------------------------------------------------------------ collision FP32
@pytest.mark.parametrize("N,ncells,dtype", [(16, 100, "f64"), (8, 3, "f64"), (24, 70, "f32")])
def test_autotune_then_parity(bz, orc, N, ncells, dtype):
    """After bz_autotune picks the work split for this batch size, results
    still match the oracle (FP64 bar, or the FP32 bound on sampled cells),
    are bitwise repeatable, and another batch size keeps its own split."""
    _note(f"autotune N={N} ncells={ncells} {dtype}")
    L, lam = 6.0, 1
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(40 + N))
    dt = bz.BZ_F64 if dtype == "f64" else bz.BZ_F32
    with bz.bz_op_create(N, L, lam, dt) as op:
        S, KH, ms = bz.bz_autotune(op, ncells)
        assert 1 <= S <= (N // 2 + 2) // 2 and KH in ((0, 1, 2, 4) if ncells <= 64 else (1, 2, 4)) and ms > 0.0
        a = _collide(bz, op, f, dt)
        b = _collide(bz, op, f, dt)
        other = _collide(bz, op, f[: min(ncells, 5)], dt)  # a different padded size when ncells > 64
    assert np.array_equal(a, b)
    sample = list(range(ncells)) if dtype == "f64" else list(range(0, ncells, 7))
    if dtype == "f64":
        ref = orc.collision(N, L, lam, f[sample])
        assert rel_l2_per_cell(a[sample], ref).max() <= F64_TOL
        assert rel_l2_per_cell(other, a[: other.shape[0]]).max() <= F64_TOL
    else:
        err, floor, ok = f32_check(orc, N, L, lam, f[sample], a[sample])
        _note("  " + f32_report(err, floor, ok, sample))
        assert ok.all(), f32_report(err, floor, ok, sample)


@pytest.mark.parametrize("N,ncells,sample,split", [(16, 256, list(range(256)), None), (24, 130, list(range(0, 130, 4)), None),
                                                   (32, 64, [0, 21, 42, 63], None), (16, 100, list(range(100)), (2, 2)),
                                                   (16, 256, list(range(256)), (1, 1)),
                                                   (32, 64, [0, 63], (4, 2)), (24, 64, [0, 31, 63], (3, 4))])
def test_collision_f32_within_bound(bz, orc, N, ncells, sample, split):
    """FP32 path against the FP64 oracle on the same FP32 input, per cell:
    1e-5 relative L2 (N = 16: all 256 cells of the headline batch at the
    default and at a one-chunk split)."""
    _note(f"collision f32 N={N} ncells={ncells} split={split}")
    L = 6.0
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(30 + N))
    with bz.bz_op_create(N, L, 1, bz.BZ_F32) as op:
        if split:
            bz.bz_set_split(op, ncells, *split)
        got = _collide(bz, op, f, bz.BZ_F32)
    err, floor, ok = f32_check(orc, N, L, 1, f[sample], got[sample])
    _note("  f32 " + f32_report(err, floor, ok, sample))
    assert ok.all(), f32_report(err, floor, ok, sample)


# ------------------------------------------------------------- projection
@pytest.mark.parametrize("in_f32", [False, True])
def test_conserve_matches_oracle(bz, orc, in_f32):
    import torch

    N, L = 16, 6.0
    rng = np.random.default_rng(8)
    qt = rng.standard_normal((37, N, N, N))
    if in_f32:
        qt = qt.astype(np.float32).astype(np.float64)
    ref, mref = orc.project(N, L, qt)
    with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
        qd = to_dev(qt, torch.float32 if in_f32 else torch.float64)
        qc = torch.empty(qt.shape, dtype=torch.float64, device="cuda")
        mom = torch.empty((37, 5), dtype=torch.float64, device="cuda")
        bz.conserve(op, 37, qd, qc, mom)
        got, gm = to_host(qc), to_host(mom)
        if not in_f32:  # in place
            bz.conserve(op, 37, qd, qd)
            assert np.array_equal(to_host(qd), got)
    assert rel_l2_per_cell(got, ref).max() <= F64_TOL
    assert np.abs(gm - mref).max() <= 1e-12 * np.abs(mref).max()


def test_conserve_flags_nonfinite_cells(bz):
    """A NaN or an Inf in a cell's Q~ sets that cell's five moments to the
    non-finite flag and makes its Qc non-finite; the other cells' moments and
    Qc are bit for bit those of a run without the bad values (FP64 and FP32
    input)."""
    import torch

    N, L, n = 8, 6.0, 6
    rng = np.random.default_rng(21)
    clean = rng.standard_normal((n, N, N, N))
    bad = clean.copy()
    bad[2, 1, 2, 3] = np.nan
    bad[4, 0, 0, 0] = np.inf
    flag = np.array([bz.BZ_MOMENTS_NONFINITE_BITS], dtype=np.uint64)
    for td in (torch.float64, torch.float32):
        with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
            out = []
            for q in (clean, bad):
                qd = to_dev(q, td)
                qc = torch.empty(q.shape, dtype=torch.float64, device="cuda")
                mom = torch.empty((n, 5), dtype=torch.float64, device="cuda")
                bz.conserve(op, n, qd, qc, mom)
                out.append((to_host(qc), to_host(mom)))
        (qc0, m0), (qc1, m1) = out
        for c in range(n):
            if c in (2, 4):
                assert np.array_equal(m1[c].view(np.uint64), np.repeat(flag, 5)), c
                assert not np.isfinite(qc1[c]).any(), c
            else:
                assert np.isfinite(m1[c]).all() and np.array_equal(m1[c], m0[c]), c
                assert np.array_equal(qc1[c], qc0[c]), c


def test_collision_plus_projection_conserves(bz):
    """C Q_c = 0 to rounding for GPU output in both precisions."""
    import torch

    N, L = 16, 6.0
    f = synth.two_maxwellian(N, L, 64, 5)
    v = synth.velocity_points(N, L)
    v1, v2, v3 = np.meshgrid(v, v, v, indexing="ij")
    C = (2 * L / N) ** 3 * np.stack([np.ones_like(v1), v1, v2, v3, v1 ** 2 + v2 ** 2 + v3 ** 2]).reshape(5, -1)
    for wd, td in ((bz.BZ_F64, torch.float64), (bz.BZ_F32, torch.float32)):
        with bz.bz_op_create(N, L, 1, wd) as op:
            fd = to_dev(f, td)
            qt = torch.empty_like(fd)
            bz.collision_eval(op, 64, fd, qt)
            qc = torch.empty(f.shape, dtype=torch.float64, device="cuda")
            bz.conserve(op, 64, qt, qc)
            q = to_host(qc).reshape(64, -1)
            scale = np.abs(to_host(qt).reshape(64, -1)).sum(axis=1).max() * np.abs(C).max()
            assert np.abs(q @ C.T).max() <= 1e-14 * scale


# ---------------------------------------------------- homogeneous time stepping
def test_bkw_euler_run_matches_oracle(bz, orc):
    """Maxwell molecules, N = 8, L = 6, BKW data at t0 = 5.5, ten forward-Euler
    steps dt = 0.01 with the projection every step, GPU vs oracle."""
    import torch

    w = synth.WORKLOADS["bkw_n8"]
    N, L, dt = w["N"], w["L"], 0.01
    f0 = synth.bkw(N, L, 5.5)[None].copy()
    ref = f0.copy()
    for _ in range(10):
        qc, _ = orc.project(N, L, orc.collision(N, L, 0, ref))
        ref = ref + dt * qc
    with bz.bz_op_create(N, L, 0, bz.BZ_F64) as op:
        fd = to_dev(f0)
        qt = torch.empty_like(fd)
        qc = torch.empty_like(fd)
        for _ in range(10):
            bz.collision_eval(op, 1, fd, qt)
            bz.conserve(op, 1, qt, qc)
            bz.bz_axpy(dt, qc, fd)
        got = to_host(fd)
    assert rel_l2_per_cell(got, ref).max() <= 1e-13


# --------------------------------------------------------------- transport
def test_transport_step_matches_oracle(bz, orc):
    import torch

    N, L, M = 8, 8.0, 24
    xf = synth.boundary_layer_faces(M, X=4.0)
    f = synth.boundary_layer_state(N, L, M)
    f[2:8] *= 1.3  # a density step so that the limiter and the wall act
    left = (bz.BZ_WALL_DIFFUSE, 2.0, (0.0, 0.2, 0.0))
    right = (bz.BZ_WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))
    dt = 0.5 * np.diff(xf).min() / L
    ref = f.copy()
    for _ in range(5):
        ref = orc.transport_step(N, L, ref, xf, dt, left=left, right=right)
    with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
        fd = to_dev(f)
        xd = to_dev(xf)
        for _ in range(5):
            bz.transport_step(op, M, fd, xd, dt, left=left, right=right)
        got = to_host(fd)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    for kind in (bz.BZ_WALL_NOFLUX, bz.BZ_WALL_DIFFUSE):
        r = (kind, 1.5, (0.0, 0.0, 0.0))
        ref2 = orc.transport_step(N, L, f, xf, dt, left=left, right=r)
        with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
            fd = to_dev(f)
            bz.transport_step(op, M, fd, to_dev(xf), dt, left=left, right=r)
            got2 = to_host(fd)
        assert np.abs(got2 - ref2).max() <= 1e-13 * np.abs(ref2).max()


# ------------------------------------------------------------------ edges
def test_edge_cases(bz):
    import torch

    N, L = 8, 6.0
    with bz.bz_op_create(N, L, 1, bz.BZ_F64) as op:
        e = torch.empty(0, dtype=torch.float64, device="cuda")
        bz.collision_eval(op, 0, e, e)  # no-op
        f = to_dev(synth.two_maxwellian(N, L, 2, 1))
        with pytest.raises(bz.BzError) as ei:
            bz.collision_eval(op, 2, f, torch.empty_like(f), dtype=bz.BZ_F32)
        assert ei.value.code == bz.BZ_EINVAL
        with pytest.raises(bz.BzError):
            bz.collision_eval(op, 2, f, f)  # aliasing
        flat = torch.zeros(2 * N ** 3 + 1, dtype=torch.float64, device="cuda")
        with pytest.raises(bz.BzError) as ei:  # cells must start on pairs of values
            bz.collision_eval(op, 2, flat[1:].view(2, N, N, N), torch.empty((2, N, N, N), dtype=torch.float64,
                                                                            device="cuda"))
        assert ei.value.code == bz.BZ_EINVAL
        with pytest.raises(bz.BzError) as ei:
            bz.transport_step(op, 4, torch.zeros((8, N, N, N), dtype=torch.float64, device="cuda"),
                              to_dev(np.linspace(0, 1, 5)), 0.01, left=(bz.BZ_WALL_DIFFUSE, 1.0, (0.1, 0, 0)))
        assert ei.value.code == bz.BZ_EINVAL
    for lam in (-3.0, 2.5):  # the radial integral diverges at lambda <= -3
        with pytest.raises(bz.BzError) as ei:
            bz.bz_op_create(16, 6.0, lam, bz.BZ_F64)
        assert ei.value.code == bz.BZ_EUNSUPPORTED
    bz.bz_set_memory_cap(1 << 20)
    try:
        with pytest.raises(bz.BzError) as ei:
            bz.bz_op_create(16, 6.0, 1, bz.BZ_F64)
        assert ei.value.code == bz.BZ_ENOMEM
    finally:
        bz.bz_set_memory_cap(0)


# ------------------------------------------------------- Strang time step
def _oracle_strang(orc, N, L, lam, f, xf, dt, eps, left, right):
    """Transport dt/2, Heun collision dt on P_N Q~, transport dt/2 (oracle pieces)."""
    f = orc.transport_step(N, L, f, xf, 0.5 * dt, left=left, right=right)
    fi = f[2:-2]
    q1, _ = orc.project(N, L, orc.collision(N, L, lam, fi))
    fs = fi + dt / eps * q1
    q2, _ = orc.project(N, L, orc.collision(N, L, lam, fs))
    f = f.copy()
    f[2:-2] = fi + 0.5 * dt / eps * (q1 + q2)
    return orc.transport_step(N, L, f, xf, 0.5 * dt, left=left, right=right)


def test_strang_step_matches_oracle_and_graph_replays(bz, orc):
    """Boundary-layer set-up (diffuse wall at T = 2, outflow far end, Kn = 0.1):
    three GPU Strang steps vs the oracle composition, then a captured HIP graph
    of three steps replayed twice (with eager work in between) is bitwise equal
    to the eager steps."""
    import torch

    N, L, M, lam, eps = 8, 8.0, 24, 1, 0.1
    xf = synth.boundary_layer_faces(M, X=4.0)
    f0 = synth.boundary_layer_state(N, L, M)
    left = (bz.BZ_WALL_DIFFUSE, 2.0, (0.0, 0.0, 0.0))
    right = (bz.BZ_WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))
    dt = 0.5 * np.diff(xf).min() / L
    ref = f0.copy()
    for _ in range(3):
        ref = _oracle_strang(orc, N, L, lam, ref, xf, dt, eps, left, right)
    with bz.bz_op_create(N, L, lam, bz.BZ_F64) as op:
        xd = to_dev(xf)
        fd = to_dev(f0)
        eager = []
        for i in range(6):
            bz.bz_strang_step(op, M, fd, xd, dt, eps, left, right)
            if i in (2, 5):
                eager.append(to_host(fd).copy())
        gd = to_dev(f0)
        with bz.bz_graph_capture_strang(op, M, gd, xd, dt, eps, 3, left, right) as g:
            g.launch()
            first = to_host(gd).copy()
            junk = torch.empty_like(fd[:M])
            bz.collision_eval(op, M, fd[2:-2], junk)  # eager work between replays
            torch.cuda.synchronize()
            g.launch()
            second = to_host(gd).copy()
    scale = np.abs(ref).max()
    assert np.abs(eager[0] - ref).max() <= 1e-12 * scale
    assert np.array_equal(first, eager[0])
    assert np.array_equal(second, eager[1])


# ------------------------------------------------------------ mixed-N batch
def _macroscopic(f, N, L):
    v = synth.velocity_points(N, L)
    dv3 = (2.0 * L / N) ** 3
    v1, v2, v3 = np.meshgrid(v, v, v, indexing="ij")
    fi = f[2:-2].reshape(f.shape[0] - 4, -1)
    rho = fi.sum(axis=1) * dv3
    u = (fi @ v1.ravel()) * dv3 / rho
    e = (fi @ (v1 ** 2 + v2 ** 2 + v3 ** 2).ravel()) * dv3
    return rho, u, (e / rho - u * u) / 3.0


def test_sudden_heating_and_cooling_of_the_wall(bz, orc):
    """Sec. 5 problem (Kn = 1, 8 / 2 cells per mean free path at the wall /
    inside, 370 cells on [0, 100]): two Strang steps match the oracle; then
    1000 steps from HIP graphs show the expected trends -- heating thins and
    heats the gas at the wall and drives it away (u > 0) behind a front that
    moves outward; cooling densifies and cools it and draws it in (u < 0) --
    with mass conserved while the disturbance is far from the outflow end and
    no growth of negative values of f."""
    import torch

    w = synth.WORKLOADS["wall_long_n16_370"]
    N, M, lam, eps = w["N"], w["ncells"], w["lam"], w["eps"]
    xf = synth.boundary_layer_faces(M, w["X"], w["alpha"])
    xc, dx = 0.5 * (xf[1:] + xf[:-1]), np.diff(xf)
    right = (bz.BZ_WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))
    for Tw, L in w["cases"]:
        _note(f"sudden wall Tw={Tw} L={L}")
        left = (bz.BZ_WALL_DIFFUSE, Tw, (0.0, 0.0, 0.0))
        f0 = synth.boundary_layer_state(N, L, M)
        dt = 0.5 * dx.min() / L
        with bz.bz_op_create(N, L, lam, bz.BZ_F64) as op:
            xd = to_dev(xf)
            fd = to_dev(f0)
            if Tw > 1.0:  # parity of the set-up against the oracle
                for _ in range(2):
                    bz.bz_strang_step(op, M, fd, xd, dt, eps, left, right)
                ref = f0.copy()
                for _ in range(2):
                    ref = _oracle_strang(orc, N, L, lam, ref, xf, dt, eps, left, right)
                assert np.abs(to_host(fd) - ref).max() <= 1e-12 * np.abs(ref).max()
                fd.copy_(to_dev(f0))
            mass0 = float((_macroscopic(f0, N, L)[0] * dx).sum())
            fronts = []
            with bz.bz_graph_capture_strang(op, M, fd, xd, dt, eps, 50, left, right) as g:
                g.launch()
                torch.cuda.synchronize()
                fd.copy_(to_dev(f0))
                for _ in range(2):
                    for _ in range(10):
                        g.launch()
                    fh = to_host(fd)
                    rho, u, T = _macroscopic(fh, N, L)
                    fronts.append(xc[np.where(np.abs(rho - 1.0) > 1e-3)[0].max()])
        assert abs(float((rho * dx).sum()) / mass0 - 1.0) <= 1e-7
        assert fh[2:-2].min() >= -1e-2 * fh[2:-2].max()
        assert fronts[1] > fronts[0] > 3.0
        if Tw > 1.0:
            assert T[0] > 1.5 and rho[0] < 0.8 and u.max() > 0.1 and u.min() > -1e-3, (T[0], rho[0], u.max(), u.min())
        else:
            assert T[0] < 0.7 and rho[0] > 1.3 and u.min() < -0.08 and u.max() < 2e-3, (T[0], rho[0], u.min(), u.max())


def _mixed_split(bz, op, ncells, N, f64):
    """Give the op, for this batch size, the k3 range count that the one-launch
    mixed convolution uses for its N (1 up to N = 16; above, 4 in FP64 and 2
    in FP32) with its own m1 chunks: the range count changes no summation
    order, but the compiled variants contract multiply-adds differently, so
    bitwise comparisons need the same one."""
    S = bz.bz_get_split(op, ncells)[0]
    bz.bz_set_split(op, ncells, S, 1 if N <= 16 else (4 if f64 else 2))


def test_ragged_mixed_n_batch(bz, orc):
    """Packed batch with N drawn from {8, 16, 24, 32} (40/30/20/10 %), its
    convolution one launch for all N: every cell equals the dense per-N
    evaluation at the same split bitwise, sampled cells match the oracle, and
    the ragged projection equals the dense one."""
    import torch

    L = 6.0
    ns, fs = synth.mixed_n(180, synth.seed_for(40))
    Ns = [8, 16, 24, 32]
    op_of = np.array([Ns.index(n) for n in ns], dtype=np.int32)
    sizes = np.array([n ** 3 for n in ns], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.concatenate([f.ravel() for f in fs])
    ops = [bz.bz_op_create(n, L, 1, bz.BZ_F64) for n in Ns]
    try:
        fd = to_dev(flat)
        qd = torch.empty_like(fd)
        qc = torch.empty_like(fd)
        mom = torch.empty((len(ns), 5), dtype=torch.float64, device="cuda")
        bz.collision_eval_ragged(ops, op_of, offs, fd, qd, bz.BZ_F64)
        bz.conserve_ragged(ops, op_of, offs, qd, qc, mom)
        got = to_host(qd)
        gotc = to_host(qc)
        for j, n in enumerate(Ns):
            sel = np.nonzero(op_of == j)[0]
            fj = np.stack([fs[i] for i in sel])
            _mixed_split(bz, ops[j], len(sel), n, True)
            dense = _collide(bz, ops[j], fj, bz.BZ_F64)
            for t, i in enumerate(sel):
                assert np.array_equal(got[offs[i]:offs[i] + n ** 3], dense[t].ravel()), (n, i)
            dd = to_dev(dense)
            dc = torch.empty_like(dd)
            bz.conserve(ops[j], len(sel), dd, dc)
            dch = to_host(dc)
            for t, i in enumerate(sel):
                assert np.array_equal(gotc[offs[i]:offs[i] + n ** 3], dch[t].ravel())
            pick = sel if n <= 16 else sel[:2]
            ref = orc.collision(n, L, 1, np.stack([fs[i] for i in pick]))
            g = np.stack([got[offs[i]:offs[i] + n ** 3] for i in pick])
            assert rel_l2_per_cell(g, ref).max() <= F64_TOL, n
        # a second call with the same layout reuses the uploaded lists
        bz.collision_eval_ragged(ops, op_of, offs, fd, qd, bz.BZ_F64)
        assert np.array_equal(to_host(qd), got)
    finally:
        for o in ops:
            o.destroy()


@pytest.mark.parametrize("fly", [False, True])
def test_ragged_mixed_n_f32_one_launch(bz, orc, fly):
    """FP32 packed batch (N from {8, 16, 24, 32}, 40/30/20/10 %), one
    convolution launch for all N: each cell bitwise equal to its op's own
    collision_eval, two sampled cells of each N within the stated FP32 bound
    of the oracle (1e-5 relative, see tests.gpu_util.f32_check).  With
    one op's weights computed on the fly the batch takes the per-op launches
    instead, with the same results."""
    import torch

    _note(f"ragged f32 fly={fly}")
    L = 6.0
    ns, fs = synth.mixed_n(150, synth.seed_for(45))
    Ns = [8, 16, 24, 32]
    op_of = np.array([Ns.index(n) for n in ns], dtype=np.int32)
    sizes = np.array([n ** 3 for n in ns], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.concatenate([f.ravel() for f in fs]).astype(np.float32)
    ops = [bz.bz_op_create_onthefly(n, L, 1, bz.BZ_F32) if (fly and n == 16) else bz.bz_op_create(n, L, 1, bz.BZ_F32)
           for n in Ns]
    try:
        fd = to_dev(flat)
        qd = torch.empty_like(fd)
        bz.collision_eval_ragged(ops, op_of, offs, fd, qd, bz.BZ_F32)
        got = to_host(qd).astype(np.float64)
        for j, n in enumerate(Ns):
            sel = np.nonzero(op_of == j)[0]
            fj = np.stack([fs[i] for i in sel]).astype(np.float32)
            if not fly:
                _mixed_split(bz, ops[j], len(sel), n, False)
            dense = _collide(bz, ops[j], fj, bz.BZ_F32)
            for t, i in enumerate(sel):
                assert np.array_equal(got[offs[i]:offs[i] + n ** 3], dense[t].ravel()), (n, i)
            pick = sel[:2]
            fp = np.stack([fs[i] for i in pick])
            g = np.stack([got[offs[i]:offs[i] + n ** 3].reshape(n, n, n) for i in pick])
            err, floor, ok = f32_check(orc, n, L, 1, fp, g)
            assert ok.all(), (n, f32_report(err, floor, ok, pick))
    finally:
        for o in ops:
            o.destroy()


def test_ragged_autotune_picks_a_form_with_same_results(bz, orc):
    """bz_autotune_ragged times both forms of the mixed convolution and the
    following ragged call uses the faster; either way each cell equals its
    op's own collision_eval at the split that form uses, bit for bit."""
    import torch

    L = 6.0
    ns, fs = synth.mixed_n(150, synth.seed_for(47))
    Ns = [8, 16, 24, 32]
    op_of = np.array([Ns.index(n) for n in ns], dtype=np.int32)
    sizes = np.array([n ** 3 for n in ns], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.concatenate([f.ravel() for f in fs]).astype(np.float32)
    ops = [bz.bz_op_create(n, L, 1, bz.BZ_F32) for n in Ns]
    try:
        one, t1, t0 = bz.bz_autotune_ragged(ops, op_of, offs, bz.BZ_F32)
        _note(f"ragged autotune: one launch {t1:.3f} ms, per-op {t0:.3f} ms -> one_launch={one}")
        assert one in (0, 1) and t1 > 0.0 and t0 > 0.0
        assert one == (1 if t1 <= t0 else 0)
        fd = to_dev(flat)
        qd = torch.empty_like(fd)
        bz.collision_eval_ragged(ops, op_of, offs, fd, qd, bz.BZ_F32)
        got = to_host(qd).astype(np.float64)
        for j, n in enumerate(Ns):
            sel = np.nonzero(op_of == j)[0]
            if one:
                _mixed_split(bz, ops[j], len(sel), n, False)
            dense = _collide(bz, ops[j], np.stack([fs[i] for i in sel]).astype(np.float32), bz.BZ_F32)
            for t, i in enumerate(sel):
                assert np.array_equal(got[offs[i]:offs[i] + n ** 3], dense[t].ravel()), (n, i)
    finally:
        for o in ops:
            o.destroy()


@pytest.mark.parametrize("form", [1, 0])
def test_ragged_step_graph_replays_match_eager(bz, form):
    """One step of an FP32 mixed-N batch (collision_eval_ragged, then
    conserve_ragged) captured in a HIP graph, in each convolution form (one
    launch for all meshes; per-mesh launches on forked streams): every replay,
    with eager work and synchronisations between replays and f refilled in
    between, equals the eager step with that form, bit for bit."""
    import torch

    _note(f"ragged step graph, form {form}")
    L = 6.0
    ns, fs = synth.mixed_n(150, synth.seed_for(49))
    _, fs2 = synth.mixed_n(150, synth.seed_for(49))
    fs2 = [0.5 * x[::-1].copy() for x in fs2]  # other data, same layout
    Ns = [8, 16, 24, 32]
    op_of = np.array([Ns.index(n) for n in ns], dtype=np.int32)
    sizes = np.array([n ** 3 for n in ns], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.concatenate([f.ravel() for f in fs]).astype(np.float32)
    flat2 = np.concatenate([f.ravel() for f in fs2]).astype(np.float32)
    ops = [bz.bz_op_create(n, L, 1, bz.BZ_F32) for n in Ns]
    try:
        bz.bz_set_ragged_form(ops, op_of, offs, bz.BZ_F32, form)

        def eager(fin):
            fd = to_dev(fin)
            qt = torch.empty_like(fd)
            qc = torch.empty(fd.shape, dtype=torch.float64, device="cuda")
            bz.collision_eval_ragged(ops, op_of, offs, fd, qt, bz.BZ_F32)
            bz.conserve_ragged(ops, op_of, offs, qt, qc)
            return to_host(qc)

        ref, ref2 = eager(flat), eager(flat2)
        assert not np.array_equal(ref, ref2)
        fd = to_dev(flat)
        qt = torch.empty_like(fd)
        qc = torch.empty(fd.shape, dtype=torch.float64, device="cuda")
        with bz.bz_graph_capture_ragged(ops, op_of, offs, fd, qt, qc, bz.BZ_F32, form=form) as g:
            for rep in range(3):
                qc.fill_(float("nan"))
                g.launch()
                assert np.array_equal(to_host(qc), ref), rep
                assert np.array_equal(eager(flat2), ref2)  # eager work between replays
            fd.copy_(to_dev(flat2))
            g.launch()
            assert np.array_equal(to_host(qc), ref2)
    finally:
        for o in ops:
            o.destroy()
