"""Throughput of the collision-operator hot path on one MI355X.

A step is one full pass of the hot path over the batch: forward 3-D FFT,
truncated weighted convolution, inverse FFT (collision_eval) and the FP64
conservation projection (conserve) for every cell.  The default workload is
256 independent cells, hard spheres, N = 16, L = 6, two-Maxwellian data,
FP64.  The JSON line reports evaluations per second (cells x steps / s), the
convolution kernel's roofline position (timed with HIP events on the launch
stream) and the FP64 CPU oracle timed on the host as a baseline.

Extra points (``points``): the FP32 batched path on the same inputs, the
autotuned split, variable hard spheres (lambda = 0.5, quadrature weights),
inelastic hard spheres (beta = 0.8), long sudden heating and cooling of the
wall (4000 Strang steps each from HIP graphs),
1024 FP32 cells at N = 24, both paths at N = 32 (512 cells), a boundary-layer
Strang step replayed from HIP graphs and a mixed-N batch, each with its
measured error against the oracle.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector, 256 CU x 64 lanes x 2 flop x 2.4 GHz
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (published; needs packed FP32)
HBM_PEAK = 8.0e12          # MI355X HBM3E bytes/s (published)


def conv_flops_per_cell(N: int) -> float:
    """Algorithmic work of the weighted convolution for one cell: 10 real flops
    (complex product, real weight, complex accumulate) per valid (k, m) pair,
    27 N^6 / 64 pairs."""
    return 10.0 * 27.0 * N ** 6 / 64.0


def conv_executed_flops_per_cell(N: int) -> float:
    """Flops the kernel actually issues for one cell: in each output row
    (k1, k2) the lines (m1, m2) and (k1 - m1 + N/2, k2 - m2 + N/2) carry the
    same products, so one line of each mirrored couple is summed (with the
    two weights added), 10 flops per (k3, m3) pair of a kept line: the sum
    over rows of half_lines(c1, c2) x 3N^2/4."""
    def cnt(k):
        return min(N - 1, k + N // 2) - max(0, k - N // 2 + 1) + 1
    lines = 0
    for k1 in range(N):
        for k2 in range(N):
            c1, c2 = cnt(k1), cnt(k2)
            lines += (c1 // 2) * c2 + ((c2 + 1) // 2 if c1 & 1 else 0)
    return 10.0 * lines * (3 * N * N // 4)


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "conv_f64_n16_256_traffic.md")
TRAFFIC_SOURCES = ("paper_1301_4195_amd/csrc/conv.hip", "paper_1301_4195_amd/csrc/schedule.hip",
                   "paper_1301_4195_amd/csrc/bz_internal.h", "paper_1301_4195_amd/build.py")


def conv_sources_digest() -> str:
    """SHA-256 over the sources that decide the convolution kernel's memory
    traffic (kernel, schedule, shared helpers, compiler flags)."""
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(rel.encode() + b"\0" + fh.read() + b"\0")
    return h.hexdigest()


def conv_traffic_bytes():
    """HBM bytes per convolution launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes, each scaled by the factor a plain copy
    of known size gives), or None when that summary is missing or was taken
    from other kernel sources than the ones built now."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("sources_sha256") != conv_sources_digest():
        return None
    return float(rec["bytes_per_launch"])


def run_gpu(bz, torch, N, L, lam, f_host, dtype, steps, warmup, tune=False, fly=False, info=None):
    """Time `steps` hot-path steps; returns (elapsed_s, conv_ms_per_launch, Qc host,
    autotune result (chunks, k3 ranges, ms) or None, split used).  With `tune`,
    bz_autotune picks the convolution's work split before the warm-up.  With
    `fly`, the op computes its weights on the fly (default slab).  `info`
    (a dict) receives the op's table bytes."""
    td = torch.float64 if dtype == bz.BZ_F64 else torch.float32
    ncells = f_host.shape[0]
    op = bz.bz_op_create_onthefly(N, L, lam, dtype) if fly else bz.bz_op_create(N, L, lam, dtype)
    try:
        if info is not None:
            info["table_bytes"] = bz.bz_op_table_bytes(op)
        bz.bz_op_reserve(op, ncells)
        tuned = bz.bz_autotune(op, ncells) if tune else None
        split = bz.bz_get_split(op, ncells)
        f = torch.from_numpy(f_host).to(td).cuda()
        qt = torch.empty_like(f)
        qc = torch.empty(f.shape, dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            bz.collision_eval(op, ncells, f, qt, stream=stream)
            bz.conserve(op, ncells, qt, qc, stream=stream)
        torch.cuda.synchronize()
        bz.bz_timing_enable(op, True)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(steps):
            bz.collision_eval(op, ncells, f, qt, stream=stream)
            bz.conserve(op, ncells, qt, qc, stream=stream)
        stop.record(stream)
        torch.cuda.synchronize()
        elapsed = start.elapsed_time(stop) / 1e3
        conv_ms, launches = bz.bz_timing_read(op)
        bz.bz_timing_enable(op, False)
        out = qc.cpu().numpy()
    finally:
        op.destroy()
    return elapsed, conv_ms / max(launches, 1), out, tuned, split


def rel_err(got, ref):
    g = got.reshape(got.shape[0], -1)
    r = ref.reshape(ref.shape[0], -1)
    return np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)


def host_cpu_model() -> str:
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(N, L, lam, f, min_seconds=10.0):
    """The FP64 oracle (collision + projection) on the host cores, repeated over
    the batch until about `min_seconds` of wall time."""
    import oracle

    oracle.build(force=False)
    ncells = f.shape[0]
    reps, t0 = 0, time.perf_counter()
    while True:
        qt = oracle.collision(N, L, lam, f)
        oracle.project(N, L, qt)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds or reps >= 50:
            break
    cores = oracle.num_threads()
    # one core, one pass over the same batch (the oracle builds each row of
    # weights once per pass, so the batch size is part of its cost)
    oracle.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        qt = oracle.collision(N, L, lam, f)
        oracle.project(N, L, qt)
        el1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(cores)
    return {"value": reps * ncells / el, "unit": "cell-evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": host_cpu_model(), "host_cpus_online": os.cpu_count(),
            "sample": f"{reps} pass(es) over the full {ncells}-cell batch (N={N}), {el:.1f} s wall",
            "one_core": {"value": ncells / el1, "cores": 1, "sample": f"one pass over the {ncells}-cell batch, {el1:.1f} s wall"}}


def unbatched_point(bz, torch, N, L, lam, f_host, passes=3):
    """The plain FP64 path: one cell per collision_eval + conserve call (the
    weights streamed once per cell instead of once per 64 cells, by the
    small-batch convolution).  Of `passes` passes through the cells the
    next-to-last is timed as a whole; the last brackets every convolution
    with HIP events, whose time gives the rate at which it streams the packed
    weight table, against HBM's 8 TB/s."""
    n = f_host.shape[0]
    op = bz.bz_op_create(N, L, lam, bz.BZ_F64)
    try:
        f = torch.from_numpy(f_host).cuda()
        qt = torch.empty_like(f)
        qc = torch.empty_like(f)
        fs, qts, qcs = [f[c] for c in range(n)], [qt[c] for c in range(n)], [qc[c] for c in range(n)]
        stream = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        el = None
        for p in range(passes):
            torch.cuda.synchronize()
            bz.bz_timing_enable(op, p == passes - 1)
            a.record(stream)
            for c in range(n):
                bz.collision_eval(op, 1, fs[c], qts[c], stream=stream)
                bz.conserve(op, 1, qts[c], qcs[c], stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            if p == passes - 2:
                el = a.elapsed_time(b) / 1e3
        conv_ms, k = bz.bz_timing_read(op)
        conv_ms /= max(k, 1)
        wbytes = bz.bz_op_table_bytes(op)
        split = bz.bz_get_split(op, 1)
        qc_h = qc.cpu().numpy()
    finally:
        op.destroy()
    sample = sorted(set(np.linspace(0, n - 1, min(n, 8)).astype(int).tolist()))
    err = rel_err(qc_h[sample], oracle_ref(N, L, lam, f_host, sample))
    return {"N": N, "ncells": n, "dtype": "f64", "batching": "one cell per call (unbatched)",
            "evals_per_s": n / el, "ms_per_cell": el / n * 1e3, "conv_ms": conv_ms,
            "convolution_form": "small-batch" if split[1] == 0 else "batched", "split": list(split),
            "weight_table_bytes": wbytes, "weight_stream_TBps": wbytes / (conv_ms * 1e-3) / 1e12,
            "weight_stream_frac_of_hbm": wbytes / (conv_ms * 1e-3) / HBM_PEAK,
            "max_rel_l2_err": float(err.max()), "cells_checked": len(sample)}


def oracle_rate(N, L, lam, f):
    """Per-cell rate of the oracle (collision + projection) on the host cores,
    one pass over the cells given."""
    import oracle

    oracle.build(force=False)
    t0 = time.perf_counter()
    oracle.project(N, L, oracle.collision(N, L, lam, f))
    el = time.perf_counter() - t0
    return {"value": f.shape[0] / el, "unit": "cell-evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{f.shape[0]} cells (N={N}), {el:.1f} s wall"}


def oracle_ref(N, L, lam, f, idx):
    """Oracle Q_c for the sampled cells."""
    import oracle

    oracle.build(force=False)
    qc, _ = oracle.project(N, L, oracle.collision(N, L, lam, f[idx]))
    return qc


def oracle_imag_ratio(N, L, lam, f, idx):
    """Largest ||Im|| / ||Re|| over the cells idx of the oracle's inverse
    transform of the truncated sum: the part the method drops by taking the
    real part (on the asymmetric grid the truncated sum is not Hermitian)."""
    import oracle

    oracle.build(force=False)
    qr, qi = oracle.collision(N, L, lam, f[idx], with_imag=True)
    r = np.linalg.norm(qi.reshape(len(idx), -1), axis=1) / np.linalg.norm(qr.reshape(len(idx), -1), axis=1)
    return float(r.max())


def moment_drift(N, L, qc):
    """Largest relative conserved-moment residual over the cells of a batch of
    Q_c: max over cells and the five moments of |C Q_c| / (|C| |Q_c|), C the
    mass, momentum and energy rows with weight dv^3."""
    v = (2.0 * L / N) * (np.arange(N) - N // 2)
    v1, v2, v3 = np.meshgrid(v, v, v, indexing="ij")
    C = np.stack([np.ones_like(v1), v1, v2, v3, v1 * v1 + v2 * v2 + v3 * v3]).reshape(5, -1)
    q = qc.reshape(qc.shape[0], -1)
    return float((np.abs(q @ C.T) / (np.abs(q) @ np.abs(C).T)).max())


def f32_stats(N, L, lam, f, idx, got):
    """Per-cell relative L2 error of the FP32 path's Q_c (cells idx of batch f,
    got = their GPU results) against the FP64 oracle on the same FP32 input;
    the same against the FP64 input (input rounding included); and, for every
    cell above 1e-5, its FP32 storage floor (the oracle's exact sum with the
    weights and f^ rounded to FP32, projected) and its cancellation ratio
    S/||Q~|| (absolute-term scale of the sum over its result)."""
    import oracle

    oracle.build(force=False)
    idx = list(idx)
    f64 = f[idx]
    fi = f64.astype(np.float32).astype(np.float64)
    qt = oracle.collision(N, L, lam, fi)
    ref, _ = oracle.project(N, L, qt)
    rel = rel_err(got, ref)
    ref64, _ = oracle.project(N, L, oracle.collision(N, L, lam, f64))
    rel64 = rel_err(got, ref64)
    over = np.nonzero(rel > 1e-5)[0]
    listed = []
    if over.size:
        r32, _ = oracle.project(N, L, oracle.collision_round32(N, L, lam, fi[over]))
        floor = rel_err(r32, ref[over])
        S = oracle.term_scale(N, L, lam, fi[over])
        qn = np.linalg.norm(qt[over].reshape(over.size, -1), axis=1)
        listed = [{"cell": int(idx[j]), "rel_l2_err": float(rel[j]), "fp32_storage_floor": float(fl),
                   "S_over_Q": float(sq)} for j, fl, sq in zip(over, floor, S / qn)]
    return {"max_rel_l2_err": float(rel.max()), "median_rel_l2_err": float(np.median(rel)),
            "cells_rel_err_over_1e-5": int(over.size), "cells_checked": int(len(rel)),
            "cells_over_1e-5": listed,
            "max_rel_l2_err_incl_input_rounding": float(rel64.max()),
            "error_reference": "FP64 oracle on the same FP32 input"}


def bkw_point(bz, torch, reps=7):
    """The Maxwell-molecule BKW run (one cell, N = 8, L = 6, lambda = 0, BKW
    data at t = 5.5, ten forward-Euler steps of 0.01 with the projection every
    step): a latency-bound chain of 30 launches, reported as wall time (the
    median of `reps` runs, HIP events around the ten steps), with its error
    against the oracle's same ten steps and its distance from the exact BKW
    solution at t = 5.6 (the discretisation's, not a parity figure)."""
    import oracle

    w = synth.WORKLOADS["bkw_n8"]
    N, L, dt, nsteps = w["N"], w["L"], 0.01, 10
    f0 = synth.bkw(N, L, 5.5)[None].copy()
    op = bz.bz_op_create(N, L, 0, bz.BZ_F64)
    try:
        f0d = torch.from_numpy(f0).cuda()
        fd = torch.empty_like(f0d)
        qt = torch.empty_like(fd)
        qc = torch.empty_like(fd)
        stream = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(reps):
            fd.copy_(f0d)
            torch.cuda.synchronize()
            a.record(stream)
            for _ in range(nsteps):
                bz.collision_eval(op, 1, fd, qt, stream=stream)
                bz.conserve(op, 1, qt, qc, stream=stream)
                bz.bz_axpy(dt, qc, fd, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        got = fd.cpu().numpy()
    finally:
        op.destroy()
    oracle.build(force=False)
    ref = f0.copy()
    for _ in range(nsteps):
        q, _ = oracle.project(N, L, oracle.collision(N, L, 0, ref))
        ref = ref + dt * q
    exact = synth.bkw(N, L, 5.5 + nsteps * dt)[None]
    ms = float(np.median(times))
    return {"workload": "bkw_n8", "N": N, "ncells": 1, "dtype": "f64", "lambda": 0, "steps": nsteps, "dt": dt,
            "ms_per_run": ms, "us_per_step": ms / nsteps * 1e3,
            "max_rel_l2_err_vs_oracle": float(rel_err(got, ref).max()),
            "rel_l2_vs_exact_bkw": float(rel_err(got, exact).max())}


def wall_point(bz, torch, steps_total=200, per_graph=20):
    """Boundary layer: 400 wall-clustered cells on [0, 20], diffuse wall T = 2
    at x = 0, outflow at x = 20, hard spheres, N = 16, L = 8, Kn = 0.1,
    dt = 0.5 min dx / L; Strang steps replayed from HIP graphs."""
    import oracle

    w = synth.WORKLOADS["wall_n16_400"]
    N, L, M, lam, eps = w["N"], w["L"], w["ncells"], w["lam"], 0.1
    xf = synth.boundary_layer_faces(M)
    f0 = synth.boundary_layer_state(N, L, M)
    dt = 0.5 * float(np.diff(xf).min()) / L
    left = (bz.BZ_WALL_DIFFUSE, 2.0, (0.0, 0.0, 0.0))
    right = (bz.BZ_WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))
    op = bz.bz_op_create(N, L, lam, bz.BZ_F64)
    try:
        xd = torch.from_numpy(xf).cuda()
        fd = torch.from_numpy(f0).cuda()
        # accuracy: two eager steps against the oracle composition
        for _ in range(2):
            bz.bz_strang_step(op, M, fd, xd, dt, eps, left, right)
        got = fd.cpu().numpy()
        oracle.build(force=False)
        ref = f0.copy()
        for _ in range(2):
            ref = oracle.transport_step(N, L, ref, xf, 0.5 * dt, left=left, right=right)
            fi = ref[2:-2]
            q1, _ = oracle.project(N, L, oracle.collision(N, L, lam, fi))
            fs = fi + dt / eps * q1
            q2, _ = oracle.project(N, L, oracle.collision(N, L, lam, fs))
            ref = ref.copy()
            ref[2:-2] = fi + 0.5 * dt / eps * (q1 + q2)
            ref = oracle.transport_step(N, L, ref, xf, 0.5 * dt, left=left, right=right)
        err = float(np.abs(got - ref).max() / np.abs(ref).max())
        # throughput: 200 steps from graphs of 20 steps
        fd.copy_(torch.from_numpy(f0))
        g = bz.bz_graph_capture_strang(op, M, fd, xd, dt, eps, per_graph, left, right)
        try:
            g.launch()
            torch.cuda.synchronize()
            fd.copy_(torch.from_numpy(f0))
            stream = torch.cuda.current_stream()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record(stream)
            for _ in range(steps_total // per_graph):
                g.launch(stream)
            b.record(stream)
            torch.cuda.synchronize()
            el = a.elapsed_time(b) / 1e3
        finally:
            g.destroy()
        mass = float(fd[2:-2].sum().item())
    finally:
        op.destroy()
    nsteps = (steps_total // per_graph) * per_graph
    return {"workload": "wall_n16_400", "N": N, "ncells": M, "dtype": "f64", "steps": nsteps,
            "ms_per_step": el / nsteps * 1e3, "steps_per_s": nsteps / el,
            "cell_evals_per_s": 2 * M * nsteps / el, "dt": dt, "eps": eps,
            "max_abs_err_2_steps_vs_oracle_rel_to_max_f": err, "final_sum_f": mass}


def macroscopic(f, N, L):
    """Density, bulk velocity u1 and temperature of every interior cell of a
    [M+4][N][N][N] state (trapezoid sums on the velocity grid)."""
    v = synth.velocity_points(N, L)
    dv3 = (2.0 * L / N) ** 3
    v1, v2, v3 = np.meshgrid(v, v, v, indexing="ij")
    fi = f[2:-2].reshape(f.shape[0] - 4, -1)
    rho = fi.sum(axis=1) * dv3
    m1 = fi @ v1.ravel() * dv3
    e = fi @ (v1 ** 2 + v2 ** 2 + v3 ** 2).ravel() * dv3
    u = m1 / rho
    return rho, u, (e / rho - u * u) / 3.0


def wall_long_point(bz, torch, steps=4000, per_graph=50, checkpoints=(1000, 2000, 4000)):
    """Sudden heating (Tw = 2) and cooling (Tw = 0.5) of the wall, Kn = 1,
    370 cells on [0, 100], thousands of Strang steps replayed from HIP graphs;
    the macroscopic state is sampled at a few times."""
    w = synth.WORKLOADS["wall_long_n16_370"]
    N, M, lam, eps = w["N"], w["ncells"], w["lam"], w["eps"]
    xf = synth.boundary_layer_faces(M, w["X"], w["alpha"])
    xc, dx = 0.5 * (xf[1:] + xf[:-1]), np.diff(xf)
    out = {"workload": "wall_long_n16_370", "N": N, "ncells": M, "dtype": "f64", "eps": eps, "cases": []}
    xd = torch.from_numpy(xf).cuda()
    for Tw, L in w["cases"]:
        op = bz.bz_op_create(N, L, lam, bz.BZ_F64)
        try:
            f0 = synth.boundary_layer_state(N, L, M)
            dt = 0.5 * float(dx.min()) / L
            fd = torch.from_numpy(f0).cuda()
            left = (bz.BZ_WALL_DIFFUSE, Tw, (0.0, 0.0, 0.0))
            right = (bz.BZ_WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))
            g = bz.bz_graph_capture_strang(op, M, fd, xd, dt, eps, per_graph, left, right)
            try:
                g.launch()
                torch.cuda.synchronize()
                fd.copy_(torch.from_numpy(f0))
                rho0 = macroscopic(f0, N, L)[0]
                mass0 = float((rho0 * dx).sum())
                done, gpu_s, samples = 0, 0.0, []
                for ck in checkpoints:
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    while done < min(ck, steps):
                        g.launch()
                        done += per_graph
                    b.record()
                    torch.cuda.synchronize()
                    gpu_s += a.elapsed_time(b) / 1e3
                    fh = fd.cpu().numpy()
                    rho, u, T = macroscopic(fh, N, L)
                    dist = np.where(np.abs(rho - 1.0) > 1e-3)[0]
                    samples.append({"step": done, "t": done * dt, "rho_wall": float(rho[0]), "T_wall": float(T[0]),
                                    "u_max": float(u.max()), "u_min": float(u.min()),
                                    "front_x": float(xc[dist.max()]) if len(dist) else 0.0,
                                    "rho_max_x_beyond_1": float(xc[xc > 1.0][np.argmax(rho[xc > 1.0])]),
                                    "mass_drift": float((rho * dx).sum() / mass0 - 1.0),
                                    "min_f_over_max_f": float(fh[2:-2].min() / fh[2:-2].max())})
            finally:
                g.destroy()
        finally:
            op.destroy()
        out["cases"].append({"Tw": Tw, "L": L, "dt": dt, "steps": done, "ms_per_step": gpu_s / done * 1e3,
                             "samples": samples})
    return out


def mixed_point(bz, torch, reps=5):
    """4096 cells, N in {8, 16, 24, 32} at 40/30/20/10 %, hard spheres, L = 6,
    FP32 transforms and convolution, FP64 projection, one packed buffer."""
    import oracle

    w = synth.WORKLOADS["mixed_4096"]
    L, lam, nc = w["L"], w["lam"], w["ncells"]
    ns, fs = synth.mixed_n(nc, synth.seed_for(w["index"]), L)
    Ns = list(synth.MIXED_N)
    op_of = np.array([Ns.index(n) for n in ns], dtype=np.int32)
    sizes = np.array([n ** 3 for n in ns], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.concatenate([f.ravel() for f in fs]).astype(np.float32)
    ops = [bz.bz_op_create(n, L, lam, bz.BZ_F32) for n in Ns]
    try:
        fd = torch.from_numpy(flat).cuda()
        qt = torch.empty_like(fd)
        qc = torch.empty(fd.shape, dtype=torch.float64, device="cuda")
        tuned = {f"N{n}": bz.bz_autotune(o, int(np.sum(op_of == i)))[:2] for i, (n, o) in enumerate(zip(Ns, ops))}
        one, ms_one, ms_per_op = bz.bz_autotune_ragged(ops, op_of, offs, bz.BZ_F32)
        bz.collision_eval_ragged(ops, op_of, offs, fd, qt, bz.BZ_F32)
        bz.conserve_ragged(ops, op_of, offs, qt, qc)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            bz.collision_eval_ragged(ops, op_of, offs, fd, qt, bz.BZ_F32, stream=stream)
            bz.conserve_ragged(ops, op_of, offs, qt, qc, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        el = a.elapsed_time(b) / 1e3
        out = qc.cpu().numpy()
        # the same step captured in a HIP graph (the autotuned form), replayed
        with bz.bz_graph_capture_ragged(ops, op_of, offs, fd, qt, qc, bz.BZ_F32) as g:
            g.launch(stream)
            torch.cuda.synchronize()
            a.record(stream)
            for _ in range(reps):
                g.launch(stream)
            b.record(stream)
            torch.cuda.synchronize()
            el_graph = a.elapsed_time(b) / 1e3
            graph_equal = bool(np.array_equal(qc.cpu().numpy(), out))
    finally:
        for o in ops:
            o.destroy()
    # error on a sample: two cells of each N (one of N = 32)
    oracle.build(force=False)
    stats = {}
    for n, k in zip(Ns, (16, 16, 8, 2)):
        idx = [i for i in range(nc) if ns[i] == n]
        sel = [idx[int(j)] for j in np.linspace(0, len(idx) - 1, k).astype(int)]
        fsel = np.stack([fs[i] for i in sel])
        got = np.stack([out[offs[i]:offs[i] + n ** 3].reshape(n, n, n) for i in sel])
        stats[f"N{n}"] = f32_stats(n, L, lam, fsel, range(len(sel)), got)
        for c in stats[f"N{n}"]["cells_over_1e-5"]:
            c["cell"] = sel[c["cell"]]
    counts = {f"N{n}": int(sum(1 for x in ns if x == n)) for n in Ns}
    return {"workload": "mixed_4096", "ncells": nc, "cells_per_N": counts, "dtype": "f32 (FP64 projection)",
            "autotuned_split": tuned,
            "convolution_form": {"chosen": "one launch" if one else "per-op launches on forked streams",
                                 "one_launch_ms": ms_one, "per_op_ms": ms_per_op},
            "ms_per_step": el / reps * 1e3, "cell_evals_per_s": nc * reps / el,
            "graph": {"ms_per_step": el_graph / reps * 1e3, "cell_evals_per_s": nc * reps / el_graph,
                      "bitwise_equal_to_eager": graph_equal},
            "algorithmic_tflops": sum(conv_flops_per_cell(n) * counts[f"N{n}"] for n in Ns) * reps / el / 1e12,
            "error_sample": stats}


def run_probes(torch):
    """Measured ceilings: FMA issue rate (FP64 and non-packed FP32, all-VGPR
    operands and one wave-uniform SGPR operand) and stream bandwidth (read
    and copy) over a 4 GiB buffer (HBM) and 64 and 160 MiB ones (resident in
    the 256 MB last-level cache, larger than the 8 x 4 MB of L2)."""
    import ctypes

    from paper_1301_4195_amd import build as hipbuild

    if not os.path.exists(hipbuild.PROBE_LIB):
        raise RuntimeError(f"{hipbuild.PROBE_LIB} not built")
    lib = ctypes.CDLL(hipbuild.PROBE_LIB)
    vp, d = ctypes.c_void_p, ctypes.c_double
    lib.bzp_fma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, vp,
                            ctypes.POINTER(d)]
    lib.bzp_stream.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int64, ctypes.c_int, vp, ctypes.c_int, vp,
                               ctypes.POINTER(d)]
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    blocks, iters = 8192, 4096
    obuf = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    for fp64 in (1, 0):
        for sgpr in (0, 1):
            ms = d()
            rc = lib.bzp_fma(fp64, sgpr, blocks, iters, obuf.data_ptr(), 5, stream, ctypes.byref(ms))
            if rc:
                raise RuntimeError(f"bzp_fma failed: {rc}")
            flops = 2.0 * 8 * iters * blocks * 256
            out[f"fma_{'f64' if fp64 else 'f32'}_{'sgpr' if sgpr else 'vgpr'}"] = {
                "tflops": flops / (ms.value * 1e-3) / 1e12,
                "wave_instr_per_s": flops / 2 / 64 / (ms.value * 1e-3), "ms": ms.value,
                "frac_of_78.6": flops / (ms.value * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
    sums = torch.empty(8192 * 256, dtype=torch.int32, device="cuda")
    for name, nbytes, reps in (("hbm_4GiB", 4 << 30, 10), ("llc_64MiB", 64 << 20, 200),
                               ("llc_160MiB", 160 << 20, 100)):
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        for copy in (0, 1):
            if copy:
                half = nbytes // 2
                dst = torch.empty(half // 4, dtype=torch.int32, device="cuda")
                n = half
            else:
                dst, n = None, nbytes
            ms = d()
            rc = lib.bzp_stream(copy, src.data_ptr(), dst.data_ptr() if dst is not None else None, n, 8192,
                                sums.data_ptr(), reps, stream, ctypes.byref(ms))
            if rc:
                raise RuntimeError(f"bzp_stream failed: {rc}")
            moved = n * (2 if copy else 1)
            out[f"{'copy' if copy else 'read'}_{name}"] = {"TBps": moved / (ms.value * 1e-3) / 1e12,
                                                          "bytes_per_launch": moved, "ms": ms.value,
                                                          "frac_of_8TBps": moved / (ms.value * 1e-3) / HBM_PEAK}
            del dst
        del src
    torch.cuda.synchronize()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-points", action="store_true", help="skip the FP32 and N=32 extra points")
    ap.add_argument("--only", choices=["f32_n16_256", "f64_n32_512", "f32_n32_512", "unbatched_f64_n16",
                                       "unbatched_f64_n32"], default=None,
                    help="time just this configuration (default split) and print one line to stderr; for "
                         "profiling a single kernel")
    ap.add_argument("--fly", action="store_true", help="with --only: an op whose weights are computed on the fly")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the timed region, copy a buffer of this many MiB three times (a plain copy "
                         "kernel of known size, to calibrate HBM traffic counters)")
    ap.add_argument("--probes", action="store_true",
                    help="run the ceiling probes (FMA issue in FP64 and FP32, memory streams over HBM- and "
                         "last-level-cache-sized buffers) and print one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (cells need no communication between GPUs, so N GPUs would "
              "each run this benchmark on their own share); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1301_4195_amd as bz

    bz.load()
    if args.probes:
        print(json.dumps({"probes": run_probes(torch)}), flush=True)
        return
    if args.only and args.only.startswith("unbatched_"):
        # the plain FP64 path, one cell per call, over `steps` cells
        wk = synth.WORKLOADS["hs_" + args.only.split("_", 2)[2] + ("_256" if args.only.endswith("16") else "_512")]
        fo = synth.two_maxwellian(wk["N"], wk["L"], args.steps, synth.seed_for(wk["index"]))
        pt = unbatched_point(bz, torch, wk["N"], wk["L"], wk["lam"], fo)
        print(f"bench --only {args.only}: {pt['evals_per_s']:.4g} evals/s, {pt['convolution_form']} convolution "
              f"{pt['conv_ms']:.4f} ms per launch (weights at {pt['weight_stream_TBps']:.2f} TB/s), "
              f"split {pt['split']}", file=sys.stderr, flush=True)
        return
    if args.only:
        dt, wname = args.only.split("_", 1)
        wk = synth.WORKLOADS["hs_" + wname]
        fo = synth.two_maxwellian(wk["N"], wk["L"], wk["ncells"], synth.seed_for(wk["index"]))
        el, cms, _, _, sp = run_gpu(bz, torch, wk["N"], wk["L"], wk["lam"], fo, bz.BZ_F64 if dt == "f64" else bz.BZ_F32,
                                    args.steps, args.warmup, fly=args.fly)
        print(f"bench --only {args.only}{' --fly' if args.fly else ''}: {wk['ncells'] * args.steps / el:.4g} evals/s, "
              f"conv {cms:.3f} ms per launch, split {sp}", file=sys.stderr, flush=True)
        return
    w = synth.WORKLOADS["hs_n16_256"]
    N, L, lam, ncells = w["N"], w["L"], w["lam"], w["ncells"]
    f = synth.two_maxwellian(N, L, ncells, synth.seed_for(w["index"]))
    print(f"bench: workload hs_n16_256 N={N} ncells={ncells} FP64, warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    elapsed, conv_ms, qc64, _, split = run_gpu(bz, torch, N, L, lam, f, bz.BZ_F64, args.steps, args.warmup)
    value = ncells * args.steps / elapsed
    flops = conv_flops_per_cell(N) * ncells
    achieved = flops / (conv_ms / 1e3) / 1e12
    sample = list(range(ncells))
    ref = oracle_ref(N, L, lam, f, sample)
    err64 = rel_err(qc64[sample], ref)
    line = {
        "metric": "collision evals/sec (cells*evals/s) at N=16,32: FP32-batched vs FP64 at stated err",
        "value": value,
        "unit": "cell-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded two-Maxwellian cells)",
        "config": {"workload": "hs_n16_256: 256 cells, hard spheres, N=16, L=6, FP64 collision_eval + conserve",
                   "N": N, "ncells": ncells, "lambda": lam, "L": L,
                   "max_rel_l2_err_vs_oracle": float(err64.max()), "err_cells_checked": len(sample),
                   "oracle_imag_over_real": oracle_imag_ratio(N, L, lam, f, [0, ncells // 2, ncells - 1])},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": conv_traffic_bytes(),
                     "kernel": f"conv_kernel<double, {N}, {split[1]}>", "split": {"m1_chunks": split[0], "k3_ranges": split[1]},
                     "kernel_ms": conv_ms,
                     "flops_per_launch": flops,
                     "executed_flops_per_launch": conv_executed_flops_per_cell(N) * ncells,
                     "executed_tflops": conv_executed_flops_per_cell(N) * ncells / (conv_ms / 1e3) / 1e12,
                     "executed_frac": conv_executed_flops_per_cell(N) * ncells / (conv_ms / 1e3) / 1e12
                     / PEAK_FP64_TFLOPS},
    }
    print(f"bench: FP64 N=16 {value:.4g} evals/s, conv {conv_ms:.3f} ms, err {err64.max():.2e}",
          file=sys.stderr, flush=True)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"bench: copy calibration {args.copy_calibration_mib} MiB x3 done", file=sys.stderr, flush=True)

    if not args.no_points:
        points = []
        el32, cms32, qc32, tu32, _ = run_gpu(bz, torch, N, L, lam, f, bz.BZ_F32, args.steps, args.warmup, tune=True)
        points.append({"N": N, "ncells": ncells, "dtype": "f32", "evals_per_s": ncells * args.steps / el32,
                       "conv_ms": cms32, "conv_tflops": flops / (cms32 / 1e3) / 1e12, "autotuned_split": tu32[:2],
                       "speedup_vs_f64": (ncells * args.steps / el32) / value,
                       "moment_drift_max": moment_drift(N, L, qc32),
                       **f32_stats(N, L, lam, f, sample, qc32[sample])})
        print(f"bench: FP32 N=16 {points[-1]['evals_per_s']:.4g} evals/s err max {points[-1]['max_rel_l2_err']:.2e}",
              file=sys.stderr, flush=True)
        # the headline configuration again, with the work split chosen by the autotuner
        elt, cmst, qct, tut, _ = run_gpu(bz, torch, N, L, lam, f, bz.BZ_F64, args.steps, args.warmup, tune=True)
        points.append({"N": N, "ncells": ncells, "dtype": "f64", "autotuned_split": tut[:2],
                       "evals_per_s": ncells * args.steps / elt, "conv_ms": cmst,
                       "conv_tflops": flops / (cmst / 1e3) / 1e12,
                       "max_rel_l2_err": float(rel_err(qct[sample], ref).max())})
        print(f"bench: FP64 N=16 autotuned (split {tut[:2]}) {points[-1]['evals_per_s']:.4g} evals/s",
              file=sys.stderr, flush=True)
        # 1024 cells at N = 24, FP32 transforms and convolution, FP64 projection
        w24 = synth.WORKLOADS["hs_n24_1024"]
        N3, n3c = w24["N"], w24["ncells"]
        f3 = synth.two_maxwellian(N3, w24["L"], n3c, synth.seed_for(w24["index"]))
        s3 = list(np.linspace(0, n3c - 1, 64).astype(int))
        st3 = max(2, args.steps // 10)
        el3, cms3, q3, tu3, _ = run_gpu(bz, torch, N3, w24["L"], w24["lam"], f3, bz.BZ_F32, st3, 1, tune=True)
        points.append({"N": N3, "ncells": n3c, "dtype": "f32", "autotuned_split": tu3[:2],
                       "evals_per_s": n3c * st3 / el3, "conv_ms": cms3,
                       "conv_tflops": conv_flops_per_cell(N3) * n3c / (cms3 / 1e3) / 1e12,
                       "moment_drift_max": moment_drift(N3, w24["L"], q3),
                       **f32_stats(N3, w24["L"], w24["lam"], f3, s3, q3[s3])})
        print(f"bench: f32 N=24 {points[-1]['evals_per_s']:.4g} evals/s err max {points[-1]['max_rel_l2_err']:.2e}",
              file=sys.stderr, flush=True)
        # variable hard spheres (lambda = 0.5): weights by quadrature of the
        # radial integral, the same convolution; same inputs as the headline
        lam_v = 0.5
        tb = time.perf_counter()
        with bz.bz_op_create(N, L, lam_v, bz.BZ_F64):
            torch.cuda.synchronize()
        build_v = time.perf_counter() - tb
        tb = time.perf_counter()
        with bz.bz_op_create(N, L, lam, bz.BZ_F64):
            torch.cuda.synchronize()
        build_c = time.perf_counter() - tb
        elv, cmsv, qcv, _, _ = run_gpu(bz, torch, N, L, lam_v, f, bz.BZ_F64, args.steps, args.warmup)
        sv = [0, ncells // 2, ncells - 1]
        refv = oracle_ref(N, L, lam_v, f, sv)
        points.append({"N": N, "ncells": ncells, "dtype": "f64", "lambda": lam_v, "evals_per_s": ncells * args.steps / elv,
                       "conv_ms": cmsv, "max_rel_l2_err": float(rel_err(qcv[sv], refv).max()), "cells_checked": len(sv),
                       "op_create_s_quadrature": build_v, "op_create_s_closed_form": build_c})
        print(f"bench: FP64 N=16 lambda=0.5 {points[-1]['evals_per_s']:.4g} evals/s err max "
              f"{points[-1]['max_rel_l2_err']:.2e}", file=sys.stderr, flush=True)
        # inelastic hard spheres (beta = 0.8, restitution 0.6): projection onto
        # mass and momentum only
        beta_i = 0.8
        opi = bz.bz_op_create_inelastic(N, L, lam, beta_i, bz.BZ_F64)
        try:
            fdi = torch.from_numpy(f).cuda()
            qti = torch.empty_like(fdi)
            qci = torch.empty_like(fdi)
            for _ in range(args.warmup):
                bz.collision_eval(opi, ncells, fdi, qti)
                bz.conserve(opi, ncells, qti, qci)
            torch.cuda.synchronize()
            a_ev, b_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a_ev.record()
            for _ in range(args.steps):
                bz.collision_eval(opi, ncells, fdi, qti)
                bz.conserve(opi, ncells, qti, qci)
            b_ev.record()
            torch.cuda.synchronize()
            eli = a_ev.elapsed_time(b_ev) / 1e3
            qci_h = qci.cpu().numpy()
        finally:
            opi.destroy()
        import oracle
        si = [0, ncells // 2, ncells - 1]
        refi, _ = oracle.project(N, L, oracle.collision(N, L, lam, f[si], beta=beta_i), energy=False)
        points.append({"N": N, "ncells": ncells, "dtype": "f64", "lambda": lam, "beta": beta_i,
                       "evals_per_s": ncells * args.steps / eli,
                       "max_rel_l2_err": float(rel_err(qci_h[si], refi).max()), "cells_checked": len(si)})
        print(f"bench: FP64 N=16 inelastic beta=0.8 {points[-1]['evals_per_s']:.4g} evals/s err max "
              f"{points[-1]['max_rel_l2_err']:.2e}", file=sys.stderr, flush=True)
        w32 = synth.WORKLOADS["hs_n32_512"]
        N2, n2 = w32["N"], w32["ncells"]
        f2 = synth.two_maxwellian(N2, L, n2, synth.seed_for(w32["index"]))
        s2 = [0, n2 // 2, n2 - 1]
        ref2 = oracle_ref(N2, L, lam, f2, s2)
        s2f = list(np.linspace(0, n2 - 1, 12).astype(int))
        flops2 = conv_flops_per_cell(N2) * n2
        rate64 = None
        for dt, name, fly in ((bz.BZ_F64, "f64", False), (bz.BZ_F32, "f32", False), (bz.BZ_F64, "f64", True)):
            st = max(2, args.steps // 10)
            inf = {}
            el, cms, q, tu, _ = run_gpu(bz, torch, N2, L, lam, f2, dt, st, 1, tune=True, fly=fly, info=inf)
            pt = {"N": N2, "ncells": n2, "dtype": name, "evals_per_s": n2 * st / el, "conv_ms": cms,
                  "conv_tflops": flops2 / (cms / 1e3) / 1e12, "autotuned_split": tu[:2],
                  "weights": "computed on the fly (default slabs)" if fly else "stored table",
                  "op_table_bytes": inf["table_bytes"]}
            if name == "f64":
                if not fly:
                    rate64 = pt["evals_per_s"]
                pt["max_rel_l2_err"] = float(rel_err(q[s2], ref2).max())
            else:
                pt["speedup_vs_f64"] = pt["evals_per_s"] / rate64
                rate32_n32 = pt["evals_per_s"]
                pt["moment_drift_max"] = moment_drift(N2, L, q)
                pt.update(f32_stats(N2, L, lam, f2, s2f, q[s2f]))
            points.append(pt)
            print(f"bench: {name} N=32 {pt['weights']} {pt['evals_per_s']:.4g} evals/s err max "
                  f"{pt['max_rel_l2_err']:.2e}, weights {pt['op_table_bytes'] / 1e6:.0f} MB", file=sys.stderr, flush=True)
        # the 48-point mesh (beyond the tables of the paper), 128 cells: stored
        # table and weights computed on the fly, in both precisions (parity
        # with the oracle is in the GPU tests; here the two forms against each
        # other)
        f48 = synth.two_maxwellian(48, L, 128, synth.seed_for(8))
        for dt, name in ((bz.BZ_F64, "f64"), (bz.BZ_F32, "f32")):
            res = {}
            for fly in (False, True):
                inf = {}
                el, cms, q, _, sp = run_gpu(bz, torch, 48, L, lam, f48, dt, 2, 1, fly=fly, info=inf)
                res[fly] = (el, cms, q, inf["table_bytes"], sp)
            for fly in (False, True):
                el, cms, q, tb, sp = res[fly]
                pt = {"N": 48, "ncells": 128, "dtype": name, "evals_per_s": 128 * 2 / el, "conv_ms": cms,
                      "conv_tflops": conv_flops_per_cell(48) * 128 / (cms / 1e3) / 1e12, "split": list(sp),
                      "weights": "computed on the fly (default slabs)" if fly else "stored table",
                      "op_table_bytes": tb}
                if fly:
                    pt["max_rel_l2_diff_vs_stored"] = float(rel_err(q, res[False][2]).max())
                points.append(pt)
                print(f"bench: {name} N=48 {pt['weights']} {pt['evals_per_s']:.4g} evals/s, "
                      f"weights {tb / 1e9:.2f} GB", file=sys.stderr, flush=True)
        # the plain FP64 path (one cell per call) at N = 16 and N = 32, and the
        # batched FP32 path's speedup over it
        for NN, ff, rate32 in ((N, f, points[0]["evals_per_s"]), (N2, f2[:8], rate32_n32)):
            pt = unbatched_point(bz, torch, NN, L, lam, ff)
            pt["speedup_of_f32_batched"] = rate32 / pt["evals_per_s"]
            points.append(pt)
            print(f"bench: FP64 N={NN} one cell per call {pt['evals_per_s']:.4g} evals/s "
                  f"(FP32 batched {pt['speedup_of_f32_batched']:.0f}x), {pt['convolution_form']} convolution "
                  f"{pt['conv_ms'] * 1e3:.1f} us = weights at {pt['weight_stream_TBps']:.2f} TB/s",
                  file=sys.stderr, flush=True)
        # the headline batch with weights computed on the fly
        inf = {}
        elf, cmsf, qcf, _, _ = run_gpu(bz, torch, N, L, lam, f, bz.BZ_F64, args.steps, args.warmup, fly=True, info=inf)
        sf = [0, ncells // 2, ncells - 1]
        points.append({"N": N, "ncells": ncells, "dtype": "f64", "weights": "computed on the fly (one slab)",
                       "evals_per_s": ncells * args.steps / elf, "conv_ms": cmsf, "op_table_bytes": inf["table_bytes"],
                       "max_rel_l2_err": float(rel_err(qcf[sf], ref[sf]).max()), "cells_checked": len(sf)})
        print(f"bench: FP64 N=16 weights on the fly {points[-1]['evals_per_s']:.4g} evals/s", file=sys.stderr,
              flush=True)
        points.append(bkw_point(bz, torch))
        print(f"bench: BKW N=8 ten Euler steps {points[-1]['us_per_step']:.1f} us/step, err vs oracle "
              f"{points[-1]['max_rel_l2_err_vs_oracle']:.2e}", file=sys.stderr, flush=True)
        print("bench: boundary-layer step (HIP graph)", file=sys.stderr, flush=True)
        points.append(wall_point(bz, torch))
        print(f"bench: wall {points[-1]['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        print("bench: sudden heating / cooling, 4000 steps each", file=sys.stderr, flush=True)
        points.append(wall_long_point(bz, torch))
        print("bench: " + ", ".join(f"Tw={c['Tw']} {c['ms_per_step']:.3f} ms/step front {c['samples'][-1]['front_x']:.1f}"
                                     for c in points[-1]["cases"]), file=sys.stderr, flush=True)
        print("bench: mixed-N 4096-cell batch", file=sys.stderr, flush=True)
        points.append(mixed_point(bz, torch))
        print(f"bench: mixed {points[-1]['cell_evals_per_s']:.4g} evals/s", file=sys.stderr, flush=True)
        line["points"] = points

    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(N, L, lam, f)
        if not args.no_points:  # the oracle's per-cell rate at N = 32 (4 cells), beside the N = 32 points
            w32 = synth.WORKLOADS["hs_n32_512"]
            line["cpu_baseline"]["n32"] = oracle_rate(
                w32["N"], L, lam, synth.two_maxwellian(w32["N"], L, w32["ncells"], synth.seed_for(w32["index"]))[:4])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
