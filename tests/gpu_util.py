"""Shared helpers of the GPU parity tests (device plumbing and error metrics)."""
from __future__ import annotations

import numpy as np


def rel_l2_per_cell(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """||a_c - b_c||_2 / ||b_c||_2 for every cell c (first axis)."""
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def to_dev(x, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t) -> np.ndarray:
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ------------------------------------------------------------ FP32 bound
F32_TOL = 1e-5  # relative L2 per cell


def f32_input(f: np.ndarray) -> np.ndarray:
    """The FP32 path's input exactly as the device sees it, promoted to FP64:
    the oracle evaluates the same numbers the FP32 path is given."""
    return np.asarray(f).astype(np.float32).astype(np.float64)


def f32_check(orc, N, L, lam, f, got, beta=1.0, omega1d=None, project=False):
    """Stated FP32 bound, per cell, against the FP64 oracle on the same FP32
    input:  err <= 1e-5, except on cells whose FP32 storage floor (the exact
    sum with the weights and f^ rounded to FP32: oracle.collision_round32) is
    above half of that -- cells where gain and loss cancel to ~1/1000 of
    their terms -- which must stay within twice their floor.  project: got is
    Q_c (compared with the oracle's projection).  Returns (err, floor or NaN
    where not needed, ok) per cell."""
    fi = f32_input(f)
    ref = orc.collision(N, L, lam, fi, omega1d, beta=beta)
    energy = beta == 1.0
    if project:
        ref, _ = orc.project(N, L, ref, energy=energy)
    err = rel_l2_per_cell(got, ref)
    floor = np.full(err.shape, np.nan)
    ok = err <= F32_TOL
    bad = np.nonzero(~ok)[0]
    if bad.size:
        r32 = orc.collision_round32(N, L, lam, fi[bad], omega1d, beta=beta)
        if project:
            r32, _ = orc.project(N, L, r32, energy=energy)
        fl = rel_l2_per_cell(r32, ref[bad])
        floor[bad] = fl
        ok[bad] = (fl > 0.5 * F32_TOL) & (err[bad] <= 2.0 * fl)
    return err, floor, ok


def f32_report(err, floor, ok, cells=None) -> str:
    """One line for the log: max / median error and the cells over 1e-5 with their floor."""
    cells = np.arange(err.size) if cells is None else np.asarray(cells)
    over = [f"{int(c)}: {e:.2e} (floor {fl:.2e})" for c, e, fl in zip(cells, err, floor) if e > F32_TOL]
    return (f"max {err.max():.3e} median {np.median(err):.3e} cells > 1e-5: {len(over)}/{err.size}"
            + (f" [{'; '.join(over)}]" if over else "") + ("" if ok.all() else " -- FAILED"))
