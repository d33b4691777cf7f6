"""Seeded synthetic inputs shared by the oracle side (tests) and the GPU side.

This module holds no arithmetic of the collision method itself: it only
draws random parameters and evaluates closed-form distribution functions
(Maxwellians, the BKW solution) at the velocity grid points
v_j = dv (j - N/2), dv = 2L/N of Sec. 3.1.

Recipes (all FP64 on the host, seed = 13014195 + workload index):

* ``two_maxwellian``: per cell, for i = 1, 2: rho_i ~ U[0.5, 2],
  V_i ~ U[-1, 1]^3, T_i ~ U[0.5, 1.5];
  f(v) = sum_i rho_i (2 pi T_i)^{-3/2} exp(-|v - V_i|^2 / (2 T_i)).
* ``bkw``: the Bobylev-Krook-Wu self-similar solution for Maxwell molecules
  with b = 1/(4 pi):  f = exp(-|v|^2/(2K)) / (2 (2 pi K)^{3/2})
  [(5K - 3)/K + (1 - K)|v|^2/K^2],  K = 1 - exp(-t/6).
* ``mixed_n``: N drawn from {8, 16, 24, 32} with p = 0.4/0.3/0.2/0.1, then
  the two-Maxwellian draw above.
* ``boundary_layer``: 400 cells on [0, 20] with faces
  x_j = 20 (exp(alpha j / 400) - 1)/(exp(alpha) - 1), alpha = 2.33, and a
  unit Maxwellian at rest in every cell.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 13014195


def seed_for(index: int) -> int:
    return BASE_SEED + int(index)


def velocity_points(N: int, L: float) -> np.ndarray:
    """The 1-D velocity mesh v_j = (2L/N)(j - N/2), j = 0..N-1."""
    return (2.0 * L / N) * (np.arange(N) - N // 2)


def _grid(N: int, L: float):
    v = velocity_points(N, L)
    return np.meshgrid(v, v, v, indexing="ij")


def maxwellian(N: int, L: float, rho: float, V, T: float) -> np.ndarray:
    v1, v2, v3 = _grid(N, L)
    d2 = (v1 - V[0]) ** 2 + (v2 - V[1]) ** 2 + (v3 - V[2]) ** 2
    return rho * (2.0 * math.pi * T) ** -1.5 * np.exp(-d2 / (2.0 * T))


def two_maxwellian_params(rng: np.random.Generator, ncells: int):
    """Per-cell (rho, V, T) for the two Maxwellians, drawn in a fixed order."""
    out = []
    for _ in range(ncells):
        cell = []
        for _i in range(2):
            rho = rng.uniform(0.5, 2.0)
            V = rng.uniform(-1.0, 1.0, size=3)
            T = rng.uniform(0.5, 1.5)
            cell.append((rho, V, T))
        out.append(cell)
    return out


def two_maxwellian(N: int, L: float, ncells: int, seed: int) -> np.ndarray:
    """[ncells, N, N, N] float64 batch of two-Maxwellian cells."""
    rng = np.random.default_rng(seed)
    params = two_maxwellian_params(rng, ncells)
    f = np.empty((ncells, N, N, N))
    for c, cell in enumerate(params):
        f[c] = sum(maxwellian(N, L, rho, V, T) for rho, V, T in cell)
    return f


def bkw_K(t: float) -> float:
    return 1.0 - math.exp(-t / 6.0)


def bkw(N: int, L: float, t: float) -> np.ndarray:
    """BKW distribution at time t on the N^3 grid, shape [N, N, N]."""
    K = bkw_K(t)
    v1, v2, v3 = _grid(N, L)
    r2 = v1 * v1 + v2 * v2 + v3 * v3
    return (np.exp(-r2 / (2.0 * K)) / (2.0 * (2.0 * math.pi * K) ** 1.5)
            * ((5.0 * K - 3.0) / K + (1.0 - K) * r2 / (K * K)))


MIXED_N = (8, 16, 24, 32)
MIXED_P = (0.4, 0.3, 0.2, 0.1)


def mixed_n(ncells: int, seed: int, L: float = 6.0):
    """Mixed-resolution batch: returns (list of N per cell, list of f arrays)."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.array(MIXED_N), size=ncells, p=np.array(MIXED_P))
    params = two_maxwellian_params(rng, ncells)
    fs = []
    for n, cell in zip(ns, params):
        fs.append(sum(maxwellian(int(n), L, rho, V, T) for rho, V, T in cell))
    return [int(n) for n in ns], fs


def boundary_layer_faces(M: int = 400, X: float = 20.0, alpha: float = 2.33) -> np.ndarray:
    """Faces of the wall-clustered 1-D mesh, x_0 = 0 at the wall."""
    j = np.arange(M + 1, dtype=np.float64)
    return X * np.expm1(alpha * j / M) / math.expm1(alpha)


def boundary_layer_state(N: int, L: float, M: int = 400) -> np.ndarray:
    """[M+4, N, N, N]: unit Maxwellian at rest in every cell, ghosts included."""
    m = maxwellian(N, L, 1.0, (0.0, 0.0, 0.0), 1.0)
    return np.broadcast_to(m, (M + 4, N, N, N)).copy()


# Workloads (sizes of the paper's experiments restated as synthetic batches).
WORKLOADS = {
    "bkw_n8": dict(index=0, N=8, L=6.0, lam=0, ncells=1, dtype="f64"),
    "hs_n16_256": dict(index=1, N=16, L=6.0, lam=1, ncells=256, dtype="f64"),
    "hs_n24_1024": dict(index=2, N=24, L=6.0, lam=1, ncells=1024, dtype="f32"),
    "wall_n16_400": dict(index=3, N=16, L=8.0, lam=1, ncells=400, dtype="f64"),
    "mixed_4096": dict(index=4, N=0, L=6.0, lam=1, ncells=4096, dtype="f32"),
    "hs_n32_512": dict(index=6, N=32, L=6.0, lam=1, ncells=512, dtype="f32"),
    # sudden heating (Tw = 2) and cooling (Tw = 0.5) of the wall over long
    # times, Sec. 5 setting: Kn = eps = 1, eight cells per mean free path at
    # the wall and two in the interior (first cell 0.125, last 0.5: faces
    # with alpha = ln 4 over [0, 100], 370 cells); velocity box L = 8 for the
    # heated gas and L = 6 for the cooled one (cases: (Tw, L))
    "wall_long_n16_370": dict(index=7, N=16, lam=1, ncells=370, dtype="f64", X=100.0,
                              alpha=math.log(4.0), eps=1.0, cases=((2.0, 8.0), (0.5, 6.0))),
}
