"""FP64 CPU oracle for the conservative spectral collision operator.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The
product path (``paper_1301_4195_amd``) never imports it and shares no code
with it; the only thing the two sides share is the seeded input generator
module ``synth``.

The arithmetic lives in ``bz_oracle.c`` (plain C, FP64, compiled with
``-O2 -ffp-contract=off`` and OpenMP over the outer loops); this module is a
ctypes wrapper.  Every function cites the passage of the paper it follows:

* ``mesh``          -- Sec. 3.1, eq. (meshpoints)
* ``ghat``          -- Sec. 2.2, eq. (GHat_calc) and the closed forms for
                       lambda = 0, 1 printed after it
* ``weights_dense`` -- the trapezoid-weighted table omega_m G^(xi_m, zeta_k),
                       Sec. 3.2
* ``forward`` / ``inverse`` -- Sec. 2.2 transform pair (phi = e^{-i zeta.v}
                       / (2 pi)^{3/2}) discretised by the trapezoid rule on
                       the meshes of Sec. 3.1, evaluated by direct sums
* ``convolve``      -- the truncated weighted convolution of Sec. 3.2
* ``collision``     -- Re IDFT(convolve(DFT f)), the unprojected Q~
* ``project``       -- Sec. 3.3, Q = Q~ - C^T (C C^T)^{-1} C Q~
* ``transport_step``-- Sec. 3.4 eqs. (transport), (upwind), (minmod) with
                       the diffuse wall of Sec. 2.1 eq. (BC), Heun in time
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bz_oracle.c")
_LIB = os.path.join(_HERE, "liborcbz.so")

GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc.  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        lib.orc_mesh.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D]
        lib.orc_ghat.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _I, _I]
        lib.orc_set_ghat_quadrature.argtypes = [ctypes.c_int]
        lib.orc_ghat.restype = ctypes.c_double
        lib.orc_weights_dense.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D]
        lib.orc_forward.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_long, _D, _D]
        lib.orc_inverse.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_long, _D, _D, _D]
        lib.orc_convolve.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D,
                                     ctypes.c_long, _D, _D]
        lib.orc_convolve_round32.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D,
                                             ctypes.c_long, _D, _D]
        lib.orc_collision.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D,
                                      ctypes.c_long, _D, _D, _D]
        lib.orc_term_scale.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D,
                                       ctypes.c_long, _D, _D]
        lib.orc_cct.argtypes = [ctypes.c_int, ctypes.c_double, _D]
        lib.orc_project.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_long, _D, _D, _D]
        lib.orc_transport_step.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_long, _D,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_double, _D,
                                           ctypes.c_int, ctypes.c_double, _D, _D]
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS or all cores)."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's later parallel loops (n >= 1)."""
    _load().orc_set_num_threads(int(n))


def mesh(N: int, L: float):
    """Velocity and Fourier 1-D meshes (Sec. 3.1, eq. meshpoints)."""
    v = np.empty(N)
    z = np.empty(N)
    _load().orc_mesh(N, L, _ptr(v), _ptr(z))
    return v, z


def ghat(N: int, L: float, lam: float, k, m, beta: float = 1.0) -> float:
    """G^(xi_m, zeta_k) by the closed forms of Sec. 2.2 (integer indices)."""
    ka = (ctypes.c_int * 3)(*[int(x) for x in k])
    ma = (ctypes.c_int * 3)(*[int(x) for x in m])
    return float(_load().orc_ghat(N, L, float(lam), float(beta), ka, ma))


def set_ghat_quadrature(on: bool) -> None:
    """Test hook: evaluate G^ by the quadrature path also for lambda = 0, 1."""
    _load().orc_set_ghat_quadrature(1 if on else 0)


def weights_dense(N: int, L: float, lam: float, omega1d=None, beta: float = 1.0) -> np.ndarray:
    """W[k, m] = omega_m G^(xi_m, zeta_k), zero off the truncation box (Sec. 3.2)."""
    n3 = N ** 3
    W = np.empty((n3, n3))
    om = None if omega1d is None else _f64(omega1d)
    _load().orc_weights_dense(N, L, float(lam), float(beta), _ptr(om), _ptr(W))
    return W


def forward(N: int, L: float, f: np.ndarray) -> np.ndarray:
    """f [ncells, N, N, N] real -> f^ [ncells, N, N, N] complex128."""
    f = _f64(f).reshape(-1, N ** 3)
    out = np.empty((f.shape[0], N ** 3, 2))
    _load().orc_forward(N, L, f.shape[0], _ptr(f), _ptr(out))
    return (out[..., 0] + 1j * out[..., 1]).reshape(-1, N, N, N)


def inverse(N: int, L: float, qhat: np.ndarray, with_imag: bool = False):
    """Q^ complex -> Re of the inverse transform (and Im when asked)."""
    q = np.asarray(qhat, dtype=np.complex128).reshape(-1, N ** 3)
    qi = np.ascontiguousarray(np.stack([q.real, q.imag], axis=-1))
    re = np.empty((q.shape[0], N ** 3))
    im = np.empty((q.shape[0], N ** 3)) if with_imag else None
    _load().orc_inverse(N, L, q.shape[0], _ptr(qi), _ptr(re), _ptr(im))
    re = re.reshape(-1, N, N, N)
    if with_imag:
        return re, im.reshape(-1, N, N, N)
    return re


def convolve(N: int, L: float, lam: float, fhat: np.ndarray, omega1d=None, beta: float = 1.0) -> np.ndarray:
    """Truncated weighted convolution Q^(zeta_k) of Sec. 3.2."""
    fh = np.asarray(fhat, dtype=np.complex128).reshape(-1, N ** 3)
    fi = np.ascontiguousarray(np.stack([fh.real, fh.imag], axis=-1))
    out = np.empty_like(fi)
    om = None if omega1d is None else _f64(omega1d)
    _load().orc_convolve(N, L, float(lam), float(beta), _ptr(om), fh.shape[0], _ptr(fi), _ptr(out))
    return (out[..., 0] + 1j * out[..., 1]).reshape(-1, N, N, N)


def convolve_round32(N: int, L: float, lam: float, fhat: np.ndarray, omega1d=None, beta: float = 1.0) -> np.ndarray:
    """The truncated sum of Sec. 3.2 with every weight and every f^ value first
    rounded to FP32, then summed exactly in FP64: the error floor of any
    evaluation that stores its weights and transform in FP32."""
    fh = np.asarray(fhat, dtype=np.complex128).reshape(-1, N ** 3)
    fi = np.ascontiguousarray(np.stack([fh.real, fh.imag], axis=-1))
    out = np.empty_like(fi)
    om = None if omega1d is None else _f64(omega1d)
    _load().orc_convolve_round32(N, L, float(lam), float(beta), _ptr(om), fh.shape[0], _ptr(fi), _ptr(out))
    return (out[..., 0] + 1j * out[..., 1]).reshape(-1, N, N, N)


def collision_round32(N: int, L: float, lam: float, f: np.ndarray, omega1d=None, beta: float = 1.0) -> np.ndarray:
    """Q~ = Re IDFT(convolve_round32(DFT f)): exact transforms, FP32-rounded
    weights and f^, exact sums.  Its distance from collision() is the FP32
    storage floor of a cell."""
    fh = forward(N, L, f)
    return inverse(N, L, convolve_round32(N, L, lam, fh, omega1d, beta))


def f32_floor(N: int, L: float, lam: float, f: np.ndarray, omega1d=None, beta: float = 1.0):
    """Per cell: ||collision_round32 - collision||_2 / ||collision||_2 for the
    cells of f (already the FP32 input, promoted).  Returns (floor, reference)."""
    ref = collision(N, L, lam, f, omega1d, beta=beta)
    r32 = collision_round32(N, L, lam, f, omega1d, beta)
    a = (r32 - ref).reshape(ref.shape[0], -1)
    b = ref.reshape(ref.shape[0], -1)
    return np.linalg.norm(a, axis=1) / np.linalg.norm(b, axis=1), ref


def term_scale(N: int, L: float, lam: float, f: np.ndarray, omega1d=None, beta: float = 1.0) -> np.ndarray:
    """Per cell, the velocity-space size of the absolute terms of the weighted
    sum: (2pi)^{-3/2} dzeta^3 N^{3/2} || sum_m |w G^| |f^_m| |f^_{k-m}| ||_2 over k.
    By Parseval this bounds the velocity-space effect of a relative
    perturbation of every term of the sum; it is the natural scale of
    floating-point error bounds for Q~ (which itself can be much smaller when
    gain and loss nearly cancel)."""
    lib = _load()
    f = _f64(f).reshape(-1, N ** 3)
    fh = np.empty((f.shape[0], N ** 3, 2))
    lib.orc_forward(N, L, f.shape[0], _ptr(f), _ptr(fh))
    tk = np.empty((f.shape[0], N ** 3))
    om = None if omega1d is None else _f64(omega1d)
    lib.orc_term_scale(N, L, float(lam), float(beta), _ptr(om), f.shape[0], _ptr(fh), _ptr(tk))
    dz = np.pi / L
    return (2.0 * np.pi) ** -1.5 * dz ** 3 * N ** 1.5 * np.linalg.norm(tk, axis=1)


def collision(N: int, L: float, lam: float, f: np.ndarray, omega1d=None, with_imag: bool = False,
              beta: float = 1.0):
    """Unprojected collision operator Q~ = Re IDFT(convolve(DFT f)), FP64."""
    f = _f64(f).reshape(-1, N ** 3)
    qt = np.empty_like(f)
    qi = np.empty_like(f) if with_imag else None
    om = None if omega1d is None else _f64(omega1d)
    _load().orc_collision(N, L, float(lam), float(beta), _ptr(om), f.shape[0], _ptr(f), _ptr(qt), _ptr(qi))
    qt = qt.reshape(-1, N, N, N)
    if with_imag:
        return qt, qi.reshape(-1, N, N, N)
    return qt


def cct(N: int, L: float) -> np.ndarray:
    """The 5x5 Gram matrix C C^T of the conservation constraints (Sec. 3.3)."""
    out = np.empty(25)
    _load().orc_cct(N, L, _ptr(out))
    return out.reshape(5, 5)


def project(N: int, L: float, qt: np.ndarray, energy: bool = True):
    """Conservation projection (Sec. 3.3).  Returns (Q_c, C Q~ per cell).
    energy=False keeps only mass and momentum (inelastic collisions)."""
    q = _f64(qt).reshape(-1, N ** 3)
    qc = np.empty_like(q)
    mom = np.empty((q.shape[0], 5))
    _load().orc_project(N, L, 5 if energy else 4, q.shape[0], _ptr(q), _ptr(qc), _ptr(mom))
    return qc.reshape(-1, N, N, N), mom


WALL_DIFFUSE, WALL_EXTRAPOLATE, WALL_NOFLUX = 0, 1, 2


def transport_step(N: int, L: float, f: np.ndarray, x_faces: np.ndarray, dt: float,
                   left=(WALL_DIFFUSE, 1.0, (0.0, 0.0, 0.0)),
                   right=(WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))) -> np.ndarray:
    """One Heun step of 1-D FV transport (Sec. 3.4).  f: [M+4, N, N, N] with
    two ghost cells at each end; returns the updated copy."""
    x = _f64(x_faces)
    M = x.shape[0] - 1
    g = _f64(f).reshape(M + 4, N ** 3).copy()
    lv = _f64(left[2])
    rv = _f64(right[2])
    _load().orc_transport_step(N, L, M, _ptr(x), float(dt), int(left[0]), float(left[1]),
                               _ptr(lv), int(right[0]), float(right[1]), _ptr(rv), _ptr(g))
    return g.reshape(M + 4, N, N, N)
