"""Independent references that pin the oracle to the mathematics of the paper.

None of these reuse the oracle's code: each computes the quantity from a
different formula of the paper (or from a classical closed-form solution),
so that a dropped term, a wrong sign or index, or a wrong 2 pi factor in the
oracle fails at least one of them.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------------------
# G^ by quadrature of its radial integral (Sec. 2.2, eq. GHat_calc), beta = 1
# ---------------------------------------------------------------------------
def _gl_nodes(order: int):
    return np.polynomial.legendre.leggauss(order)


def ghat_radial_quadrature(N: int, L: float, lam: int, k, m, panels: int = 64, order: int = 24):
    """Composite Gauss-Legendre of
    4pi/(2pi)^{3/2} int_0^{r0} r^{lam+2}[sinc(r|z|/2) sinc(r|xi - z/2|) - sinc(r|xi|)] dr
    with r0 = L.  Returns (value, int |integrand| dr) so callers can scale tolerances."""
    c = N // 2
    dz = math.pi / L
    zeta = dz * (np.asarray(k, dtype=float) - c)
    xi = dz * (np.asarray(m, dtype=float) - c)
    a = np.linalg.norm(zeta) / 2.0
    b = np.linalg.norm(xi - zeta / 2.0)
    s = np.linalg.norm(xi)
    x, w = _gl_nodes(order)
    edges = np.linspace(0.0, L, panels + 1)
    lo, hi = edges[:-1, None], edges[1:, None]
    r = (0.5 * (hi - lo) * x[None, :] + 0.5 * (hi + lo)).ravel()
    wr = (0.5 * (hi - lo) * w[None, :]).ravel()
    sinc = lambda t: np.sinc(t / math.pi)  # sin(t)/t
    f = r ** (lam + 2) * (sinc(a * r) * sinc(b * r) - sinc(s * r))
    g = r ** (lam + 2) * (np.abs(sinc(a * r) * sinc(b * r)) + np.abs(sinc(s * r)))
    pref = 4.0 * math.pi / (2.0 * math.pi) ** 1.5
    return pref * float(np.dot(wr, f)), pref * float(np.dot(wr, g))


def ghat_mpmath(N: int, L: float, lam: float, k, m, dps: int = 30, beta: float = 1.0) -> float:
    """Same integral with mpmath at high precision (independent of numpy);
    beta < 1 is the inelastic form sinc(beta r|z|/2) sinc(r|xi - beta z/2|)."""
    import mpmath as mp

    mp.mp.dps = dps
    c = N // 2
    dz = mp.pi / L
    bt = mp.mpf(beta)
    zeta = [dz * (int(ki) - c) for ki in k]
    xi = [dz * (int(mi) - c) for mi in m]
    a = bt * mp.sqrt(sum(z * z for z in zeta)) / 2
    b = mp.sqrt(sum((x - bt * z / 2) ** 2 for x, z in zip(xi, zeta)))
    s = mp.sqrt(sum(x * x for x in xi))

    def sinc(t):
        return mp.mpf(1) if t == 0 else mp.sin(t) / t

    f = lambda r: r ** (lam + 2) * (sinc(a * r) * sinc(b * r) - sinc(s * r))
    val = mp.quad(f, mp.linspace(0, L, 9))
    return float(4 * mp.pi / (2 * mp.pi) ** mp.mpf(1.5) * val)


# ---------------------------------------------------------------------------
# Fourier transform of a Maxwellian (closed form)
# ---------------------------------------------------------------------------
def maxwellian_fourier(N: int, L: float, rho: float, V, T: float) -> np.ndarray:
    """(2pi)^{-3/2} int rho (2 pi T)^{-3/2} e^{-|v-V|^2/(2T)} e^{-i zeta.v} dv
    = (2pi)^{-3/2} rho e^{-i zeta.V} e^{-T |zeta|^2 / 2}."""
    z = (math.pi / L) * (np.arange(N) - N // 2)
    z1, z2, z3 = np.meshgrid(z, z, z, indexing="ij")
    ph = z1 * V[0] + z2 * V[1] + z3 * V[2]
    return (2.0 * math.pi) ** -1.5 * rho * np.exp(-1j * ph) * np.exp(-0.5 * T * (z1 ** 2 + z2 ** 2 + z3 ** 2))


# ---------------------------------------------------------------------------
# BKW: exact Q = df/dt for Maxwell molecules, b = 1/(4 pi)
# ---------------------------------------------------------------------------
def bkw_dfdt(N: int, L: float, t: float) -> np.ndarray:
    """d/dt of the BKW solution at the grid points (exact, by hand):
    f = e^{-r2/2K} (2 pi K)^{-3/2} / 2 [ (5K-3)/K + (1-K) r2 / K^2 ],
    dK/dt = (1-K)/6."""
    K = 1.0 - math.exp(-t / 6.0)
    v = (2.0 * L / N) * (np.arange(N) - N // 2)
    v1, v2, v3 = np.meshgrid(v, v, v, indexing="ij")
    r2 = v1 * v1 + v2 * v2 + v3 * v3
    G = np.exp(-r2 / (2.0 * K)) * (2.0 * math.pi * K) ** -1.5 / 2.0
    dG = G * (r2 / (2.0 * K * K) - 1.5 / K)
    P = (5.0 * K - 3.0) / K + (1.0 - K) * r2 / (K * K)
    dP = 3.0 / (K * K) + r2 * (-1.0 / (K * K) - 2.0 * (1.0 - K) / K ** 3)
    return (dG * P + G * dP) * (1.0 - K) / 6.0


# ---------------------------------------------------------------------------
# Brute-force 5-D quadrature of the collision integral (Sec. 2, eq. Q_general)
# ---------------------------------------------------------------------------
def _sphere_rule(ncos: int, nphi: int):
    x, w = _gl_nodes(ncos)
    phi = (np.arange(nphi) + 0.5) * (2.0 * math.pi / nphi)
    ct = np.repeat(x, nphi)
    st = np.sqrt(1.0 - ct * ct)
    ph = np.tile(phi, ncos)
    pts = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    wts = np.repeat(w, nphi) * (2.0 * math.pi / nphi)
    return pts, wts  # weights sum to 4 pi


def collision_brute_force(fun, v, lam: int, rmax: float = 9.0, nr: int = 36,
                          sph_u=(16, 32), sph_s=(20, 40)) -> float:
    """Q(f,f)(v) = int_{R^3} int_{S^2} |u|^lam (1/4pi) [f(v')f(v*') - f(v)f(v*)] dsigma dv*,
    with v' = v + (|u| sigma - u)/2, v*' = v* - (|u| sigma - u)/2, u = v - v*.
    v* = v - u is integrated in spherical coordinates around v (Gauss-Legendre
    in |u|, product rule on the sphere), sigma with a second product rule."""
    v = np.asarray(v, dtype=float)
    x, w = _gl_nodes(nr // 3)
    edges = np.linspace(0.0, rmax, 4)
    rr = np.concatenate([0.5 * (edges[i + 1] - edges[i]) * x + 0.5 * (edges[i + 1] + edges[i]) for i in range(3)])
    wr = np.concatenate([0.5 * (edges[i + 1] - edges[i]) * w for i in range(3)])
    U, WU = _sphere_rule(*sph_u)
    S, WS = _sphere_rule(*sph_s)
    fv = fun(v[None, :])[0]
    total = 0.0
    for r, w_r in zip(rr, wr):
        u = r * U                                   # [nu, 3]
        vs = v[None, :] - u                         # v*
        loss = fv * fun(vs)                         # [nu]
        # gain: v' = v - u/2 + r sigma/2, v*' = v - u/2 - r sigma/2
        mid = v[None, None, :] - 0.5 * u[:, None, :]
        half = 0.5 * r * S[None, :, :]
        gain = fun((mid + half).reshape(-1, 3)).reshape(len(U), len(S)) * \
            fun((mid - half).reshape(-1, 3)).reshape(len(U), len(S))
        gain = gain @ WS / (4.0 * math.pi)
        total += w_r * r ** (2 + lam) * float(np.dot(WU, gain - loss))
    return total


def maxwellian_mixture(params):
    """Callable f(v) for sum_i rho_i (2 pi T_i)^{-3/2} exp(-|v - V_i|^2/(2 T_i))."""
    def fun(pts):
        out = np.zeros(pts.shape[0])
        for rho, V, T in params:
            d2 = ((pts - np.asarray(V)[None, :]) ** 2).sum(axis=1)
            out += rho * (2.0 * math.pi * T) ** -1.5 * np.exp(-d2 / (2.0 * T))
        return out
    return fun


# ---------------------------------------------------------------------------
# Energy loss of inelastic collisions on a Maxwellian (closed form)
# ---------------------------------------------------------------------------
def inelastic_energy_rate(lam: float, beta: float, rho: float, T: float) -> float:
    """int Q(M, M) |v|^2 dv for the law v' = v + (beta/2)(|u| sigma - u),
    B = |u|^lam b, isotropic b with int b dsigma = 1.  A collision changes
    |v|^2 + |v*|^2 by -beta(1 - beta)|u|^2 (1 - cos theta), whose sigma-average
    is -beta(1 - beta)|u|^2; symmetrising the weak form gives
    -(1/2) beta (1 - beta) rho^2 <|u|^{lam+2}>, u = v - v* ~ N(0, 2T I), and
    <|u|^p> = (2T)^{p/2} 2^{p/2} Gamma((3 + p)/2) / Gamma(3/2)."""
    p = lam + 2.0
    mom = (2.0 * T) ** (p / 2) * 2.0 ** (p / 2) * math.gamma((3.0 + p) / 2) / math.gamma(1.5)
    return -0.5 * beta * (1.0 - beta) * rho * rho * mom
