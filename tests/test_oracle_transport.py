"""Pins of the oracle's finite-volume transport (Sec. 3.4) and wall (Sec. 2.1)."""
import math

import numpy as np

import synth


def _mesh(M, X=10.0, alpha=1.5):
    j = np.arange(M + 1, dtype=float)
    return X * np.expm1(alpha * j / M) / math.expm1(alpha)


def _mass(f, xf, N, L):
    dx = np.diff(xf)
    dv = 2 * L / N
    return float((f[2:-2].reshape(len(dx), -1).sum(axis=1) * dx).sum() * dv ** 3)


def test_constant_state_is_preserved(orc):
    """Free streaming of a spatially constant f is exact with extrapolated ghosts."""
    N, L, M = 8, 4.0, 20
    xf = _mesh(M)
    m = synth.maxwellian(N, L, 1.0, (0.2, 0.0, 0.0), 1.0)
    f = np.broadcast_to(m, (M + 4, N, N, N)).copy()
    ex = (orc.WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))
    g = orc.transport_step(N, L, f, xf, 0.01, left=ex, right=ex)
    assert np.abs(g[2:-2] - f[2:-2]).max() <= 1e-15 * m.max()


def test_diffuse_walls_conserve_mass(orc):
    """With diffuse walls at both ends, sigma_w makes the net wall flux zero, so
    total mass is conserved to rounding (eq. BC) while the gas heats up."""
    N, L, M = 8, 6.0, 24
    xf = _mesh(M, X=4.0)
    f = synth.boundary_layer_state(N, L, M)
    wl = (orc.WALL_DIFFUSE, 2.0, (0.0, 0.0, 0.0))
    wr = (orc.WALL_DIFFUSE, 1.5, (0.0, 0.3, 0.0))
    m0 = _mass(f, xf, N, L)
    dt = 0.4 * np.diff(xf).min() / L
    for _ in range(20):
        f = orc.transport_step(N, L, f, xf, dt, left=wl, right=wr)
    assert abs(_mass(f, xf, N, L) - m0) <= 1e-13 * m0
    assert not np.allclose(f[2], synth.boundary_layer_state(N, L, M)[2])


def test_noflux_wall_blocks_inflow(orc):
    """No-flux boundary: nothing enters, so mass can only decrease."""
    N, L, M = 8, 6.0, 16
    xf = _mesh(M, X=4.0)
    f = synth.boundary_layer_state(N, L, M)
    nf = (orc.WALL_NOFLUX, 1.0, (0.0, 0.0, 0.0))
    m0 = _mass(f, xf, N, L)
    f = orc.transport_step(N, L, f, xf, 0.4 * np.diff(xf).min() / L, left=nf, right=nf)
    assert _mass(f, xf, N, L) < m0


def _advect(orc, M, t_end=1.0):
    N, L = 4, 1.0  # v1 in {-1, -0.5, 0, 0.5}
    xf = _mesh(M, X=10.0, alpha=1.0)
    xc = 0.5 * (xf[1:] + xf[:-1])
    v = synth.velocity_points(N, L)
    prof = lambda x: 1.0 + 0.5 * np.tanh(x - 5.0)
    f = np.empty((M + 4, N, N, N))
    for i in range(N):
        f[2:-2, i] = prof(xc)[:, None, None]
    f[:2] = f[2]
    f[-2:] = f[-3]
    dt = 0.25 * np.diff(xf).min() / L
    steps = int(math.ceil(t_end / dt))
    dt = t_end / steps
    ex = (orc.WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))
    for _ in range(steps):
        f = orc.transport_step(N, L, f, xf, dt, left=ex, right=ex)
    sel = (xc > 2.5) & (xc < 7.5)
    dx = np.diff(xf)[sel]
    err = 0.0
    for i in range(N):
        exact = prof(xc - v[i] * t_end)
        err += float((np.abs(f[2:-2, i, 0, 0][sel] - exact[sel]) * dx).sum())
    return err


def test_second_order_in_space_and_time(orc):
    """Minmod-limited upwind + Heun on a smooth monotone profile on a stretched
    mesh converges at second order in L1 (error ratio -> 4 per refinement;
    the limiter clips at the inflection point, so L-infinity is lower order)."""
    e1 = _advect(orc, 40)
    e2 = _advect(orc, 80)
    assert e1 / e2 > 3.0, (e1, e2)


def test_minmod_scheme_is_tvd(orc):
    """A step profile develops no new extrema (total variation does not grow)."""
    N, L, M = 4, 1.0, 60
    xf = _mesh(M, X=10.0, alpha=0.5)
    xc = 0.5 * (xf[1:] + xf[:-1])
    f = np.empty((M + 4, N, N, N))
    f[2:-2] = np.where(xc < 4.0, 2.0, 1.0)[:, None, None, None]
    f[:2] = f[2]
    f[-2:] = f[-3]
    ex = (orc.WALL_EXTRAPOLATE, 1.0, (0.0, 0.0, 0.0))
    tv0 = np.abs(np.diff(f[2:-2], axis=0)).sum(axis=0)
    for _ in range(40):
        f = orc.transport_step(N, L, f, xf, 0.4 * np.diff(xf).min() / L, left=ex, right=ex)
    tv1 = np.abs(np.diff(f[2:-2], axis=0)).sum(axis=0)
    assert np.all(tv1 <= tv0 + 1e-12)
    assert f[2:-2].max() <= 2.0 + 1e-12 and f[2:-2].min() >= 1.0 - 1e-12
