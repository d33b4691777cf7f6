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


def _steady_between_walls(orc, Tw, Vw, rho, steps=20):
    """A spatially uniform Maxwellian at the walls' temperature and tangential
    velocity, between two diffuse walls, is a steady state of the discrete
    scheme: the interior fluxes cancel, and the wall re-emits exactly the
    incoming half of the same Maxwellian (sigma_w = rho once the outgoing and
    incoming discrete fluxes balance).  N = 16, L = 8 puts the one unmatched
    grid speed v1 = -L at exp(-L^2 / (2 Tw)) < 1e-17 of the peak, so the
    discrete balance is exact to rounding."""
    N, L, M = 16, 8.0, 12
    xf = _mesh(M, X=3.0)
    m = synth.maxwellian(N, L, rho, Vw, Tw)
    f0 = np.broadcast_to(m, (M + 4, N, N, N)).copy()
    wall = (orc.WALL_DIFFUSE, Tw, tuple(Vw))
    dt = 0.4 * np.diff(xf).min() / L
    f = f0
    for _ in range(steps):
        f = orc.transport_step(N, L, f, xf, dt, left=wall, right=wall)
    return np.abs(f[2:-2] - f0[2:-2]).max() / m.max()


def test_diffuse_wall_emits_its_maxwellian_at_rest(orc):
    """Eq. (BC): the emitted half-Maxwellian has the wall temperature."""
    assert _steady_between_walls(orc, 0.8, (0.0, 0.0, 0.0), 1.0) <= 1e-12


def test_diffuse_wall_emits_its_drifting_maxwellian(orc):
    """Eq. (BC) with a tangential wall velocity: the emitted Maxwellian drifts
    with the wall (V_w = (0, 0.4, -0.3)); a gas moving with the wall at the
    wall temperature stays put."""
    assert _steady_between_walls(orc, 0.8, (0.0, 0.4, -0.3), 1.3) <= 1e-12


def test_diffuse_wall_temperature_and_velocity_are_observable(orc):
    """The same state next to walls at another temperature, or moving
    another way, is not steady: the two steady-state pins above would catch a
    wall Maxwellian with the wrong temperature or drift."""
    N, L, M = 16, 8.0, 12
    xf = _mesh(M, X=3.0)
    m = synth.maxwellian(N, L, 1.0, (0.0, 0.0, 0.0), 0.8)
    f0 = np.broadcast_to(m, (M + 4, N, N, N)).copy()
    dt = 0.4 * np.diff(xf).min() / L
    for wall in ((orc.WALL_DIFFUSE, 0.9, (0.0, 0.0, 0.0)), (orc.WALL_DIFFUSE, 0.8, (0.0, 0.1, 0.0))):
        f = orc.transport_step(N, L, f0, xf, dt, left=wall, right=wall)
        assert np.abs(f[2:-2] - f0[2:-2]).max() / m.max() > 1e-4
