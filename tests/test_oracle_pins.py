"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test compares the oracle with an independent route to the same number
(quadrature of a different formula, a classical closed-form solution, brute
force, a textbook solver) or with an exact invariant.
"""
import math

import numpy as np
import pytest

import synth
from tests import pins

L6 = 6.0


def _rand_pairs(N, n, seed):
    rng = np.random.default_rng(seed)
    return [(rng.integers(0, N, 3), rng.integers(0, N, 3)) for _ in range(n)]


def _special_pairs(N):
    """Pairs that hit each closed-form branch: B = 0, A = B (p = 0), |xi| = 0."""
    c = N // 2
    out = []
    # B = |2m - k - c|^2 = 0: 2m = k + c
    out.append(((c + 2, c, c - 2), (c + 1, c, c - 1)))
    # A = B > 0: |k - c| = |2m - k - c|, e.g. k - c = (2,0,0), 2m - k - c = (0,2,0)
    out.append(((c + 2, c, c), (c + 1, c + 1, c)))
    # |xi| = 0
    out.append(((c + 3, c - 1, c + 1), (c, c, c)))
    # near-coincident |zeta|/2 and |xi - zeta/2| (small p r0)
    out.append(((c + 5, c + 5, c - 4), (c + 1, c + 3, c - 4)))
    return out


@pytest.mark.parametrize("lam", [0, 1])
@pytest.mark.parametrize("N", [8, 16, 32])
def test_ghat_closed_form_matches_radial_quadrature(orc, lam, N):
    """Closed forms (Sec. 2.2, after eq. GHat_calc) vs composite Gauss-Legendre
    of the radial integral eq. GHat_calc itself, incl. every limiting branch."""
    worst = 0.0
    for k, m in _rand_pairs(N, 60, 11 + N + lam) + _special_pairs(N):
        g = orc.ghat(N, L6, lam, k, m)
        q, scale = pins.ghat_radial_quadrature(N, L6, lam, k, m)
        worst = max(worst, abs(g - q) / scale)
    assert worst < 1e-13, worst


@pytest.mark.parametrize("lam", [0, 1])
def test_ghat_matches_high_precision_integral(orc, lam):
    """30-digit mpmath quadrature of eq. GHat_calc at a few pairs (incl. small p)."""
    N = 16
    for k, m in _special_pairs(N) + _rand_pairs(N, 4, 5 + lam):
        g = orc.ghat(N, L6, lam, k, m)
        ref = pins.ghat_mpmath(N, L6, lam, k, m)
        assert abs(g - ref) <= 2e-14 * max(abs(ref), 1.0), (k, m, g, ref)


@pytest.mark.parametrize("lam", [0, 1])
def test_ghat_zero_row_and_symmetry(orc, lam):
    """G(u, 0) = 0 (eq. G_sinc) makes the zeta = 0 row vanish exactly; G^ depends
    on |zeta|, |xi - zeta/2| and |xi| only, so it is invariant under a common
    permutation of the coordinate axes of (k, m)."""
    N = 16
    c = N // 2
    rng = np.random.default_rng(3)
    for _ in range(50):
        m = rng.integers(0, N, 3)
        assert orc.ghat(N, L6, lam, (c, c, c), m) == 0.0
    for k, m in _rand_pairs(N, 40, 7):
        g = orc.ghat(N, L6, lam, k, m)
        for perm in ([1, 2, 0], [2, 0, 1], [0, 2, 1]):
            assert orc.ghat(N, L6, lam, np.asarray(k)[perm], np.asarray(m)[perm]) == g


@pytest.mark.parametrize("N", [8, 16, 32])
def test_ghat_quadrature_path_matches_closed_forms(orc, N):
    """The quadrature path used for other exponents (Sec. 2.2, last paragraph:
    the radial integral of eq. GHat_calc by numerical quadrature), forced at
    lambda = 0 and 1, reproduces the closed forms, every branch included."""
    pairs = _rand_pairs(N, 40, 21 + N) + _special_pairs(N)
    closed = {lam: [orc.ghat(N, L6, lam, k, m) for k, m in pairs] for lam in (0, 1)}
    try:
        orc.set_ghat_quadrature(True)
        quad = {lam: [orc.ghat(N, L6, lam, k, m) for k, m in pairs] for lam in (0, 1)}
    finally:
        orc.set_ghat_quadrature(False)
    for lam in (0, 1):
        err = max(abs(a - b) for a, b in zip(closed[lam], quad[lam])) / L6 ** (lam + 3)
        assert err < 1e-14, (lam, err)


@pytest.mark.parametrize("lam", [0.5, -1.5, 1.7])
def test_ghat_general_lambda_matches_high_precision_integral(orc, lam):
    """Non-integer exponents (variable hard and soft potentials): the oracle's
    quadrature vs a 30-digit mpmath quadrature of eq. GHat_calc."""
    N = 16
    for k, m in _special_pairs(N) + _rand_pairs(N, 3, 9):
        g = orc.ghat(N, L6, lam, k, m)
        ref = pins.ghat_mpmath(N, L6, lam, k, m)
        assert abs(g - ref) <= 1e-14 * L6 ** (lam + 3), (k, m, g, ref)


def test_ghat_general_lambda_zero_row_and_symmetry(orc):
    """G(u, 0) = 0 and the axis-permutation invariance hold on the quadrature
    path too (exactly: the same nodes see the same three lengths)."""
    N, lam = 16, 0.5
    c = N // 2
    rng = np.random.default_rng(4)
    for _ in range(20):
        assert orc.ghat(N, L6, lam, (c, c, c), rng.integers(0, N, 3)) == 0.0
    for k, m in _rand_pairs(N, 10, 8):
        g = orc.ghat(N, L6, lam, k, m)
        for perm in ([1, 2, 0], [2, 0, 1]):
            assert orc.ghat(N, L6, lam, np.asarray(k)[perm], np.asarray(m)[perm]) == g


def test_ghat_bulk_table_equals_per_pair(orc):
    """On the quadrature path the bulk routines evaluate G^ once per distinct
    (|k - N/2|^2, |2m - k - N/2|^2, |m - N/2|^2) triple; the dense table must
    equal the per-pair evaluation bitwise."""
    N, lam = 8, 0.5
    c = N // 2
    W = orc.weights_dense(N, L6, lam)
    dz3 = (math.pi / L6) * (math.pi / L6) * (math.pi / L6)
    for k, m in _rand_pairs(N, 200, 12):
        if np.all((np.asarray(k) - m + c >= 0) & (np.asarray(k) - m + c < N)):
            kk = (k[0] * N + k[1]) * N + k[2]
            mm = (m[0] * N + m[1]) * N + m[2]
            assert W[kk, mm] == dz3 * orc.ghat(N, L6, lam, k, m)


@pytest.mark.parametrize("beta", [0.8, 0.55])
def test_ghat_inelastic_matches_high_precision_integral(orc, beta):
    """Inelastic weights (beta < 1 in eqs. G_eqn, GHat_calc) vs 30-digit
    mpmath quadrature of the same radial integral."""
    N = 16
    for lam in (0, 1):
        for k, m in _special_pairs(N) + _rand_pairs(N, 2, 19):
            g = orc.ghat(N, L6, lam, k, m, beta=beta)
            ref = pins.ghat_mpmath(N, L6, lam, k, m, beta=beta)
            assert abs(g - ref) <= 1e-14 * L6 ** (lam + 3), (lam, k, m, g, ref)


@pytest.mark.parametrize("lam,beta", [(0, 0.8), (1, 0.8), (0.5, 0.9)])
def test_inelastic_energy_loss_of_a_maxwellian(orc, lam, beta):
    """Inelastic collisions cool a Maxwellian at the rate that the collision
    law fixes in closed form (tests/pins.inelastic_energy_rate).  The discrete
    operator's energy moment C_4 Q~ converges to it spectrally: within 2 % at
    N = 16 and at least ten times closer than at N = 8.  Mass stays exactly
    conserved (G(u, 0) = 0 also for beta < 1)."""
    exact = pins.inelastic_energy_rate(lam, beta, 1.0, 1.0)
    err = {}
    for N in (8, 16):
        f = synth.maxwellian(N, L6, 1.0, (0.0, 0.0, 0.0), 1.0)[None]
        qt = orc.collision(N, L6, lam, f, beta=beta)
        _, mom = orc.project(N, L6, qt, energy=False)
        assert abs(mom[0, 0]) <= 1e-14 * np.abs(qt).sum() * (2 * L6 / N) ** 3
        err[N] = abs(mom[0, 4] - exact)
    assert err[16] <= 0.02 * abs(exact), (err, exact)
    assert err[16] <= 0.1 * err[8], err


def test_projection_without_energy_row(orc):
    """The inelastic constraint set (Sec. 3.3: energy is not preserved) keeps
    mass and momentum: C_4 Q = 0 and agreement with a textbook KKT solve on the
    four rows."""
    N = 8
    rng = np.random.default_rng(6)
    qt = rng.standard_normal((2, N, N, N))
    qc, mom = orc.project(N, L6, qt, energy=False)
    dv = 2 * L6 / N
    v = synth.velocity_points(N, L6)
    v1, v2, v3 = np.meshgrid(v, v, v, indexing="ij")
    C = dv ** 3 * np.stack([np.ones_like(v1), v1, v2, v3]).reshape(4, -1)
    for c in range(2):
        q = qt[c].ravel()
        assert np.abs(C @ qc[c].ravel()).max() <= 1e-13 * np.abs(C).max() * np.abs(q).sum()
        n = q.size
        K = np.zeros((n + 4, n + 4))
        K[:n, :n] = np.eye(n)
        K[:n, n:] = C.T
        K[n:, :n] = C
        sol = np.linalg.lstsq(K, np.concatenate([q, np.zeros(4)]), rcond=None)[0][:n]
        assert np.abs(sol - qc[c].ravel()).max() <= 1e-11 * np.abs(q).max()


def test_weights_dense_truncation_box(orc):
    """The dense table is zero exactly where zeta_k - xi_m leaves the grid, and
    the number of kept pairs is (3N^2/4)^3 (counted by brute force)."""
    N = 8
    W = orc.weights_dense(N, L6, 1)
    c = N // 2
    idx = np.indices((N, N, N)).reshape(3, -1).T
    n = idx[:, None, :] - idx[None, :, :] + c  # [k, m, 3]
    inside = np.all((n >= 0) & (n < N), axis=2)
    assert inside.sum() == (3 * N * N // 4) ** 3
    assert np.all(W[~inside] == 0.0)
    kc = (c * N + c) * N + c
    assert np.all(W[kc] == 0.0)
    assert np.count_nonzero(W[inside]) > 0.99 * inside.sum() - N ** 3


def test_forward_transform_of_maxwellian(orc):
    """f^ of a Maxwellian vs its analytic transform (2pi)^{-3/2} rho
    e^{-i zeta.V} e^{-T|zeta|^2/2}: pins the 2pi factors, dv^3 and the centring
    phases of the transform pair (Sec. 2.2 / 3.1).  With T = 0.5 and L = 6 the
    velocity-domain truncation is e^{-(L-|V|)^2/(2T)} ~ 1e-13; aliasing from
    zeta +- 2pi/dv is e^{-T(pi/dv)^2/2} ~ 2e-8 at the edge of the N = 32
    Fourier grid and below 1e-16 on its central half."""
    N = 32
    rho, V, T = 1.3, (0.4, -0.3, 0.2), 0.5
    f = synth.maxwellian(N, L6, rho, V, T)
    fh = orc.forward(N, L6, f[None])[0]
    ref = pins.maxwellian_fourier(N, L6, rho, V, T)
    scale = np.abs(ref).max()
    assert np.abs(fh - ref).max() <= 1e-7 * scale
    q = slice(N // 4, 3 * N // 4 + 1)
    assert np.abs(fh[q, q, q] - ref[q, q, q]).max() <= 1e-12 * scale


def test_transform_round_trip(orc):
    """The discrete pair is exact: (2pi)^{-3} (dv dzeta N)^3 = 1."""
    N = 16
    f = synth.two_maxwellian(N, L6, 2, 99)
    back, im = orc.inverse(N, L6, orc.forward(N, L6, f), with_imag=True)
    assert np.abs(back - f).max() <= 1e-14 * np.abs(f).max()
    assert np.abs(im).max() <= 1e-14 * np.abs(f).max()


@pytest.mark.parametrize("lam", [0, 1, 0.5])
def test_mass_of_unprojected_operator_vanishes(orc, lam):
    """G^(xi, 0) = 0 gives Q^(0) = 0 exactly, i.e. sum_j Q~_j = 0 to rounding."""
    N = 16
    f = synth.two_maxwellian(N, L6, 3, 7)
    qt = orc.collision(N, L6, lam, f)
    for c in range(3):
        assert abs(qt[c].sum()) <= 1e-14 * np.abs(qt[c]).sum()


def test_projection_is_the_constrained_minimiser(orc):
    """Sec. 3.3: C Q = 0, P^2 = P, agreement with a textbook KKT solve, and
    Q = Q~ when Q~ already satisfies the constraints."""
    N = 8
    rng = np.random.default_rng(5)
    qt = rng.standard_normal((2, N, N, N))
    qc, mom = orc.project(N, L6, qt)
    dv = 2 * L6 / N
    v = synth.velocity_points(N, L6)
    v1, v2, v3 = np.meshgrid(v, v, v, indexing="ij")
    C = dv ** 3 * np.stack([np.ones_like(v1), v1, v2, v3, v1 ** 2 + v2 ** 2 + v3 ** 2]).reshape(5, -1)
    for c in range(2):
        q = qt[c].ravel()
        assert np.allclose(mom[c], C @ q, rtol=1e-13, atol=1e-13 * np.abs(C @ q).max())
        assert np.abs(C @ qc[c].ravel()).max() <= 1e-13 * np.abs(C).max() * np.abs(q).sum()
        n = q.size
        K = np.zeros((n + 5, n + 5))
        K[:n, :n] = np.eye(n)
        K[:n, n:] = C.T
        K[n:, :n] = C
        sol = np.linalg.lstsq(K, np.concatenate([q, np.zeros(5)]), rcond=None)[0][:n]
        assert np.abs(sol - qc[c].ravel()).max() <= 1e-11 * np.abs(q).max()
    qcc, _ = orc.project(N, L6, qc)
    assert np.abs(qcc - qc).max() <= 1e-13 * np.abs(qc).max()


@pytest.mark.parametrize("N,bound", [(8, 0.45), (16, 1.0e-2), (24, 3.0e-4)])
def test_bkw_convergence(orc, N, bound):
    """Maxwell molecules, b = 1/(4pi): Q_c(f_BKW(t0)) approaches the exact
    df/dt of the BKW solution; the bounds follow the spectral convergence
    (errors 0.43, 8.9e-3, 2.1e-4 at N = 8, 16, 24)."""
    t0 = 5.5
    f = synth.bkw(N, L6, t0)
    qc, _ = orc.project(N, L6, orc.collision(N, L6, 0, f[None]))
    ex = pins.bkw_dfdt(N, L6, t0)
    err = np.linalg.norm(qc[0] - ex) / np.linalg.norm(ex)
    assert err < bound, err


def test_maxwellian_is_near_equilibrium(orc):
    """Q(M, M) = 0 for the continuous operator: the discrete Q_c of a
    Maxwellian decays with N (hard spheres)."""
    res = []
    for N in (8, 16):
        m = synth.maxwellian(N, L6, 1.0, (0.0, 0.0, 0.0), 1.0)
        qc, _ = orc.project(N, L6, orc.collision(N, L6, 1, m[None]))
        res.append(np.abs(qc).max() / m.max())
    assert res[1] < 1e-3 and res[1] < res[0] / 100.0, res


def test_collision_matches_brute_force_integral(orc):
    """The whole discrete chain (transform, weights, truncated trapezoid
    convolution, inverse, projection) against direct 5-D quadrature of the
    collision integral eq. Q_general with the collision law eq.
    velocity_interact, hard spheres, at grid points of an N = 24 mesh."""
    N = 24
    params = [(1.0, (0.3, 0.0, 0.0), 0.6), (0.5, (-0.5, 0.2, 0.0), 0.9)]
    f = sum(synth.maxwellian(N, L6, r, V, T) for r, V, T in params)
    qc, _ = orc.project(N, L6, orc.collision(N, L6, 1, f[None]))
    v = synth.velocity_points(N, L6)
    fun = pins.maxwellian_mixture(params)
    scale = np.abs(qc).max()
    for i, j, k in [(13, 12, 11), (10, 13, 12)]:
        bf = pins.collision_brute_force(fun, (v[i], v[j], v[k]), 1, nr=30, sph_u=(14, 28), sph_s=(18, 36))
        assert abs(bf - qc[0, i, j, k]) <= 1e-4 * scale, (bf, qc[0, i, j, k])


def test_homogeneous_euler_run_conserves_moments(orc):
    """Ten forward-Euler steps f <- f + dt Q_c (Sec. 3.3 semi-discrete form) from
    BKW data keep mass, momentum and energy to rounding, and stay close to the
    BKW solution at t0 + 0.1 (loosely: the N = 8 operator error is large)."""
    N, dt = 8, 0.01
    f = synth.bkw(N, L6, 5.5)[None].copy()
    dv = 2 * L6 / N
    v = synth.velocity_points(N, L6)
    v1, v2, v3 = np.meshgrid(v, v, v, indexing="ij")
    rows = [np.ones_like(v1), v1, v2, v3, v1 ** 2 + v2 ** 2 + v3 ** 2]
    m0 = np.array([(r * f[0]).sum() * dv ** 3 for r in rows])
    for _ in range(10):
        qc, _ = orc.project(N, L6, orc.collision(N, L6, 0, f))
        f = f + dt * qc
    m1 = np.array([(r * f[0]).sum() * dv ** 3 for r in rows])
    assert np.abs(m1 - m0).max() <= 1e-14 * np.abs(m0).max()
    ref = synth.bkw(N, L6, 5.6)
    assert np.linalg.norm(f[0] - ref) / np.linalg.norm(ref) < 0.05


def test_term_scale_bounds_the_operator(orc):
    """The absolute-term scale dominates |Q~| (triangle inequality + Parseval)
    and equals a dense-table evaluation of sum_m |W||f^||f^| at N = 8."""
    N = 8
    f = synth.two_maxwellian(N, L6, 4, 21)
    S = orc.term_scale(N, L6, 1, f)
    qt = orc.collision(N, L6, 1, f)
    assert np.all(np.linalg.norm(qt.reshape(4, -1), axis=1) <= S * (1 + 1e-12))
    W = orc.weights_dense(N, L6, 1)
    fh = orc.forward(N, L6, f).reshape(4, -1)
    c = N // 2
    idx = np.indices((N, N, N)).reshape(3, -1).T
    n = idx[:, None, :] - idx[None, :, :] + c
    valid = np.all((n >= 0) & (n < N), axis=2)
    nlin = np.where(valid, (n[..., 0] * N + n[..., 1]) * N + n[..., 2], 0)
    for cell in range(4):
        T = (np.abs(W) * np.abs(fh[cell])[None, :] * np.abs(fh[cell])[nlin] * valid).sum(axis=1)
        ref = (2 * math.pi) ** -1.5 * (math.pi / L6) ** 3 * N ** 1.5 * np.linalg.norm(T)
        assert abs(S[cell] - ref) <= 1e-12 * ref


def test_round32_sum_equals_dense_brute_force(orc):
    """The FP32-storage floor sum: every weight and every f^ value rounded to
    FP32 (numpy's round-to-nearest), then summed exactly, equals a dense-table
    brute force at N = 8; rounding nothing reproduces the plain sum, and the
    floor it gives lies within the forward-error bound 2u of the absolute
    terms."""
    N = 8
    f = synth.two_maxwellian(N, L6, 3, 22)
    fh = orc.forward(N, L6, f)
    got = orc.convolve_round32(N, L6, 1, fh).reshape(3, -1)
    W32 = orc.weights_dense(N, L6, 1).astype(np.float32).astype(np.float64)
    c = N // 2
    idx = np.indices((N, N, N)).reshape(3, -1).T
    n = idx[:, None, :] - idx[None, :, :] + c
    valid = np.all((n >= 0) & (n < N), axis=2)
    nlin = np.where(valid, (n[..., 0] * N + n[..., 1]) * N + n[..., 2], 0)
    fr = fh.reshape(3, -1)
    fr = fr.real.astype(np.float32).astype(np.float64) + 1j * fr.imag.astype(np.float32).astype(np.float64)
    for cell in range(3):
        ref = (W32 * fr[cell][None, :] * fr[cell][nlin] * valid).sum(axis=1)
        assert np.abs(got[cell] - ref).max() <= 1e-14 * np.abs(ref).max()
    exact = orc.convolve(N, L6, 1, fh).reshape(3, -1)
    assert not np.array_equal(got, exact)
    floor, ref_qt = orc.f32_floor(N, L6, 1, f)
    S = orc.term_scale(N, L6, 1, f)
    qn = np.linalg.norm(ref_qt.reshape(3, -1), axis=1)
    assert np.all(floor > 0) and np.all(floor * qn <= 2 * 2.0 ** -24 * 2 * S)
