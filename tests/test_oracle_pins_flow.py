"""Pins of the oracle's characteristic tracing, field interpolation, moments
and macroscopic right-hand side against closed forms and the moment
equations of the Vlasov--Poisson system.

Every expected value is derived independently of the oracle's own formula:
the exact RK4 map of a linear ODE (the fourth-order Taylor polynomial of the
matrix exponential), Lagrange interpolation's exactness on polynomials,
Gaussian moments, and the time derivatives of the conserved densities that
the Vlasov equation implies (section 2.2, eqs. (macro_sys), (macro_sys_comp),
(electric_field_flux)).
"""
import math

import numpy as np
import pytest

from oracle import feet as FT
from oracle import grid as G
from oracle import ht as HT
from oracle import lomac as LM
from oracle import macro as MA
import slar_inputs as SI


# ------------------------------------------------- characteristics (eq. (SL_basic_formulation))
def _rk4_matrix(A, tau):
    """One classical RK4 step of y' = A y is y -> T4(tau A) y with the
    degree-4 Taylor polynomial T4 of the exponential."""
    M = tau * A
    out = np.eye(A.shape[0])
    term = np.eye(A.shape[0])
    for k in range(1, 5):
        term = term @ M / k
        out = out + term
    return out


def _grid_2d2v(nx=32, nv=16, L=4 * math.pi, vmax=6.0):
    lo = (0.0, 0.0, -vmax, -vmax)
    hi = (L, L, vmax, vmax)
    n = (nx, nx, nv, nv)
    return lo, hi, n


@pytest.mark.parametrize("cv", [1.0, 2.0 / 3.0])
def test_rk4_feet_constant_field_closed_form(cv):
    """Constant frozen field e: the backward characteristic of
    dx/dt = c v, dv/dt = -e over tau is x* = x - c v tau - c e tau^2 / 2,
    v* = v + e tau (a quadratic in time, which RK4 integrates exactly)."""
    lo, hi, n = _grid_2d2v()
    e = np.array([0.37, -0.81])
    E = np.stack([np.full(n[:2], e[0]), np.full(n[:2], e[1])])
    idx = SI.random_requests(n, 500, seed=21)
    tau = 0.7
    foot = FT.feet(idx, lo, hi, n, 2, 2, tau, cv, E)
    P = FT.grid_points(idx, lo, hi, n)
    x, v = P[:, :2], P[:, 2:]
    assert np.abs(foot[:, :2] - (x - cv * v * tau - cv * e * tau * tau / 2)).max() < 1e-13
    assert np.abs(foot[:, 2:] - (v + e * tau)).max() < 1e-13


@pytest.mark.parametrize("cv,a", [(1.0, (0.3, -0.45)), (2.0 / 3.0, (-0.2, 0.6))])
def test_rk4_feet_linear_field_is_the_rk4_map(cv, a):
    """Linear frozen field E_m(x) = a_m (x_m - c_m), sampled on the grid:
    the degree-4 field interpolation is exact for it away from the periodic
    seam, and per dimension the backward characteristic solves
    (X - c, V)' = [[0, -cv], [a, 0]] (X - c, V), whose one-step RK4 map is
    T4(tau A).  Grid points and stages stay two cells or more inside the
    seam, so the comparison is exact to rounding."""
    lo, hi, n = _grid_2d2v()
    L = hi[0] - lo[0]
    c = (L / 2, L / 2 + 0.3)
    xs = [G.centres(lo[m], hi[m], n[m]) for m in range(2)]
    X1, X2 = np.meshgrid(xs[0], xs[1], indexing="ij")
    E = np.stack([a[0] * (X1 - c[0]), a[1] * (X2 - c[1])])
    rng = np.random.default_rng(5)
    # x within 2.5 of the centre, |v| <= 2.2: with tau = 0.6 every stage
    # point moves by less than 1.5, far from the seam at 0 / L
    mid = n[0] // 2
    idx = np.stack([rng.integers(mid - 6, mid + 6, 400), rng.integers(mid - 6, mid + 6, 400),
                    rng.integers(3, 13, 400), rng.integers(3, 13, 400)], axis=1)
    tau = 0.6
    foot = FT.feet(idx, lo, hi, n, 2, 2, tau, cv, E)
    P = FT.grid_points(idx, lo, hi, n)
    for m in range(2):
        A = np.array([[0.0, -cv], [a[m], 0.0]])
        T = _rk4_matrix(A, tau)
        y0 = np.stack([P[:, m] - c[m], P[:, 2 + m]])
        y1 = T @ y0
        assert np.abs(foot[:, m] - c[m] - y1[0]).max() < 1e-12
        assert np.abs(foot[:, 2 + m] - y1[1]).max() < 1e-12


def test_rk4_feet_linear_field_1d1v():
    """The same RK4 map pin for the 1D1V tree (dx = 1)."""
    L, vmax = 4 * math.pi, 6.0
    lo, hi, n = (0.0, -vmax), (L, vmax), (64, 32)
    x = G.centres(lo[0], hi[0], n[0])
    a, c, cv, tau = 0.25, L / 2, 1.0, 0.8
    E = (a * (x - c))[None]
    idx = np.stack(np.meshgrid(np.arange(22, 42), np.arange(8, 24), indexing="ij"), -1).reshape(-1, 2)
    foot = FT.feet(idx, lo, hi, n, 1, 2, tau, cv, E)
    P = FT.grid_points(idx, lo, hi, n)
    y1 = _rk4_matrix(np.array([[0.0, -cv], [a, 0.0]]), tau) @ np.stack([P[:, 0] - c, P[:, 1]])
    assert np.abs(foot[:, 0] - c - y1[0]).max() < 1e-12
    assert np.abs(foot[:, 1] - y1[1]).max() < 1e-12


# ----------------------------------------------- off-grid field interpolation
def _quartic(t, coef):
    return sum(cf * t ** k for k, cf in enumerate(coef))


def test_interp_periodic_exact_on_quartics_inside():
    """Degree-4 tensor-product Lagrange interpolation reproduces any product
    of polynomials of degree <= 4 at points whose stencils do not wrap."""
    n, L = (24, 20), (3.0, 2.0)
    lo = (0.5, -1.0)
    h = [L[m] / n[m] for m in range(2)]
    xs = [G.centres(lo[m], lo[m] + L[m], n[m]) for m in range(2)]
    c1 = np.array([0.3, -1.1, 0.7, 0.25, -0.4])
    c2 = np.array([-0.2, 0.5, 1.3, -0.6, 0.15])
    X1, X2 = np.meshgrid(xs[0], xs[1], indexing="ij")
    field = _quartic(X1 - 2.0, c1) * _quartic(X2 + 0.1, c2)
    rng = np.random.default_rng(3)
    pts = np.stack([rng.uniform(lo[0] + 3 * h[0], lo[0] + L[0] - 3 * h[0], 300),
                    rng.uniform(lo[1] + 3 * h[1], lo[1] + L[1] - 3 * h[1], 300)], axis=1)
    got = G.interp_periodic(field, lo, h, pts, 5)
    ref = _quartic(pts[:, 0] - 2.0, c1) * _quartic(pts[:, 1] + 0.1, c2)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # a degree-5 term is not reproduced: the pin can fail
    bad = G.interp_periodic(field + X1 ** 5, lo, h, pts, 5)
    assert np.abs(bad - ref - pts[:, 0] ** 5).max() > 1e-7


def test_interp_periodic_wraps_the_stencil():
    """A periodic field that near the seam equals a quartic of the unwrapped
    coordinate is interpolated exactly within two cells of the seam, from
    either side (the stencil indices wrap mod N)."""
    N, L, lo = 40, 5.0, -1.0
    h = L / N
    x = G.centres(lo, lo + L, N)
    seam = lo + L
    t = np.mod(x - seam + L / 2, L) - L / 2        # signed distance to the seam, unwrapped
    coef = np.array([0.4, -0.9, 0.3, 1.2, -0.7])
    field = _quartic(t, coef)
    rng = np.random.default_rng(8)
    s = rng.uniform(-2 * h, 2 * h, 200)
    pts = np.mod(seam + s - lo, L) + lo              # physical points on both sides of the seam
    got = G.interp_periodic(field, (lo,), (h,), pts[:, None], 5)
    assert np.abs(got - _quartic(s, coef)).max() <= 1e-12


# ------------------------------------------------------------------- moments
def _maxwellian_tensor(n_x, u, T, vg):
    """f(x, v) = n(x) (2 pi T(x))^{-1} exp(-|v - u(x)|^2 / (2 T(x))) on a 2D2V grid."""
    V1, V2 = np.meshgrid(vg[0], vg[1], indexing="ij")
    d1 = V1[None, None] - u[0][..., None, None]
    d2 = V2[None, None] - u[1][..., None, None]
    Tx = T[..., None, None]
    return n_x[..., None, None] / (2 * math.pi * Tx) * np.exp(-(d1 * d1 + d2 * d2) / (2 * Tx))


def _drifting_state(nx=16, nv=48, vmax=10.0):
    L = 2 * math.pi
    x = G.centres(0.0, L, nx)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    n_x = 1.0 + 0.2 * np.cos(X1) + 0.1 * np.sin(X2)
    u = (0.3 * np.sin(X2), 0.2 * np.cos(X1))
    T = 1.0 + 0.1 * np.cos(X1 + X2)
    vg = [G.centres(-vmax, vmax, nv)] * 2
    dv = (2 * vmax / nv) ** 2
    return L, n_x, u, T, vg, dv


def test_dense_moments_match_gaussian_closed_forms():
    """For f = n M(v; u, T) (d_v = 2): <1> = n, <v> = n u, <|v|^2> =
    n (2T + |u|^2), <v_a v_b> = n (T delta_ab + u_a u_b), <|v|^2 v_a> =
    n u_a (4T + |u|^2); the order is 1, v_1, v_2, |v|^2, v1v1, v1v2, v2v2,
    |v|^2 v_1, |v|^2 v_2 (eq. (macro_sys_comp) fluxes after the raw moments)."""
    L, n_x, u, T, vg, dv = _drifting_state()
    f = _maxwellian_tensor(n_x, u, T, vg)
    M = HT.dense_moments(f, 2, vg, dv)
    u2 = u[0] ** 2 + u[1] ** 2
    ref = [n_x, n_x * u[0], n_x * u[1], n_x * (2 * T + u2),
           n_x * (T + u[0] ** 2), n_x * u[0] * u[1], n_x * (T + u[1] ** 2),
           n_x * u[0] * (4 * T + u2), n_x * u[1] * (4 * T + u2)]
    for q in range(9):
        assert np.abs(M[q] - ref[q]).max() < 1e-12, q


def test_ht_moments_equal_dense_moments_with_correction():
    """HT.moments (frame contraction, plus the appended LoMaC columns) equals
    the moments of the dense reconstruction for all nine psi."""
    n = (6, 7, 10, 9)
    F = SI.random_ht(4, n, (3, 4, 5, 4, 5, 6), seed=77)
    rng = np.random.default_rng(78)
    F["corr"] = {"C": rng.standard_normal((4, n[0], n[1])), "Q": rng.standard_normal((4, n[2], n[3]))}
    vg = [G.centres(-3.0, 3.0, n[2]), G.centres(-2.0, 4.0, n[3])]
    dv = (6.0 / n[2]) * (6.0 / n[3])
    a = HT.moments(F, vg, dv)
    b = HT.dense_moments(HT.full(F), 2, vg, dv)
    assert a.shape == b.shape == (9, n[0], n[1])
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


# -------------------------------------------- macroscopic right-hand side
def _fft_deriv(f, axis, L):
    N = f.shape[axis]
    k = np.fft.fftfreq(N, d=L / N) * 2 * math.pi
    shape = [1] * f.ndim
    shape[axis] = N
    return np.real(np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(f, axis=axis), axis=axis))


def _field(n_e, n_i, L):
    """E = -grad phi with -Laplace phi = n_i - n_e on the nonzero modes."""
    N = n_e.shape[0]
    k = np.fft.fftfreq(N, d=L / N) * 2 * math.pi
    K1, K2 = np.meshgrid(k, k, indexing="ij")
    k2 = K1 ** 2 + K2 ** 2
    rh = np.fft.fft2(n_i - n_e)
    ph = np.where(k2 > 0, rh / np.where(k2 > 0, k2, 1.0), 0.0)
    phi = np.real(np.fft.ifft2(ph))
    return np.stack([-_fft_deriv(phi, 0, L), -_fft_deriv(phi, 1, L)])


def test_macro_rhs_equals_vlasov_moment_equations():
    """At U = U(F*) (no correction) the right-hand side R of U' = -R(U)
    must equal minus the time derivative of the conserved densities that
    the Vlasov equation d_t f = -v.grad_x f + E.grad_v f implies, computed
    here from the moments of a dense drifting Maxwellian:
      d_t n        = -div <v f>
      d_t (n u)_a  = -sum_b d_b <v_a v_b f> - n E_a
      d_t e        = -div (1/2 <|v|^2 v f>) - E.<v f> + E.d_t E,
    with e = 1/2 <|v|^2 f> + 1/2 |E|^2 and d_t E the field of d_t n_e (the
    Poisson map is affine).  The inputs are band-limited well below the
    Nyquist mode, so the discrete spectral product rule is exact and the
    local energy identity behind the flux F_ep holds to rounding."""
    L, n_x, u, T, vg, dv = _drifting_state()
    f = _maxwellian_tensor(n_x, u, T, vg)
    Mstar = HT.dense_moments(f, 2, vg, dv)
    n_i = float(n_x.mean())
    lengths = [L, L]
    U = LM.conserved_from_raw(Mstar[:4], n_i, lengths)
    g = np.exp(-0.5 * vg[0] ** 2)
    B = LM.basis([g / np.linalg.norm(g)] * 2, vg, [vg[0][1] - vg[0][0]] * 2)
    sysm = MA.MacroSystem(Mstar, B, n_i, lengths, dv, vg, U, 1.0)
    R = sysm.rhs(U)

    E = _field(Mstar[0], n_i, L)
    M1 = Mstar[1:3]
    P = [[Mstar[4], Mstar[5]], [Mstar[5], Mstar[6]]]
    Q = Mstar[7:9]
    dn = -(_fft_deriv(M1[0], 0, L) + _fft_deriv(M1[1], 1, L))
    dmom = [-(_fft_deriv(P[a][0], 0, L) + _fft_deriv(P[a][1], 1, L)) - Mstar[0] * E[a] for a in range(2)]
    dE = _field(Mstar[0] + dn, n_i, L) - _field(Mstar[0], n_i, L)
    de = (-(_fft_deriv(0.5 * Q[0], 0, L) + _fft_deriv(0.5 * Q[1], 1, L))
          - (E[0] * M1[0] + E[1] * M1[1]) + (E[0] * dE[0] + E[1] * dE[1]))
    dU = np.stack([dn, dmom[0], dmom[1], de])
    scale = np.abs(dU).max()
    assert np.abs(-R - dU).max() <= 1e-12 * scale
    # the energy equation is not trivially satisfied: its terms are O(1e-1)
    assert np.abs(de).max() > 1e-2


# ------------------------------------------- exponential integrator (eq. (slarvp))
def test_cf3_slar_vp_is_third_order_in_time():
    """Section 4.1: the SLAR_VP step is third order in time.  Self-convergence
    at a fixed 64^2 mesh (1D1V Landau, alpha 0.3, k 0.5, degree-4 stencils,
    no truncation loss: tol 1e-13, full rank) to T = 1.2 with dt = 0.4, 0.2,
    0.1: successive differences shrink by about 2^3 (7.2 measured).  A wrong
    stage time, final velocity multiplier or a swapped final-field pair
    drops the ratio to about 2."""
    N, T = 64, 1.2
    from oracle import step as ST
    p = SI.config("landau1d", n=N).with_(alpha=0.3, order=5, split=False, tol=1e-13, rmax=N, lomac=False)
    out = {}
    for dt in (0.4, 0.2, 0.1):
        q = p.with_(dt=dt)
        o = ST.Oracle(q, probes=SI.probe_indices(N, N, 64, 5))
        F, _ = o.run(SI.initial_ht(q), int(round(T / dt)))
        out[dt] = HT.full(F)
    e1 = np.abs(out[0.4] - out[0.2]).max()
    e2 = np.abs(out[0.2] - out[0.1]).max()
    assert 5.5 < e1 / e2 < 11.0, (e1, e2)
