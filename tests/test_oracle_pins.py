"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it pins.  None of them re-types the oracle's
formula: they use brute force, closed forms, invariants and library
routines (SVD, linear solves, the Faddeeva function).
"""
import math
import os

import numpy as np
import pytest

import slar_inputs as SI
from oracle import cross as CR
from oracle import feet as FT
from oracle import grid as G
from oracle import ht as HT
from oracle import lomac as LM
from oracle import macro as MA
from oracle import nested_cross as NC
from oracle import spectral as SP
from oracle import step as ST
from oracle import timeint as TI

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ grid
def test_grid_points_printed_values():
    """Section 4.2 prints v_70 = 11/16 (two-stream slice) and v_64 = -dv/2
    (bump-on-tail slice) on 128-cell velocity grids: cell centres."""
    rows = [l.split() for l in open(os.path.join(GOLD, "grid_points.txt")) if l.strip() and not l.startswith("#")]
    assert rows
    for lo, hi, n, i1, val in rows:
        c = G.centres(float(lo), float(hi), int(n))
        assert abs(c[int(i1) - 1] - float(val)) < 1e-14


def test_quadratic_weights_closed_form():
    """Eq. (1d_quadratic_interp_weight): partition of unity, exact on
    quadratics, nodal at xi in {-1, 0, 1}; the general Lagrange form of width 3
    gives the same numbers."""
    xi = np.linspace(-0.5, 0.5, 41)
    w = G.quadratic_weights(xi)
    assert np.allclose(w.sum(-1), 1.0, atol=1e-15)
    for poly in (lambda t: 1 + 0 * t, lambda t: t, lambda t: t * t):
        exact = poly(xi)
        interp = w @ np.array([poly(-1.0), poly(0.0), poly(1.0)])
        assert np.allclose(interp, exact, atol=1e-14)
    assert np.allclose(G.lagrange_weights(xi, 3), w, atol=1e-15)
    assert np.allclose(G.quadratic_weights(np.array([0.0])), [[0, 1, 0]])


def test_quartic_weights_exact_on_quartics():
    """Width-5 stencil (the higher-order extension of section 3.1)."""
    xi = np.linspace(-0.5, 0.5, 33)
    w = G.lagrange_weights(xi, 5)
    nodes = np.arange(-2, 3, dtype=float)
    for deg in range(5):
        assert np.allclose(w @ nodes ** deg, xi ** deg, atol=1e-13)
    # a quintic is not reproduced (degree 4 exactly, not more)
    assert np.abs(w @ nodes ** 5 - xi ** 5).max() > 1e-3


def test_locate_half_open_cells():
    lo, h = -1.0, 0.25
    j, xi = G.locate(np.array([-1.0, -0.875, -0.75 + 1e-12, 0.999]), lo, h)
    assert list(j) == [0, 0, 1, 7]
    assert np.all(xi >= -0.5) and np.all(xi < 0.5)


# ----------------------------------------------------- HT-SL sampling (P2)
def _brute(F, rows, wts):
    return HT.block_interp(HT.full(F)[None], rows, wts)[:, 0]


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("width", [3, 5])
def test_ht_sample_equals_full_grid_interpolation_1d1v(kind, width):
    """Section 3.1: the leaf-contraction evaluation equals eq. (tp_interp) on
    the reconstructed tensor, for any ranks and feet."""
    p = SI.config("landau1d", n=20)
    F = SI.random_ht(2, p.n, (5, 7), seed=11)
    idx = SI.random_requests(p.n, 400, 2)
    E = 0.8 * SI.random_field((p.n[0],), 4)[None]
    foot = FT.feet(idx, p.lo, p.hi, p.n, 1, kind, 1.3, 1.0, E)
    rows, wts = FT.stencils(foot, idx, p.lo, p.hi, p.n, width, kind, 1)
    a = HT.sample(F, rows, wts)
    b = _brute(F, rows, wts)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()


@pytest.mark.parametrize("with_corr", [False, True])
def test_ht_sample_equals_full_grid_interpolation_2d2v(with_corr):
    p = SI.config("landau2d", n=10)
    F = SI.random_ht(4, p.n, (3, 4, 5, 2, 6, 4), seed=5)
    if with_corr:
        rng = np.random.default_rng(9)
        F["corr"] = {"C": rng.standard_normal((4, 10, 10)), "Q": rng.standard_normal((4, 10, 10))}
    idx = SI.random_requests(p.n, 600, 3)
    E = 0.5 * np.stack([SI.random_field((10, 10), 7), SI.random_field((10, 10), 8)])
    foot = FT.feet(idx, p.lo, p.hi, p.n, 2, 2, 0.9, 1.0, E)
    rows, wts = FT.stencils(foot, idx, p.lo, p.hi, p.n, 3, 2, 2)
    a = HT.sample(F, rows, wts)
    b = _brute(F, rows, wts)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


# ------------------------------------------------- stability analysis (P3-P5)
def _g1d(lam, zeta):
    m = np.round(lam)
    th = lam - m
    return np.exp(-1j * m * zeta) * (1 + th ** 2 * (np.cos(zeta) - 1) - 1j * th * np.sin(zeta))


def test_amplification_factor_of_x_shift():
    """Appendix A: a Fourier mode e^{i j zeta} is multiplied by
    g = e^{-i m zeta} (1 + th^2 (cos zeta - 1) - i th sin zeta), lam = m + th,
    for constant-coefficient advection with CFL lam = v tau / dx."""
    Nx, Nv = 32, 9
    lo, hi = (0.0, -3.0), (2 * math.pi, 3.0)
    kmode = 3
    x = G.centres(lo[0], hi[0], Nx)
    j = np.arange(Nx)
    zeta = 2 * math.pi * kmode / Nx
    F = {"leaves": [np.stack([np.cos(zeta * j), np.sin(zeta * j)], 1), np.eye(Nv)],
         "root": np.zeros((2, Nv))}
    F["root"][0, :] = 1.0       # F[i, v] = cos(zeta i) for every v
    tau = 0.37
    idx = np.stack(np.meshgrid(np.arange(Nx), np.arange(Nv), indexing="ij"), -1).reshape(-1, 2)
    foot = FT.feet(idx, lo, hi, (Nx, Nv), 1, 0, tau, 1.0)
    rows, wts = FT.stencils(foot, idx, lo, hi, (Nx, Nv), 3, 0, 1)
    out = HT.sample(F, rows, wts).reshape(Nx, Nv)
    v = G.centres(lo[1], hi[1], Nv)
    dx = (hi[0] - lo[0]) / Nx
    for c in range(Nv):
        g = _g1d(v[c] * tau / dx, zeta)
        expect = np.real(g * np.exp(1j * zeta * j))
        assert np.abs(out[:, c] - expect).max() < 1e-13
        assert abs(g) <= 1 + 1e-15


def test_integer_shift_is_exact_and_zero_step_is_identity():
    """Appendix A: an integer CFL is a pure circular shift; tau = 0 leaves
    every entry unchanged."""
    Nx, Nv = 16, 4
    lo, hi = (0.0, 0.5), (16.0, 4.5)       # dx = 1, v = 1, 2, 3, 4
    F = SI.random_ht(2, (Nx, Nv), (4, 3), seed=1)
    full = HT.full(F)
    idx = np.stack(np.meshgrid(np.arange(Nx), np.arange(Nv), indexing="ij"), -1).reshape(-1, 2)
    for tau, shift in ((1.0, 1), (0.0, 0)):
        foot = FT.feet(idx, lo, hi, (Nx, Nv), 1, 0, tau, 1.0)
        rows, wts = FT.stencils(foot, idx, lo, hi, (Nx, Nv), 3, 0, 1)
        out = HT.sample(F, rows, wts).reshape(Nx, Nv)
        for c in range(Nv):
            s = shift * (c + 1)
            assert np.abs(out[:, c] - np.roll(full[:, c], s)).max() < 1e-14


def test_l2_nonincrease_full_grid():
    """Theorem 1: ||F^{n+1}|| <= ||F^n|| for the constant-coefficient problem
    at any step size (full-grid update, 2D)."""
    rng = np.random.default_rng(0)
    N = 24
    f = rng.standard_normal((N, N))
    lo, hi = (0.0, 0.0), (1.0, 1.0)
    idx = np.stack(np.meshgrid(np.arange(N), np.arange(N), indexing="ij"), -1).reshape(-1, 2)
    P = FT.grid_points(idx, lo, hi, (N, N))
    for a in ((0.3, -0.7), (2.6, 11.2), (-7.45, 0.01)):
        foot = P - np.array(a) * 0.05
        rows, wts = [], []
        for m in range(2):
            j, xi = G.locate(foot[:, m], lo[m], 1.0 / N)
            rows.append(G.stencil_rows(j, 3, N)); wts.append(G.quadratic_weights(xi))
        g = HT.block_interp(f[None], rows, wts)[:, 0]
        assert np.linalg.norm(g) <= np.linalg.norm(f) * (1 + 1e-14)


# -------------------------------------------------------- cross approx (P6-P8)
def test_aca_recovers_exact_low_rank_matrix():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((50, 4)) @ rng.standard_normal((4, 70))
    U, V, info = CR.aca(lambda i: A[i], lambda j: A[:, j], lambda I, J: A[I, J], 50, 70,
                        1e-12, 20, 0, SI.probe_indices(50, 70, 64, 1))
    assert info["rank"] <= 5
    assert np.abs(U @ V.T - A).max() < 1e-12 * np.abs(A).max()


def test_slar_reproduces_landau_f0_exactly():
    """An exactly low-rank input (Landau f0: ranks x-leaves 2, others 1) is
    recovered exactly with its true ranks by a zero step."""
    p = SI.config("landau2d", n=12)
    o = ST.Oracle(p, probes=SI.probe_indices(144, 144, 64, 2))
    F0 = SI.initial_ht(p)
    Fn = o.slar(F0, 0, 0.0, 1.0, None)
    assert HT.ranks(Fn) == (2, 2, 1, 1, 1, 1)
    assert np.abs(HT.full(Fn) - HT.full(F0)).max() < 1e-14


def test_slar_matches_full_grid_update_within_tolerance():
    """SLAR(F) vs the dense SL-FD update of the same tensor: error of the
    order of eps_Base ||F|| (cross + truncation), on a 12^4 grid."""
    p = SI.config("landau2d", n=12).with_(tol=1e-6, rmax=40, alpha=0.3)
    o = ST.Oracle(p, probes=SI.probe_indices(144, 144, 64, 3))
    F0 = SI.initial_ht(p)
    E = o.efield(F0)
    Fn = o.slar(F0, 2, 0.5, 1.0, E)
    idx = np.stack(np.unravel_index(np.arange(12 ** 4), (12,) * 4), 1)
    foot = FT.feet(idx, p.lo, p.hi, p.n, 2, 2, 0.5, 1.0, E)
    rows, wts = FT.stencils(foot, idx, p.lo, p.hi, p.n, 3, 2, 2)
    dense = _brute(F0, rows, wts).reshape((12,) * 4)
    err = np.linalg.norm(HT.full(Fn) - dense) / np.linalg.norm(dense)
    assert err < 5 * p.tol


# ------------------------------------------- nested HT cross (next: row 3)
def _lookup(A):
    return lambda idx: A[idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]]


def _probes4(n, m, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, n[a], m) for a in range(4)], 1)


@pytest.mark.parametrize("n,ranks", [((7, 6, 8, 5), (3, 2, 3, 4, 4, 4)),
                                     ((12, 12, 12, 12), (5, 5, 5, 5, 8, 8)),
                                     ((10, 9, 11, 8), (4, 5, 3, 4, 6, 6))])
def test_nested_cross_recovers_exact_ht_ranks(n, ranks):
    """A tensor of exact HT ranks is reproduced to rounding by the nested
    skeleton, with exactly those ranks (brute force: full reconstruction)."""
    A = HT.full(SI.random_ht(4, n, ranks, seed=21))
    F, info = NC.nested_cross(_lookup(A), n, 1e-12, 30, _probes4(n, 64, 22), seed_index=(1, 2, 3, 1))
    assert np.linalg.norm(HT.full(F) - A) <= 1e-11 * np.linalg.norm(A)
    assert info["ranks"] == list(ranks)
    assert info["samples"] < A.size


def test_nested_cross_reproduces_its_sampled_blocks():
    """The skeleton interpolates: every entry of A[R1 x R2, P_v] and of
    A[P_x, R3 x R4] that it sampled is reproduced exactly."""
    n = (9, 8, 10, 7)
    A = HT.full(SI.random_ht(4, n, (4, 3, 5, 3, 5, 5), seed=23))
    A = A + 1e-3 * np.sin(np.arange(A.size).reshape(A.shape))      # not of low rank
    F, info = NC.nested_cross(_lookup(A), n, 1e-4, 30, _probes4(n, 64, 24))
    B = HT.full(F)
    s = info["sets"]
    for a in s["R"][0]:
        for b in s["R"][1]:
            for (j1, j2) in s["Pv"]:
                assert abs(B[a, b, j1, j2] - A[a, b, j1, j2]) <= 1e-10 * np.abs(A).max()
    for (i1, i2) in s["Px"]:
        for p in s["R"][2]:
            for q in s["R"][3]:
                assert abs(B[i1, i2, p, q] - A[i1, i2, p, q]) <= 1e-9 * np.abs(A).max()


def test_nested_cross_matches_full_grid_sl_update():
    """Nested cross of the SL-FD update (entries from the dense update of a
    12^4 Landau state, section 3.1) against that dense update: error of the
    order of the tolerance."""
    p = SI.config("landau2d", n=12).with_(tol=1e-6, rmax=40, alpha=0.3)
    o = ST.Oracle(p, probes=SI.probe_indices(144, 144, 64, 3))
    F0 = SI.initial_ht(p)
    E = o.efield(F0)
    idx = np.stack(np.unravel_index(np.arange(12 ** 4), (12,) * 4), 1)
    foot = FT.feet(idx, p.lo, p.hi, p.n, 2, 2, 0.5, 1.0, E)
    rows, wts = FT.stencils(foot, idx, p.lo, p.hi, p.n, 3, 2, 2)
    dense = _brute(F0, rows, wts).reshape((12,) * 4)
    F, info = NC.nested_cross(_lookup(dense), (12,) * 4, p.tol, 64, _probes4((12,) * 4, 64, 25),
                              seed_index=(0, 0, 6, 6))
    err = np.linalg.norm(HT.full(F) - dense) / np.linalg.norm(dense)
    assert err < 5 * p.tol, err
    assert info["converged"]


def test_nested_cross_zero_and_rank_one():
    n = (6, 5, 7, 4)
    F, info = NC.nested_cross(_lookup(np.zeros(n)), n, 1e-8, 10, _probes4(n, 16, 26))
    assert np.all(HT.full(F) == 0.0) and info["ranks"] == [0] * 6
    rng = np.random.default_rng(27)
    a = [rng.standard_normal(k) + 2.0 for k in n]
    A = np.einsum("i,j,k,l->ijkl", *a)
    F, info = NC.nested_cross(_lookup(A), n, 1e-10, 10, _probes4(n, 16, 28))
    assert info["ranks"] == [1] * 6
    assert np.abs(HT.full(F) - A).max() <= 1e-12 * np.abs(A).max()


def test_nested_cross_samples_grow_linearly_in_n():
    """Fixed HT ranks, n doubled: the nested skeleton samples grow about
    linearly in n; cross approximation on the {x}|{v} matricisation would
    sample k (N_x + N_v) = 2 k n^2 entries, four times more."""
    ranks = (3, 3, 3, 3, 4, 4)
    s = []
    for n in (16, 32):
        A = HT.full(SI.random_ht(4, (n,) * 4, ranks, seed=29))
        F, info = NC.nested_cross(_lookup(A), (n,) * 4, 1e-12, 20, _probes4((n,) * 4, 64, 30))
        assert np.linalg.norm(HT.full(F) - A) <= 1e-10 * np.linalg.norm(A)
        s.append(info["samples"])
    assert s[1] < 2.5 * s[0]
    assert s[1] < 2 * 4 * 32 ** 2


def test_truncation_error_bound_and_leading_singular_vectors():
    """HSVD error <= eps ||F|| and column 0 of each leaf = the leading left
    singular vector of that mode's matricisation (Supplement B)."""
    rng = np.random.default_rng(2)
    n = 9
    Ft = SI.random_ht(4, (n,) * 4, (4, 4, 4, 4, 6, 6), seed=7)
    A = HT.full(Ft).reshape(n * n, n * n) + 1e-7 * rng.standard_normal((n * n, n * n))
    tol = 1e-4
    Fh = CR.truncate_dense(A, (n, n), (n, n), tol, 81)
    R = HT.full(Fh).reshape(n * n, n * n)
    assert np.linalg.norm(R - A) <= tol * np.linalg.norm(A) * (1 + 1e-12)
    T = HT.full(Fh)
    for mu in range(4):
        M = np.moveaxis(T, mu, 0).reshape(n, -1)
        u, s, _ = np.linalg.svd(M)
        c0 = Fh["leaves"][mu][:, 0]
        assert abs(abs(u[:, 0] @ c0) - 1.0) < 1e-8


def test_recompress_matches_dense_svd():
    rng = np.random.default_rng(8)
    U = rng.standard_normal((40, 7)); V = rng.standard_normal((30, 7))
    X, s, Y, _, _ = CR.recompress(U, V, 1e-14, 40, 2)
    sd = np.linalg.svd(U @ V.T, compute_uv=False)
    assert np.allclose(s, sd[: len(s)], rtol=1e-12)
    assert np.abs(X @ np.diag(s) @ Y.T - U @ V.T).max() < 1e-12 * np.abs(U @ V.T).max()


# ------------------------------------------------------------- Poisson (P10)
def test_poisson_closed_form_and_zero_mean():
    """rho = -alpha cos(kx) (n_e = 1 + alpha cos kx, n_i = 1) gives
    E = -(alpha/k) sin(kx), eqs. (Poisson), (Efromphi)."""
    k, a = 0.5, 0.3
    L = 2 * math.pi / k
    x = G.centres(0.0, L, 64)
    _, E = SP.poisson(1 + a * np.cos(k * x), 1.0, [L])
    assert np.abs(E[0] + (a / k) * np.sin(k * x)).max() < 1e-13
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    _, E2 = SP.poisson(1 + a * np.cos(k * X1) + a * np.cos(k * X2), 1.0, [L, L])
    assert np.abs(E2[1] + (a / k) * np.sin(k * X2)).max() < 1e-13
    assert abs(E2.sum()) < 1e-11


def test_discrete_identities_sum_div_and_sum_rho_E():
    """Spectral compatibility (section 3.2.3): sum D.F = 0, sum rho E = 0."""
    f = SI.random_field((24, 20), 3, smooth=False)
    F = np.stack([SI.random_field((24, 20), 4, smooth=False), SI.random_field((24, 20), 5, smooth=False)])
    L = [3.0, 5.0]
    assert abs(SP.div(F, L).sum()) < 1e-11
    _, E = SP.poisson(1.0 + 0.3 * f, 1.0, L)
    rho = -0.3 * f
    assert np.abs((rho[None] * E).sum(axis=(1, 2))).max() < 1e-11


# --------------------------------------------------------------- LoMaC (P9)
def _rand_basis(seed=0, dv=2, n=12):
    rng = np.random.default_rng(seed)
    vg = [G.centres(-5, 5, n) for _ in range(dv)]
    u1 = [np.exp(-0.5 * (v - rng.uniform(-1, 1)) ** 2) * (1 + 0.2 * rng.standard_normal(n)) for v in vg]
    u1 = [u / np.linalg.norm(u) for u in u1]
    return LM.basis(u1, vg, [10.0 / n] * dv), vg


def test_q_basis_is_orthogonal_and_norms_factorise():
    """Supplement B: Q_0, Q_{1,mu}, Q_2 are orthogonal in <.,.>_{v;omega^-1}
    and their squared norms are the stated products of 1D norms."""
    B, vg = _rand_basis()
    h = 10.0 / 12
    Om = np.multiply.outer(B["g"][0]["omega"], B["g"][1]["omega"])
    Q = B["Q"]
    Gm = np.einsum("aij,bij->ab", Q, Q / Om[None] * h * h)
    off = Gm - np.diag(np.diag(Gm))
    assert np.abs(off).max() < 1e-12 * np.abs(np.diag(Gm)).max()
    assert np.allclose(np.diag(Gm), B["NQ"], rtol=1e-12)
    assert Om.min() >= LM.DELTA ** 2


def test_projection_preserves_moments_and_is_idempotent():
    """Eq. (moments_pres_disc), R(U(F)) = P*F and P*(P*F) = P*F."""
    B, vg = _rand_basis(1)
    rng = np.random.default_rng(3)
    Fd = rng.random((6, 5, 12, 12))
    dvol = (10.0 / 12) ** 2
    PF = LM.project_dense(Fd, 2, B, vg, dvol)
    Mf = HT.dense_moments(Fd, 2, vg, dvol)[:4]
    Mp = HT.dense_moments(PF, 2, vg, dvol)[:4]
    assert np.abs(Mf - Mp).max() < 1e-12 * np.abs(Mf).max()
    PPF = LM.project_dense(PF, 2, B, vg, dvol)
    assert np.abs(PPF - PF).max() < 1e-12 * np.abs(PF).max()
    L = [3.0, 4.0]
    U = LM.conserved_from_raw(Mf, 1.0, L)
    RU = LM.expand(LM.coefficients(LM.raw_from_conserved(U, 1.0, L), B), B["Q"])
    assert np.abs(RU - PF).max() < 1e-12 * np.abs(PF).max()


def test_gaussian_weight_symmetric_grid():
    """A Maxwellian weight on a symmetric grid: gamma = beta = 0 and eta is the
    discrete second moment ratio sum v^2 w / sum w (pure odd/even symmetry)."""
    v = G.centres(-6, 6, 32)
    u = np.exp(-0.5 * v * v)
    g = LM.gram_schmidt_1d(u / np.linalg.norm(u), v, 12 / 32)
    assert abs(g["gamma"]) < 1e-14 and abs(g["beta"]) < 1e-13
    assert abs(g["eta"] - np.sum(v * v * u) / np.sum(u)) < 1e-13


# ---------------------------------------------------------------- solvers
def test_fgmres_solves_linear_system():
    rng = np.random.default_rng(0)
    A = np.eye(60) + 0.3 * rng.standard_normal((60, 60)) / math.sqrt(60)
    b = rng.standard_normal(60)
    x, its = MA.fgmres(lambda v: A @ v, b, 1e-12, restart=20, maxit=400)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-9 * np.linalg.norm(x)
    # a preconditioner that is the exact inverse converges in one iteration
    Ainv = np.linalg.inv(A)
    x2, its2 = MA.fgmres(lambda v: A @ v, b, 1e-10, restart=20, maxit=400, precond=lambda v: Ainv @ v)
    assert its2 == 1 and np.linalg.norm(x2 - x) < 1e-8 * np.linalg.norm(x)


def test_lomac_step_conserves_and_matches_macro_state():
    """Section 3.2.2-3.2.3 with the spectral identities: U(F^{n+1}) = U^{n+1}
    and total mass, momentum and energy are conserved to round-off."""
    p = SI.config("landau2d", n=16).with_(rmax=20, alpha=0.2)
    o = ST.Oracle(p, probes=SI.probe_indices(256, 256, 64, 7))
    F = SI.initial_ht(p)
    U = o.conserved(F)
    d0 = o.diagnostics(F)
    Unm1 = None
    for n in range(2):
        Fs = o.slar_vp(F, p.dt)
        F, Unew, info = o.lomac(Fs, U, Unm1, p.dt)
        assert info["converged"]
        Unm1, U = U, Unew
        Uk = o.conserved(F)
        assert np.abs(Uk - U).max() < 1e-12 * np.abs(U).max()
    d = o.diagnostics(F)
    assert abs(d["mass"] - d0["mass"]) < 1e-12 * d0["mass"]
    assert abs(d["energy"] - d0["energy"]) < 1e-12 * d0["energy"]
    assert max(abs(m) for m in d["momentum"]) < 1e-12 * d0["mass"]


# ---------------------------------------------------------- Landau (P12)
def _landau_root(k):
    from scipy.special import wofz
    from scipy.optimize import fsolve

    def f(z):
        w = complex(z[0], z[1])
        zeta = w / (math.sqrt(2) * k)
        Z = 1j * math.sqrt(math.pi) * wofz(zeta)
        D = 1 + (1 + zeta * Z) / k ** 2
        return [D.real, D.imag]

    r = fsolve(f, [1.4, -0.15], xtol=1e-13)
    return r[0], r[1]


def test_linear_landau_rate_1d1v():
    """Linear Landau damping at k = 0.5: the electric energy envelope decays
    as exp(2 gamma t) with gamma from the Maxwellian dispersion relation
    (-0.1533); split 1D1V workload on 64^2."""
    om, gam = _landau_root(0.5)
    assert abs(gam + 0.1533) < 1e-3
    p = SI.config("landau1d").with_(T=15.0)
    o = ST.Oracle(p)
    _, hist = o.run(SI.initial_ht(p), 150)
    ee = np.log([h["elec_energy"] for h in hist])
    t = np.arange(len(ee)) * p.dt
    pk = [i for i in range(1, len(ee) - 1) if ee[i] > ee[i - 1] and ee[i] >= ee[i + 1]]
    slope = np.polyfit(t[pk], ee[pk], 1)[0]
    assert abs(slope / 2 - gam) < 0.05 * abs(gam), (slope / 2, gam)
    # oscillation: energy peaks are half a plasma period apart
    per = np.mean(np.diff(t[pk]))
    assert abs(per - math.pi / om) < 0.1


# ------------------------------------------------------------- CNN (P16)
def test_cnn_gradient_matches_central_differences():
    """The CNN oracle's backward pass against central finite differences of
    its forward pass (the pin the GPU gradients are checked against)."""
    from oracle import cnn as CN
    rng = np.random.default_rng(5)
    shapes = [(3, 4), (4, 4), (4, 2)]
    theta = 0.3 * rng.standard_normal(CN.nparams(shapes))
    x = rng.standard_normal((2, 3, 6, 5))
    y = rng.standard_normal((2, 2, 6, 5))
    g = CN.grad(theta, shapes, x, y)
    idx = rng.choice(len(theta), 25, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta); e[i] = h
        fd = (CN.loss(theta + e, shapes, x, y) - CN.loss(theta - e, shapes, x, y)) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_cnn_conv_is_periodic_cross_correlation():
    from oracle import cnn as CN
    x = np.zeros((1, 1, 5, 5)); x[0, 0, 0, 0] = 1.0
    w = np.zeros((1, 1, 3, 3)); w[0, 0, 0, 0] = 2.0      # tap (dy, dx) = (0, 0) reads in[y-1, x-1]
    out = CN.conv(x, w, np.zeros(1))
    assert out[0, 0, 1, 1] == 2.0 and abs(out).sum() == 2.0


def test_cnn_features_invariants():
    """Network input: U channels standardised one by one (mean 0, std 1),
    residual channels of rms 1 over all channels together (not one by one),
    invariance under any scaling of v and any affine map of each U channel,
    and a constant U channel mapped to zero."""
    from oracle import cnn as CN
    rng = np.random.default_rng(11)
    K, H, W = 4, 6, 5
    v = rng.standard_normal((K, H, W)) * np.array([1.0, 3.0, 0.1, 7.0])[:, None, None]
    U = rng.standard_normal((K, H, W)) * np.array([2.0, 0.5, 9.0, 1.0])[:, None, None] + 4.0
    f = CN.features(v, U)
    assert f.shape == (2 * K, H, W)
    assert abs(np.sqrt(np.mean(f[:K] ** 2)) - 1.0) < 1e-14
    # channel scales are kept relative to each other (one rms for all)
    assert np.allclose(f[:K] / v, f[0, 0, 0] / v[0, 0, 0], rtol=1e-13, atol=0)
    for c in range(K):
        assert abs(f[K + c].mean()) < 1e-13
        # the std guard adds 1e-12 |mean| / std (< 1e-10 here) to the std
        assert abs(f[K + c].std() - 1.0) < 1e-10
    a = rng.uniform(0.5, 2.0, K)[:, None, None]
    b = rng.uniform(-3.0, 3.0, K)[:, None, None]
    assert np.allclose(CN.features(-37.0 * v, a * U + b)[:K], -f[:K], rtol=1e-13, atol=1e-15)
    assert np.allclose(CN.features(v, a * U + b)[K:], f[K:], rtol=1e-10, atol=1e-12)
    U2 = U.copy(); U2[3] = 2.5
    f2 = CN.features(v, U2)
    assert np.all(np.isfinite(f2)) and np.all(f2[K + 3] == 0.0)
    assert np.all(CN.features(np.zeros_like(v), U)[:K] == 0.0)


def test_cnn_apply_and_target_are_inverse():
    """An untrained network (last layer zero) leaves the spectral
    preconditioner unchanged, and the training target of the pair
    (w, apply(w)) is exactly the network output scaled back by rms(w)."""
    from oracle import cnn as CN
    rng = np.random.default_rng(12)
    K, H, W = 4, 5, 4
    shapes = [(2 * K, 6), (6, K)]
    theta = 0.3 * rng.standard_normal(CN.nparams(shapes))
    w = rng.standard_normal((K, H, W)); U = rng.standard_normal((K, H, W))
    pw = rng.standard_normal((K, H, W))
    th0 = theta.copy(); th0[CN.nparams([shapes[0]]):] = 0.0
    assert np.array_equal(CN.apply(th0, shapes, w, U, pw), pw)
    z = CN.apply(theta, shapes, w, U, pw)
    out, _ = CN.forward(theta, shapes, CN.features(w, U)[None])
    assert np.allclose(CN.target(z, pw, w), out[0], rtol=1e-12, atol=1e-14)
    assert np.allclose(CN.apply(theta, shapes, 5.0 * w, U, 5.0 * pw), 5.0 * z, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------
# Macroscopic time integrators (section 4: S-stable DIRK-3 start-up, then
# variable-step BDF-3).

def test_dirk3_tableau_is_third_order_stiffly_accurate_and_l_stable():
    """Order conditions up to three, c = A 1, last row = b, and the stability
    function R(z) = 1 + z b^T (I - z A)^{-1} 1 is bounded by 1 on the
    imaginary axis and vanishes at infinity (L-stability: 1 - b^T A^{-1} 1)."""
    A, b, c = TI.dirk3()
    one = np.ones(3)
    assert np.allclose(A @ one, c, atol=1e-15, rtol=0)
    assert np.allclose(A[2], b, atol=0, rtol=0)
    assert np.allclose(np.triu(A, 1), 0.0, atol=0, rtol=0)
    assert abs(b @ one - 1.0) < 1e-14
    assert abs(b @ c - 0.5) < 1e-14
    assert abs(b @ (c * c) - 1.0 / 3.0) < 1e-14
    assert abs(b @ A @ c - 1.0 / 6.0) < 1e-14
    assert abs(A[0, 0] - A[1, 1]) == 0.0 and abs(A[1, 1] - A[2, 2]) == 0.0
    assert abs(1.0 - b @ np.linalg.solve(A, one)) < 1e-13
    for y in np.linspace(-50.0, 50.0, 401):
        z = 1j * y
        R = 1.0 + z * (b @ np.linalg.solve(np.eye(3) - z * A, one))
        assert abs(R) <= 1.0 + 1e-12


def test_bdf_weights_reduce_to_textbook_and_are_exact_for_cubics():
    """Equal steps: backward Euler, BDF2 (4/3, -1/3; 2h/3) and BDF3 (18/11,
    -9/11, 2/11; 6h/11).  Any distinct nodes: U(t0) - sum_j c_j U(t_j) =
    beta U'(t0) holds exactly for every cubic (the weights differentiate the
    interpolating polynomial)."""
    h = 0.37
    c, beta = TI.bdf([h, 0.0])
    assert np.allclose(c, [1.0], rtol=1e-15) and abs(beta - h) < 1e-16
    c, beta = TI.bdf([2 * h, h, 0.0])
    assert np.allclose(c, [4.0 / 3.0, -1.0 / 3.0], rtol=1e-14) and abs(beta - 2 * h / 3) < 1e-15
    c, beta = TI.bdf([3 * h, 2 * h, h, 0.0])
    assert np.allclose(c, [18 / 11, -9 / 11, 2 / 11], rtol=1e-14) and abs(beta - 6 * h / 11) < 1e-15
    rng = np.random.default_rng(5)
    for _ in range(20):
        steps = rng.uniform(0.05, 0.5, 3)
        t = np.cumsum(np.concatenate([[0.0], steps]))[::-1]      # t0 > t1 > t2 > t3
        c, beta = TI.bdf(t)
        assert abs(c.sum() - 1.0) < 1e-13
        coef = rng.standard_normal(4)
        P = np.polynomial.Polynomial(coef)
        lhs = P(t[0]) - sum(c[j] * P(t[1 + j]) for j in range(3))
        assert abs(lhs - beta * P.deriv()(t[0])) < 1e-12 * (1 + np.abs(coef).sum())


def _linear_run(lam, hs):
    """u' = -lam u (R(u) = lam u) from u(0) = 1 with the step sequencing of
    the kinetic driver: two DIRK-3 start-up steps, then BDF-3."""
    Us, ts = [np.array([1.0])], [0.0]

    def stage(i, tau, U_hist, beta):
        return U_hist / (1.0 + beta * lam), (lambda u: lam * u)

    for n, h in enumerate(hs):
        if n < 2:
            U = TI.dirk3_step(Us[-1], h, stage)
        else:
            U_hist, beta = TI.bdf_history(Us, ts, h)
            U = U_hist / (1.0 + beta * lam)
        Us.append(U)
        ts.append(ts[-1] + h)
    return float(Us[-1][0]), ts[-1]


def test_dirk3_bdf3_sequencing_converges_at_third_order():
    """The shared step sequencing (stage history sums, BDF history) on
    u' = -lam u: the error at T = 2 falls by ~8 per halving of the step,
    with equal steps and with steps alternating by a ratio 1.25."""
    lam = 1.3
    for pattern in ([1.0], [1.0, 1.25]):
        errs = []
        for m in (20, 40, 80):
            base = 2.0 / m
            hs = [base * pattern[i % len(pattern)] for i in range(m)]
            hs = [x * 2.0 / sum(hs) for x in hs]
            u, T = _linear_run(lam, hs)
            errs.append(abs(u - np.exp(-lam * T)))
        rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert all(2.7 < r < 3.3 for r in rates), (pattern, errs, rates)


@pytest.mark.parametrize("name,N", [("landau1d_paper", 32), ("stronglandau1d", 24),
                                    ("bumpontail1d", 40), ("bumpontail2d", 10)])
def test_paper_workload_initial_data(name, N):
    """The low-rank initial HT of each section 4 setup reconstructs the
    printed initial condition at every cell centre, and its step is the
    CFL-5 step dt = 5 dx / v_max."""
    p = SI.config(name, n=N)
    F = HT.full(SI.initial_ht(p))
    xs = [SI.cell_centres(p.lo[m], p.hi[m], p.n[m]) for m in range(p.d)]
    G_ = np.meshgrid(*xs, indexing="ij")
    if p.dx == 1:
        x, v = G_
        if p.kind == "landau":
            f = (1 + p.alpha * np.cos(0.5 * x)) * np.exp(-v * v / 2) / math.sqrt(2 * math.pi)
        else:
            s2p = math.sqrt(2 * math.pi)
            f = (1 + 0.04 * np.cos(0.3 * x)) * (9 / (10 * s2p) * np.exp(-v * v / 2)
                                               + 2 / (10 * s2p) * np.exp(-(v - 4.5) ** 2 / (2 * 0.5)))
    else:
        x1, x2, v1, v2 = G_
        vt = 2.4
        f = (1 + 0.04 * np.cos(0.3 * x1) * np.cos(0.3 * x2)) / (2 * math.sqrt(2 * math.pi)) ** 2 * (
            17 / (40 * math.pi) * np.exp(-(v1 * v1 + v2 * v2) / 2)
            + 3 / (40 * math.pi * vt) * np.exp(-((v1 - 4.5) ** 2 + v2 * v2) / (2 * vt)))
    assert np.abs(F - f).max() < 1e-15 * max(1.0, np.abs(f).max())
    dx = (p.hi[0] - p.lo[0]) / p.n[0]
    assert abs(p.dt - 5 * dx / p.hi[p.dx]) < 1e-15
    assert p.integrator == "dirk3_bdf3" and not p.split and p.order == 3


def test_cur_core_reproduces_skeleton_and_exact_low_rank():
    """CUR identities behind the regularised skeleton: with W invertible and
    no truncation, C W^+ R is the cross itself (it interpolates its pivot
    fibers); for a matrix of rank r whose pivot block has rank r, the
    rank-r truncated core gives the matrix exactly (A = C W^+ R when
    rank W = rank A)."""
    rng = np.random.default_rng(12)
    A = rng.standard_normal((40, 5)) @ rng.standard_normal((5, 50))
    U, V, info = CR.aca(lambda i: A[i], lambda j: A[:, j], lambda I, J: A[I, J], 40, 50,
                        1e-14, 5, 0, None)
    Uc, Vc = CR.cur_core(U, V, info["pivots"], 5)
    assert np.abs(Uc @ Vc.T - U @ V.T).max() < 1e-12 * np.abs(A).max()
    assert np.abs(Uc @ Vc.T - A).max() < 1e-12 * np.abs(A).max()
    # a rank-12 matrix crossed with 9 terms, core truncated to 4: the result
    # has rank 4 and reproduces C W_4^+ R built from the sampled fibers
    B = rng.standard_normal((30, 12)) @ rng.standard_normal((12, 35))
    U, V, info = CR.aca(lambda i: B[i], lambda j: B[:, j], lambda I, J: B[I, J], 30, 35,
                        1e-14, 9, 0, None)
    I = [p[0] for p in info["pivots"]]; J = [p[1] for p in info["pivots"]]
    Uc, Vc = CR.cur_core(U, V, info["pivots"], 4)
    assert Uc.shape[1] == 4 and np.linalg.matrix_rank(Uc @ Vc.T) == 4
    Y, s, Zt = np.linalg.svd(B[np.ix_(I, J)])
    ref = B[:, J] @ (Zt[:4].T @ np.diag(1.0 / s[:4]) @ Y[:, :4].T) @ B[I, :]
    assert np.abs(Uc @ Vc.T - ref).max() < 1e-10 * np.abs(ref).max()


def test_correction_filter_keeps_totals_and_resolved_band():
    """The band-limited LoMaC correction: the zero mode (hence mass,
    momentum and energy totals) is unchanged to rounding, modes up to a
    sixth of the Nyquist index to 1e-4, a mode at half the Nyquist index is
    scaled by e^-(36/256) = 0.868815 per axis, the Nyquist mode is removed
    (e^-36), the scaling is a tensor product over the axes, and the result
    is real."""
    rng = np.random.default_rng(3)
    n = 24
    U0 = rng.standard_normal((4, n, n))
    x = np.arange(n) * 2 * math.pi / n
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    const = np.full((n, n), 0.7)
    Uf = LM.filter_correction(U0 + const[None], U0)
    assert np.abs(Uf - U0 - const[None]).max() < 1e-14
    low = np.cos(2 * X1 + 0.3) * np.sin(X2)               # modes |m| <= 2 = n / 12
    U = U0 + low[None] * np.arange(1, 5)[:, None, None]
    Uf = LM.filter_correction(U, U0)
    assert np.abs(Uf - U).max() < 1e-4 * 4
    half = np.cos(6 * X1 + 0.4)                            # |m| = 6 = Nyquist / 2 along axis 0
    Uf = LM.filter_correction(U0 + half[None], U0)
    assert np.abs(Uf - U0 - 0.868815 * half[None]).max() < 1e-6
    both = np.cos(6 * X1) * np.cos(6 * X2)                 # half the Nyquist index on both axes
    Uf = LM.filter_correction(U0 + both[None], U0)
    assert np.abs(Uf - U0 - 0.868815 ** 2 * both[None]).max() < 1e-6
    nyq = np.cos(math.pi * np.arange(n))[:, None] * np.ones((1, n))   # pure Nyquist along axis 0
    Uf = LM.filter_correction(U0 + nyq[None], U0)
    assert np.abs(Uf - U0).max() < 1e-14 + 3e-16 * n
    Ur = U0 + rng.standard_normal((4, n, n))
    Uf = LM.filter_correction(Ur, U0)
    assert np.isrealobj(Uf)
    assert np.abs(Uf.sum(axis=(1, 2)) - Ur.sum(axis=(1, 2))).max() < 1e-12
    assert np.linalg.norm(Uf - U0) < np.linalg.norm(Ur - U0)


def test_frame_sampling_equals_leaf_to_root_contraction():
    """Eq. (tp_interp) evaluated on the node frames (x frame, v frame times
    the root) gives the leaf-to-root HT contraction's value at every foot."""
    p = SI.config("landau2d", n=10)
    F = SI.random_ht(4, p.n, (3, 4, 5, 3, 6, 5), seed=44)
    idx = SI.random_requests(p.n, 400, 8)
    E = 0.5 * np.stack([SI.random_field((10, 10), 1), SI.random_field((10, 10), 2)])
    foot = FT.feet(idx, p.lo, p.hi, p.n, 2, 2, 0.6, 1.0, E)
    rows, wts = FT.stencils(foot, idx, p.lo, p.hi, p.n, 3, 2, 2)
    a = HT.sample(F, rows, wts)
    X = HT.x_frame(F)
    P = np.tensordot(HT.v_frame(F), F["root"], axes=([2], [1]))
    b = HT.sample_frames(X, P, rows, wts)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_dispersion_roots_of_linear_theory():
    """The rates the long GPU runs are checked against: Landau damping at
    k = 0.5 (-0.1534), the purely growing two-stream root for beams at
    +-2.4, k = 0.2 (0.2258), and the bump-on-tail root of the section 4
    setup (0.9587 + 0.1917 i)."""
    import math
    from dispersion import root_beams, root_maxwellians
    om, gam = root_beams(0.5, 0.0, [1.4, -0.15])
    assert abs(gam + 0.1534) < 1e-3 and abs(om - 1.4157) < 1e-3
    om, gam = root_beams(0.2, 2.4, [0.0, 0.2])
    assert abs(om) < 1e-8 and abs(gam - 0.2258) < 1e-3
    p = SI.config("bumpontail1d")
    n_p, n_b, u, vt = p.bump
    comps = [(n_p * math.sqrt(2 * math.pi), 0.0, 1.0), (n_b * math.sqrt(2 * math.pi * vt), u, vt)]
    om, gam = root_maxwellians(p.k, comps, [1.0, 0.2])
    assert abs(om - 0.9587) < 1e-3 and abs(gam - 0.1917) < 1e-3
