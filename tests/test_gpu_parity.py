"""GPU parity: every C-ABI entry point against the CPU FP64 oracle on the
same seeded inputs.  Tolerances (normwise max|a-b|/max|b|):
  FP64 arithmetic 1e-12; FP32 contractions 1e-6 (single-precision sums of
  at most a few thousand O(1) terms with orthonormal leaves).
Samples whose foot lies on a cell face (two valid stencils) are compared
with both oracle readings."""
import math

import numpy as np
import pytest

import slar_inputs as SI
from oracle import feet as FT
from oracle import ht as HT
from oracle import spectral as SP
from oracle import step as ST

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_29027_amd import lib as L  # noqa: E402
from gpu_util import dev, ht_to_dev, normwise, ht_from_dev  # noqa: E402


def _oracle_samples(F, p, idx, kind, tau, cv, E, width):
    foot = FT.feet(idx, p.lo, p.hi, p.n, p.dx, kind, tau, cv, E)
    rows, wts = FT.stencils(foot, idx, p.lo, p.hi, p.n, width, kind, p.dx)
    amb = FT.face_ambiguous(foot, p.lo, p.hi, p.n, kind, p.dx)
    return HT.sample(F, rows, wts), amb


CASES = [
    ("landau1d", 20, 0, 5, 1.7), ("landau1d", 20, 1, 5, 1.3), ("landau1d", 20, 2, 5, 0.9),
    ("landau1d", 33, 2, 3, 2.2), ("landau2d", 10, 2, 3, 0.8), ("landau2d", 9, 0, 3, 0.6),
]


@pytest.mark.parametrize("name,N,kind,width,tau", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ht_sample_matches_oracle(name, N, kind, width, tau, prec):
    p = SI.config(name, n=N)
    d = p.d
    ranks = (6, 9) if d == 2 else (4, 5, 3, 6, 7, 5)
    F = SI.random_ht(d, p.n, ranks, seed=21)
    idx = SI.random_requests(p.n, 1000 + 37, seed=5)        # ragged tail
    nx = p.n[: p.dx]
    E1 = np.stack([0.6 * SI.random_field(nx, 40 + m) for m in range(p.dx)])
    E2 = np.stack([0.6 * SI.random_field(nx, 50 + m) for m in range(p.dx)])
    cE = (-1.0 / 12.0, 3.0 / 4.0)
    Eo = FT.frozen_field([E1, E2], cE)
    ref, amb = _oracle_samples(F, p, idx, kind, tau, 1.0, Eo, width)
    tdt = torch.float64 if prec == "f64" else torch.float32
    T = ht_to_dev(F, tdt)
    H = L.make_ht(T, d, L.F64 if prec == "f64" else L.F32)
    g = L.make_grid(p)
    out = torch.zeros(len(idx), dtype=tdt, device="cuda")
    adv = L.make_adv(kind, tau, 1.0, dev(E1), dev(E2), cE, order=width)
    L.slar_ht_sample(g, H, adv, dev(idx, torch.int32), out)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    tol = 1e-12 if prec == "f64" else 1e-6
    keep = ~amb
    assert keep.sum() > 0.9 * len(idx)
    assert normwise(got[keep], ref[keep]) < tol


# Ranks that take one, two and four 16-column matrix-core tiles, ranks that
# are not multiples of the 4-deep K step, r12 != r34, the rank cap 64, both
# trees and both stencil widths; 221 entries = three whole 64-entry blocks
# and a ragged one.
HIGH_RANK = [
    ("landau2d", 32, (13, 18, 21, 10, 29, 17), 3),
    ("landau2d", 64, (40, 37, 45, 33, 61, 50), 3),
    ("landau2d", 64, (64, 64, 64, 64, 64, 64), 3),
    ("landau1d", 64, (27, 21), 5),
    ("landau1d", 128, (64, 55), 3),
    ("landau1d", 48, (3, 47), 5),
]


@pytest.mark.parametrize("name,N,ranks,width", HIGH_RANK)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ht_sample_high_rank_within_rounding_bound(name, N, ranks, width, prec):
    """FP64: every entry lies within the rounding-error bound of its
    contraction, |f~ - f| <= gamma_n |f|(x), gamma_n = n u / (1 - n u), where
    |f|(x) is the same contraction of the absolute values of the weights,
    leaves, transfer tensors and root (computed by the oracle) and n bounds
    the roundings along any term: W-point sum and product (W + 2), the
    Khatri-Rao product, the K = r_a r_b sum with its products, the root sum
    over r_k, the product with the left factor and the column sums
    (n = K + r_k + r_n + W + 16).  Random Gaussian transfer tensors cancel
    strongly (|f|(x) / |f| ~ 1e5 at rank 64), so in FP32 that bound says
    nothing; there the bar is normwise, 3e-5, the size of FP32 sums of up
    to 4096 terms of comparable magnitude (sqrt(4096) 2^-24 ~ 4e-6, with
    margin).  FP64 also meets 1e-12 normwise."""
    p = SI.config(name, n=N)
    d = p.d
    F = SI.random_ht(d, p.n, ranks, seed=31)
    idx = SI.random_requests(p.n, 3 * 64 + 29, seed=6)
    E = np.stack([0.6 * SI.random_field(p.n[: p.dx], 60 + m) for m in range(p.dx)])
    foot = FT.feet(idx, p.lo, p.hi, p.n, p.dx, 2, 0.9, 1.0, E)
    rows, wts = FT.stencils(foot, idx, p.lo, p.hi, p.n, width, 2, p.dx)
    amb = FT.face_ambiguous(foot, p.lo, p.hi, p.n, 2, p.dx)
    ref = HT.sample(F, rows, wts)
    Fa = {k: ([np.abs(x) for x in v] if k == "leaves" else np.abs(v)) for k, v in F.items()}
    scale = HT.sample(Fa, rows, [np.abs(w) for w in wts])
    if d == 2:
        K, rk, rn = ranks[1], ranks[1], ranks[0]
    else:
        K, rk, rn = max(ranks[0] * ranks[1], ranks[2] * ranks[3]), ranks[5], ranks[4]
    u = 2.0 ** -53 if prec == "f64" else 2.0 ** -24
    nr = K + rk + rn + width + 16
    gamma = nr * u / (1 - nr * u)
    tdt = torch.float64 if prec == "f64" else torch.float32
    H = L.make_ht(ht_to_dev(F, tdt), d, L.F64 if prec == "f64" else L.F32)
    g = L.make_grid(p)
    out = torch.zeros(len(idx), dtype=tdt, device="cuda")
    adv = L.make_adv(2, 0.9, 1.0, dev(E), order=width)
    L.slar_ht_sample(g, H, adv, dev(idx, torch.int32), out)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    keep = ~amb
    assert keep.sum() > 0.9 * len(idx)
    err = np.abs(got - ref)[keep]
    if prec == "f64":
        assert np.all(err <= gamma * scale[keep]), float(np.max(err / (gamma * scale[keep])))
    assert normwise(got[keep], ref[keep]) < (1e-12 if prec == "f64" else 3e-5)


def test_ht_sample_empty_request_and_invalid_args():
    p = SI.config("landau2d", n=8)
    F = SI.random_ht(4, p.n, (2, 2, 2, 2, 2, 2), seed=1)
    T = ht_to_dev(F)
    H = L.make_ht(T, 4, L.F64)
    g = L.make_grid(p)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    idx = torch.zeros((0, 4), dtype=torch.int32, device="cuda")
    L.slar_ht_sample(g, H, L.make_adv(0, 0.1), idx, out)
    with pytest.raises(L.SlarError):
        L.slar_ht_sample(g, H, L.make_adv(2, 0.1, 1.0, None), dev(np.zeros((4, 4)), torch.int32), out)


@pytest.mark.parametrize("name,N", [("landau1d", 24), ("landau2d", 12)])
@pytest.mark.parametrize("prec", [L.F64, L.F32])
def test_frame_sampler_matches_oracle(name, N, prec):
    p = SI.config(name, n=N)
    d = p.d
    ranks = (7, 5) if d == 2 else (4, 5, 3, 6, 9, 7)
    F = SI.random_ht(d, p.n, ranks, seed=3)
    g = L.make_grid(p)
    ws = L.Workspace(g, 40)
    T = ht_to_dev(F)
    H = L.make_ht(T, d, L.F64)
    Nx = int(np.prod(p.n[: p.dx])); Nv = int(np.prod(p.n[p.dx:]))
    X = torch.zeros((Nx, 12), dtype=torch.float64, device="cuda")
    P = torch.zeros((Nv, 12), dtype=torch.float64, device="cuda")
    Fr = L.slar_frames_from_ht(g, H, L.frames(X, P, 0), ws)
    width = p.order if d == 2 else 3
    E = np.stack([0.5 * SI.random_field(p.n[: p.dx], 7 + m) for m in range(p.dx)])
    idx = SI.random_requests(p.n, 2000 + 3, seed=9)
    ref, amb = _oracle_samples(F, p, idx, 2, 0.7, 1.0, E, width)
    out = torch.zeros(len(idx), dtype=torch.float64, device="cuda")
    L.slar_frame_sample(g, Fr, L.make_adv(2, 0.7, 1.0, dev(E), order=width), prec, dev(idx, torch.int32), out, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    tol = 1e-12 if prec == L.F64 else 1e-6
    assert normwise(got[~amb], ref[~amb]) < tol
    # frames themselves equal the node frames of the oracle
    Xo = HT.x_frame(F).reshape(Nx, -1)
    Po = (HT.v_frame(F).reshape(Nv, -1) @ F["root"].T)
    assert normwise(X[:, : Fr.r].cpu().numpy(), Xo) < 1e-13
    assert normwise(P[:, : Fr.r].cpu().numpy(), Po) < 1e-13


@pytest.mark.parametrize("shape", [(64,), (48,), (32, 32), (24, 40), (128, 128)])
def test_poisson_matches_oracle(shape):
    dx = len(shape)
    L_ = [4 * math.pi, 3.0][:dx]
    p = SI.Problem("t", dx, dx, tuple(shape) * 2, tuple([0.0] * dx + [-6.0] * dx),
                   tuple(L_ + [6.0] * dx), "landau", 0.1, 0.5)
    g = L.make_grid(p)
    ws = L.Workspace(g, 8)
    ne = 1.0 + 0.3 * SI.random_field(shape, 11, smooth=False)
    phi_o, E_o = SP.poisson(ne, 1.0, L_)
    phi = torch.zeros(int(np.prod(shape)), dtype=torch.float64, device="cuda")
    E = torch.zeros((dx, int(np.prod(shape))), dtype=torch.float64, device="cuda")
    L.slar_poisson(g, dev(ne.ravel()), 1.0, phi, E, ws)
    torch.cuda.synchronize()
    assert normwise(phi.cpu().numpy(), phi_o.ravel()) < 1e-12
    assert normwise(E.cpu().numpy(), E_o.reshape(dx, -1)) < 1e-12


@pytest.mark.parametrize("name,N", [("landau1d", 32), ("landau2d", 12)])
def test_moments_match_oracle(name, N):
    p = SI.config(name, n=N)
    d = p.d
    F = SI.random_ht(d, p.n, (5, 6) if d == 2 else (3, 4, 5, 3, 6, 5), seed=8)
    o = ST.Oracle(p)
    Mo = o.moments(F)
    g = L.make_grid(p)
    ws = L.Workspace(g, 16)
    T = ht_to_dev(F)
    H = L.make_ht(T, d, L.F64)
    Nx = int(np.prod(p.n[: p.dx])); Nv = int(np.prod(p.n[p.dx:]))
    X = torch.zeros((Nx, 8), dtype=torch.float64, device="cuda")
    P = torch.zeros((Nv, 8), dtype=torch.float64, device="cuda")
    Fr = L.slar_frames_from_ht(g, H, L.frames(X, P, 0), ws)
    M = torch.zeros((Mo.shape[0], Nx), dtype=torch.float64, device="cuda")
    L.slar_moments(g, Fr, M, ws)
    torch.cuda.synchronize()
    Mg = M.cpu().numpy()
    for q in range(Mo.shape[0]):
        assert normwise(Mg[q], Mo[q].ravel()) < 1e-12, q


def _lowrank_input(nx, nv, k, seed, decay=0.5):
    """Exactly rank-k factors with geometrically decaying weights."""
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((k, nx)) * (decay ** np.arange(k))[:, None]
    V = rng.standard_normal((k, nv))
    return U, V


@pytest.mark.parametrize("name,N,k,tol", [("landau1d", 64, 12, 1e-6), ("landau2d", 10, 20, 1e-6),
                                          ("landau2d", 16, 30, 1e-5), ("landau2d", 24, 9, 1e-8)])
def test_truncate_matches_oracle(name, N, k, tol):
    """slar_truncate vs the oracle's QR + SVD truncation on the same factors:
    same ranks; reconstructed tensors agree to 1e-12 (the refined leaf bases
    are as accurate as SVDs of the unfoldings; the unrefined Gram
    eigenvectors alone would carry eps sigma_1^2 / theta)."""
    from oracle import cross as CR
    p = SI.config(name, n=N)
    nx = tuple(p.n[: p.dx]); nv = tuple(p.n[p.dx:])
    Nx = int(np.prod(nx)); Nv = int(np.prod(nv))
    U, V = _lowrank_input(Nx, Nv, k, seed=N + k)
    Fo = CR.truncate_lowrank(U.T, V.T, nx, nv, tol, 40)
    g = L.make_grid(p)
    ws = L.Workspace(g, 40)
    Ud = dev(U); Vd = dev(V)
    lr = L.LowRank(k, Ud.data_ptr(), Vd.data_ptr())
    from paper_2606_29027_amd.solver import Solver
    s = Solver(p.with_(rmax=40), L.F64)
    H, T = s.ht_buf[0]
    L.slar_truncate(g, lr, tol, 40, H, ws)
    torch.cuda.synchronize()
    Fg = ht_from_dev(H, T, p.d, p.n)
    assert tuple(H.rank[: (2 if p.d == 2 else 6)]) == HT.ranks(Fo)
    err = normwise(HT.full(Fg), HT.full(Fo))
    assert err < 1e-12, err
    # column 0 of every leaf is the leading left singular vector of its mode
    for m in range(p.d):
        assert abs(abs(Fg["leaves"][m][:, 0] @ Fo["leaves"][m][:, 0]) - 1) < 1e-10
