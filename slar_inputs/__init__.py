"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only *draws* inputs: problem parameters, random hierarchical
Tucker (HT) factors, request multi-indices, the analytic initial data sampled
on the cell-centred grid, and the random probe indices the cross
approximation uses for its a-posteriori check.  It contains none of the
method's arithmetic (no interpolation, no characteristics, no contraction,
no projection).  Every generator is a pure function of its seed.

Layout conventions (shared by both sides because they are *input* formats):
  * phase-space dimension order is (x_1..x_dx, v_1..v_dv);
  * a grid is described by per-dimension (lo, hi, N); cell centres are
    lo + (i + 1/2) (hi - lo)/N, i = 0..N-1 (section 3.1, uniform cell-centred
    tensor grid; cell I_i with centre x_i);
  * a 2-leaf HT (1D1V) is {"leaves": [Ux, Uv], "root": B} with
    F[i, j] = sum_ab Ux[i, a] B[a, b] Uv[j, b];
  * a 4-leaf HT on the tree {{x1,x2},{v1,v2}} is
    {"leaves": [U1, U2, U3, U4], "B12": [r1, r2, r12], "B34": [r3, r4, r34],
     "root": [r12, r34]} with
    F = sum U1[i1,a] U2[i2,b] B12[a,b,c] root[c,e] U3[i3,p] U4[i4,q] B34[p,q,e].
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Problem", "config", "CONFIG_NAMES", "cell_centres", "initial_ht",
    "random_ht", "graded_ht", "random_requests", "fiber_requests", "probe_indices",
    "batched_instances", "random_field", "PAPER_WORKLOADS",
]


@dataclasses.dataclass(frozen=True)
class Problem:
    """One Vlasov--Poisson workload: grid, initial data and solver knobs."""
    name: str
    dx: int                      # spatial dimensions
    dv: int                      # velocity dimensions
    n: tuple                     # cells per dimension, len dx+dv
    lo: tuple
    hi: tuple
    kind: str                    # "landau" | "twostream"
    alpha: float
    k: float
    v0: float = 0.0
    tol: float = 1e-6            # baseline cross/truncation tolerance
    rmax: int = 40
    dt: float = 0.1
    T: float = 1.0
    order: int = 3               # interpolation stencil width (3 or 5)
    split: bool = False          # Strang splitting (1D1V workload)
    lomac: bool = True
    bdf: int = 2
    integrator: str = "bdf2"      # or "dirk3_bdf3" (the paper's section 4 choice)
    bump: tuple = ()              # bump-on-tail (n_p, n_b, u, v_t)
    kcross: int = 0               # cross-approximation term cap (0: min(2 rmax, 128))
    lomac_filter: bool = True     # band-limited LoMaC correction (mode filter)

    @property
    def d(self) -> int:
        return self.dx + self.dv

    @property
    def cross_cap(self) -> int:
        """Most terms one cross approximation may take before the truncation
        caps the rank at rmax."""
        return self.kcross if self.kcross > 0 else min(2 * self.rmax, 128)

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def config(name: str, n: Optional[int] = None) -> Problem:
    """The five benchmark workloads; ``n`` overrides the cells per dimension
    (used for small parity cases on the same physics)."""
    p4 = 4.0 * math.pi
    if name == "landau1d":        # 1D1V weak Landau, split, 5-point stencil
        N = n or 64
        return Problem(name, 1, 1, (N, N), (0.0, -6.0), (p4, 6.0), "landau",
                       0.01, 0.5, tol=1e-6, rmax=64, dt=0.1, T=5.0, order=5,
                       split=True, lomac=False)
    if name == "landau2d":        # 2D2V weak Landau + LoMaC
        N = n or 64
        return Problem(name, 2, 2, (N,) * 4, (0.0, 0.0, -6.0, -6.0),
                       (p4, p4, 6.0, 6.0), "landau", 0.01, 0.5, tol=1e-6,
                       rmax=40, dt=0.2, T=10.0)
    if name == "twostream2d":     # 2D2V two-stream, bimodal in v1 only
        N = n or 128
        L = 10.0 * math.pi
        return Problem(name, 2, 2, (N,) * 4, (0.0, 0.0, -8.0, -8.0),
                       (L, L, 8.0, 8.0), "twostream", 0.001, 0.2, v0=2.4,
                       tol=1e-5, rmax=60, dt=0.1, T=40.0)
    if name == "stronglandau2d":  # 2D2V strong Landau, learned preconditioner
        N = n or 128
        return Problem(name, 2, 2, (N,) * 4, (0.0, 0.0, -6.0, -6.0),
                       (p4, p4, 6.0, 6.0), "landau", 0.5, 0.5, tol=1e-5,
                       rmax=60, dt=0.2, T=30.0)
    # --- the paper's own section 4 setups (CFL 5 read as dt = 5 dx / v_max,
    # unsplit CF3 with 3-point stencils, LoMaC, DIRK-3 start-up + BDF-3)
    if name in ("landau1d_paper", "stronglandau1d"):
        N = n or 256
        weak = name == "landau1d_paper"
        return Problem(name, 1, 1, (N, N), (0.0, -2.0 * math.pi), (p4, 2.0 * math.pi), "landau",
                       0.01 if weak else 0.5, 0.5, tol=1e-5 if weak else 1e-4, rmax=64,
                       dt=5.0 * (p4 / N) / (2.0 * math.pi), T=40.0, order=3,
                       integrator="dirk3_bdf3")
    if name == "bumpontail1d":
        N = n or 256
        Lx = 20.0 * math.pi / 3.0
        s2p = math.sqrt(2.0 * math.pi)
        return Problem(name, 1, 1, (N, N), (0.0, -13.0), (Lx, 13.0), "bumpontail", 0.04, 0.3,
                       tol=1e-4, rmax=64, dt=5.0 * (Lx / N) / 13.0, T=40.0, order=3,
                       integrator="dirk3_bdf3", bump=(9.0 / (10.0 * s2p), 2.0 / (10.0 * s2p), 4.5, 0.5))
    if name == "bumpontail2d":
        N = n or 128
        Lx = 20.0 * math.pi / 3.0
        vt = 2.4
        return Problem(name, 2, 2, (N,) * 4, (0.0, 0.0, -13.0, -13.0), (Lx, Lx, 13.0, 13.0),
                       "bumpontail", 0.04, 0.3, tol=1e-4, rmax=60, dt=5.0 * (Lx / N) / 13.0,
                       T=30.0, integrator="dirk3_bdf3",
                       bump=(17.0 / (40.0 * math.pi), 3.0 / (40.0 * math.pi * vt), 4.5, vt))
    raise KeyError(name)


CONFIG_NAMES = ("landau1d", "landau2d", "twostream2d", "stronglandau2d")
# section 4 setups of the paper run on the same path
PAPER_WORKLOADS = ("landau1d_paper", "stronglandau1d", "bumpontail1d", "bumpontail2d")


def cell_centres(lo: float, hi: float, n: int) -> np.ndarray:
    h = (hi - lo) / n
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * h


def _maxwell(v: np.ndarray) -> np.ndarray:
    return np.exp(-0.5 * v * v) / math.sqrt(2.0 * math.pi)


def initial_ht(p: Problem) -> dict:
    """Exact low-rank HT of the analytic initial condition on the grid.

    Landau: f0 = (1 + alpha sum_mu cos(k x_mu)) prod_mu M(v_mu).
    Two-stream (bimodal in v1 only): the v1 factor is
    exp(-(v-v0)^2/2) + exp(-(v+v0)^2/2), normalised with 1/(4 pi) overall.
    Bump-on-tail (section 4): 1D1V (1 + alpha cos kx)(n_p e^{-v^2/2} +
    n_b e^{-(v-u)^2/(2 v_t)}); 2D2V (1 + alpha cos kx_1 cos kx_2) / (8 pi)
    (n_p e^{-|v|^2/2} + n_b e^{-((v_1-u)^2 + v_2^2)/(2 v_t)}).
    """
    xs = [cell_centres(p.lo[m], p.hi[m], p.n[m]) for m in range(p.d)]
    if p.dx == 1:
        x = xs[0]
        Ux = np.stack([np.ones_like(x), np.cos(p.k * x)], axis=1)
        if p.kind == "bumpontail":
            n_p, n_b, u, vt = p.bump
            v = xs[1]
            Uv = (n_p * np.exp(-0.5 * v * v) + n_b * np.exp(-0.5 * (v - u) ** 2 / vt))[:, None]
        else:
            Uv = _maxwell(xs[1])[:, None]
        B = np.array([[1.0], [p.alpha]])
        return {"leaves": [Ux, Uv], "root": B}
    U1 = np.stack([np.ones_like(xs[0]), np.cos(p.k * xs[0])], axis=1)
    U2 = np.stack([np.ones_like(xs[1]), np.cos(p.k * xs[1])], axis=1)
    B12 = np.zeros((2, 2, 1))
    B12[0, 0, 0] = 1.0
    if p.kind == "bumpontail":
        B12[1, 1, 0] = p.alpha                  # product of the two cosines
        n_p, n_b, u, vt = p.bump
        v1, v2 = xs[2], xs[3]
        U3 = np.stack([np.exp(-0.5 * v1 * v1), np.exp(-0.5 * (v1 - u) ** 2 / vt)], axis=1)
        U4 = np.stack([np.exp(-0.5 * v2 * v2), np.exp(-0.5 * v2 * v2 / vt)], axis=1)
        B34 = np.zeros((2, 2, 1))
        B34[0, 0, 0] = n_p / (8.0 * math.pi)
        B34[1, 1, 0] = n_b / (8.0 * math.pi)
        return {"leaves": [U1, U2, U3, U4], "B12": B12, "B34": B34, "root": np.ones((1, 1))}
    B12[1, 0, 0] = p.alpha
    B12[0, 1, 0] = p.alpha
    if p.kind == "landau":
        U3 = _maxwell(xs[2])[:, None]
        U4 = _maxwell(xs[3])[:, None]
    elif p.kind == "twostream":
        v1, v2 = xs[2], xs[3]
        U3 = (np.exp(-0.5 * (v1 - p.v0) ** 2) + np.exp(-0.5 * (v1 + p.v0) ** 2))[:, None]
        U4 = np.exp(-0.5 * v2 * v2)[:, None] / (4.0 * math.pi)
    else:
        raise KeyError(p.kind)
    B34 = np.ones((1, 1, 1))
    root = np.ones((1, 1))
    return {"leaves": [U1, U2, U3, U4], "B12": B12, "B34": B34, "root": root}


def random_ht(d: int, n: Sequence[int], ranks: Sequence[int], seed: int) -> dict:
    """Random HT with orthonormal leaves and Gaussian transfer tensors.

    ``ranks`` = (r_x, r_v) for d == 2 and (r1, r2, r3, r4, r12, r34) for d == 4.
    """
    rng = np.random.default_rng(seed)

    def leaf(N, r):
        q, _ = np.linalg.qr(rng.standard_normal((N, r)))
        return np.ascontiguousarray(q)

    if d == 2:
        rx, rv = ranks
        return {"leaves": [leaf(n[0], rx), leaf(n[1], rv)],
                "root": rng.standard_normal((rx, rv)) / math.sqrt(rx * rv)}
    r1, r2, r3, r4, r12, r34 = ranks
    return {
        "leaves": [leaf(n[0], r1), leaf(n[1], r2), leaf(n[2], r3), leaf(n[3], r4)],
        "B12": rng.standard_normal((r1, r2, r12)) / math.sqrt(r1 * r2),
        "B34": rng.standard_normal((r3, r4, r34)) / math.sqrt(r3 * r4),
        "root": rng.standard_normal((r12, r34)) / math.sqrt(r12 * r34),
    }


def graded_ht(n: Sequence[int], r_leaf: int, r_root: int, decay: float, seed: int) -> dict:
    """A 4-leaf HT in orthogonal form with geometrically decaying root
    singular values (root = diag(decay^c), c < r_root): leaves and the
    matricised transfer tensors [r1 r2][r12] have orthonormal columns, so the
    node frames are orthonormal and ||F||_F = ||root||_F.  A stand-in for a
    truncated solution state (a few dominant terms, a long small tail)."""
    rng = np.random.default_rng(seed)

    def orth(rows, cols):
        q, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
        return np.ascontiguousarray(q)

    r = r_leaf
    return {
        "leaves": [orth(n[m], r) for m in range(4)],
        "B12": orth(r * r, r_root).reshape(r, r, r_root),
        "B34": orth(r * r, r_root).reshape(r, r, r_root),
        "root": np.diag(decay ** np.arange(r_root)),
    }


def random_requests(n: Sequence[int], count: int, seed: int) -> np.ndarray:
    """Uniform random grid multi-indices, int32 [count][d]."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, N, size=count) for N in n], axis=1).astype(np.int32)


def fiber_requests(n: Sequence[int], dx: int, row: int, col: int) -> np.ndarray:
    """All multi-indices of one row fiber (x fixed at linear index ``row``,
    every v) followed by one column fiber (v fixed at ``col``, every x) of the
    {x}|{v} matricisation; row-major linearisation in each group."""
    nx = list(n[:dx]); nv = list(n[dx:])
    xi = np.array(np.unravel_index(row, nx)).reshape(1, dx)
    vj = np.array(np.unravel_index(col, nv)).reshape(1, len(nv))
    allv = np.stack(np.unravel_index(np.arange(int(np.prod(nv))), nv), axis=1)
    allx = np.stack(np.unravel_index(np.arange(int(np.prod(nx))), nx), axis=1)
    r = np.concatenate([np.repeat(xi, len(allv), 0), allv], axis=1)
    c = np.concatenate([allx, np.repeat(vj, len(allx), 0)], axis=1)
    return np.concatenate([r, c], 0).astype(np.int32)


def probe_indices(nrows: int, ncols: int, count: int, seed: int) -> np.ndarray:
    """Random (row, col) entries of the {x}|{v} matricisation used by the
    cross approximation's a-posteriori check: int32 [count][2]."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, nrows, size=count),
                     rng.integers(0, ncols, size=count)], axis=1).astype(np.int32)


def random_field(shape: Sequence[int], seed: int, smooth: bool = True) -> np.ndarray:
    """A seeded smooth periodic real field (a few random Fourier modes)."""
    rng = np.random.default_rng(seed)
    out = np.zeros(shape)
    grids = np.meshgrid(*[np.arange(s) / s for s in shape], indexing="ij")
    modes = 4 if smooth else 32
    for _ in range(modes):
        ks = [int(rng.integers(-3 if smooth else -s // 2, 4 if smooth else s // 2)) for s in shape]
        ph = rng.uniform(0, 2 * math.pi)
        arg = sum(2 * math.pi * k * g for k, g in zip(ks, grids))
        out += rng.standard_normal() * np.cos(arg + ph)
    return out


def batched_instances(count: int = 64, sizes: Sequence[int] = (32, 48, 64, 96, 128),
                      sizes_1d: Optional[Sequence[int]] = None) -> List[Problem]:
    """Independent Landau instances of uneven size (per-instance seed i):
    1D1V or 2D2V with probability 1/2, N per dimension from
    {32, 48, 64, 96, 128}, alpha ~ U[0.005, 0.5], k ~ U[0.3, 0.6],
    x in [0, 2 pi / k) so the perturbation is periodic, v in [-6, 6].
    ``sizes`` / ``sizes_1d`` replace the size menu of the 2D2V / 1D1V
    instances (small test cases) without changing the other draws."""
    s2 = list(sizes)
    s1 = list(sizes if sizes_1d is None else sizes_1d)
    out = []
    for i in range(count):
        rng = np.random.default_rng(i)
        two = bool(rng.integers(0, 2))
        dims = 4 if two else 2
        menu = s2 if two else s1
        ns = tuple(int(menu[rng.integers(0, len(menu))]) for _ in range(dims))
        alpha = float(rng.uniform(0.005, 0.5))
        k = float(rng.uniform(0.3, 0.6))
        L = 2.0 * math.pi / k
        if two:
            out.append(Problem(f"inst{i}", 2, 2, ns, (0.0, 0.0, -6.0, -6.0),
                               (L, L, 6.0, 6.0), "landau", alpha, k, tol=1e-6,
                               rmax=40, dt=0.1, T=2.0, lomac=False))
        else:
            out.append(Problem(f"inst{i}", 1, 1, ns, (0.0, -6.0), (L, 6.0),
                               "landau", alpha, k, tol=1e-6, rmax=40, dt=0.1,
                               T=2.0, lomac=False))
    return out
