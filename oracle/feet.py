"""Feet of the characteristics (oracle).

The SL-FD update sets f(x_i, t^{n+1}) = f(x*, t^n) with x* the foot of the
characteristic through the grid point (section 3.1, eq.
(SL_basic_formulation)).  For Vlasov--Poisson with q_e = -1, m_e = 1
(section 2.1) the characteristics of a linear sub-flow with frozen field E
and velocity multiplier c are  dx/dt = c v,  dv/dt = -E(x).

Three kinds of sub-flow are used:
  kind 0 (x-shift, split):   x* = x - c v tau,  v* = v            (exact)
  kind 1 (v-shift, split):   x* = x,            v* = v + E(x) tau (exact, E on the grid)
  kind 2 (frozen-field flow of the third-order exponential integrator):
        integrate backwards in time with one classical RK4 step of size tau
        (the paper asks for "a high-order RK integrator"), E evaluated off the
        grid by periodic degree-4 tensor-product Lagrange interpolation.

A sample is described by its grid multi-index; the output is the foot in
physical coordinates, shape (S, d).  For the split kinds the coordinates that
do not move keep their exact grid index (weight exactly 1 at the centre).
"""
from __future__ import annotations

import numpy as np

from . import grid as G


def grid_points(idx: np.ndarray, lo, hi, n) -> np.ndarray:
    idx = np.asarray(idx)
    d = idx.shape[1]
    out = np.empty(idx.shape, dtype=np.float64)
    for m in range(d):
        out[:, m] = G.centres(lo[m], hi[m], n[m])[idx[:, m]]
    return out


def frozen_field(E_list, coefs):
    """E_eff = sum_i c_i E_i on the grid (the combined field of a CF3 stage)."""
    out = None
    for c, E in zip(coefs, E_list):
        term = c * np.asarray(E, dtype=np.float64)
        out = term if out is None else out + term
    return out


def feet(idx, lo, hi, n, dx: int, kind: int, tau: float, cv: float, E=None):
    """Physical foot coordinates for the grid points ``idx`` (S, d).

    ``E`` has shape (dx, N_x1..N_xdx) (the frozen field, already combined).
    """
    idx = np.asarray(idx)
    P = grid_points(idx, lo, hi, n)
    d = P.shape[1]
    dv = d - dx
    X = P[:, :dx].copy()
    V = P[:, dx:].copy()
    hx = [G.spacing(lo[m], hi[m], n[m]) for m in range(dx)]
    if kind == 0:
        return np.concatenate([X - cv * tau * V, V], axis=1)
    if kind == 1:
        Eg = np.stack([E[m][tuple(idx[:, q] for q in range(dx))] for m in range(dv)], axis=1)
        return np.concatenate([X, V + tau * Eg], axis=1)
    if kind != 2:
        raise ValueError("kind")

    def Eat(Xp):
        return np.stack([G.interp_periodic(E[m], lo[:dx], hx, Xp, 5) for m in range(dv)], axis=1)

    # backward characteristic: d/ds (X, V) = (-c V, +E(X)), s in [0, tau]
    k1x, k1v = -cv * V, Eat(X)
    k2x, k2v = -cv * (V + 0.5 * tau * k1v), Eat(X + 0.5 * tau * k1x)
    k3x, k3v = -cv * (V + 0.5 * tau * k2v), Eat(X + 0.5 * tau * k2x)
    k4x, k4v = -cv * (V + tau * k3v), Eat(X + tau * k3x)
    Xs = X + (tau / 6.0) * (k1x + 2.0 * k2x + 2.0 * k3x + k4x)
    Vs = V + (tau / 6.0) * (k1v + 2.0 * k2v + 2.0 * k3v + k4v)
    return np.concatenate([Xs, Vs], axis=1)


def stencils(foot: np.ndarray, idx, lo, hi, n, width: int, kind: int, dx: int):
    """Per-dimension wrapped stencil rows and weights for each foot.

    Returns (rows, wts): lists over dimensions of arrays (S, width).  For the
    split kinds the dimensions that do not move use the exact grid index
    with weight e_centre.
    """
    d = foot.shape[1]
    rows, wts = [], []
    for m in range(d):
        h = G.spacing(lo[m], hi[m], n[m])
        moving = (kind == 2) or (kind == 0 and m < dx) or (kind == 1 and m >= dx)
        if moving:
            j, xi = G.locate(foot[:, m], lo[m], h)
            w = G.quadratic_weights(xi) if width == 3 else G.lagrange_weights(xi, width)
        else:
            j = np.asarray(idx)[:, m].astype(np.int64)
            w = np.zeros((foot.shape[0], width))
            w[:, width // 2] = 1.0
        rows.append(G.stencil_rows(j, width, n[m]))
        wts.append(w)
    return rows, wts


def face_ambiguous(foot: np.ndarray, lo, hi, n, kind: int, dx: int, rel: float = 1e-9):
    """Mask of samples whose foot sits on a cell face to within ``rel`` cells
    in some moving dimension: there both neighbouring stencils are valid
    readings of "the cell containing x*"."""
    d = foot.shape[1]
    amb = np.zeros(foot.shape[0], dtype=bool)
    for m in range(d):
        moving = (kind == 2) or (kind == 0 and m < dx) or (kind == 1 and m >= dx)
        if not moving:
            continue
        h = G.spacing(lo[m], hi[m], n[m])
        s = (foot[:, m] - lo[m]) / h
        amb |= np.abs(s - np.round(s)) < rel * np.maximum(1.0, np.abs(s))
    return amb
