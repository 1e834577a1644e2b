"""Uniform cell-centred grids and local Lagrange stencils (oracle).

Section 3.1: the domain in each coordinate is cut into N uniform cells
I_i = [x_{i-1/2}, x_{i+1/2}] with centres x_i and spacing h; phase space is
periodic in every coordinate (section 2.1), so stencil indices wrap mod N.

Cell location of a characteristic foot (the paper only says the foot "lies in
the cell I_j"; faces are shared by two cells): half-open cells
[x_{j-1/2}, x_{j+1/2}), i.e. j = floor((x* - lo)/h) and
xi = (x* - x_j)/h in [-1/2, 1/2).

Stencil: width 3 is the quadratic rule of eq. (1d_quadratic_interp_weight)
on {j-1, j, j+1}; width 5 is the natural extension the paper mentions
(degree 4 on {j-2..j+2}), with Lagrange weights
l_m(xi) = prod_{n != m} (xi - n)/(m - n).
"""
from __future__ import annotations

import numpy as np


def spacing(lo: float, hi: float, n: int) -> float:
    return (hi - lo) / n


def centres(lo: float, hi: float, n: int) -> np.ndarray:
    """x_i = lo + (i + 1/2) h, i = 0..n-1 (0-based form of x_i = a + (i-1/2)h)."""
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * spacing(lo, hi, n)


def locate(xstar, lo: float, h: float):
    """Cell index (unwrapped) and normalised coordinate of a foot."""
    s = (np.asarray(xstar, dtype=np.float64) - lo) / h
    j = np.floor(s)
    xi = s - j - 0.5
    return j.astype(np.int64), xi


def lagrange_weights(xi, width: int) -> np.ndarray:
    """Lagrange weights on the integer nodes -(width//2)..(width//2).

    Returns an array of shape xi.shape + (width,).  For width 3 this is
    (xi(xi-1)/2, 1-xi^2, xi(xi+1)/2), eq. (1d_quadratic_interp_weight).
    """
    xi = np.asarray(xi, dtype=np.float64)
    half = width // 2
    nodes = list(range(-half, half + 1))
    out = np.empty(xi.shape + (width,))
    for a, m in enumerate(nodes):
        w = np.ones_like(xi)
        for nn in nodes:
            if nn != m:
                w = w * (xi - nn) / (m - nn)
        out[..., a] = w
    return out


def quadratic_weights(xi) -> np.ndarray:
    """Eq. (1d_quadratic_interp_weight) written exactly as printed."""
    xi = np.asarray(xi, dtype=np.float64)
    return np.stack([0.5 * xi * (xi - 1.0), 1.0 - xi * xi, 0.5 * xi * (xi + 1.0)], axis=-1)


def stencil_rows(j, width: int, n: int) -> np.ndarray:
    """Wrapped stencil indices j-(w//2) .. j+(w//2) (mod n), shape j.shape+(w,)."""
    half = width // 2
    off = np.arange(-half, half + 1)
    return np.mod(np.asarray(j)[..., None] + off, n)


def interp_periodic(field: np.ndarray, lo, h, pts: np.ndarray, width: int = 5) -> np.ndarray:
    """Tensor-product Lagrange interpolation of a periodic grid field.

    ``field`` has shape (N_1..N_D); ``pts`` has shape (S, D).  Used for the
    frozen electric field at off-grid positions while tracing characteristics
    (the paper does not say how E is evaluated off the grid; degree-4 Lagrange
    keeps the tracing error below the interpolation error of f).
    """
    D = field.ndim
    S = pts.shape[0]
    idx = []
    wts = []
    for m in range(D):
        j, xi = locate(pts[:, m], lo[m], h[m])
        idx.append(stencil_rows(j, width, field.shape[m]))
        wts.append(lagrange_weights(xi, width))
    out = np.zeros(S)
    # plain sum over the width^D block
    for flat in range(width ** D):
        offs = np.unravel_index(flat, (width,) * D)
        w = np.ones(S)
        ind = []
        for m in range(D):
            w = w * wts[m][:, offs[m]]
            ind.append(idx[m][:, offs[m]])
        out += w * field[tuple(ind)]
    return out
