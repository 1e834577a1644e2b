"""Hierarchical Tucker tensors and the HT-SL entry evaluation (oracle).

Section 3.1: with leaf bases U^(mu) (N_mu x r_mu) and transfer tensors, the
tensor-product interpolation <F_J, W> of eq. (tp_interp) is evaluated by
  c^(mu) = w(xi_mu) U^(mu)_{J_mu}      (1 x r_mu, per leaf)
followed by contraction with the transfer tensors up to the root, O(d r^3)
per point.  Two trees are used (section 4, 2D2V rank labels r1..r4, r12,
r34): the 2-leaf tree {x}{v} (a matrix, 1D1V) and {{x1,x2},{v1,v2}}.

A tensor here is a dict (input layout documented in ``slar_inputs``) plus an
optional exact additive correction ``corr = {"C": (K, Nx...), "Q": (K, Nv...)}``
meaning F + sum_k C_k (x) Q_k; this is how the LoMaC-corrected state of
eq. (LoMaC_update_discrete) is held without re-truncation.
"""
from __future__ import annotations

import itertools

import numpy as np


def ndim(F) -> int:
    return len(F["leaves"])


def x_frame(F) -> np.ndarray:
    """Node frame of the x subtree, shape (N_x..., r_x-root)."""
    L = F["leaves"]
    if len(L) == 2:
        return L[0]
    return np.einsum("ia,jb,abc->ijc", L[0], L[1], F["B12"])


def v_frame(F) -> np.ndarray:
    L = F["leaves"]
    if len(L) == 2:
        return L[1]
    return np.einsum("kp,lq,pqe->kle", L[2], L[3], F["B34"])


def full(F) -> np.ndarray:
    """Dense reconstruction (small grids only)."""
    X = x_frame(F)
    V = v_frame(F)
    out = np.tensordot(np.tensordot(X, F["root"], axes=([X.ndim - 1], [0])), V,
                       axes=([X.ndim - 1], [V.ndim - 1]))
    if F.get("corr") is not None:
        C, Q = F["corr"]["C"], F["corr"]["Q"]
        out = out + np.tensordot(C, Q, axes=([0], [0]))
    return out


def block_interp(T: np.ndarray, rows, wts) -> np.ndarray:
    """sum over the stencil block of T[k, rows] * prod weights -> (S, K).

    T has shape (K, N_1..N_D); rows/wts are lists over D of (S, width).
    This is eq. (tp_interp) applied to a dense (small-dimensional) tensor.
    """
    D = len(rows)
    S, w = rows[0].shape
    out = np.zeros((S, T.shape[0]))
    for offs in itertools.product(range(w), repeat=D):
        wt = np.ones(S)
        ind = []
        for m in range(D):
            wt = wt * wts[m][:, offs[m]]
            ind.append(rows[m][:, offs[m]])
        vals = T[(slice(None),) + tuple(ind)]          # (K, S)
        out += wt[:, None] * vals.T
    return out


def sample(F, rows, wts, chunk: int = 4096) -> np.ndarray:
    """HT-SL value at each foot given per-dimension stencil rows and weights.

    Follows section 3.1 literally: leaf interpolation, then transfer
    contractions up to the root.
    """
    L = F["leaves"]
    S = rows[0].shape[0]
    out = np.empty(S)
    for s0 in range(0, S, chunk):
        sl = slice(s0, min(S, s0 + chunk))
        c = [np.einsum("sw,swr->sr", wts[m][sl], L[m][rows[m][sl]]) for m in range(len(L))]
        if len(L) == 2:
            out[sl] = np.einsum("sa,ab,sb->s", c[0], F["root"], c[1])
        else:
            t12 = np.einsum("sa,abc->sbc", c[0], F["B12"])
            y12 = np.einsum("sb,sbc->sc", c[1], t12)
            t34 = np.einsum("sp,pqe->sqe", c[2], F["B34"])
            y34 = np.einsum("sq,sqe->se", c[3], t34)
            out[sl] = np.einsum("sc,ce,se->s", y12, F["root"], y34)
    if F.get("corr") is not None:
        d = len(L)
        dx = d // 2
        cx = block_interp(F["corr"]["C"], rows[:dx], wts[:dx])
        cq = block_interp(F["corr"]["Q"], rows[dx:], wts[dx:])
        out = out + np.sum(cx * cq, axis=1)
    return out


def sample_frames(X: np.ndarray, P: np.ndarray, rows, wts) -> np.ndarray:
    """The same SL-FD value from the frame form F[I, J] = sum_c X[I, c] P[J, c]
    (X of shape (N_x1.., r), P of shape (N_v1.., r); the root folded into P):
    eq. (tp_interp) applied to each frame separately, then the length-r dot
    product.  This is what the cross approximation samples."""
    dx = X.ndim - 1
    cx = block_interp(np.moveaxis(X, -1, 0), rows[:dx], wts[:dx])
    cp = block_interp(np.moveaxis(P, -1, 0), rows[dx:], wts[dx:])
    return np.sum(cx * cp, axis=1)


# ---------------------------------------------------------------- moments

def psi_list(vgrids):
    """Velocity test functions in the fixed output order
    [1, v_1..v_dv, |v|^2, v_mu v_nu (mu <= nu), |v|^2 v_mu]
    (raw moments, eq. (raw moments), then the flux moments of
    eq. (macro_sys_comp)).  Returns dense arrays on the velocity grid."""
    dv = len(vgrids)
    Vs = np.meshgrid(*vgrids, indexing="ij")
    v2 = sum(V * V for V in Vs)
    out = [np.ones_like(Vs[0])]
    out += [Vs[m] for m in range(dv)]
    out.append(v2)
    for a in range(dv):
        for b in range(a, dv):
            out.append(Vs[a] * Vs[b])
    out += [v2 * Vs[m] for m in range(dv)]
    return out


def moments(F, vgrids, dvol: float) -> np.ndarray:
    """M_psi(x) = sum_k F(x, v_k) psi(v_k) w^v_k for every psi of psi_list,
    eqs. (disc_m0)-(disc_m2) and the flux moments; shape (npsi, N_x...)."""
    X = x_frame(F)
    V = v_frame(F)
    psis = psi_list(vgrids)
    dxn = X.ndim - 1
    res = []
    for psi in psis:
        m = np.tensordot(psi, V, axes=(list(range(psi.ndim)), list(range(psi.ndim)))) * dvol
        M = np.tensordot(X, F["root"] @ m, axes=([dxn], [0]))
        if F.get("corr") is not None:
            C, Q = F["corr"]["C"], F["corr"]["Q"]
            q = np.tensordot(Q, psi, axes=(list(range(1, Q.ndim)), list(range(psi.ndim)))) * dvol
            M = M + np.tensordot(q, C, axes=([0], [0]))
        res.append(M)
    return np.stack(res)


def dense_moments(Ffull: np.ndarray, dx: int, vgrids, dvol: float) -> np.ndarray:
    """Same moments straight from a dense tensor (pin for ``moments``)."""
    psis = psi_list(vgrids)
    ax = tuple(range(dx, Ffull.ndim))
    return np.stack([np.sum(Ffull * psi, axis=ax) * dvol for psi in psis])


def ranks(F):
    L = F["leaves"]
    if len(L) == 2:
        return (L[0].shape[1], L[1].shape[1])
    return tuple(U.shape[1] for U in L) + (F["B12"].shape[2], F["B34"].shape[2])
