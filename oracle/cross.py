"""Cross approximation and HT truncation (oracle).

The paper builds the updated HT tensor by HTACA, which samples selected
entries (typically fibers) through the SL-FD evaluator and finishes with an
HOSVD-type truncation on the dimension tree (introduction, section 3.1 and
Supplement B, section "Discrete velocity weight"); the sampling algorithm
itself is deferred to the authors' earlier work.  The reading implemented
here:

ACA with partial pivoting on the {x}|{v} matricisation A (rows: spatial
multi-index, columns: velocity multi-index, both row-major):
  1. start at row pivot i = first_row;
  2. residual row a = A[i,:] - sum_l u_l[i] v_l; column pivot
     j = lowest index with |a_j| >= (1 - 1e-10) max|a| (near-ties resolved
     to the lowest index so that round-off cannot flip the choice);
  3. if max|a| <= tol ||S_k||_F / sqrt(nrows ncols) (the probe threshold
     below), row i is already reproduced and the error estimate is zero: go
     to the probe check of step 7;
  4. v = a / a_j; u = A[:,j] - sum_l v_l[j] u_l; keep (u, v);
  5. ||S_k||_F^2 += 2 sum_{l<k} (u_l.u)(v_l.v) + |u|^2 |v|^2; stop when
     |u||v| <= tol ||S_k||_F or k = kmax;
  6. otherwise next row pivot = unused row maximising |u| (same tie rule);
  7. on stopping, check the given random probe entries: if some residual
     exceeds tol ||S_k||_F / sqrt(nrows ncols), continue from the row of the
     largest such residual.

Term cap: the cross may take up to kmax terms (min(2 rmax, 128) in the
workloads).  If it stops at that cap before meeting its tolerance, the
skeleton C W^-1 R (pivot columns C, pivot rows R, pivot block W) is
replaced by C W_r^+ R, the pseudo-inverse of W truncated at the HT rank cap
r = rmax (``cur_core``); a skeleton cut off by the cap has no error control,
and its interpolation through W^-1 let the error grow from step to step on
the strong-Landau workload, where the truncated core did not.

Truncation (recompression + HT): QR of both factor sets, SVD of the small
core, root rank = smallest r with tail sqrt(sum_{i>=r} s_i^2) <= theta,
theta = tol ||F||_F / sqrt(2d-3) (one share of the error budget per tree
edge), capped at rmax.  For the 4-leaf tree each leaf basis is the leading
left singular subspace of the mode matricisation of (frame * diag(s)),
truncated with the same theta, and the transfer tensor is the projection of
the frame onto the leaf bases.  Column 0 of every leaf is therefore the
leading left singular vector of that mode (Supplement B).  Singular vectors
are sign-fixed: the entry of largest magnitude (lowest index on ties) is
positive.
"""
from __future__ import annotations

import math

import numpy as np

TIE_REL = 1e-10


def argmax_tie(a: np.ndarray, mask=None) -> int:
    m = np.abs(a)
    if mask is not None:
        m = np.where(mask, m, -1.0)
    top = m.max()
    return int(np.flatnonzero(m >= top * (1.0 - TIE_REL))[0]) if top > 0 else int(np.argmax(m))


def aca(row_fn, col_fn, pts_fn, nrows: int, ncols: int, tol: float, kmax: int,
        first_row: int = 0, probes=None):
    """Returns (U (nrows, k), V (ncols, k), info)."""
    Us, Vs = [], []
    used = np.zeros(nrows, dtype=bool)
    norm2 = 0.0
    i = first_row
    info = {"samples": 0, "pivots": [], "probe_rounds": 0, "converged": False}
    while len(Us) < kmax:
        a = np.array(row_fn(i), dtype=np.float64)
        info["samples"] += ncols
        for u, v in zip(Us, Vs):
            a = a - u[i] * v
        used[i] = True
        j = argmax_tie(a)
        amax = abs(a[j])
        # a residual row below the probe threshold is already reproduced:
        # the error estimate is zero, so finish (subject to the probes)
        thr = tol * math.sqrt(norm2) / math.sqrt(nrows * ncols)
        if amax == 0.0 or amax <= thr:
            if _probe_continue(Us, Vs, pts_fn, probes, tol, norm2, nrows, ncols, used, info):
                i = info["next_row"]
                continue
            info["converged"] = True
            break
        v = a / a[j]
        b = np.array(col_fn(j), dtype=np.float64)
        info["samples"] += nrows
        for u_, v_ in zip(Us, Vs):
            b = b - v_[j] * u_
        u = b
        cross = 0.0
        for u_, v_ in zip(Us, Vs):
            cross += float(u_ @ u) * float(v_ @ v)
        norm2 = norm2 + 2.0 * cross + float(u @ u) * float(v @ v)
        Us.append(u)
        Vs.append(v)
        info["pivots"].append((i, j))
        if math.sqrt(float(u @ u) * float(v @ v)) <= tol * math.sqrt(max(norm2, 0.0)):
            if _probe_continue(Us, Vs, pts_fn, probes, tol, norm2, nrows, ncols, used, info):
                i = info["next_row"]
                continue
            info["converged"] = True
            break
        if used.all():
            break
        i = argmax_tie(u, ~used)
    if not Us:                       # identically zero tensor
        Us.append(np.zeros(nrows)); Vs.append(np.eye(ncols, 1)[:, 0])
    U = np.stack(Us, axis=1)
    V = np.stack(Vs, axis=1)
    info["rank"] = U.shape[1]
    return U, V, info


def cur_core(U: np.ndarray, V: np.ndarray, pivots, rmax: int):
    """Regularised skeleton of a cross that stopped at its term cap.

    The cross U V^T interpolates its pivot rows I and columns J, so with the
    sampled fibers C = A[:, J], R = A[I, :] and W = A[I, J] it equals
    C W^-1 R.  When the cap was hit before the tolerance, W^-1 is replaced
    by the pseudo-inverse of W truncated to its leading min(rmax, rank W)
    singular triplets: A ~ C W_r^+ R, returned as factors (U', V') with
    U' = C Z_r diag(1/s_r) and V' = R^T Y_r for W = Y diag(s) Z^T."""
    I = np.array([p[0] for p in pivots], dtype=np.int64)
    J = np.array([p[1] for p in pivots], dtype=np.int64)
    C = U @ V[J].T               # A[:, J]: the cross reproduces its pivot columns
    R = (U[I] @ V.T)             # A[I, :]
    W = U[I] @ V[J].T            # A[I, J]
    Y, s, Zt = np.linalg.svd(W)
    r = int(min(rmax, np.count_nonzero(s > 1e-14 * s[0]))) if s[0] > 0 else 1
    r = max(r, 1)
    Uc = C @ (Zt[:r].T / s[:r][None, :])
    Vc = R.T @ Y[:, :r]
    return Uc, Vc


def _probe_continue(Us, Vs, pts_fn, probes, tol, norm2, nrows, ncols, used, info) -> bool:
    if probes is None or len(probes) == 0 or not Us:
        return False
    I = probes[:, 0].astype(np.int64)
    J = probes[:, 1].astype(np.int64)
    vals = np.array(pts_fn(I, J), dtype=np.float64)
    info["samples"] += len(I)
    for u, v in zip(Us, Vs):
        vals = vals - u[I] * v[J]
    thr = tol * math.sqrt(max(norm2, 0.0)) / math.sqrt(nrows * ncols)
    bad = np.abs(vals) > thr
    bad &= ~used[I]
    if not bad.any():
        return False
    info["probe_rounds"] += 1
    info["next_row"] = int(I[argmax_tie(vals, bad)])
    return True


def sign_fix(Q: np.ndarray) -> np.ndarray:
    """Flip columns so their largest-|entry| (lowest index on ties) is > 0."""
    Q = Q.copy()
    for c in range(Q.shape[1]):
        p = argmax_tie(Q[:, c])
        if Q[p, c] < 0:
            Q[:, c] = -Q[:, c]
    return Q


def tail_rank(s: np.ndarray, theta: float, rmax: int) -> int:
    """Smallest r >= 1 with sqrt(sum_{i >= r} s_i^2) <= theta, capped at rmax."""
    tails = np.sqrt(np.cumsum((s ** 2)[::-1])[::-1])  # tails[r] = ||s[r:]||
    r = len(s)
    for cand in range(len(s)):
        if tails[cand] <= theta:
            r = cand
            break
    return int(max(1, min(r, rmax)))


def recompress(U: np.ndarray, V: np.ndarray, tol: float, rmax: int, d: int):
    """U V^T -> X diag(s) Y^T with orthonormal X, Y (sign-fixed on X)."""
    Qu, Ru = np.linalg.qr(U)
    Qv, Rv = np.linalg.qr(V)
    W, s, Zt = np.linalg.svd(Ru @ Rv.T)
    normF = float(np.sqrt(np.sum(s ** 2)))
    theta = tol * normF / math.sqrt(max(2 * d - 3, 1))
    r = tail_rank(s, theta, rmax)
    X = Qu @ W[:, :r]
    Y = Qv @ Zt.T[:, :r]
    for c in range(r):
        p = argmax_tie(X[:, c])
        if X[p, c] < 0:
            X[:, c] = -X[:, c]
            Y[:, c] = -Y[:, c]
    return X, s[:r].copy(), Y, theta, normF


def leaf_basis(A: np.ndarray, theta: float, rmax: int) -> np.ndarray:
    """Leading left singular subspace of A (rows = the leaf's grid)."""
    Uu, s, _ = np.linalg.svd(A, full_matrices=False)
    r = tail_rank(s, theta, rmax)
    return sign_fix(Uu[:, :r])


def to_ht(X, s, Y, nx, nv, theta: float, rmax: int) -> dict:
    """Frames (rows x-grid / v-grid, orthonormal) + root singular values -> HT."""
    r = len(s)
    if len(nx) == 1:
        return {"leaves": [X, Y], "root": np.diag(s)}
    out = {"root": np.diag(s)}
    leaves = []
    for frame, (na, nb), key in ((X, nx, "B12"), (Y, nv, "B34")):
        Fr = frame.reshape(na, nb, r)
        Fs = Fr * s[None, None, :]
        Ua = leaf_basis(Fs.reshape(na, nb * r), theta, rmax)
        Ub = leaf_basis(np.transpose(Fs, (1, 0, 2)).reshape(nb, na * r), theta, rmax)
        out[key] = np.einsum("ia,jb,ijc->abc", Ua, Ub, Fr)
        leaves += [Ua, Ub]
    out["leaves"] = leaves
    return out


def truncate_lowrank(U, V, nx, nv, tol: float, rmax: int) -> dict:
    d = len(nx) + len(nv)
    X, s, Y, theta, _ = recompress(U, V, tol, rmax, d)
    return to_ht(X, s, Y, nx, nv, theta, rmax)


def truncate_dense(Fm: np.ndarray, nx, nv, tol: float, rmax: int) -> dict:
    """HSVD of a dense matricisation (pin for the factored path)."""
    Uu, s, Vt = np.linalg.svd(Fm, full_matrices=False)
    d = len(nx) + len(nv)
    theta = tol * float(np.sqrt(np.sum(s ** 2))) / math.sqrt(max(2 * d - 3, 1))
    r = tail_rank(s, theta, rmax)
    X = Uu[:, :r].copy(); Y = Vt[:r].T.copy()
    for c in range(r):
        p = argmax_tie(X[:, c])
        if X[p, c] < 0:
            X[:, c] = -X[:, c]; Y[:, c] = -Y[:, c]
    return to_ht(X, s[:r].copy(), Y, nx, nv, theta, rmax)
