"""Nested hierarchical-Tucker cross approximation (oracle, FP64 NumPy).

Test infrastructure only: imported by tests/, never by the product path.

Not a step of the paper's method.  The paper builds its HT tensors with
HTACA (cross approximation on the {x}|{v} matricisation, whose fibers have
N_x or N_v entries, then an HOSVD on the tree), and it names the rank
sensitivity of that sampler as the cost driver it wants to remove (section
4, 2D2V two-stream discussion; section 5).  This is the nested form of
cross approximation on a dimension tree after Ballani, Grasedyck and Kluge
(Linear Algebra Appl. 438, 2013): every index set is chosen inside products
of the sets of neighbouring tree nodes, so that only fibers of length N_mu
and small blocks of entries are ever sampled.

Tree {{1,2},{3,4}}, A of shape (n1, n2, n3, n4), row-major pair indices.

Index sets:
  leaf mu:   rows R_mu (subset of [n_mu]); complements Q_mu chosen inside
             (rows of the sibling leaf) x (complement of the parent node),
             both enlarged by the sweep's enrichment indices E;
  node x:    rows P_x inside (R_1 + E_1) x (R_2 + E_2), node v likewise;
             the complement of x is P_v and that of v is P_x.

Skeleton (interpolation) form built from those sets:
  leaves     W_mu = A^(mu)[:, Q_mu] A^(mu)[R_mu, Q_mu]^-1      (n_mu x r_mu)
  transfers  B12[a, b, d] = A[R_1[a], R_2[b], P_v[d]]
             B34[p, q, c] = A[P_x[c], R_3[p], R_4[q]]
  root       A[P_x, P_v]^-1   (rows indexed by P_v, columns by P_x)
so that A ~ X S^-1 V^T with X = (W_1 (x) W_2) B12, V = (W_3 (x) W_4) B34
and S = A[P_x, P_v].  X reproduces A[R_1 x R_2, P_v] exactly (W_mu is the
identity on R_mu) and interpolates between those rows; the root pivots may
lie off the leaf grid (Ballani-Grasedyck-Kluge nest them inside it), so a
component that vanishes on the grid can still enter through the probes.

Pivot search, one sweep: the enrichment E is `enrich` probes taken in
rotation plus the worst failing probe of the previous sweep.  For each leaf
in the order 1, 2, 3, 4, the candidate matrix
A^(mu)[:, (sibling rows + E) x (parent complement + E)] (the rows a sibling
chose in this sweep, once chosen) is searched by the ACA of
``oracle.cross.aca`` (partial pivoting, tie rule, stopping test, and its
probe restart with the entries of E inside the matrix as probes) for R_mu
and Q_mu; then the root matrix A[(R_1 + E_1) x (R_2 + E_2),
(R_3 + E_3) x (R_4 + E_4)] is searched the same way for P_x and P_v.  After
every sweep from the second on, the probes are checked against the
skeleton; the search stops when every probe error is at most
tol ||F||_F / sqrt(N_x N_v) (the ACA probe threshold, ||F||_F the norm of
the skeleton), else after `max_sweeps`.  Every leaf and root search runs
at tol / 10: a skeleton's error constant is larger than a truncated SVD's
and six node approximations compound, so searches at tol itself leave probe
errors up to twenty times the threshold on SL-FD updates of Landau data.

Samples (distinct entries): a leaf search samples r_mu rows and r_mu
columns of its candidate matrix, about r_mu (n_mu + (r_sib + e)(k + e)),
and the root search k ((r_1 + e)(r_2 + e) + (r_3 + e)(r_4 + e)); the
skeleton reuses them.  This grows like d N r^2 + r^3 against the
k (N_x + N_v) = k (N^2 + N^2) of cross approximation on the {x}|{v}
matricisation.

Parity pins (tests/test_oracle_pins.py): exact recovery of tensors of
exact HT rank, the interpolation property on every sampled transfer entry,
the sample count, and the error on smooth Vlasov data against the full
tensor.
"""
from __future__ import annotations

import math

import numpy as np

from .cross import aca


def _pairs(rows_a, rows_b):
    return [(a, b) for a in rows_a for b in rows_b]


def _leaf_candidates(mu, R, Px, Pv):
    """Complement multi-indices (3-tuples in the order of the other axes)."""
    if mu == 0:
        return [(i2, j1, j2) for i2 in R[1] for (j1, j2) in Pv]
    if mu == 1:
        return [(i1, j1, j2) for i1 in R[0] for (j1, j2) in Pv]
    if mu == 2:
        return [(i1, i2, j2) for (i1, i2) in Px for j2 in R[3]]
    return [(i1, i2, j1) for (i1, i2) in Px for j1 in R[2]]


def _leaf_index(mu, t, comp):
    """Full multi-index with value t on axis mu and the complement comp."""
    c = list(comp)
    c.insert(mu, t)
    return tuple(c)


class _Sampler:
    """Entry oracle with a cache: `count` is the number of distinct entries
    evaluated (a skeleton reuses the fibers and blocks its search sampled)."""

    def __init__(self, f):
        self.f = f
        self.cache = {}
        self.count = 0

    def __call__(self, idx):
        idx = np.asarray(idx, dtype=np.int64).reshape(-1, 4)
        keys = [tuple(int(v) for v in row) for row in idx]
        new = [i for i, k in enumerate(keys) if k not in self.cache]
        if new:
            vals = np.asarray(self.f(idx[new]), dtype=np.float64)
            for i, v in zip(new, vals):
                self.cache[keys[i]] = float(v)
            self.count += len(new)
        return np.array([self.cache[k] for k in keys], dtype=np.float64)


def _leaf_matrix(S, mu, n, cands):
    idx = [_leaf_index(mu, t, c) for c in cands for t in range(n[mu])]
    return S(idx).reshape(len(cands), n[mu]).T          # (n_mu, |cands|)


def _search(row_fn, col_fn, pts_fn, nrows, ncols, tol, kmax, first_row, probes):
    """ACA with partial pivoting on an implicit matrix (rows and columns are
    sampled only as the pivots need them), with the probe restart of
    ``oracle.cross.aca``: row and column pivots."""
    pr = np.asarray(probes, dtype=np.int64).reshape(-1, 2) if len(probes) else None
    _, _, info = aca(row_fn, col_fn, pts_fn, nrows, ncols, tol, kmax, first_row=first_row, probes=pr)
    rows = [p[0] for p in info["pivots"]]
    cols = [p[1] for p in info["pivots"]]
    return rows, cols


def _leaf_search(S, a, n, cands, tol, kmax, first_row, E):
    row = lambda i: S([_leaf_index(a, i, c) for c in cands])
    col = lambda j: S([_leaf_index(a, t, cands[j]) for t in range(n[a])])
    pts = lambda I, J: S([_leaf_index(a, int(i), cands[int(j)]) for i, j in zip(I, J)])
    where = {c: j for j, c in enumerate(cands)}
    probes = []
    for e in E:
        comp = tuple(e[b] for b in range(4) if b != a)
        if comp in where:
            probes.append((e[a], where[comp]))
    return _search(row, col, pts, n[a], len(cands), tol, kmax, first_row, probes)


def _root_search(S, rx, rv, tol, kmax, first_row, E):
    row = lambda i: S([(rx[i][0], rx[i][1], p, q) for (p, q) in rv])
    col = lambda j: S([(a, b, rv[j][0], rv[j][1]) for (a, b) in rx])
    pts = lambda I, J: S([(rx[int(i)][0], rx[int(i)][1], rv[int(j)][0], rv[int(j)][1]) for i, j in zip(I, J)])
    wx = {p: i for i, p in enumerate(rx)}
    wv = {p: j for j, p in enumerate(rv)}
    probes = [(wx[(e[0], e[1])], wv[(e[2], e[3])]) for e in E
              if (e[0], e[1]) in wx and (e[2], e[3]) in wv]
    return _search(row, col, pts, len(rx), len(rv), tol, kmax, first_row, probes)


def norm_ht(F) -> float:
    """Frobenius norm of the skeleton HT from its frames."""
    L = F["leaves"]
    X = np.einsum("ia,jb,abd->ijd", L[0], L[1], F["B12"]).reshape(-1, F["B12"].shape[2])
    V = np.einsum("kp,lq,pqc->klc", L[2], L[3], F["B34"]).reshape(-1, F["B34"].shape[2])
    G = (X.T @ X) @ F["root"] @ (V.T @ V) @ F["root"].T
    return math.sqrt(max(float(np.trace(G)), 0.0))


def build(S, n, R, Q, Px, Pv):
    """Skeleton HT from the index sets (dict in the layout of oracle.ht)."""
    leaves = []
    for mu in range(4):
        C = _leaf_matrix(S, mu, n, Q[mu])                      # n_mu x r_mu
        leaves.append(C @ np.linalg.inv(C[R[mu], :]))
    kx, kv = len(Px), len(Pv)
    b12 = S([(a, b, j1, j2) for a in R[0] for b in R[1] for (j1, j2) in Pv])
    B12 = b12.reshape(len(R[0]), len(R[1]), kv)
    b34 = S([(i1, i2, p, q) for (i1, i2) in Px for p in R[2] for q in R[3]])
    B34 = np.transpose(b34.reshape(kx, len(R[2]), len(R[3])), (1, 2, 0))
    core = S([(i1, i2, j1, j2) for (i1, i2) in Px for (j1, j2) in Pv]).reshape(kx, kv)
    root = np.linalg.inv(core)                                 # (kv x kx): [d, c]
    # the HT root pairs x-frame column d (P_v) with v-frame column c (P_x)
    return {"leaves": leaves, "B12": B12, "B34": B34, "root": root}


def _evaluate(F, idx):
    L = F["leaves"]
    idx = np.asarray(idx, dtype=np.int64)
    X = np.einsum("sa,sb,abd->sd", L[0][idx[:, 0]], L[1][idx[:, 1]], F["B12"])
    V = np.einsum("sp,sq,pqc->sc", L[2][idx[:, 2]], L[3][idx[:, 3]], F["B34"])
    return np.einsum("sd,dc,sc->s", X, F["root"], V)


def _zero_ht(n):
    z = [np.zeros((n[m], 1)) for m in range(4)]
    return {"leaves": z, "B12": np.zeros((1, 1, 1)), "B34": np.zeros((1, 1, 1)),
            "root": np.zeros((1, 1))}


def _union(a, b):
    out = list(a)
    for x in b:
        if x not in out:
            out.append(x)
    return out


def nested_cross(f, n, tol: float, kmax: int, probes, seed_index=(0, 0, 0, 0),
                 enrich: int = 4, max_sweeps: int = 12, node_tol: float | None = None):
    """f(idx (m, 4) int) -> values; probes (m, 4) int: seeded multi-indices
    that both enrich the candidate sets and check the result; node_tol: the
    tolerance of every leaf and root search (default tol / 10).
    Returns (F dict, info)."""
    ntol = tol / 10.0 if node_tol is None else node_tol
    S = _Sampler(f)
    n = tuple(int(v) for v in n)
    Nx, Nv = n[0] * n[1], n[2] * n[3]
    pr = np.asarray(probes, dtype=np.int64).reshape(-1, 4)
    m = len(pr)
    R = [[int(seed_index[a])] for a in range(4)]
    Px = [(R[0][0], R[1][0])]
    Pv = [(R[2][0], R[3][0])]
    Q = [None] * 4
    info = {"sweeps": 0, "probe_rounds": 0, "converged": False}
    forced = []
    F = None
    for sweep in range(max_sweeps):
        # enrichment: `enrich` probes in rotation, plus the last failed probe
        E = _union([], [tuple(int(v) for v in pr[(sweep * enrich + t) % m]) for t in range(min(enrich, m))])
        E = _union(E, forced)
        Ru = [_union(R[a], [e[a] for e in E]) for a in range(4)]
        Pxu = _union(Px, [(e[0], e[1]) for e in E])
        Pvu = _union(Pv, [(e[2], e[3]) for e in E])
        # leaves in order; a leaf sees the rows its sibling chose this sweep
        done = [False] * 4
        for a in range(4):
            Rc = [R[b] if done[b] else Ru[b] for b in range(4)]
            cands = _leaf_candidates(a, Rc, Pxu, Pvu)
            rows, cols = _leaf_search(S, a, n, cands, ntol, kmax, R[a][0], E)
            if not rows:
                info.update(samples=S.count, ranks=[0] * 6)
                return _zero_ht(n), info
            R[a] = rows
            Q[a] = [cands[c] for c in cols]
            done[a] = True
        # root, over the new leaf rows with the enrichment indices added: the
        # root pivots need not lie on the leaf interpolation grid (the frames
        # interpolate between its points), and a component that vanishes on
        # that grid is seen through the probes
        rx = _pairs(_union(R[0], [e[0] for e in E]), _union(R[1], [e[1] for e in E]))
        rv = _pairs(_union(R[2], [e[2] for e in E]), _union(R[3], [e[3] for e in E]))
        rows, cols = _root_search(S, rx, rv, ntol, kmax, rx.index(Px[0]) if Px[0] in rx else 0, E)
        if not rows:
            info.update(samples=S.count, ranks=[0] * 6)
            return _zero_ht(n), info
        Px = [rx[i] for i in rows]
        Pv = [rv[j] for j in cols]
        info["sweeps"] = sweep + 1
        F = build(S, n, R, Q, Px, Pv)
        # probe check (from the second sweep on, so that every leaf has seen
        # node sets chosen by a root search)
        vals = S(pr)
        err = np.abs(vals - _evaluate(F, pr))
        thr = tol * norm_ht(F) / math.sqrt(Nx * Nv)
        bad = np.flatnonzero(err > thr)
        if len(bad) == 0 and sweep >= 1:
            info["converged"] = True
            break
        forced = [tuple(int(v) for v in pr[bad[np.argmax(err[bad])]])] if len(bad) else []
        info["probe_rounds"] += 1 if len(bad) else 0
    info["samples"] = S.count
    info["ranks"] = [len(r) for r in R] + [len(Px), len(Pv)]
    info["sets"] = {"R": R, "Q": Q, "Px": Px, "Pv": Pv}
    return F, info


def skeleton_samples(n, ranks) -> int:
    """Entries the skeleton itself samples: leaf fibers, both transfer
    blocks and the core (ranks = r1, r2, r3, r4, k)."""
    r1, r2, r3, r4, k = ranks
    return n[0] * r1 + n[1] * r2 + n[2] * r3 + n[3] * r4 + k * (r1 * r2 + r3 * r4) + k * k
