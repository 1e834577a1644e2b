"""Time integrators of the macroscopic LoMaC system (oracle; test infrastructure).

Section 3.2.3 couples the kinetic SLAR update to an implicit solve of the
macroscopic moment system U' = -R(U), R(U) = D.F(U) - S(U).  Section 4 runs
it with the S-stable three-stage DIRK method of Alexander (1977, Theorem 5)
for the start-up steps and the classical variable-step BDF-3 of Gear (1971)
after them; every stage or step is one nonlinear system

    G(U) = U - sum_j c_j U_j + sum_j d_j R_j + beta R(U) = 0,

with history states U_j, explicit stage terms R_j (earlier DIRK stages) and
an implicit weight beta.  This module only produces those weights.

* ``dirk3``: gamma is the root in (1/6, 1/2) of 6 x^3 - 18 x^2 + 9 x - 1 = 0;
  c = (gamma, (1 + gamma)/2, 1); rows of A: (gamma), ((1 - gamma)/2, gamma),
  (b1, b2, gamma) with b1 = -(6 gamma^2 - 16 gamma + 1)/4,
  b2 = (6 gamma^2 - 20 gamma + 5)/4; the last row is b (stiffly accurate).
  Stage i at t_n + c_i h: U_i = U_n - h sum_{j<=i} a_ij R(U_j), i.e.
  c = (1), d_j = h a_ij (j < i), beta = h a_ii.
* ``dirk3_step`` / ``bdf_history`` sequence one step given a stage solver;
  the kinetic driver (``step``) and the tests share them.
* ``bdf``: the derivative at t_{n+1} of the polynomial interpolating
  (t_{n+1}, U), (t_n, U_n), ..., (t_{n+1-k}, U_{n+1-k}) equals -R(U).  With
  Lagrange basis l_j on those nodes (node 0 = t_{n+1}),
    l_0'(t_0) = sum_{m>0} 1 / (t_0 - t_m),
    l_j'(t_0) = prod_{m != 0, j} (t_0 - t_m) / prod_{m != j} (t_j - t_m),
  so c_j = -l_j'(t_0) / l_0'(t_0) and beta = 1 / l_0'(t_0).  With equal
  steps k = 3 gives the textbook 18/11, -9/11, 2/11 and beta = 6h/11.
"""
from __future__ import annotations

import numpy as np


def dirk3():
    """(A [3][3], b [3], c [3]) of the S-stable three-stage DIRK."""
    roots = np.roots([6.0, -18.0, 9.0, -1.0])
    g = [float(r.real) for r in roots if abs(r.imag) < 1e-12 and 1.0 / 6.0 < r.real < 0.5]
    assert len(g) == 1
    g = g[0]
    b1 = -(6.0 * g * g - 16.0 * g + 1.0) / 4.0
    b2 = (6.0 * g * g - 20.0 * g + 5.0) / 4.0
    A = np.array([[g, 0.0, 0.0],
                  [(1.0 - g) / 2.0, g, 0.0],
                  [b1, b2, g]])
    c = np.array([g, (1.0 + g) / 2.0, 1.0])
    return A, A[2].copy(), c


def bdf(times):
    """Variable-step BDF weights.  times = [t_{n+1}, t_n, ..., t_{n+1-k}]
    (k + 1 distinct values).  Returns (c [k], beta)."""
    t = [float(x) for x in times]
    k = len(t) - 1
    l0 = sum(1.0 / (t[0] - t[m]) for m in range(1, k + 1))
    c = []
    for j in range(1, k + 1):
        num = 1.0
        for m in range(1, k + 1):
            if m != j:
                num *= t[0] - t[m]
        den = 1.0
        for m in range(k + 1):
            if m != j:
                den *= t[j] - t[m]
        c.append(-(num / den) / l0)
    return np.array(c), 1.0 / l0


def dirk3_step(U_n, h, stage):
    """One DIRK-3 step.  stage(i, tau_i, U_hist, beta) solves stage i
    (tau_i = c_i h after t_n) for U_i in U_i - U_hist + beta R_i(U_i) = 0 and
    returns (U_i, R_i) with R_i the right-hand side callable of that stage.
    Returns U_3, the new state (the last row of A is b)."""
    A, _, c = dirk3()
    R = []
    for i in range(3):
        U_hist = U_n - h * sum(A[i][j] * R[j] for j in range(i)) if i else U_n
        U_i, rhs = stage(i, c[i] * h, U_hist, A[i][i] * h)
        if i < 2:
            R.append(rhs(U_i))
    return U_i


def bdf_history(Us, ts, h):
    """Combined history and implicit weight of a variable-step BDF-3 step
    from t_n = ts[-1] to ts[-1] + h, with states Us[-1], Us[-2], Us[-3] at
    ts[-1], ts[-2], ts[-3]."""
    cw, beta = bdf([ts[-1] + h, ts[-1], ts[-2], ts[-3]])
    return sum(cw[j] * Us[-1 - j] for j in range(3)), beta
