"""Implicit macroscopic update and its Jacobian-free Newton--Krylov solve (oracle).

Section 3.2.3, eqs. (BE_macro), (BE_nonlinear_system): with the LoMaC
closure, the conserved variables U = (n, m n u, e) solve
  G(U) = U - U_hist + b dt ( D.F(U) - S(U) ) = 0,
  backward Euler: U_hist = U^n, b = 1;  BDF2: U_hist = 4/3 U^n - 1/3 U^{n-1},
  b = 2/3 (the start-up step is BE); the paper's own DIRK-3 start-up and
  variable-step BDF-3 give other U_hist and b (``timeint``).
The flux (eq. (macro_sys_comp)) is taken from the corrected kinetic state
F(U) = F* + sum_k dC_k(U) Q_k (eq. (LoMaC_update_discrete)):
  mass      <v f>,
  momentum  <v (x) v f>,
  energy    1/2 <|v|^2 v f> + F_ep,  F_ep = -phi grad(d_t phi) + J phi
            (eq. (electric_field_flux)), J = q_e M_1 = -M_1,
            -Laplace(d_t phi) = -div J,
and S = (0, rho_e E, 0) with rho_e = q_e n_e = -U_0, E from the Poisson
solve of U_0.  All x-derivatives are spectral (see ``spectral``).

JFNK: Newton from the SLAR state U(F*), finite-difference Jacobian-vector
products, restarted GMRES (right-preconditioned flexible GMRES when a
preconditioner is given), classical Gram--Schmidt with one
re-orthogonalisation.  Tolerances 1e-10 (Newton) and 1e-4 (Krylov) as in
section 4; read as: Newton stops when ||G||_2 / sqrt(#unknowns) <= 1e-10,
GMRES when its residual drops by 1e-4.  The mean of each component of G is
exactly mean(U) - mean(U_hist) (the divergence and the source have zero mean
by the discrete identities of the spectral operators), so on that subspace
the Jacobian is the identity: each Newton update sets the mean of the step
to -mean(G) exactly, which makes total mass, momentum and energy
conserved to round-off.
"""
from __future__ import annotations

import math

import numpy as np

from . import lomac as LM
from . import spectral as SP


class MacroSystem:
    """Everything G(U) needs, frozen for one time step."""

    def __init__(self, Mstar, B, n_i, lengths, dvol_v, vgrids, U_hist, beta_dt):
        from .ht import psi_list
        self.dv = B["dv"]
        self.B = B
        self.n_i = n_i
        self.lengths = lengths
        self.Mstar = Mstar                        # all psi moments of F*
        self.Cstar = LM.coefficients(Mstar[: self.dv + 2], B)
        self.psiQ = LM.velocity_integrals(B, psi_list(vgrids), dvol_v)  # (npsi, K)
        self.U_hist = U_hist
        self.beta_dt = beta_dt

    def corrected_moments(self, U):
        Mraw = LM.raw_from_conserved(U, self.n_i, self.lengths)
        dC = LM.coefficients(Mraw, self.B) - self.Cstar
        return self.Mstar + np.tensordot(self.psiQ, dC, axes=([1], [0])), dC

    def residual(self, U: np.ndarray) -> np.ndarray:
        return U - self.U_hist + self.beta_dt * self.rhs(U)

    def rhs(self, U: np.ndarray) -> np.ndarray:
        """R(U) = D.F(U) - S(U), so that the moment system reads U' = -R(U)."""
        dv = self.dv
        L = self.lengths
        M, _ = self.corrected_moments(U)
        # moment order: 0:1, 1..dv: v_mu, dv+1: |v|^2, then v_mu v_nu (mu<=nu), then |v|^2 v_mu
        off_vv = dv + 2
        pair = {}
        c = off_vv
        for a in range(dv):
            for b in range(a, dv):
                pair[(a, b)] = pair[(b, a)] = c
                c += 1
        off_e = c
        phi, E = SP.poisson(U[0], self.n_i, L)
        J = -M[1: dv + 1]
        dtphi = SP.inv_neg_laplace(-SP.div(J, L), L)
        gdt = SP.grad(dtphi, L)
        Fep = -phi[None] * gdt + J * phi[None]
        divF = np.empty_like(U)
        divF[0] = SP.div(M[1: dv + 1], L)
        for a in range(dv):
            divF[1 + a] = SP.div(np.stack([M[pair[(a, b)]] for b in range(dv)]), L)
        divF[dv + 1] = SP.div(0.5 * M[off_e: off_e + dv] + Fep, L)
        S = np.zeros_like(U)
        S[1: dv + 1] = -U[0][None] * E
        return divF - S


def fgmres(Aop, b, tol, restart=50, maxit=500, precond=None, record=None):
    """Right-preconditioned flexible GMRES(m) with CGS2; returns (x, iters)."""
    n = b.size
    bn = float(np.linalg.norm(b))
    x = np.zeros(n)
    if bn == 0.0:
        return x, 0
    its = 0
    r = b.copy()
    while its < maxit:
        beta = float(np.linalg.norm(r))
        if beta <= tol * bn:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart); sn = np.zeros(restart)
        g = np.zeros(restart + 1); g[0] = beta
        jlast = 0
        for j in range(restart):
            z = precond(V[j]) if precond is not None else V[j]
            Z.append(z)
            w = Aop(z)
            if record is not None:
                record.append((w.copy(), z.copy()))
            Vm = np.stack(V, axis=1)
            h = Vm.T @ w
            w = w - Vm @ h
            h2 = Vm.T @ w
            w = w - Vm @ h2
            h = h + h2
            H[: j + 1, j] = h
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] > 0:
                V.append(w / H[j + 1, j])
            else:
                V.append(np.zeros(n))
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den if den > 0 else 1.0
            sn[j] = H[j + 1, j] / den if den > 0 else 0.0
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            jlast = j
            if abs(g[j + 1]) <= tol * bn or its >= maxit or H[j, j] == 0.0:
                break
        k = jlast + 1
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1: k] @ y[i + 1: k]) / H[i, i] if H[i, i] != 0 else 0.0
        x = x + np.stack(Z[:k], axis=1) @ y
        r = b - Aop(x)
        if float(np.linalg.norm(r)) <= tol * bn:
            break
    return x, its


def jfnk(system: MacroSystem, U0: np.ndarray, newton_tol=1e-10, krylov_tol=1e-4,
         max_newton=30, restart=50, maxit=500, precond=None, record=None):
    """Returns (U, info) with Newton/Krylov counts and the final RMS residual."""
    U = U0.copy()
    shape = U.shape
    nunk = U.size
    info = {"newton": 0, "krylov": 0, "rms": [], "converged": False}
    eps = np.finfo(np.float64).eps
    for it in range(max_newton + 1):
        g = system.residual(U)
        rms = float(np.linalg.norm(g)) / math.sqrt(nunk)
        info["rms"].append(rms)
        if rms <= newton_tol:
            info["converged"] = True
            break
        if it == max_newton:
            break
        gf = g.ravel()
        Un = float(np.linalg.norm(U))

        def Jv(v, U=U, gf=gf):
            vn = float(np.linalg.norm(v))
            if vn == 0.0:
                return np.zeros_like(v)
            h = math.sqrt(eps) * (1.0 + Un) / vn
            return (system.residual(U + h * v.reshape(shape)).ravel() - gf) / h

        pc = None
        if precond is not None:
            pc = (lambda v, U=U: precond(v.reshape(shape), U).ravel())
        d, k = fgmres(Jv, -gf, krylov_tol, restart, maxit, pc, record)
        d = d.reshape(shape)
        # exact Newton step on the per-component mean (identity Jacobian there)
        axes = tuple(range(1, U.ndim))
        d = d - d.mean(axis=axes, keepdims=True) - g.mean(axis=axes, keepdims=True)
        U = U + d
        info["newton"] += 1
        info["krylov"] += k
    info["U"] = U
    return U, info
