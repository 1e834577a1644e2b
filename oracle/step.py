"""One SLAR / SLAR_VP / LoMaC time step and run driver (oracle).

  * SLAR(F; a, dt, eps_Base): the updated tensor is built by the cross
    approximation (``cross``) from SL-FD entry evaluations (``feet`` +
    ``ht.sample``), section 3.1;
  * SLAR_VP (eq. (slarvp)): third-order commutator-free exponential
    integrator of Celledoni, Marthinsen and Owren, three frozen-field linear
    advections per step:
        E1 = E[f^n];  Y2 = S_{h/3}[v, -E1] f^n
        E2 = E[Y2];   Y3 = S_{2h/3}[v, -E2] f^n
        E3 = E[Y3];   f* = S_h[(2/3) v, -(-E1/12 + 3 E3/4)] Y2
    (the coefficient set is the published CF3 scheme; the paper cites it
    without printing it);
  * 1D1V Strang splitting X(h/2) V(h) X(h/2), E recomputed after the first
    half step (used for the split 1D1V workload; the paper itself avoids
    splitting);
  * LoMaC step (fig. "Fluid correction diagram"): weight and basis from F*,
    JFNK on G(U) = 0, exact correction F^{n+1} = F* + sum dC_k Q_k, with
    U^{n+1} the macroscopic state carried to the next step; the implicit
    macroscopic integrator is BE then BDF2, or (section 4) two S-stable
    DIRK-3 start-up steps, each stage one SLAR_VP from F^n to its stage time
    and one JFNK solve, then variable-step BDF-3 (``timeint``);
  * background ion density n_i = mean_x n_e(x, 0) (stationary neutralising
    ions, section 2.1).
"""
from __future__ import annotations

import math

import numpy as np

from . import cross as CR
from . import feet as FT
from . import grid as G
from . import ht as HT
from . import lomac as LM
from . import macro as MA
from . import spectral as SP
from . import timeint as TI


class Oracle:
    def __init__(self, p, probes=None, delta: float = LM.DELTA, newton_tol: float = 1e-10):
        self.p = p
        self.dx, self.dv = p.dx, p.dv
        self.n = tuple(p.n)
        self.lo = tuple(p.lo)
        self.hi = tuple(p.hi)
        self.nx = self.n[: p.dx]
        self.nv = self.n[p.dx:]
        self.lengths = [self.hi[m] - self.lo[m] for m in range(p.dx)]
        self.h = [G.spacing(self.lo[m], self.hi[m], self.n[m]) for m in range(p.d)]
        self.vgrids = [G.centres(self.lo[m], self.hi[m], self.n[m]) for m in range(p.dx, p.d)]
        self.dvol_x = float(np.prod(self.h[: p.dx]))
        self.dvol_v = float(np.prod(self.h[p.dx:]))
        self.probes = probes
        self.delta = delta
        self.n_i = None
        self.newton_tol = newton_tol
        self.stats = []

    # ------------------------------------------------------------ sampling
    def entries(self, F, idx, kind, tau, cv, E):
        foot = FT.feet(idx, self.lo, self.hi, self.n, self.dx, kind, tau, cv, E)
        rows, wts = FT.stencils(foot, idx, self.lo, self.hi, self.n, self.p.order, kind, self.dx)
        return HT.sample(F, rows, wts)

    def _idx(self, I, J):
        I = np.atleast_1d(I); J = np.atleast_1d(J)
        xi = np.stack(np.unravel_index(I, self.nx), axis=1)
        vj = np.stack(np.unravel_index(J, self.nv), axis=1)
        return np.concatenate([xi, vj], axis=1)

    def slar(self, F, kind, tau, cv, E):
        nrows = int(np.prod(self.nx)); ncols = int(np.prod(self.nv))

        def row(i):
            return self.entries(F, self._idx(np.full(ncols, i), np.arange(ncols)), kind, tau, cv, E)

        def col(j):
            return self.entries(F, self._idx(np.arange(nrows), np.full(nrows, j)), kind, tau, cv, E)

        def pts(I, J):
            return self.entries(F, self._idx(I, J), kind, tau, cv, E)

        kc = self.p.cross_cap
        U, V, info = CR.aca(row, col, pts, nrows, ncols, self.p.tol, kc, 0, self.probes)
        info["capped"] = (not info["converged"]) and U.shape[1] >= kc
        if info["capped"] and U.shape[1] > self.p.rmax:
            U, V = CR.cur_core(U, V, info["pivots"], self.p.rmax)
        Fn = CR.truncate_lowrank(U, V, self.nx, self.nv, self.p.tol, self.p.rmax)
        info["ranks"] = HT.ranks(Fn)
        self.stats.append(info)
        return Fn

    # -------------------------------------------------------------- fields
    def moments(self, F):
        return HT.moments(F, self.vgrids, self.dvol_v)

    def efield(self, F):
        M0 = self.moments(F)[0]
        if self.n_i is None:
            self.n_i = float(np.mean(M0))
        return SP.poisson(M0, self.n_i, self.lengths)[1]

    # --------------------------------------------------------------- steps
    def slar_vp(self, F, h):
        E1 = self.efield(F)
        Y2 = self.slar(F, 2, h / 3.0, 1.0, E1)
        E2 = self.efield(Y2)
        Y3 = self.slar(F, 2, 2.0 * h / 3.0, 1.0, E2)
        E3 = self.efield(Y3)
        Ec = FT.frozen_field([E1, E3], [-1.0 / 12.0, 3.0 / 4.0])
        return self.slar(Y2, 2, h, 2.0 / 3.0, Ec)

    def strang(self, F, h):
        self.efield(F)                      # fixes n_i at the first call
        F1 = self.slar(F, 0, 0.5 * h, 1.0, None)
        E = self.efield(F1)
        F2 = self.slar(F1, 1, h, 1.0, E)
        return self.slar(F2, 0, 0.5 * h, 1.0, None)

    def conserved(self, F):
        M = self.moments(F)
        if self.n_i is None:
            self.n_i = float(np.mean(M[0]))
        return LM.conserved_from_raw(M[: self.dv + 2], self.n_i, self.lengths)

    def lomac(self, Fs, U_n, U_nm1, h, precond=None, record=None):
        """Returns (F^{n+1}, U^{n+1}, jfnk info); BE, then BDF2."""
        if U_nm1 is None or self.p.bdf == 1:
            U_hist, b = U_n, 1.0
        else:
            U_hist, b = (4.0 * U_n - U_nm1) / 3.0, 2.0 / 3.0
        return self.lomac_solve(Fs, U_hist, b * h, precond, record)

    def lomac_solve(self, Fs, U_hist, beta_dt, precond=None, record=None):
        """LoMaC closure of F*, the implicit solve of
        U - U_hist + beta_dt R(U) = 0, and the exact correction."""
        L = Fs["leaves"]
        u1 = [L[self.dx + m][:, 0] for m in range(self.dv)]
        B = LM.basis(u1, self.vgrids, self.h[self.dx:], self.delta)
        Mstar = self.moments(Fs)
        U0 = LM.conserved_from_raw(Mstar[: self.dv + 2], self.n_i, self.lengths)
        sysm = MA.MacroSystem(Mstar, B, self.n_i, self.lengths, self.dvol_v, self.vgrids,
                              U_hist, beta_dt)
        U, info = MA.jfnk(sysm, U0, newton_tol=self.newton_tol, precond=precond, record=record)
        if getattr(self.p, "lomac_filter", False):
            U = LM.filter_correction(U, U0)
        Mraw = LM.raw_from_conserved(U, self.n_i, self.lengths)
        dC = LM.coefficients(Mraw, B) - sysm.Cstar
        Fn = dict(Fs)
        Fn["corr"] = {"C": dC, "Q": B["Q"]}
        info["basis"] = B
        info["system"] = sysm
        return Fn, U, info

    def diagnostics(self, F, U=None):
        M = self.moments(F)
        if self.n_i is None:
            self.n_i = float(np.mean(M[0]))
        _, E = SP.poisson(M[0], self.n_i, self.lengths)
        ep = SP.field_energy_density(E)
        dv = self.dv
        out = {
            "elec_energy": float(np.sum(ep) * self.dvol_x),
            "mass": float(np.sum(M[0]) * self.dvol_x),
            "momentum": [float(np.sum(M[1 + m]) * self.dvol_x) for m in range(dv)],
            "energy": float(np.sum(0.5 * M[dv + 1] + ep) * self.dvol_x),
        }
        return out

    def dirk3_step(self, F, U_n, h, precond=None):
        """One step of the S-stable three-stage DIRK (``timeint``): stage i
        takes F*_i = SLAR_VP(F^n; c_i h) (the stage distribution at
        t_n + c_i h) and solves its implicit system with the LoMaC closure
        of F*_i; the last stage (c = 1) is the new state.  Returns
        (F^{n+1}, U^{n+1}, info summed over the stages)."""
        info = {"newton": 0, "krylov": 0, "converged": True}
        last = {}

        def stage(i, tau, U_hist, beta):
            Fs = self.slar_vp(F, tau)
            Fi, Ui, inf = self.lomac_solve(Fs, U_hist, beta, precond)
            for key in ("newton", "krylov"):
                info[key] += inf[key]
            info["converged"] &= inf["converged"]
            last["F"] = Fi
            return Ui, inf["system"].rhs

        U = TI.dirk3_step(U_n, h, stage)
        return last["F"], U, info

    def bdf3_step(self, F, Us, ts, h, precond=None):
        """One variable-step BDF-3 step of size h after the states Us at
        times ts (the last three are used)."""
        U_hist, beta = TI.bdf_history(Us, ts, h)
        Fs = self.slar_vp(F, h)
        return self.lomac_solve(Fs, U_hist, beta, precond)

    def run(self, F, steps, lomac=None, precond=None, callback=None, integrator=None, dts=None):
        """integrator: "bdf2" (BE start-up, then fixed-step BDF2) or
        "dirk3_bdf3" (two DIRK-3 start-up steps, then variable-step BDF-3);
        dts: optional per-step sizes (default p.dt)."""
        p = self.p
        lomac = p.lomac if lomac is None else lomac
        integrator = integrator or p.integrator
        U_n = self.conserved(F) if lomac else None
        U_nm1 = None
        Us, ts = [U_n], [0.0]
        hist = [self.diagnostics(F)]
        for n in range(steps):
            h = p.dt if dts is None else dts[n]
            if lomac and integrator == "dirk3_bdf3":
                if n < 2:
                    F, U_new, info = self.dirk3_step(F, Us[-1], h, precond)
                else:
                    F, U_new, info = self.bdf3_step(F, Us, ts, h, precond)
                Us.append(U_new)
                ts.append(ts[-1] + h)
            elif lomac:
                Fs = self.strang(F, h) if p.split else self.slar_vp(F, h)
                F, U_new, info = self.lomac(Fs, U_n, U_nm1, h, precond)
                U_nm1, U_n = U_n, U_new
            else:
                Fs = self.strang(F, h) if p.split else self.slar_vp(F, h)
                F, info = Fs, {}
            d = self.diagnostics(F)
            d["ranks"] = HT.ranks(F)
            d["newton"] = info.get("newton")
            d["krylov"] = info.get("krylov")
            hist.append(d)
            if callback is not None:
                callback(n, F, d)
        return F, hist
