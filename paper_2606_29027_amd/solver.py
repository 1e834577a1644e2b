"""One LoMaC-SLAR time step on the GPU, as a sequence of C-ABI calls.

The step follows the flowchart of section 3.2 ("Fluid correction diagram"):
SLAR_VP (eq. (slarvp), three frozen-field sub-flows of the third-order
commutator-free exponential integrator, each one cross approximation +
truncation) gives F*; the LoMaC closure of F* is prepared, the macroscopic
system is solved by JFNK (backward Euler for the first step, BDF2 after), and
the exact correction F^{n+1} = F* + sum_k dC_k Q_k is appended in frame form.
The split 1D1V workload uses Strang splitting X(h/2) V(h) X(h/2) instead.
With p.integrator == "dirk3_bdf3" the macroscopic integrator is the one of
section 4: two S-stable DIRK-3 start-up steps (each stage one SLAR_VP from
F^n to its stage time, one closure and one implicit solve), then
variable-step BDF-3; step sizes may vary from step to step.

This module only sequences library calls and owns the device buffers
(PyTorch allocations); it does no arithmetic of the method itself.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import lib as L

KCAP = 72          # frame columns (rank cap 64 + LoMaC columns)
RCAP = 64          # HT rank cap
CCAP = 128         # cross-approximation terms


class Solver:
    def __init__(self, p, precision: int = L.F64, probes=None, delta: float = 1e-12,
                 precond: int = 0, cnn=None, newton_tol: float = 1e-10, krylov_tol: float = 1e-4,
                 strict: bool = True, work=None):
        self.p = p
        self.grid = L.make_grid(p)
        # work: optional caller device memory for the library workspace
        # (slar_workspace_create_in), at least slar_workspace_bytes long
        self.ws = L.Workspace(self.grid, min(p.rmax, RCAP), work=work)
        self.prec = precision
        # the truncation's leaf refinement buys FP64-level agreement; with FP32
        # frame tables the sampling error is far above the Gram accuracy
        L.slar_leaf_refine(self.ws, precision == L.F64)
        self.delta = delta
        self.precond = precond
        self.cnn = cnn
        self.newton_tol = newton_tol
        self.krylov_tol = krylov_tol
        # strict: a macroscopic solve that misses the Newton tolerance raises
        # SlarError(SLAR_E_NOCONV) after the step's records are stored;
        # otherwise the step is completed and reported with converged False
        self.strict = strict
        self.macro_log = []           # per solve: Newton records (rms, krylov, lin. residual, restarts)
        self.fallbacks = 0            # learned-preconditioner solves redone with plain GMRES
        self.d = p.dx + p.dv
        self.Nx = int(np.prod(p.n[: p.dx]))
        self.Nv = int(np.prod(p.n[p.dx:]))
        self.nmom = 5 if p.dv == 1 else 9
        self.K = p.dv + 2
        f64 = dict(dtype=torch.float64, device="cuda")
        z = lambda *s: torch.zeros(*s, **f64)   # noqa: E731
        self.frames_buf = [(z(self.Nx, KCAP), z(self.Nv, KCAP)) for _ in range(4)]
        self.ht_buf = [self._ht_buffers() for _ in range(2)]
        self.kcross = min(p.cross_cap, CCAP)
        self.U = z(self.kcross, self.Nx)
        self.V = z(self.kcross, self.Nv)
        self.M = z(self.nmom, self.Nx)
        self.E = [z(p.dx, self.Nx) for _ in range(3)]
        self.Ubuf = [z(self.K, self.Nx) for _ in range(4)]
        self.Rstage = [z(self.K, self.Nx) for _ in range(2)]
        self.Ustage = [z(self.K, self.Nx) for _ in range(2)]
        self.U_hist = []              # DIRK-3/BDF-3: newest last, at times self.t_hist
        self.t_hist = []
        self.probes = None if probes is None else torch.as_tensor(
            np.ascontiguousarray(probes), dtype=torch.int32, device="cuda")
        self.n_i = None
        self.state = None            # current frames (L.Frames)
        self.state_slot = 0
        self.U_n = None
        self.U_nm1 = None
        self.stats = []
        # host wall time of the phases whose calls synchronise their stream
        # (work queued before them is counted in them)
        self.tphase = {"cross": 0.0, "truncation": 0.0, "macro": 0.0}

    # -------------------------------------------------------------- buffers
    def _ht_buffers(self):
        p = self.p
        f64 = dict(dtype=torch.float64, device="cuda")
        T = {"leaves": [torch.zeros(p.n[m] * RCAP, **f64) for m in range(self.d)],
             "root": torch.zeros(RCAP * RCAP, **f64)}
        if self.d == 4:
            T["B12"] = torch.zeros(RCAP * RCAP * RCAP, **f64)
            T["B34"] = torch.zeros(RCAP * RCAP * RCAP, **f64)
        H = L.HT()
        H.d = self.d
        H.dtype = L.F64
        for m in range(self.d):
            H.leaf[m] = T["leaves"][m].data_ptr()
        H.root = T["root"].data_ptr()
        if self.d == 4:
            H.B12 = T["B12"].data_ptr(); H.B34 = T["B34"].data_ptr()
        H._keep = T
        return H, T

    def _frames(self, slot, r=0):
        X, P = self.frames_buf[slot]
        return L.frames(X, P, r)

    # ---------------------------------------------------------------- setup
    def set_initial(self, F0: dict):
        """Upload an initial HT (host arrays, oracle layout) and build its frames."""
        T = {"leaves": [torch.as_tensor(np.ascontiguousarray(U), dtype=torch.float64, device="cuda")
                        for U in F0["leaves"]],
             "root": torch.as_tensor(np.ascontiguousarray(F0["root"]), dtype=torch.float64, device="cuda")}
        if self.d == 4:
            for key in ("B12", "B34"):
                b = F0[key]
                T[key] = torch.as_tensor(np.ascontiguousarray(b.reshape(b.shape[0] * b.shape[1], b.shape[2])),
                                         dtype=torch.float64, device="cuda")
        H = L.make_ht(T, self.d, L.F64)
        self.state = L.slar_frames_from_ht(self.grid, H, self._frames(0), self.ws)
        self.state_slot = 0
        L.slar_moments(self.grid, self.state, self.M, self.ws)
        torch.cuda.synchronize()
        # stationary neutralising ions: mean initial electron density
        self.n_i = float(self.M[0].double().mean().item())
        if self.p.lomac:
            self.U_n = self.Ubuf[0]
            L.slar_conserved(self.grid, self.state, self.n_i, self.U_n, self.ws)
            self.U_nm1 = None
            self.U_hist, self.t_hist = [self.U_n], [0.0]

    # ---------------------------------------------------------- components
    def efield(self, F: L.Frames, out):
        L.slar_moments(self.grid, F, self.M, self.ws)
        L.slar_poisson(self.grid, self.M[0], self.n_i, None, out, self.ws)
        return out

    def slar(self, src: L.Frames, adv, ht_slot: int, frame_slot: int):
        """One SLAR call: cross approximation + truncation + frames."""
        t0 = time.perf_counter()
        lr, info, st = L.slar_cross_update(self.grid, src, adv, self.prec, self.p.tol, self.kcross,
                                           self.probes, self.U, self.V, self.ws)
        t1 = time.perf_counter()
        H, _ = self.ht_buf[ht_slot]
        L.slar_truncate(self.grid, lr, self.p.tol, min(self.p.rmax, RCAP), H, self.ws)
        self.tphase["cross"] += t1 - t0
        self.tphase["truncation"] += time.perf_counter() - t1
        F = L.slar_frames_from_ht(self.grid, H, self._frames(frame_slot), self.ws)
        self.stats.append({"rank": info.rank, "samples": int(info.samples), "iters": info.iterations,
                           "probe_rounds": info.probe_rounds, "converged": info.converged,
                           "ranks": tuple(H.rank[: (2 if self.d == 2 else 6)])})
        return F, H

    def _free_slots(self, n):
        return [s for s in range(4) if s != self.state_slot][:n]

    def slar_vp(self, h):
        """Third-order commutator-free exponential integrator, section 3.1."""
        p = self.p
        sY2, sY3, sFs = self._free_slots(3)
        E1 = self.efield(self.state, self.E[0])
        Y2, _ = self.slar(self.state, L.make_adv(2, h / 3.0, 1.0, E1), 0, sY2)
        E2 = self.efield(Y2, self.E[1])
        Y3, _ = self.slar(self.state, L.make_adv(2, 2.0 * h / 3.0, 1.0, E2), 1, sY3)
        E3 = self.efield(Y3, self.E[2])
        Fs, Hs = self.slar(Y2, L.make_adv(2, h, 2.0 / 3.0, E1, E3, (-1.0 / 12.0, 3.0 / 4.0)), 1, sFs)
        return Fs, Hs, sFs

    def strang(self, h):
        o = self.p.order
        s1, s2, s3 = self._free_slots(3)
        F1, _ = self.slar(self.state, L.make_adv(0, 0.5 * h, 1.0, order=o), 0, s1)
        E = self.efield(F1, self.E[0])
        F2, _ = self.slar(F1, L.make_adv(1, h, 1.0, E, order=o), 1, s2)
        F3, H3 = self.slar(F2, L.make_adv(0, 0.5 * h, 1.0, order=o), 0, s3)
        return F3, H3, s3

    def _solve(self, Hs, Fs, hist, stages, beta, U_out):
        L.slar_lomac_prepare(self.grid, Hs, Fs, self.delta, self.n_i, self.ws)
        t0 = time.perf_counter()
        st, (nn, nk) = L.slar_macro_solve_system(self.grid, hist, stages, beta, self.newton_tol,
                                                 self.krylov_tol, self.precond,
                                                 None if self.cnn is None else self.cnn.handle, U_out, self.ws)
        if self.p.lomac_filter:
            L.slar_lomac_filter(self.grid, U_out, self.ws)
        self.tphase["macro"] += time.perf_counter() - t0
        self.macro_log.append(L.slar_macro_history(self.ws))
        self.fallbacks += int(L.slar_macro_fallbacks(self.ws)[1])
        return st == L.SLAR_OK, nn, nk

    def _step_dirk3_bdf3(self, h):
        """One step of the section 4 integrator (see the module docstring)."""
        U_n, t_n = self.U_hist[-1], self.t_hist[-1]
        U_new = [u for u in self.Ubuf if all(u is not v for v in self.U_hist[-3:])][0]
        ok, nn, nk = True, 0, 0
        if len(self.U_hist) < 3:
            A, c = L.slar_dirk3_tableau()
            for i in range(3):
                Fs, Hs, slot = self.slar_vp(c[i] * h)
                U_i = U_new if i == 2 else self.Ustage[i]
                stages = [(self.Rstage[j], h * A[i][j]) for j in range(i)]
                o, a, b = self._solve(Hs, Fs, [(U_n, 1.0)], stages, h * A[i][i], U_i)
                ok, nn, nk = ok and o, nn + a, nk + b
                if i < 2:
                    L.slar_macro_rhs(self.grid, U_i, self.Rstage[i], self.ws)
        else:
            cw, beta = L.slar_bdf_weights([t_n + h, t_n, self.t_hist[-2], self.t_hist[-3]])
            Fs, Hs, slot = self.slar_vp(h)
            hist = [(self.U_hist[-1 - j], cw[j]) for j in range(3)]
            ok, nn, nk = self._solve(Hs, Fs, hist, [], beta, U_new)
        out_slot = [s for s in range(4) if s != slot][0]
        Fn = L.slar_lomac_project(self.grid, Fs, U_new, self._frames(out_slot), self.ws)
        self.U_hist = (self.U_hist + [U_new])[-3:]
        self.t_hist = (self.t_hist + [t_n + h])[-3:]
        self.U_nm1, self.U_n = U_n, U_new
        self.state, self.state_slot = Fn, out_slot
        return {"newton": nn, "krylov": nk, "converged": ok}

    def step(self, h=None):
        """One time step of size h (default p.dt)."""
        p = self.p
        h = p.dt if h is None else h
        t0 = time.perf_counter()
        if p.lomac and p.integrator == "dirk3_bdf3":
            info = self._step_dirk3_bdf3(h)
            torch.cuda.synchronize()
            info["seconds"] = time.perf_counter() - t0
            return self._finish(info)
        Fs, Hs, slot = self.strang(h) if p.split else self.slar_vp(h)
        info = {}
        if p.lomac:
            L.slar_lomac_prepare(self.grid, Hs, Fs, self.delta, self.n_i, self.ws)
            U_new = [u for u in self.Ubuf if u is not self.U_n and u is not self.U_nm1][0]
            bdf = 1 if (self.U_nm1 is None or p.bdf == 1) else 2
            tm = time.perf_counter()
            st, (nn, nk) = L.slar_macro_solve(self.grid, self.U_n, self.U_nm1 if bdf == 2 else None, h, bdf,
                                              self.newton_tol, self.krylov_tol, self.precond,
                                              None if self.cnn is None else self.cnn.handle, U_new, self.ws)
            if p.lomac_filter:
                L.slar_lomac_filter(self.grid, U_new, self.ws)
            self.tphase["macro"] += time.perf_counter() - tm
            self.macro_log.append(L.slar_macro_history(self.ws))
            self.fallbacks += int(L.slar_macro_fallbacks(self.ws)[1])
            out_slot = [s for s in range(4) if s not in (slot,)][0]
            Fn = L.slar_lomac_project(self.grid, Fs, U_new, self._frames(out_slot), self.ws)
            self.U_nm1, self.U_n = self.U_n, U_new
            self.state, self.state_slot = Fn, out_slot
            info = {"newton": nn, "krylov": nk, "converged": st == L.SLAR_OK}
        else:
            self.state, self.state_slot = Fs, slot
        torch.cuda.synchronize()
        info["seconds"] = time.perf_counter() - t0
        return self._finish(info)

    def _finish(self, info):
        if "converged" in info:
            info["newton_log"] = self.macro_log[-1] if self.macro_log else []
            if self.strict and not info["converged"]:
                raise L.SlarError(L.SLAR_E_NOCONV, "macroscopic Newton solve of the step "
                                  f"(final RMS residual {info['newton_log'][-1][0]:.3e})"
                                  if info["newton_log"] else "macroscopic Newton solve of the step")
        return info

    # ---------------------------------------------------------- diagnostics
    def dense(self):
        """Full tensor (small grids only), shape p.n, via the frames on host."""
        F = self.state
        X, P = self.frames_buf[self.state_slot]
        A = X[:, : F.r].cpu().numpy() @ P[:, : F.r].cpu().numpy().T
        return A.reshape(tuple(self.p.n))

    def diagnostics(self):
        p = self.p
        L.slar_moments(self.grid, self.state, self.M, self.ws)
        L.slar_poisson(self.grid, self.M[0], self.n_i, None, self.E[0], self.ws)
        M = self.M.cpu().numpy()
        E = self.E[0].cpu().numpy()
        dvol = float(np.prod([(p.hi[m] - p.lo[m]) / p.n[m] for m in range(p.dx)]))
        ep = 0.5 * np.sum(E * E, axis=0)
        return {"elec_energy": float(ep.sum() * dvol), "mass": float(M[0].sum() * dvol),
                "momentum": [float(M[1 + m].sum() * dvol) for m in range(p.dv)],
                "energy": float((0.5 * M[p.dv + 1] + ep).sum() * dvol)}
