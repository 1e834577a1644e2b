"""Many independent Vlasov--Poisson instances stepped together.

Every instance is advanced by the same SLAR_VP step as the one-instance
driver (section 3.1: the three frozen-field sub-flows of the third-order
commutator-free exponential integrator, each one cross approximation plus
truncation), but each stage is one batched library call for all instances:
slar_batch_efield and slar_batch_truncate (every step one grouped launch
over all instances) and slar_batch_cross_update (persistent multi-instance
launches replayed from a captured hipGraph).  Instances differ in dimension, grid
size and rank; they share tolerance, rank cap and time step.

This module only sequences library calls and owns the device buffers; it
does no arithmetic of the method.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import lib as L

KCAP = 72
RCAP = 64          # HT rank cap
CCAP = 128         # cross-approximation terms


class _Inst:
    """Device buffers of one instance."""

    def __init__(self, p):
        self.p = p
        self.d = p.dx + p.dv
        self.Nx = int(np.prod(p.n[: p.dx]))
        self.Nv = int(np.prod(p.n[p.dx:]))
        self.nmom = 5 if p.dv == 1 else 9
        f64 = dict(dtype=torch.float64, device="cuda")
        z = lambda *s: torch.zeros(*s, **f64)   # noqa: E731
        self.frames_buf = [(z(self.Nx, KCAP), z(self.Nv, KCAP)) for _ in range(4)]
        self.ht = [self._ht() for _ in range(2)]
        self.U = z(CCAP, self.Nx)
        self.V = z(CCAP, self.Nv)
        self.M = z(self.nmom, self.Nx)
        self.E = [z(p.dx, self.Nx) for _ in range(3)]
        self.n_i = None

    def _ht(self):
        p = self.p
        f64 = dict(dtype=torch.float64, device="cuda")
        T = {"leaves": [torch.zeros(p.n[m] * RCAP, **f64) for m in range(self.d)],
             "root": torch.zeros(RCAP * RCAP, **f64)}
        if self.d == 4:
            T["B12"] = torch.zeros(RCAP ** 3, **f64)
            T["B34"] = torch.zeros(RCAP ** 3, **f64)
        return T

    def ht_desc(self, slot):
        T = self.ht[slot]
        H = L.HT()
        H.d = self.d
        H.dtype = L.F64
        for m in range(self.d):
            H.leaf[m] = T["leaves"][m].data_ptr()
        H.root = T["root"].data_ptr()
        if self.d == 4:
            H.B12 = T["B12"].data_ptr(); H.B34 = T["B34"].data_ptr()
        H._keep = T
        return H

    def frames(self, slot, r=0):
        X, P = self.frames_buf[slot]
        return L.frames(X, P, r)


class BatchSolver:
    def __init__(self, problems, probes=None, tol=None, rmax=None):
        self.problems = list(problems)
        for p in self.problems:
            if p.split or p.order != 3 or p.lomac:
                raise ValueError("batched instances use the unsplit 3-point SLAR_VP step without LoMaC")
        dts = {p.dt for p in self.problems}
        if len(dts) != 1:
            raise ValueError("instances must share the time step")
        self.dt = dts.pop()
        self.tol = tol if tol is not None else max(p.tol for p in self.problems)
        self.rmax = min(rmax if rmax is not None else max(p.rmax for p in self.problems), RCAP)
        # the cross of every instance may run past the rank cap (the
        # truncation caps the rank); the shared cap follows the same rule
        self.kcross = min(2 * self.rmax, CCAP) if rmax is not None else \
            min(max(p.cross_cap for p in self.problems), CCAP)
        self.batch = L.Batch([L.make_grid(p) for p in self.problems], self.rmax)
        # FP32 frame tables: their sampling error is far above the Gram
        # accuracy of the leaf bases, so the truncation skips the refinement
        for ws in self.batch.ws:
            L.slar_leaf_refine(ws, False)
        self.inst = [_Inst(p) for p in self.problems]
        self.probes = None
        if probes is not None:
            self.probes = [torch.as_tensor(np.ascontiguousarray(pr), dtype=torch.int32, device="cuda")
                           for pr in probes]
        self.state = None          # list of Frames
        self.state_slot = 0
        self.stats = []
        # host wall time per stage: the field solves are only enqueued (their
        # device time lands in the cross call, which synchronises); the cross
        # and truncation calls return once their work is done
        self.tphase = {"efield": 0.0, "cross": 0.0, "truncation": 0.0}

    @property
    def count(self):
        return len(self.inst)

    # ---------------------------------------------------------------- setup
    def set_initial(self, F0s):
        """Upload initial HTs (host arrays, oracle layout) and build frames."""
        self.state = []
        for q, (I, F0) in enumerate(zip(self.inst, F0s)):
            T = {"leaves": [torch.as_tensor(np.ascontiguousarray(U), dtype=torch.float64, device="cuda")
                            for U in F0["leaves"]],
                 "root": torch.as_tensor(np.ascontiguousarray(F0["root"]), dtype=torch.float64, device="cuda")}
            if I.d == 4:
                for key in ("B12", "B34"):
                    b = F0[key]
                    T[key] = torch.as_tensor(np.ascontiguousarray(b.reshape(b.shape[0] * b.shape[1], b.shape[2])),
                                             dtype=torch.float64, device="cuda")
            H = L.make_ht(T, I.d, L.F64)
            ws = self.batch.ws[q]
            F = L.slar_frames_from_ht(ws.grid, H, I.frames(0), ws)
            L.slar_moments(ws.grid, F, I.M, ws)
            self.state.append(F)
        torch.cuda.synchronize()
        for I in self.inst:
            I.n_i = float(I.M[0].double().mean().item())
        self.state_slot = 0

    # --------------------------------------------------------------- stages
    def efield(self, F, e):
        t0 = time.perf_counter()
        self.batch.efield(F, [I.n_i for I in self.inst], [I.M for I in self.inst], [I.E[e] for I in self.inst])
        self.tphase["efield"] += time.perf_counter() - t0
        return [I.E[e] for I in self.inst]

    def slar(self, src, advs, ht_slot, frame_slot):
        t0 = time.perf_counter()
        lrs, info, _ = self.batch.cross_update(src, advs, self.tol, self.kcross, self.probes,
                                               [I.U for I in self.inst], [I.V for I in self.inst])
        t1 = time.perf_counter()
        hts = [I.ht_desc(ht_slot) for I in self.inst]
        outs = [I.frames(frame_slot) for I in self.inst]
        self.batch.truncate(lrs, self.tol, self.rmax, hts, outs)
        self.tphase["cross"] += t1 - t0
        self.tphase["truncation"] += time.perf_counter() - t1
        self.stats.append({"ranks": [x.rank for x in info], "samples": int(sum(x.samples for x in info)),
                           "samples_q": [int(x.samples) for x in info], "src_ranks": [f.r for f in src],
                           "iters": max(x.iterations for x in info)})
        return outs, hts

    def _free_slots(self, n):
        return [s for s in range(4) if s != self.state_slot][:n]

    def tune(self, reps=2):
        """Autotune the batched cross approximation on the first sub-flow of
        the current state (outputs are scratch)."""
        E1 = self.efield(self.state, 0)
        advs = [L.make_adv(2, self.dt / 3.0, 1.0, E) for E in E1]
        return self.batch.tune(self.state, advs, self.tol, self.kcross, self.probes,
                               [I.U for I in self.inst], [I.V for I in self.inst], reps)

    def step(self):
        """One SLAR_VP step of every instance."""
        h = self.dt
        t0 = time.perf_counter()
        sY2, sY3, sFs = self._free_slots(3)
        E1 = self.efield(self.state, 0)
        Y2, _ = self.slar(self.state, [L.make_adv(2, h / 3.0, 1.0, E) for E in E1], 0, sY2)
        E2 = self.efield(Y2, 1)
        Y3, _ = self.slar(self.state, [L.make_adv(2, 2.0 * h / 3.0, 1.0, E) for E in E2], 1, sY3)
        E3 = self.efield(Y3, 2)
        Fs, _ = self.slar(Y2, [L.make_adv(2, h, 2.0 / 3.0, a, b, (-1.0 / 12.0, 3.0 / 4.0))
                               for a, b in zip(E1, E3)], 1, sFs)
        self.state, self.state_slot = Fs, sFs
        torch.cuda.synchronize()
        return {"seconds": time.perf_counter() - t0}

    # ---------------------------------------------------------- diagnostics
    def dense(self, q):
        F = self.state[q]
        X, P = self.inst[q].frames_buf[self.state_slot]
        A = X[:, : F.r].cpu().numpy() @ P[:, : F.r].cpu().numpy().T
        return A.reshape(tuple(self.problems[q].n))

    def elec_energy(self):
        """Electric energy of every instance (field of the current state)."""
        E = self.efield(self.state, 0)
        out = []
        for p, e in zip(self.problems, E):
            dvol = float(np.prod([(p.hi[m] - p.lo[m]) / p.n[m] for m in range(p.dx)]))
            out.append(float(0.5 * (e * e).sum().item() * dvol))
        return out
