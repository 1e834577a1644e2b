"""ctypes binding of ``libslar.so`` (argument marshalling only).

Every function here converts torch tensors / Python numbers to the C ABI of
``include/slar.h`` and raises on a non-OK status.  No arithmetic of the
method happens in Python: every step runs in the HIP kernels of the library.
Device memory and streams come from PyTorch.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslar.so")

SLAR_OK, SLAR_E_INVAL, SLAR_E_NOMEM, SLAR_E_RANK_CAP, SLAR_E_NOCONV, SLAR_E_NUMERIC, SLAR_E_HIP = range(7)
F32, F64 = 0, 1

EXPORTS = (
    "slar_status_str", "slar_workspace_create", "slar_workspace_bytes", "slar_workspace_create_in",
    "slar_workspace_destroy", "slar_ht_sample",
    "slar_frames_from_ht", "slar_frame_sample", "slar_cross_update", "slar_nested_cross", "slar_truncate",
    "slar_moments", "slar_poisson", "slar_conserved", "slar_lomac_prepare", "slar_macro_solve",
    "slar_lomac_project", "slar_cnn_create", "slar_cnn_destroy", "slar_cnn_nparams",
    "slar_cnn_set_params", "slar_cnn_get_params", "slar_cnn_forward", "slar_cnn_grad",
    "slar_cnn_train_step", "slar_record_krylov", "slar_recorded_pairs", "slar_timing_enable", "slar_leaf_refine",
    "slar_timing_read", "slar_batch_create", "slar_batch_destroy", "slar_batch_workspace",
    "slar_batch_cross_update", "slar_batch_truncate", "slar_batch_efield", "slar_batch_get_config",
    "slar_batch_set_config", "slar_batch_tune", "slar_batch_timing", "slar_batch_timing_reset",
    "slar_macro_solve_system", "slar_macro_rhs", "slar_dirk3_tableau", "slar_bdf_weights",
    "slar_cnn_correct", "slar_macro_history", "slar_macro_fallbacks", "slar_lomac_filter",
    "slar_poisson_noalloc",
)


class Grid(C.Structure):
    _fields_ = [("dx", C.c_int32), ("dv", C.c_int32), ("n", C.c_int32 * 4),
                ("lo", C.c_double * 4), ("hi", C.c_double * 4)]


class HT(C.Structure):
    _fields_ = [("d", C.c_int32), ("rank", C.c_int32 * 6), ("dtype", C.c_int32),
                ("leaf", C.c_void_p * 4), ("B12", C.c_void_p), ("B34", C.c_void_p),
                ("root", C.c_void_p)]


class Frames(C.Structure):
    _fields_ = [("r", C.c_int32), ("ld", C.c_int32), ("X", C.c_void_p), ("P", C.c_void_p)]


class Adv(C.Structure):
    _fields_ = [("kind", C.c_int32), ("order", C.c_int32), ("tau", C.c_double),
                ("cv", C.c_double), ("E", C.c_void_p * 2), ("cE", C.c_double * 2)]


class LowRank(C.Structure):
    _fields_ = [("k", C.c_int32), ("U", C.c_void_p), ("V", C.c_void_p)]


class CrossInfo(C.Structure):
    _fields_ = [("rank", C.c_int32), ("iterations", C.c_int32), ("probe_rounds", C.c_int32),
                ("converged", C.c_int32), ("samples", C.c_int64)]


class NestedInfo(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("probe_rounds", C.c_int32), ("converged", C.c_int32),
                ("rank", C.c_int32 * 6), ("samples", C.c_int64)]


class MacroSystem(C.Structure):
    _fields_ = [("nhist", C.c_int32), ("U", C.c_void_p * 3), ("c", C.c_double * 3),
                ("nstage", C.c_int32), ("R", C.c_void_p * 3), ("d", C.c_double * 3),
                ("beta", C.c_double)]


class SlarError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {status_str(status)} ({status})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; fails loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: run __graft_entry__.build() first")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "slar_status_str": (C.c_char_p, [i32]),
        "slar_workspace_create": (i32, [P(Grid), i32, P(vp)]),
        "slar_workspace_bytes": (i32, [P(Grid), i32, P(C.c_size_t)]),
        "slar_workspace_create_in": (i32, [P(Grid), i32, vp, C.c_size_t, P(vp)]),
        "slar_workspace_destroy": (i32, [vp]),
        "slar_ht_sample": (i32, [P(Grid), P(HT), P(Adv), i64, vp, vp, vp]),
        "slar_frames_from_ht": (i32, [P(Grid), P(HT), P(Frames), vp, vp]),
        "slar_frame_sample": (i32, [P(Grid), P(Frames), P(Adv), i32, i64, vp, vp, vp, vp]),
        "slar_cross_update": (i32, [P(Grid), P(Frames), P(Adv), i32, dbl, i32, i32, vp,
                                    P(LowRank), P(CrossInfo), vp, vp]),
        "slar_nested_cross": (i32, [P(Grid), P(Frames), P(Adv), i32, dbl, i32, i32, vp, vp, P(HT),
                                    P(NestedInfo), vp, vp]),
        "slar_truncate": (i32, [P(Grid), P(LowRank), dbl, i32, P(HT), vp, vp]),
        "slar_moments": (i32, [P(Grid), P(Frames), vp, vp, vp]),
        "slar_poisson": (i32, [P(Grid), vp, dbl, vp, vp, vp, vp]),
        "slar_conserved": (i32, [P(Grid), P(Frames), dbl, vp, vp, vp]),
        "slar_lomac_prepare": (i32, [P(Grid), P(HT), P(Frames), dbl, dbl, vp, vp]),
        "slar_macro_solve": (i32, [P(Grid), vp, vp, dbl, i32, dbl, dbl, i32, vp, vp, P(i32), vp, vp]),
        "slar_lomac_project": (i32, [P(Grid), P(Frames), vp, P(Frames), vp, vp]),
        "slar_cnn_create": (i32, [i32, P(i32), i32, i32, P(vp)]),
        "slar_cnn_destroy": (i32, [vp]),
        "slar_cnn_nparams": (i32, [vp]),
        "slar_cnn_set_params": (i32, [vp, vp, i32]),
        "slar_cnn_get_params": (i32, [vp, vp, i32]),
        "slar_cnn_forward": (i32, [vp, i32, i32, i32, vp, vp, vp]),
        "slar_cnn_grad": (i32, [vp, i32, i32, i32, vp, vp, vp, P(C.c_float), vp]),
        "slar_cnn_train_step": (i32, [vp, i32, i32, i32, vp, vp, C.c_float, P(C.c_float), vp]),
        "slar_record_krylov": (i32, [vp, vp, vp, i32]),
        "slar_recorded_pairs": (i32, [vp]),
        "slar_timing_enable": (i32, [vp, i32]),
        "slar_leaf_refine": (i32, [vp, i32]),
        "slar_timing_read": (i32, [vp, P(C.c_double)]),
        "slar_batch_create": (i32, [i32, P(Grid), i32, P(vp)]),
        "slar_batch_destroy": (i32, [vp]),
        "slar_batch_workspace": (vp, [vp, i32]),
        "slar_batch_cross_update": (i32, [vp, P(Frames), P(Adv), dbl, i32, i32, P(vp), P(LowRank),
                                          P(CrossInfo), vp]),
        "slar_batch_truncate": (i32, [vp, P(LowRank), dbl, i32, P(HT), P(Frames), P(i32), vp]),
        "slar_batch_efield": (i32, [vp, P(Frames), P(dbl), P(vp), P(vp), vp]),
        "slar_batch_get_config": (i32, [vp, P(i32)]),
        "slar_batch_set_config": (i32, [vp, P(i32)]),
        "slar_batch_tune": (i32, [vp, P(Frames), P(Adv), dbl, i32, i32, P(vp), P(LowRank), i32, vp]),
        "slar_batch_timing": (i32, [vp, P(C.c_double)]),
        "slar_batch_timing_reset": (i32, [vp]),
        "slar_macro_solve_system": (i32, [P(Grid), P(MacroSystem), dbl, dbl, i32, vp, vp, P(i32), vp, vp]),
        "slar_macro_rhs": (i32, [P(Grid), vp, vp, vp, vp]),
        "slar_cnn_correct": (i32, [P(Grid), vp, vp, vp, vp, vp, vp]),
        "slar_dirk3_tableau": (i32, [P(dbl), P(dbl)]),
        "slar_bdf_weights": (i32, [i32, P(dbl), P(dbl), P(dbl)]),
        "slar_macro_history": (i32, [vp, P(dbl), i32]),
        "slar_macro_fallbacks": (i32, [vp, P(i32)]),
        "slar_lomac_filter": (i32, [P(Grid), vp, vp, vp]),
        "slar_poisson_noalloc": (i32, [P(Grid), vp, dbl, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_str(s: int) -> str:
    return load().slar_status_str(int(s)).decode()


def _check(status, where, ok=(SLAR_OK,)):
    if status not in ok:
        raise SlarError(status, where)
    return status


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_grid(p) -> Grid:
    g = Grid()
    g.dx, g.dv = p.dx, p.dv
    for m in range(p.dx + p.dv):
        g.n[m] = int(p.n[m]); g.lo[m] = float(p.lo[m]); g.hi[m] = float(p.hi[m])
    return g


def slar_workspace_bytes(grid: Grid, rmax: int) -> int:
    n = C.c_size_t(0)
    _check(load().slar_workspace_bytes(C.byref(grid), int(rmax), C.byref(n)), "slar_workspace_bytes")
    return int(n.value)


class Workspace:
    """Library workspace; with ``work`` (a device tensor of at least
    slar_workspace_bytes bytes, 256-byte aligned) its device buffers are
    carved from that memory, which the object keeps alive."""

    def __init__(self, grid: Grid, rmax: int, work=None):
        self.grid = grid
        h = C.c_void_p()
        if work is None:
            _check(load().slar_workspace_create(C.byref(grid), int(rmax), C.byref(h)), "slar_workspace_create")
        else:
            nbytes = work.numel() * work.element_size()
            _check(load().slar_workspace_create_in(C.byref(grid), int(rmax), C.c_void_p(work.data_ptr()),
                                                   C.c_size_t(nbytes), C.byref(h)), "slar_workspace_create_in")
        self._work = work
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.slar_workspace_destroy(self.h)
            self.h = None


def make_ht(tensors: dict, d: int, dtype: int) -> HT:
    """tensors: {"leaves": [...], "B12", "B34", "root"} of contiguous device tensors."""
    H = HT()
    H.d = d
    H.dtype = dtype
    L = tensors["leaves"]
    for m in range(d):
        H.leaf[m] = L[m].data_ptr()
        H.rank[m] = L[m].shape[1]
    H.root = tensors["root"].data_ptr()
    if d == 4:
        H.B12 = tensors["B12"].data_ptr(); H.B34 = tensors["B34"].data_ptr()
        H.rank[4] = tensors["root"].shape[0]; H.rank[5] = tensors["root"].shape[1]
    H._keep = tensors
    return H


def make_adv(kind, tau, cv=1.0, E=None, E2=None, cE=(1.0, 0.0), order=3) -> Adv:
    a = Adv()
    a.kind, a.order, a.tau, a.cv = int(kind), int(order), float(tau), float(cv)
    a.E[0] = None if E is None else E.data_ptr()
    a.E[1] = None if E2 is None else E2.data_ptr()
    a.cE[0], a.cE[1] = float(cE[0]), float(cE[1])
    a._keep = (E, E2)          # the descriptor owns references to its tensors
    return a


def frames(X, P, r) -> Frames:
    f = Frames()
    f.r, f.ld = int(r), int(X.shape[1])
    f.X, f.P = X.data_ptr(), P.data_ptr()
    f._keep = (X, P)
    return f


# ------------------------------------------------------------ entry points
def slar_ht_sample(grid, H, adv, idx, out):
    _check(load().slar_ht_sample(C.byref(grid), C.byref(H), C.byref(adv), int(idx.shape[0]),
                                 _ptr(idx), _ptr(out), _stream()), "slar_ht_sample")


def slar_frames_from_ht(grid, H, F: Frames, ws):
    _check(load().slar_frames_from_ht(C.byref(grid), C.byref(H), C.byref(F), ws.h, _stream()),
           "slar_frames_from_ht")
    return F


def slar_frame_sample(grid, F, adv, dtype, idx, out, ws):
    _check(load().slar_frame_sample(C.byref(grid), C.byref(F), C.byref(adv), int(dtype),
                                    int(idx.shape[0]), _ptr(idx), _ptr(out), ws.h, _stream()),
           "slar_frame_sample")


def slar_cross_update(grid, src, adv, dtype, tol, kmax, probes, U, V, ws):
    lr = LowRank(0, U.data_ptr(), V.data_ptr())
    lr._keep = (U, V)
    info = CrossInfo()
    nprobe = 0 if probes is None else int(probes.shape[0])
    st = load().slar_cross_update(C.byref(grid), C.byref(src), C.byref(adv), int(dtype),
                                  float(tol), int(kmax), nprobe, _ptr(probes), C.byref(lr),
                                  C.byref(info), ws.h, _stream())
    _check(st, "slar_cross_update", ok=(SLAR_OK, SLAR_E_RANK_CAP))
    return lr, info, st


def slar_nested_cross(grid, src, adv, dtype, tol, kmax, probes, seed, out: HT, ws):
    """Nested HT cross of the SL-FD update (d = 4).  probes: host int32
    (m, 4) array, seed: 4 ints; out: HT of FP64 device buffers with the
    capacities documented in slar.h (ranks are written).  Returns
    (info, status); SLAR_E_NOCONV is returned, not raised."""
    import numpy as np
    pr = np.ascontiguousarray(np.asarray(probes, dtype=np.int32).reshape(-1, 4))
    sd = np.ascontiguousarray(np.asarray(seed, dtype=np.int32).reshape(4))
    info = NestedInfo()
    st = load().slar_nested_cross(C.byref(grid), C.byref(src), C.byref(adv), int(dtype), float(tol),
                                  int(kmax), int(pr.shape[0]), pr.ctypes.data_as(C.c_void_p),
                                  sd.ctypes.data_as(C.c_void_p), C.byref(out), C.byref(info), ws.h,
                                  _stream())
    _check(st, "slar_nested_cross", ok=(SLAR_OK, SLAR_E_NOCONV))
    return info, st


def slar_truncate(grid, lr, tol, rmax, out_ht: HT, ws):
    st = load().slar_truncate(C.byref(grid), C.byref(lr), float(tol), int(rmax), C.byref(out_ht),
                              ws.h, _stream())
    _check(st, "slar_truncate", ok=(SLAR_OK, SLAR_E_RANK_CAP))
    return st


def slar_moments(grid, F, M, ws):
    _check(load().slar_moments(C.byref(grid), C.byref(F), _ptr(M), ws.h, _stream()), "slar_moments")


def slar_poisson(grid, n_e, n_i, phi, E, ws):
    _check(load().slar_poisson(C.byref(grid), _ptr(n_e), float(n_i), _ptr(phi), _ptr(E), ws.h,
                               _stream()), "slar_poisson")


def slar_poisson_noalloc(grid, n_e, n_i, phi, E):
    """slar_poisson without a workspace or device allocation."""
    _check(load().slar_poisson_noalloc(C.byref(grid), _ptr(n_e), float(n_i), _ptr(phi), _ptr(E), _stream()),
           "slar_poisson_noalloc")
    return E


def slar_conserved(grid, F, n_i, U, ws):
    _check(load().slar_conserved(C.byref(grid), C.byref(F), float(n_i), _ptr(U), ws.h, _stream()),
           "slar_conserved")


def slar_lomac_prepare(grid, H, F, delta, n_i, ws):
    _check(load().slar_lomac_prepare(C.byref(grid), C.byref(H), C.byref(F), float(delta),
                                     float(n_i), ws.h, _stream()), "slar_lomac_prepare")


def slar_macro_solve(grid, U_n, U_nm1, dt, bdf, newton_tol, krylov_tol, precond, cnn, U_out, ws):
    iters = (C.c_int32 * 2)()
    st = load().slar_macro_solve(C.byref(grid), _ptr(U_n), _ptr(U_nm1), float(dt), int(bdf),
                                 float(newton_tol), float(krylov_tol), int(precond), cnn, _ptr(U_out),
                                 iters, ws.h, _stream())
    _check(st, "slar_macro_solve", ok=(SLAR_OK, SLAR_E_NOCONV))
    return st, (iters[0], iters[1])


def slar_macro_solve_system(grid, hist, stages, beta, newton_tol, krylov_tol, precond, cnn, U_out, ws):
    """hist: [(U_j, c_j)] (1..3), stages: [(R_j, d_j)] (0..3)."""
    S = MacroSystem()
    S.nhist = len(hist)
    for j, (U, c) in enumerate(hist):
        S.U[j] = U.data_ptr(); S.c[j] = float(c)
    S.nstage = len(stages)
    for j, (R, d) in enumerate(stages):
        S.R[j] = R.data_ptr(); S.d[j] = float(d)
    S.beta = float(beta)
    iters = (C.c_int32 * 2)()
    st = load().slar_macro_solve_system(C.byref(grid), C.byref(S), float(newton_tol), float(krylov_tol),
                                        int(precond), cnn, _ptr(U_out), iters, ws.h, _stream())
    _check(st, "slar_macro_solve_system", ok=(SLAR_OK, SLAR_E_NOCONV))
    return st, (iters[0], iters[1])


def slar_macro_history(ws):
    """Per-Newton records of the last macro solve: list of (rms, krylov,
    true relative linear residual, restarts)."""
    out = (C.c_double * (4 * 32))()
    n = load().slar_macro_history(ws.h, out, 32)
    if n < 0:
        raise SlarError(SLAR_E_INVAL, "slar_macro_history")
    return [tuple(out[4 * i: 4 * i + 4]) for i in range(min(n, 32))]


def slar_macro_fallbacks(ws):
    """(solves that fell back to plain GMRES since creation, last solve did)."""
    last = C.c_int32(0)
    n = load().slar_macro_fallbacks(ws.h, C.byref(last))
    if n < 0:
        raise SlarError(SLAR_E_INVAL, "slar_macro_fallbacks")
    return n, bool(last.value)


def slar_macro_rhs(grid, U, R_out, ws):
    _check(load().slar_macro_rhs(C.byref(grid), _ptr(U), _ptr(R_out), ws.h, _stream()), "slar_macro_rhs")
    return R_out


def slar_dirk3_tableau():
    A = (C.c_double * 9)()
    c = (C.c_double * 3)()
    _check(load().slar_dirk3_tableau(A, c), "slar_dirk3_tableau")
    return [[A[3 * i + j] for j in range(3)] for i in range(3)], [c[i] for i in range(3)]


def slar_bdf_weights(times):
    k = len(times) - 1
    t = (C.c_double * (k + 1))(*[float(x) for x in times])
    c = (C.c_double * max(k, 1))()
    beta = C.c_double()
    _check(load().slar_bdf_weights(int(k), t, c, C.byref(beta)), "slar_bdf_weights")
    return [c[j] for j in range(k)], beta.value


def slar_lomac_filter(grid, U, ws):
    _check(load().slar_lomac_filter(C.byref(grid), _ptr(U), ws.h, _stream()), "slar_lomac_filter")
    return U


def slar_lomac_project(grid, Fs, U_new, out: Frames, ws):
    _check(load().slar_lomac_project(C.byref(grid), C.byref(Fs), _ptr(U_new), C.byref(out), ws.h,
                                     _stream()), "slar_lomac_project")
    return out


# ------------------------------------------------------- learned preconditioner
def slar_cnn_correct(grid, cnn, v, U, z, ws):
    """z += rms(v) CNN(features(v, U)) in place (device [K][Nx] FP64)."""
    _check(load().slar_cnn_correct(C.byref(grid), cnn.handle, _ptr(v), _ptr(U), _ptr(z), ws.h, _stream()),
           "slar_cnn_correct")
    return z


class Cnn:
    """Handle of a device CNN (see slar.h); parameters as a host float32 array."""

    def __init__(self, channels, max_batch, max_pixels):
        self.channels = list(channels)
        arr = (C.c_int32 * len(channels))(*channels)
        h = C.c_void_p()
        _check(load().slar_cnn_create(len(channels) - 1, arr, int(max_batch), int(max_pixels),
                                      C.byref(h)), "slar_cnn_create")
        self.handle = h
        self.nparams = load().slar_cnn_nparams(h)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.slar_cnn_destroy(self.handle)
            self.handle = None

    def set_params(self, theta):
        import numpy as np
        t = np.ascontiguousarray(theta, dtype=np.float32)
        _check(load().slar_cnn_set_params(self.handle, t.ctypes.data_as(C.c_void_p), len(t)),
               "slar_cnn_set_params")

    def get_params(self):
        import numpy as np
        t = np.zeros(self.nparams, dtype=np.float32)
        _check(load().slar_cnn_get_params(self.handle, t.ctypes.data_as(C.c_void_p), len(t)),
               "slar_cnn_get_params")
        return t

    def forward(self, x, y):
        B, _, H, W = x.shape
        _check(load().slar_cnn_forward(self.handle, B, H, W, _ptr(x), _ptr(y), _stream()),
               "slar_cnn_forward")

    def grad(self, x, y):
        import numpy as np
        B, _, H, W = x.shape
        g = np.zeros(self.nparams, dtype=np.float32)
        loss = C.c_float()
        _check(load().slar_cnn_grad(self.handle, B, H, W, _ptr(x), _ptr(y),
                                    g.ctypes.data_as(C.c_void_p), C.byref(loss), _stream()),
               "slar_cnn_grad")
        return g, loss.value

    def train_step(self, x, y, lr):
        B, _, H, W = x.shape
        loss = C.c_float()
        _check(load().slar_cnn_train_step(self.handle, B, H, W, _ptr(x), _ptr(y), float(lr),
                                          C.byref(loss), _stream()), "slar_cnn_train_step")
        return loss.value


def slar_record_krylov(ws, feats, targs, capacity):
    _check(load().slar_record_krylov(ws.h, _ptr(feats), _ptr(targs), int(capacity)),
           "slar_record_krylov")


def slar_recorded_pairs(ws) -> int:
    return int(load().slar_recorded_pairs(ws.h))


def slar_leaf_refine(ws, on: bool):
    """Switch the refinement pass of the truncation's leaf bases."""
    _check(load().slar_leaf_refine(ws.h, 1 if on else 0), "slar_leaf_refine")


def slar_timing_enable(ws, on, every: int = 1):
    """on: False / True; every: time every n-th cross iteration."""
    _check(load().slar_timing_enable(ws.h, int(every) if on else 0), "slar_timing_enable")


def slar_timing_read(ws):
    out = (C.c_double * 8)()
    _check(load().slar_timing_read(ws.h, out), "slar_timing_read")
    keys = ("row_ms", "row_launches", "row_bytes", "col_ms", "col_launches", "col_bytes")
    return {k: out[i] for i, k in enumerate(keys)}


# ------------------------------------------------------------------ batches
def _array(T, items):
    arr = (T * len(items))(*items)
    arr._keep = [getattr(x, "_keep", None) for x in items]
    return arr


def _ptrs(tensors):
    arr = (C.c_void_p * len(tensors))(*[None if t is None else t.data_ptr() for t in tensors])
    arr._keep = list(tensors)
    return arr


class Batch:
    """Handle of a multi-instance batch (slar_batch_*)."""

    def __init__(self, grids, rmax: int):
        self.grids = list(grids)
        self.count = len(self.grids)
        h = C.c_void_p()
        arr = (Grid * self.count)(*self.grids)
        _check(load().slar_batch_create(self.count, arr, int(rmax), C.byref(h)), "slar_batch_create")
        self.h = h
        # views of the per-instance workspaces (owned by the batch)
        self.ws = [_BorrowedWorkspace(g, load().slar_batch_workspace(h, q)) for q, g in enumerate(self.grids)]

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.slar_batch_destroy(self.h)
            self.h = None

    def cross_update(self, src, advs, tol, kmax, probes, U, V):
        lrs = [LowRank(0, u.data_ptr(), v.data_ptr()) for u, v in zip(U, V)]
        out = _array(LowRank, lrs)
        info = (CrossInfo * self.count)()
        nprobe = 0 if probes is None else int(probes[0].shape[0])
        pp = None if probes is None else _ptrs(probes)
        st = load().slar_batch_cross_update(self.h, _array(Frames, src), _array(Adv, advs), float(tol),
                                            int(kmax), nprobe, pp, out, info, _stream())
        _check(st, "slar_batch_cross_update", ok=(SLAR_OK, SLAR_E_RANK_CAP))
        res = []
        for q in range(self.count):
            lr = LowRank(out[q].k, out[q].U, out[q].V)
            lr._keep = (U[q], V[q])
            res.append(lr)
        return res, list(info), st

    def truncate(self, lrs, tol, rmax, hts, frames_out=None):
        status = (C.c_int32 * self.count)()
        hts_arr = _array(HT, hts)
        fr = None if frames_out is None else _array(Frames, frames_out)
        st = load().slar_batch_truncate(self.h, _array(LowRank, lrs), float(tol), int(rmax), hts_arr, fr,
                                        status, _stream())
        _check(st, "slar_batch_truncate", ok=(SLAR_OK, SLAR_E_RANK_CAP))
        for q in range(self.count):             # ranks written by the library
            hts[q].rank[:] = hts_arr[q].rank[:]
            if frames_out is not None:
                frames_out[q].r = fr[q].r
        return list(status)

    def efield(self, F, n_i, M, E):
        nis = (C.c_double * self.count)(*[float(x) for x in n_i])
        _check(load().slar_batch_efield(self.h, _array(Frames, F), nis, _ptrs(M), _ptrs(E), _stream()),
               "slar_batch_efield")

    def config(self):
        cfg = (C.c_int32 * 8)()
        _check(load().slar_batch_get_config(self.h, cfg), "slar_batch_get_config")
        keys = ("grid", "group", "chunk", "team_r16", "team_r32", "team_rmax", "captures")
        return {k: int(cfg[i]) for i, k in enumerate(keys)}

    def set_config(self, grid, group, chunk, teams=(16, 16, 16)):
        cfg = (C.c_int32 * 8)(int(grid), int(group), int(chunk), *[int(t) for t in teams], 0, 0)
        _check(load().slar_batch_set_config(self.h, cfg), "slar_batch_set_config")

    def tune(self, src, advs, tol, kmax, probes, U, V, reps=2):
        lrs = [LowRank(0, u.data_ptr(), v.data_ptr()) for u, v in zip(U, V)]
        nprobe = 0 if probes is None else int(probes[0].shape[0])
        pp = None if probes is None else _ptrs(probes)
        _check(load().slar_batch_tune(self.h, _array(Frames, src), _array(Adv, advs), float(tol), int(kmax),
                                      nprobe, pp, _array(LowRank, lrs), int(reps), _stream()),
               "slar_batch_tune")
        return self.config()

    def timing(self):
        out = (C.c_double * 4)()
        _check(load().slar_batch_timing(self.h, out), "slar_batch_timing")
        return {"cross_ms": out[0], "chunks": out[1], "iterations": out[2], "calls": out[3]}

    def timing_reset(self):
        _check(load().slar_batch_timing_reset(self.h), "slar_batch_timing_reset")


class _BorrowedWorkspace:
    """A workspace owned by a batch (usable with the one-instance calls)."""

    def __init__(self, grid, handle):
        if not handle:
            raise RuntimeError("slar_batch_workspace returned NULL")
        self.grid = grid
        self.h = C.c_void_p(handle)
