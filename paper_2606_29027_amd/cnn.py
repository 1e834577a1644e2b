"""Learned preconditioner: data collection, training and loading.

The network (kernels in csrc/cnn.hip) corrects the exact per-mode spectral
preconditioner inside flexible GMRES.  Training pairs come from the solver
itself: every flexible-GMRES step of a recording run stores the network
input for w = J z and the target (z - P_spec(w)) / rms(w); the network is
then fitted by Adam on the mean squared error with the library's own forward
and backward kernels.  Parameters are initialised from a seeded generator
with the last layer at zero (an untrained network is the spectral
preconditioner itself).
"""
from __future__ import annotations

import math
import os
import time

import numpy as np
import torch

from . import lib as L

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "cnn_precond.npz")
HIDDEN = 16


def channels(dv: int = 2, hidden: int = HIDDEN):
    K = dv + 2
    return [2 * K, hidden, hidden, K]


def init_params(chs, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    nl = len(chs) - 1
    for l in range(nl):
        ci, co = chs[l], chs[l + 1]
        if l == nl - 1:
            w = np.zeros((co, ci, 3, 3))
        else:
            w = rng.standard_normal((co, ci, 3, 3)) * math.sqrt(1.0 / (9 * ci))
        parts += [w.ravel(), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def make(max_batch: int = 8, max_pixels: int = 128 * 128, seed: int = 0) -> L.Cnn:
    net = L.Cnn(channels(), max_batch, max_pixels)
    net.set_params(init_params(net.channels, seed))
    return net


def collect(problems, steps: int, capacity: int, probes_seed: int = 7, skip=None):
    """Run recording solves (spectral preconditioner) and return a list of
    (features, targets, (H, W)) device tensors, one entry per problem.
    skip[i] steps of problem i run before recording starts (later-time
    systems, where the spectral part is less exact)."""
    import slar_inputs as SI
    from .solver import Solver
    out = []
    for i, p in enumerate(problems):
        Nx = int(np.prod(p.n[: p.dx])); Nv = int(np.prod(p.n[p.dx:]))
        K = p.dv + 2
        feats = torch.zeros((capacity, 2 * K, Nx), dtype=torch.float32, device="cuda")
        targs = torch.zeros((capacity, K, Nx), dtype=torch.float32, device="cuda")
        s = Solver(p, L.F32, probes=SI.probe_indices(Nx, Nv, 64, probes_seed), precond=1)
        s.set_initial(SI.initial_ht(p))
        for _ in range(skip[i] if skip else 0):
            s.step()
        L.slar_record_krylov(s.ws, feats, targs, capacity)
        for _ in range(steps):
            s.step()
            if L.slar_recorded_pairs(s.ws) >= capacity:
                break
        n = L.slar_recorded_pairs(s.ws)
        L.slar_record_krylov(s.ws, None, None, 0)
        H, W = p.n[0], p.n[1]
        out.append((feats[:n].reshape(n, 2 * K, H, W).contiguous(),
                    targs[:n].reshape(n, K, H, W).contiguous(), (H, W)))
        del s
    return out


def train(net: L.Cnn, data, iters: int = 300, batch: int = 8, lr: float = 2e-3, seed: int = 0):
    """Adam on the recorded pairs; returns the loss history."""
    rng = np.random.default_rng(seed)
    hist = []
    for it in range(iters):
        feats, targs, _ = data[it % len(data)]
        n = feats.shape[0]
        if n == 0:
            continue
        idx = torch.as_tensor(rng.choice(n, size=min(batch, n), replace=False), device="cuda")
        x = feats.index_select(0, idx).contiguous()
        y = targs.index_select(0, idx).contiguous()
        hist.append(net.train_step(x, y, lr))
    return hist


def save(net: L.Cnn, path: str = WEIGHTS, meta: dict | None = None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=net.get_params(), channels=np.array(net.channels),
             **({k: np.array(v) for k, v in (meta or {}).items()}))


def load_trained(p=None, path: str = WEIGHTS, train_if_missing: bool = True) -> L.Cnn:
    """The committed trained network, or a freshly trained one (cfg-2/3-type
    problems) if no weight file is present."""
    net = make()
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        net.set_params(z["params"])
        return net
    if not train_if_missing:
        raise FileNotFoundError(path)
    data = collect(training_problems(), steps=150, capacity=200, skip=TRAINING_SKIP)
    train(net, data, iters=1500)
    return net


def training_problems():
    """Newton systems of the 2D2V weak Landau (64^4) and two-stream (128^4)
    workloads."""
    import slar_inputs as SI
    return [SI.config("landau2d"), SI.config("twostream2d")]


# steps run before recording: weak Landau from t = 4, two-stream from t = 15
# (the growing mode has left the linear regime's start-up)
TRAINING_SKIP = (20, 150)
