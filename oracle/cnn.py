"""Convolutional preconditioner network (oracle, FP64 NumPy).

Not part of the paper: a small periodic convolutional network used as a
learned right preconditioner of the Krylov solve of the macroscopic system
(the paper names preconditioning of that solve as future work, section 5).
Layers: 3x3 periodic cross-correlation
  out[o, y, x] = b[o] + sum_{c, dy, dx} w[o, c, dy, dx] in[c, y + dy - 1, x + dx - 1]
with tanh after every layer but the last.  Loss: mean squared error over
all output entries.  Parameters are packed per layer as w (Co, Ci, 3, 3)
then b (Co).

Network input and target inside the Krylov solve (K = d_v + 2 conserved
components on the N_x-point spatial grid):
  input  = [v / rms(v) ; (U_c - mean U_c) / std U_c for each c]  (2K channels)
  output correction z = P_spec(v) + rms(v) net(input),
  training target (z - P_spec(w)) / rms(w) for a recorded pair (w = J z, z),
with rms(v) over all K N_x entries and mean/std per channel of U.

Parity: the network is pinned by central finite differences of this forward
pass; the input and target definitions by their invariants (standardised U
channels, unit-rms residual channels, invariance under scaling of v).
"""
from __future__ import annotations

import numpy as np


def unpack(theta: np.ndarray, shapes):
    out = []
    o = 0
    for ci, co in shapes:
        w = theta[o: o + co * ci * 9].reshape(co, ci, 3, 3); o += co * ci * 9
        b = theta[o: o + co]; o += co
        out.append((w, b))
    return out


def nparams(shapes) -> int:
    return sum(co * ci * 9 + co for ci, co in shapes)


def conv(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x (B, Ci, H, W) -> (B, Co, H, W), periodic."""
    out = np.zeros((x.shape[0], w.shape[0]) + x.shape[2:])
    for dy in range(3):
        for dx in range(3):
            xs = np.roll(np.roll(x, -(dy - 1), axis=2), -(dx - 1), axis=3)
            out += np.einsum("oc,bchw->bohw", w[:, :, dy, dx], xs)
    return out + b[None, :, None, None]


def forward(theta, shapes, x):
    acts = [x]
    a = x
    layers = unpack(theta, shapes)
    for li, (w, b) in enumerate(layers):
        z = conv(a, w, b)
        a = np.tanh(z) if li < len(layers) - 1 else z
        acts.append(a)
    return a, acts


def loss(theta, shapes, x, y) -> float:
    out, _ = forward(theta, shapes, x)
    return float(np.mean((out - y) ** 2))


def grad(theta, shapes, x, y):
    """Gradient of the mean squared error with respect to the parameters."""
    out, acts = forward(theta, shapes, x)
    layers = unpack(theta, shapes)
    g = 2.0 * (out - y) / out.size
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        w, b = layers[li]
        if li < len(layers) - 1:
            g = g * (1.0 - acts[li + 1] ** 2)
        a_in = acts[li]
        gw = np.zeros_like(w)
        for dy in range(3):
            for dx in range(3):
                xs = np.roll(np.roll(a_in, -(dy - 1), axis=2), -(dx - 1), axis=3)
                gw[:, :, dy, dx] = np.einsum("bohw,bchw->oc", g, xs)
        gb = g.sum(axis=(0, 2, 3))
        grads.append((gw, gb))
        # gradient w.r.t. the layer input: transpose correlation
        gin = np.zeros_like(a_in)
        for dy in range(3):
            for dx in range(3):
                t = np.einsum("oc,bohw->bchw", w[:, :, dy, dx], g)
                gin += np.roll(np.roll(t, dy - 1, axis=2), dx - 1, axis=3)
        g = gin
    grads.reverse()
    return np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])


def features(v: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Network input for residual v and state U, both (K, H, W): (2K, H, W).
    The std of a U channel gets 1e-12 |mean| + 1e-300 added (a constant
    channel maps to zero instead of dividing by zero)."""
    rms = np.sqrt(np.mean(v ** 2))
    vin = v / rms if rms > 0.0 else np.zeros_like(v)
    mean = U.mean(axis=(1, 2), keepdims=True)
    std = np.sqrt(np.maximum((U ** 2).mean(axis=(1, 2), keepdims=True) - mean ** 2, 0.0))
    std = std + 1e-12 * np.abs(mean) + 1e-300
    return np.concatenate([vin, (U - mean) / std], axis=0)


def target(z: np.ndarray, pw: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Training target for the pair (w = J z, z) with P_spec(w) = pw."""
    rms = np.sqrt(np.mean(w ** 2))
    return (z - pw) / rms if rms > 0.0 else np.zeros_like(z)


def apply(theta, shapes, v: np.ndarray, U: np.ndarray, pv: np.ndarray) -> np.ndarray:
    """Preconditioned vector z = P_spec(v) + rms(v) net(features(v, U)),
    with P_spec(v) = pv given."""
    out, _ = forward(theta, shapes, features(v, U)[None])
    return pv + np.sqrt(np.mean(v ** 2)) * out[0]
