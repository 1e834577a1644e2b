"""Convolutional preconditioner network (oracle, FP64 NumPy).

Not part of the paper: a small periodic convolutional network used as a
learned right preconditioner of the Krylov solve of the macroscopic system
(the paper names preconditioning of that solve as future work, section 5).
Layers: 3x3 periodic cross-correlation
  out[o, y, x] = b[o] + sum_{c, dy, dx} w[o, c, dy, dx] in[c, y + dy - 1, x + dx - 1]
with tanh after every layer but the last.  Loss: mean squared error over
all output entries.  Parameters are packed per layer as w (Co, Ci, 3, 3)
then b (Co).

Parity: pinned by central finite differences of this forward pass.
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
