"""FP64 oracle of the learned flexible-GMRES stage: a small circular CNN.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network maps a normalised Krylov vector v / ||v|| (real and imaginary
parts as two channels on the n x n grid) to an approximation of the
sparsifying preconditioner's output M v / ||v||.  Layers: 3 x 3
cross-correlations with circular (periodic) padding, no bias, ReLU after
every layer but the last; channels 2 -> 32 -> 32 -> 32 -> 32 -> 32 -> 2.
Training minimises the mean over a batch of ||net(x) - t||^2 / ||t||^2 with
Adam (Kingma and Ba).  Everything is written out with numpy loops over the
nine taps; no blocking or fusion.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (2, 32, 32, 32, 32, 32, 2)
TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def conv_forward(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """y[b, o, i, j] = sum_{c, dy, dx} w[o, c, dy+1, dx+1] x[b, c, (i+dy) mod H, (j+dx) mod W]."""
    B, Cin, H, W = x.shape
    Cout = w.shape[0]
    y = np.zeros((B, Cout, H, W))
    for dy, dx in TAPS:
        xs = np.roll(x, shift=(-dy, -dx), axis=(2, 3))          # xs[..., i, j] = x[..., i+dy, j+dx]
        y += np.einsum("oc,bchw->bohw", w[:, :, dy + 1, dx + 1], xs)
    return y


def conv_backward_data(gy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient of conv_forward w.r.t. x: gx[b,c,i,j] = sum w[o,c,dy+1,dx+1] gy[b,o,i-dy,j-dx]."""
    gx = np.zeros((gy.shape[0], w.shape[1]) + gy.shape[2:])
    for dy, dx in TAPS:
        gys = np.roll(gy, shift=(dy, dx), axis=(2, 3))           # gys[..., i, j] = gy[..., i-dy, j-dx]
        gx += np.einsum("oc,bohw->bchw", w[:, :, dy + 1, dx + 1], gys)
    return gx


def conv_backward_weight(gy: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Gradient w.r.t. w: gw[o,c,dy+1,dx+1] = sum_{b,i,j} gy[b,o,i,j] x[b,c,i+dy,j+dx]."""
    gw = np.zeros((gy.shape[1], x.shape[1], 3, 3))
    for dy, dx in TAPS:
        xs = np.roll(x, shift=(-dy, -dx), axis=(2, 3))
        gw[:, :, dy + 1, dx + 1] = np.einsum("bohw,bchw->oc", gy, xs)
    return gw


def init_weights(seed: int, channels=CHANNELS):
    """He-style normal initialisation, one (Cout, Cin, 3, 3) array per layer."""
    rng = np.random.default_rng(seed)
    ws = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        ws.append(rng.standard_normal((cout, cin, 3, 3)) * np.sqrt(2.0 / (9 * cin)))
    return ws


def forward(ws, x):
    """Returns the output and the list of layer inputs / pre-activations for backward."""
    acts = [x]
    pre = []
    h = x
    for li, w in enumerate(ws):
        z = conv_forward(h, w)
        pre.append(z)
        h = np.maximum(z, 0.0) if li < len(ws) - 1 else z
        acts.append(h)
    return h, acts, pre


def loss(y: np.ndarray, t: np.ndarray) -> float:
    """Mean over the batch of ||y - t||^2 / ||t||^2."""
    num = np.sum((y - t) ** 2, axis=(1, 2, 3))
    den = np.sum(t ** 2, axis=(1, 2, 3))
    return float(np.mean(num / den))


def loss_grad(y: np.ndarray, t: np.ndarray) -> np.ndarray:
    den = np.sum(t ** 2, axis=(1, 2, 3))
    return 2.0 * (y - t) / den[:, None, None, None] / y.shape[0]


def backward(ws, acts, pre, gy):
    """Gradients of the loss w.r.t. every weight array, given dL/dy."""
    grads = [None] * len(ws)
    g = gy
    for li in range(len(ws) - 1, -1, -1):
        if li < len(ws) - 1:
            g = g * (pre[li] > 0)
        grads[li] = conv_backward_weight(g, acts[li])
        if li > 0:
            g = conv_backward_data(g, ws[li])
    return grads


class Adam:
    """Adam with bias correction (lr, beta1, beta2, eps as in Kingma and Ba)."""

    def __init__(self, shapes, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros(s) for s in shapes]
        self.v = [np.zeros(s) for s in shapes]
        self.t = 0

    def step(self, ws, grads):
        self.t += 1
        out = []
        for i, (w, g) in enumerate(zip(ws, grads)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * g * g
            mh = self.m[i] / (1 - self.b1 ** self.t)
            vh = self.v[i] / (1 - self.b2 ** self.t)
            out.append(w - self.lr * mh / (np.sqrt(vh) + self.eps))
        return out


def to_channels(v: np.ndarray) -> np.ndarray:
    """Complex grid functions (B, n, n) -> real (B, 2, n, n)."""
    return np.stack([v.real, v.imag], axis=1)


def from_channels(x: np.ndarray) -> np.ndarray:
    return x[:, 0] + 1j * x[:, 1]
