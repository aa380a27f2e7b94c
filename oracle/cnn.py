"""FP64 reference of the learned force closure (test infrastructure only).

The closure is a small 3D convolutional network that maps the local
state of a binary mixture to the force densities N_a = n_a Phi_a of the
kinetic equation (Sec. 2, eq. evolution; Sec. 3, eq. splitforce):

  input  x  [14][Z][Y][X]: (n_0, n_1), (j_0, j_1) and the pressure gradients
                           of n_0 and n_1, each after affine scaling
  layers    4 convolutions with 3x3x3 kernels on the periodic lattice,
            channels 14 -> 32 -> 32 -> 32 -> 6, SiLU after the first three
  output y  [6][Z][Y][X]:  N_0 and N_1 (three components each) after scaling

Convolution (cross-correlation, periodic):
  y[o, r] = b[o] + sum_i sum_{d in {-1,0,1}^3} W[o, i, d + 1] x[i, r + d]
SiLU: s(z) = z / (1 + exp(-z)).
Loss: mean squared error over all outputs.
Adam: first/second moment estimates with bias correction.

Plain loops over the 27 taps with numpy rolls; no reordering beyond that.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
CHANNELS = (14, 32, 32, 32, 6)


def shift(x: np.ndarray, d) -> np.ndarray:
    """x[..., z + dz, y + dy, x + dx] on the periodic grid."""
    dz, dy, dx = d
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(-3, -2, -1))


def conv3d(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x [Ci][Z][Y][X], W [Co][Ci][3][3][3], b [Co] -> [Co][Z][Y][X]."""
    Co = W.shape[0]
    y = np.zeros((Co,) + x.shape[1:])
    for d in TAPS:
        w = W[:, :, d[0] + 1, d[1] + 1, d[2] + 1]           # [Co][Ci]
        y += np.tensordot(w, shift(x, d), axes=([1], [0]))
    return y + b[:, None, None, None]


def conv3d_dgrad(gy: np.ndarray, W: np.ndarray) -> np.ndarray:
    """d loss / d x from d loss / d y:  gx[i, r] = sum_o sum_d W[o, i, d] gy[o, r - d]."""
    Ci = W.shape[1]
    gx = np.zeros((Ci,) + gy.shape[1:])
    for d in TAPS:
        w = W[:, :, d[0] + 1, d[1] + 1, d[2] + 1]
        gx += np.tensordot(w, shift(gy, (-d[0], -d[1], -d[2])), axes=([0], [0]))
    return gx


def conv3d_wgrad(gy: np.ndarray, x: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """d loss / d W [Co][Ci][3][3][3] and d loss / d b [Co]."""
    Co, Ci = gy.shape[0], x.shape[0]
    gW = np.zeros((Co, Ci, 3, 3, 3))
    for d in TAPS:
        xs = shift(x, d)
        gW[:, :, d[0] + 1, d[1] + 1, d[2] + 1] = np.tensordot(gy, xs, axes=([1, 2, 3], [1, 2, 3]))
    return gW, gy.sum(axis=(1, 2, 3))


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def init_params(seed: int = 0, channels=CHANNELS) -> List[Dict[str, np.ndarray]]:
    """He-style initialisation (uniform, fan-in 27 Ci)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    layers = []
    for ci, co in zip(channels[:-1], channels[1:]):
        lim = np.sqrt(6.0 / (27 * ci))
        layers.append({"W": rng.uniform(-lim, lim, size=(co, ci, 3, 3, 3)), "b": np.zeros(co)})
    return layers


def forward(layers, x):
    """Returns the output and the per-layer caches (input, pre-activation)."""
    caches = []
    h = x
    for l, L in enumerate(layers):
        z = conv3d(h, L["W"], L["b"])
        caches.append((h, z))
        h = silu(z) if l < len(layers) - 1 else z
    return h, caches


def backward(layers, caches, gy):
    """Gradients of every W and b given d loss / d output; also d loss / d input."""
    grads = [None] * len(layers)
    g = gy
    for l in range(len(layers) - 1, -1, -1):
        h, z = caches[l]
        if l < len(layers) - 1:
            g = g * silu_grad(z)
        gW, gb = conv3d_wgrad(g, h)
        grads[l] = {"W": gW, "b": gb}
        g = conv3d_dgrad(g, layers[l]["W"])
    return grads, g


def mse(y, t):
    return float(np.mean((y - t) ** 2)), 2.0 * (y - t) / y.size


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (in place on p, m, v); t is the 1-based step count."""
    m *= b1
    m += (1 - b1) * g
    v *= b2
    v += (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p -= lr * mh / (np.sqrt(vh) + eps)
