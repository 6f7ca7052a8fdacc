"""Plain FP64 reference of the surrogate network (forward, weighted squared
error, backward) for checking the device kernels.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.  The network maps 64
inputs through three hidden layers of 256 SiLU units to 32 outputs; the
parameter vector is laid out as W0[256][64] b0 W1[256][256] b1 W2[256][256]
b2 W3[32][256] b3 (W row-major as W[out][in]).

With ``bf16=True`` the quantities the device keeps in BF16 are rounded to
BF16 (round to nearest even) at the same points: inputs, weights, hidden
activations, the output-error gradient and the back-propagated
pre-activation gradients.  Everything else is FP64.  With ``bf16=False``
the network is plain FP64, which the finite-difference pins check.

SiLU: s(z) = z / (1 + e^-z), s'(z) = sigma(z) (1 + z (1 - sigma(z))).
"""

from __future__ import annotations

import numpy as np

IN, HID, OUT = 64, 256, 32
SHAPES = [(HID, IN), (HID, HID), (HID, HID), (OUT, HID)]


def offsets():
    """(weight offset, bias offset) of each layer in the parameter vector."""
    out, o = [], 0
    for (a, b) in SHAPES:
        out.append((o, o + a * b))
        o += a * b + a
    return out, o


OFFSETS, NPARAMS = offsets()


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params):
    params = np.asarray(params, dtype=np.float64)
    layers = []
    for (wo, bo), (a, b) in zip(OFFSETS, SHAPES):
        layers.append((params[wo:wo + a * b].reshape(a, b), params[bo:bo + a]))
    return layers


def _silu(z):
    return z / (1.0 + np.exp(-z))


def _dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, bf16: bool = True, keep: bool = False):
    """Outputs y[rows][32]; with keep, also the per-layer inputs and
    pre-activations."""
    r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(params)
    h = r(x)
    acts, zs = [h], []
    for L, (W, b) in enumerate(layers):
        z = h @ r(W).T + b
        if L < 3:
            zs.append(z)
            h = r(_silu(z))
            acts.append(h)
        else:
            y = z
    if keep:
        return y, acts, zs
    return y


def loss_grad(params, x, targets, colw, scale: float = 1.0, bf16: bool = True):
    """(loss, gradient) of scale * sum_r sum_c colw[c] (y - t)^2."""
    r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(params)
    y, acts, zs = forward(params, x, bf16, keep=True)
    d = y - targets
    loss = scale * float(np.sum(colw[None, :] * d * d))
    dz = r(2.0 * colw[None, :] * d * scale)
    grad = np.zeros(NPARAMS)
    for L in range(3, -1, -1):
        W, _ = layers[L]
        wo, bo = OFFSETS[L]
        a_in = acts[L]
        grad[wo:wo + W.size] = (dz.T @ a_in).ravel()
        grad[bo:bo + W.shape[0]] = dz.sum(0)
        if L == 0:
            break
        dz = r((dz @ r(W)) * _dsilu(zs[L - 1]))
    return loss, grad


def init_params(seed: int = 0):
    """The initialisation the training driver uses: W ~ U(-a, a) with
    a = sqrt(6 / (in + out)) (Glorot), zero biases."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAMS)
    for (wo, bo), (a, b) in zip(OFFSETS, SHAPES):
        lim = np.sqrt(6.0 / (a + b))
        p[wo:wo + a * b] = rng.uniform(-lim, lim, size=a * b)
    return p
