"""Pins of the network oracle (oracle/mlp_oracle.py): the FP64 gradient
against central finite differences of the loss, the BF16 rounding against
its definition, and the layout against an independent composition of the
layers."""

import numpy as np
import pytest

from oracle import mlp_oracle as M


def _data(rows=24, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 0.5, size=(rows, M.IN))
    t = rng.normal(0, 0.3, size=(rows, M.OUT))
    colw = np.ones(M.OUT)
    colw[-1] = 0.0
    colw[-2] = 2.5
    return x, t, colw


def test_fp64_gradient_matches_finite_differences():
    params = M.init_params(3) + 0.01
    x, t, colw = _data()
    loss, g = M.loss_grad(params, x, t, colw, scale=0.7, bf16=False)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(M.NPARAMS, 40, replace=False),
                          [bo for _, bo in M.OFFSETS], [wo for wo, _ in M.OFFSETS]])
    for k in idx:
        h = 1e-6
        a = params.copy()
        b = params.copy()
        a[k] += h
        b[k] -= h
        fd = (M.loss_grad(a, x, t, colw, 0.7, bf16=False)[0] -
              M.loss_grad(b, x, t, colw, 0.7, bf16=False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_forward_equals_explicit_composition():
    params = M.init_params(5)
    x, _, _ = _data(7, 2)
    W0 = params[:256 * 64].reshape(256, 64)
    b0 = params[256 * 64:256 * 64 + 256]
    h = x @ W0.T + b0
    h = h / (1 + np.exp(-h))
    o = 256 * 64 + 256
    for _ in range(2):
        W = params[o:o + 65536].reshape(256, 256)
        b = params[o + 65536:o + 65536 + 256]
        h = h @ W.T + b
        h = h / (1 + np.exp(-h))
        o += 65536 + 256
    W3 = params[o:o + 32 * 256].reshape(32, 256)
    b3 = params[o + 32 * 256:]
    assert b3.size == 32 and M.NPARAMS == o + 32 * 256 + 32 == 156448
    np.testing.assert_allclose(M.forward(params, x, bf16=False), h @ W3.T + b3, rtol=1e-13,
                               atol=1e-13)


def test_bf16_round_to_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, 1.0 + 2 ** -7,
                     -2.5, 3.0e38, 1e-40, 0.0])
    got = M.bf16_round(vals)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even -> 1 + 2^-6
    exp = np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0, 1.0 + 2 ** -7, -2.5, 2.9975474e38,
                    np.float32(1e-40), 0.0])
    np.testing.assert_allclose(got[:6], exp[:6], rtol=0, atol=0)
    assert abs(got[6] - 3.0e38) / 3.0e38 < 2 ** -8
    assert got[8] == 0.0
    # every result is representable in BF16 (low 16 bits zero)
    bits = got.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)


def test_bf16_gradient_is_close_to_fp64():
    """Rounding at the BF16 points moves the gradient by about 2^-8
    relative, no more."""
    params = M.init_params(7)
    x, t, colw = _data(64, 4)
    _, g64 = M.loss_grad(params, x, t, colw, bf16=False)
    _, g16 = M.loss_grad(params, x, t, colw, bf16=True)
    assert np.linalg.norm(g16 - g64) <= 0.05 * np.linalg.norm(g64)
