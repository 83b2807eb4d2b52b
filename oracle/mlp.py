"""FP64 reference of the MLP equation-of-state surrogate and of the
reduced-precision population codec.

TEST INFRASTRUCTURE ONLY (part of the oracle; see ``oracle/__init__.py``).

The surrogate maps (rho, e) to (T, P, c_s^2) of the van der Waals fluid; it
stands in for the caloric inversion (eq. lbm_temp; an iterative solve for a
general equation of state).  Network: 2 -> 64 -> 64 -> 3, ReLU hidden
activations (max(z, 0)), linear output.  Parameter vector layout (4547 values):
  W1[64][2], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]
(row j of W holds the weights into output unit j).
Inputs are min-max scaled to [-1, 1]; outputs are z-scored:
  xhat_d = 2 (x_d - lo_d) / (hi_d - lo_d) - 1,   y_k = yhat_k s_k + m_k.
Loss on a batch of B samples: L = 1/(3B) sum_b sum_k (yhat_bk - that_bk)^2
with that = (y_target - m) / s.  Optimiser: Adam.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 2, 64, 3
SIZES = [N_H * N_IN, N_H, N_H * N_H, N_H, N_OUT * N_H, N_OUT]
N_PARAMS = sum(SIZES)  # 4547


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    assert p.size == N_PARAMS
    o = np.cumsum([0] + SIZES)
    W1 = p[o[0]:o[1]].reshape(N_H, N_IN)
    b1 = p[o[1]:o[2]]
    W2 = p[o[2]:o[3]].reshape(N_H, N_H)
    b2 = p[o[3]:o[4]]
    W3 = p[o[4]:o[5]].reshape(N_OUT, N_H)
    b3 = p[o[5]:o[6]]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.reshape(-1), b1, W2.reshape(-1), b2, W3.reshape(-1), b3])


def normalize_inputs(x, lo, hi):
    """x: (B, 2) raw (rho, e); returns (B, 2) in [-1, 1]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return 2.0 * (np.asarray(x, dtype=np.float64) - lo) / (hi - lo) - 1.0


def forward(params, xn):
    """xn: (B, 2) normalised inputs; returns yhat (B, 3) and the activations."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    h1 = np.maximum(xn @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    y = h2 @ W3.T + b3
    return y, (xn, h1, h2)


def loss_grad(params, xn, tn):
    """MSE loss and its gradient with respect to the parameter vector."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    y, (x, h1, h2) = forward(params, xn)
    B = x.shape[0]
    r = y - tn
    L = np.sum(r * r) / (3.0 * B)
    dy = 2.0 * r / (3.0 * B)                 # dL/dyhat
    dW3 = dy.T @ h2
    db3 = dy.sum(0)
    dz2 = (dy @ W3) * (h2 > 0.0)             # ReLU' = 1 where the unit is active
    dW2 = dz2.T @ h1
    db2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (h1 > 0.0)
    dW1 = dz1.T @ x
    db1 = dz1.sum(0)
    return L, pack(dW1, db1, dW2, db2, dW3, db3)


def adam(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# Reduced-precision codec: FP32 -> BF16 / FP16, round to nearest, ties to even
# ---------------------------------------------------------------------------
def bf16_bits(x32):
    """BF16 bit patterns of float32 values, round-to-nearest-even on the 16
    discarded mantissa bits.  NaN inputs map to a quiet NaN."""
    u = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) & 0xFFFF
    nan = np.isnan(np.asarray(x32, dtype=np.float32))
    r = np.where(nan, 0x7FC0, r)
    return r.astype(np.uint16)


def bf16_to_f32(bits):
    return (np.asarray(bits, dtype=np.uint32) << 16).astype(np.uint32).view(np.float32)


def f16_bits(x32):
    """IEEE binary16 bit patterns (numpy's conversion rounds to nearest even)."""
    return np.asarray(x32, dtype=np.float32).astype(np.float16).view(np.uint16)


def f16_to_f32(bits):
    return np.asarray(bits, dtype=np.uint16).view(np.float16).astype(np.float32)


def encode_deviation(f32, ref32, kind):
    """Stored code of f - f_ref (the subtraction in FP32, then rounding)."""
    d = (np.asarray(f32, dtype=np.float32) - np.asarray(ref32, dtype=np.float32)).astype(np.float32)
    return bf16_bits(d) if kind == "bf16" else f16_bits(d)


def decode_deviation(bits, ref32, kind):
    d = bf16_to_f32(bits) if kind == "bf16" else f16_to_f32(bits)
    return (np.asarray(ref32, dtype=np.float32) + d).astype(np.float32)
