"""FP64 oracle of the warm-start network: a fully connected ReLU network, its mean-
squared-error loss, backpropagation and the Adam update.  TEST INFRASTRUCTURE ONLY
(see oracle/__init__).

The thesis has no learned component (its future-work chapter names learning-based
methods); this oracle is the textbook definition of each step, written with plain
matrix products so the GPU kernels can be checked against it:
  forward   a_0 = x,  z_l = a_{l-1} W_l^T + b_l,  a_l = max(z_l, 0) (hidden layers),
            y = z_L (linear output);
  loss      L = mean over batch and outputs of (y - t)^2;
  backward  d_L = dL/dy = 2 (y - t) / (B n_out);  dW_l = d_l^T a_{l-1};  db_l = sum_b d_l;
            d_{l-1} = (d_l W_l) * [a_{l-1} > 0];
  Adam      m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
            p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)   (Kingma & Ba 2015).
Parameters are one flat vector: for each layer W_l (out x in, row-major) then b_l.

`bf16=True` rounds both operands of every matrix product to bfloat16 (round to
nearest even) before multiplying in FP64: the kernels' bf16 mode feeds its matrix
cores exactly those values, so the ReLU decisions of both sides agree (a decision
taken in the kernel's precision), and only the fp32 accumulation differs.
"""
from __future__ import annotations

import numpy as np


def to_bf16(a):
    """Round values to the nearest bfloat16 (ties to even), returned as float64.

    bfloat16 is the upper half of an IEEE binary32 word, so rounding to nearest even
    adds 0x7FFF plus the lowest kept bit to the word and drops the low 16 bits; a
    finite value that rounds past the largest bfloat16 becomes infinity.  A NaN stays
    a NaN (the carry must not run into its exponent).  Float64 input is first
    rounded to float32, which is what the kernels hold before their conversion."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def _mm(a, b, bf16):
    return (to_bf16(a) @ to_bf16(b)) if bf16 else a @ b


def n_params(widths):
    return sum(widths[l + 1] * widths[l] + widths[l + 1] for l in range(len(widths) - 1))


def unpack(params, widths):
    out, off = [], 0
    for l in range(len(widths) - 1):
        i, o = widths[l], widths[l + 1]
        W = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((W, b))
    return out


def forward(params, widths, x, bf16=False):
    """Returns (y, activations) with activations[l] = a_l for l = 0..L-1."""
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    a = np.asarray(x, dtype=np.float64)
    acts = [a]
    for l, (W, b) in enumerate(layers):
        z = _mm(a, W.T, bf16) + b
        if l < len(layers) - 1:
            a = np.maximum(z, 0.0)
            acts.append(a)
        else:
            a = z
    return a, acts


def mse(y, t):
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, widths, acts, dy, bf16=False):
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    grads = []
    d = np.asarray(dy, dtype=np.float64)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a_prev = acts[l]
        grads.append((_mm(d.T, a_prev, bf16), d.sum(0)))
        if l > 0:
            d = _mm(d, W, bf16) * (a_prev > 0)
    grads.reverse()
    return np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])


def adam(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
