"""Oracle: the child-patch predictor network of the learned adjacent zone.

TEST INFRASTRUCTURE ONLY (see ``oracle/grid.py``).  Not from the paper: the paper's adjacent
zone (Sec. 2.3) adds the children of every significant point; the learned mask replaces that
blanket rule by a small network that proposes which child patches are needed.

Network (plain definition, FP64):
    h1 = relu(x W1 + b1)      x: 64 features,  W1: 64 x 128
    h2 = relu(h1 W2 + b2)     W2: 128 x 128
    z  = h2 W3 + b3           W3: 128 x 4
    p  = sigmoid(z)           probability that child patch c (c = 0..3) is needed
Loss: mean over samples and the 4 outputs of the binary cross-entropy
    l(z, y) = -(y log p + (1 - y) log(1 - p)) = softplus(z) - y z.
Parameters are one flat vector in the order W1 (row-major, [in][out]), b1, W2, b2, W3, b3.

Optimiser: Adam (Kingma & Ba 2015), bias-corrected,
    m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
    theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

``emulate_bf16=True`` rounds, as the GPU does, the operands of every matrix product to bfloat16
(round to nearest even): x, the weights, the hidden activations, and in the backward pass the
output error and the back-propagated errors; sums stay in FP64 here.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 64, 128, 4
SHAPES = [(N_IN, N_H), (N_H,), (N_H, N_H), (N_H,), (N_H, N_OUT), (N_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)


def bf16(a):
    """Round FP64/FP32 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    r = ((bits + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(np.asarray(theta[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def _r(a, on):
    return bf16(a) if on else a


def forward(theta, X, emulate_bf16=False):
    """Logits z (n x 4) and the activations needed by the backward pass."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    e = emulate_bf16
    x = _r(X, e)
    a1 = x @ _r(W1, e) + b1
    h1 = np.maximum(a1, 0.0)
    a2 = _r(h1, e) @ _r(W2, e) + b2
    h2 = np.maximum(a2, 0.0)
    z = _r(h2, e) @ _r(W3, e) + b3
    return z, (x, a1, h1, a2, h2)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def loss(theta, X, Y, emulate_bf16=False):
    z, _ = forward(theta, X, emulate_bf16)
    return float(np.mean(np.logaddexp(0.0, z) - Y * z))


def grad(theta, X, Y, emulate_bf16=False):
    """Gradient of `loss` with respect to the flat parameter vector (backpropagation)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    e = emulate_bf16
    z, (x, a1, h1, a2, h2) = forward(theta, X, e)
    n = X.shape[0]
    dz = (sigmoid(z) - Y) / (n * N_OUT)          # d loss / d z
    dzr = _r(dz, e)
    gW3 = _r(h2, e).T @ dzr
    gb3 = dz.sum(0)
    dh2 = (dzr @ _r(W3, e).T) * (a2 > 0)
    dh2r = _r(dh2, e)
    gW2 = _r(h1, e).T @ dh2r
    gb2 = dh2.sum(0)
    dh1 = (dh2r @ _r(W2, e).T) * (a1 > 0)
    dh1r = _r(dh1, e)
    gW1 = x.T @ dh1r
    gb1 = dh1.sum(0)
    return pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
