"""Oracle 3D convolutional preconditioner network, forward and backward, FP64.

Part of the CPU oracle (test infrastructure only).

The paper names no preconditioner.  This is the learned preconditioner of the
build: three periodic 3x3x3 convolutions (3 -> 16 -> 16 -> 2 channels, with
bias), SiLU between them.  Input channels for one band are
[Re r~, Im r~, h^2 (V_loc - theta)] with r~ = r / ||r|| * sqrt(Ng); the two
output channels are the real and imaginary parts of the correction.

Convolution is cross-correlation with circular padding:
    out[o, x] = b[o] + sum_i sum_{d in {-1,0,1}^3} w[o, i, d] * in[i, x + d],
written with 27 ``np.roll`` shifts, and its backward pass is derived by hand:
    dL/db[o]       = sum_x g[o, x]
    dL/dw[o, i, d] = sum_x g[o, x] in[i, x + d]
    dL/din[i, y]   = sum_o sum_d w[o, i, d] g[o, y - d].
SiLU is z * sigmoid(z).  The loss of one pair (t_hat, t) is
||t_hat/||t_hat|| - t/||t|| ||^2, invariant to the scale of either.
Adam follows Kingma and Ba (2015).
"""
from __future__ import annotations

import math

import numpy as np

OFFSETS = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)]
CHANNELS = (3, 16, 16, 2)


def shift(a: np.ndarray, d) -> np.ndarray:
    """s[..., x] = a[..., x + d] (periodic) over the last three axes."""
    return np.roll(a, shift=(-d[0], -d[1], -d[2]), axis=(-3, -2, -1))


def conv3d(inp: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """inp (Cin, n, n, n), w (Cout, Cin, 3, 3, 3), b (Cout,)."""
    cout = w.shape[0]
    out = np.zeros((cout,) + inp.shape[1:], dtype=np.float64)
    for d in OFFSETS:
        s = shift(inp, d)
        wd = w[:, :, d[0] + 1, d[1] + 1, d[2] + 1]  # (Cout, Cin)
        out += np.tensordot(wd, s, axes=([1], [0]))
    return out + b[:, None, None, None]


def conv3d_backward(inp: np.ndarray, w: np.ndarray, g: np.ndarray):
    """Returns (dinp, dw, db) for out = conv3d(inp, w, b) and dL/dout = g."""
    dw = np.zeros_like(w)
    dinp = np.zeros_like(inp)
    for d in OFFSETS:
        s = shift(inp, d)
        dw[:, :, d[0] + 1, d[1] + 1, d[2] + 1] = np.tensordot(g, s, axes=([1, 2, 3], [1, 2, 3]))
        wd = w[:, :, d[0] + 1, d[1] + 1, d[2] + 1]
        # contribution to dinp at y from g at y - d
        gd = shift(g, (-d[0], -d[1], -d[2]))
        dinp += np.tensordot(wd, gd, axes=([0], [0]))
    db = g.sum(axis=(1, 2, 3))
    return dinp, dw, db


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def init_params(seed: int = 2, channels=CHANNELS):
    """Kaiming-uniform weights (fan_in = Cin * 27) and zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        bound = math.sqrt(6.0 / (cin * 27))
        w = rng.uniform(-bound, bound, size=(cout, cin, 3, 3, 3))
        params.append((w, np.zeros(cout)))
    return params


def round_bf16(a) -> np.ndarray:
    """Nearest bfloat16 of each value, ties to even, returned as float64.

    bfloat16 is the upper half of an IEEE binary32 (sign, 8 exponent bits,
    7 fraction bits): the value is first rounded to binary32, then its lower
    16 bits are rounded away (round half to even on bit 16).  NaN stays NaN.
    """
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = np.where(nan, ((u >> 16) | 0x40) & 0xFFFF, r)
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def forward(params, x: np.ndarray, bf16: bool = False):
    """Returns (output, cache) for one sample x (3, n, n, n).  With ``bf16``
    every layer's input and weights are rounded to bfloat16 first (the
    matrix-core arithmetic of the GPU network; products and sums stay exact
    here, bias and SiLU unrounded)."""
    acts = [x]
    pre = []
    h = x
    for k, (w, b) in enumerate(params):
        if bf16:
            z = conv3d(round_bf16(h), round_bf16(w), b)
        else:
            z = conv3d(h, w, b)
        pre.append(z)
        h = silu(z) if k < len(params) - 1 else z
        acts.append(h)
    return h, (acts, pre)


def forward_residual(params, x: np.ndarray):
    """Residual variant: output = net(x) + x[:2] (the network corrects its
    first two input channels).  The gradient with respect to the parameters
    is that of ``forward`` for the same output gradient."""
    out, cache = forward(params, x)
    return out + x[:2], cache


def backward(params, cache, gout: np.ndarray, bf16: bool = False):
    """Gradients [(dw, db), ...] and d input for dL/doutput = gout.  With
    ``bf16`` the two operands of every convolution product (the layer input
    and the output gradient for dw; the weights and the output gradient for
    d input) are rounded to bfloat16 first; db sums the unrounded gradient."""
    acts, pre = cache
    grads = [None] * len(params)
    g = gout
    for k in range(len(params) - 1, -1, -1):
        if k < len(params) - 1:
            g = g * silu_grad(pre[k])
        w, _ = params[k]
        if bf16:
            dinp, dw, _ = conv3d_backward(round_bf16(acts[k]), round_bf16(w), round_bf16(g))
            db = g.sum(axis=(1, 2, 3))
        else:
            dinp, dw, db = conv3d_backward(acts[k], w, g)
        grads[k] = (dw, db)
        g = dinp
    return grads, g


def normalised_loss(pred: np.ndarray, target: np.ndarray):
    """Returns (loss, dloss/dpred) for ||p/||p|| - t/||t|| ||^2."""
    pn = math.sqrt(float(np.sum(pred * pred)))
    tn = math.sqrt(float(np.sum(target * target)))
    u = pred / pn
    v = target / tn
    diff = u - v
    loss = float(np.sum(diff * diff))
    gu = 2.0 * diff
    gp = (gu - u * float(np.sum(u * gu))) / pn
    return loss, gp


def adam_update(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (returns new p, m, v); t counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def make_input(r: np.ndarray, V: np.ndarray, theta: float, n: int, h: float) -> np.ndarray:
    """Network input for one residual r (Ng complex): (3, n, n, n)."""
    Ng = n ** 3
    rn = r / np.linalg.norm(r) * math.sqrt(Ng)
    x = np.empty((3, n, n, n))
    x[0] = np.real(rn).reshape(n, n, n)
    x[1] = np.imag(rn).reshape(n, n, n)
    x[2] = (h * h * (V - theta)).reshape(n, n, n)
    return x
