"""FP64 numpy oracle of the surrogate's convolution layers.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg).

A layer maps an image batch x[n, h, w, ci] on a periodic grid to
    y[n, h, w, co] = b[co] + sum_{t, ci} x[n, h + d dy_t, w + d dx_t, ci] * W[t, ci, co]
with the nine taps t = 3 (dy + 1) + (dx + 1), dy, dx in {-1, 0, 1}, the
dilation d >= 1 (circular padding), optionally followed by a ReLU.  The gradients below are
the adjoints of that definition; they are pinned against central finite
differences of `conv_forward` in tests/test_conv_oracle.py.
"""
import numpy as np

OFFSETS = [(t // 3 - 1, t % 3 - 1) for t in range(9)]


def shifted(x, dy, dx):
    """s[n, h, w] = x[n, h + dy, w + dx] (periodic)."""
    return np.roll(x, shift=(-dy, -dx), axis=(1, 2))


def conv_forward(x, W, b=None, relu=False, dil=1):
    x = np.asarray(x, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    y = np.zeros(x.shape[:3] + (W.shape[2],))
    for t, (dy, dx) in enumerate(OFFSETS):
        y += shifted(x, dil * dy, dil * dx) @ W[t]
    if b is not None:
        y += np.asarray(b, dtype=np.float64)
    if relu:
        y = np.maximum(y, 0.0)
    return y


def conv_backward(x, W, dy_out, dil=1):
    """Gradients of the linear part: (dx, dW, db) for upstream gradient dy_out."""
    x = np.asarray(x, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    g = np.asarray(dy_out, dtype=np.float64)
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for t, (dy, dxo) in enumerate(OFFSETS):
        dy, dxo = dil * dy, dil * dxo
        # y[p] gets x[p + off] W[t]  =>  x[q] receives g[q - off] W[t]^T
        dx += shifted(g @ W[t].T, -dy, -dxo)
        xs = shifted(x, dy, dxo)
        dW[t] = xs.reshape(-1, x.shape[-1]).T @ g.reshape(-1, g.shape[-1])
    db = g.reshape(-1, g.shape[-1]).sum(axis=0)
    return dx, dW, db


def bf16_round(a):
    """Round float64 values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba 2015); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
