"""Pins of the surrogate's convolution oracle: the backward formulas against
central finite differences of the forward definition, the identity filter,
translation equivariance of the circular padding, the bfloat16 rounding
against numpy's IEEE float32 bit layout, and Adam against its textbook
first step (the update equals -lr * sign(g) when eps is negligible)."""
import numpy as np
import pytest

from oracle import conv_oracle as C


def rand(shape, seed):
    return np.random.default_rng(seed).normal(size=shape)


def test_identity_filter_and_bias():
    x = rand((2, 5, 6, 4), 0)
    W = np.zeros((9, 4, 4))
    W[4] = np.eye(4)  # centre tap
    b = np.arange(4.0)
    assert np.allclose(C.conv_forward(x, W, b), x + b)
    # a single off-centre tap is a periodic shift
    W2 = np.zeros((9, 4, 4))
    W2[5] = np.eye(4)  # (dy, dx) = (0, +1)
    assert np.allclose(C.conv_forward(x, W2)[:, :, :-1], x[:, :, 1:])
    assert np.allclose(C.conv_forward(x, W2)[:, :, -1], x[:, :, 0])


def dense_conv_loops(x, K):
    """Plain periodic convolution with a (2r+1) x (2r+1) kernel K[a, b, ci, co]
    (a, b index offsets -r..r), summed by explicit loops."""
    n, h, w, ci = x.shape
    r = (K.shape[0] - 1) // 2
    y = np.zeros((n, h, w, K.shape[3]))
    for i in range(h):
        for j in range(w):
            for a in range(2 * r + 1):
                for b in range(2 * r + 1):
                    y[:, i, j] += x[:, (i + a - r) % h, (j + b - r) % w] @ K[a, b]
    return y


@pytest.mark.parametrize("dil", [1, 2, 3, 5])
def test_dilated_conv_is_zero_stuffed_dense_conv(dil):
    x = rand((2, 7, 9, 2), 10 + dil)
    W = rand((9, 2, 3), 20 + dil)
    K = np.zeros((2 * dil + 1, 2 * dil + 1, 2, 3))
    for t in range(9):
        K[dil * (t // 3), dil * (t % 3)] = W[t]
    assert np.allclose(C.conv_forward(x, W, dil=dil), dense_conv_loops(x, K))


def test_translation_equivariance():
    x = rand((1, 7, 9, 3), 1)
    W = rand((9, 3, 5), 2)
    y = C.conv_forward(x, W)
    ys = C.conv_forward(np.roll(x, (2, -3), axis=(1, 2)), W)
    assert np.allclose(np.roll(y, (2, -3), axis=(1, 2)), ys)


@pytest.mark.parametrize("relu,dil", [(False, 1), (True, 1), (True, 2), (False, 3)])
def test_backward_matches_finite_differences(relu, dil):
    x = rand((2, 4, 5, 3), 3)
    W = rand((9, 3, 2), 4)
    b = rand((2,), 5)
    g = rand((2, 4, 5, 2), 6)

    def loss(x_, W_, b_):
        return float(np.sum(C.conv_forward(x_, W_, b_, relu, dil) * g))

    y_lin = C.conv_forward(x, W, b, dil=dil)
    gl = g * (y_lin > 0) if relu else g
    dx, dW, db = C.conv_backward(x, W, gl, dil)
    h = 1e-6
    rng = np.random.default_rng(7)
    for _ in range(12):
        i = tuple(rng.integers(s) for s in x.shape)
        e = np.zeros_like(x)
        e[i] = h
        fd = (loss(x + e, W, b) - loss(x - e, W, b)) / (2 * h)
        assert abs(fd - dx[i]) < 1e-6 * max(1, abs(fd))
        j = tuple(rng.integers(s) for s in W.shape)
        e = np.zeros_like(W)
        e[j] = h
        fd = (loss(x, W + e, b) - loss(x, W - e, b)) / (2 * h)
        assert abs(fd - dW[j]) < 1e-6 * max(1, abs(fd))
    for k in range(2):
        e = np.zeros_like(b)
        e[k] = h
        fd = (loss(x, W, b + e) - loss(x, W, b - e)) / (2 * h)
        assert abs(fd - db[k]) < 1e-6 * max(1, abs(fd))


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.14159265, 1e-3])
    r = C.bf16_round(v)
    # representable: 8 significant bits
    m, e = np.frexp(r)
    assert np.allclose(m * 2 ** 8, np.round(m * 2 ** 8))
    assert r[0] == 1.0 and r[1] == 1.0            # tie rounds to even
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == 1.0 + 2 ** -6                   # tie rounds to even (up)
    assert np.all(np.abs(r - v) <= 2 ** -8 * np.abs(v) + 1e-30)  # half an ulp


def test_adam_first_step():
    w = rand((10,), 8)
    g = rand((10,), 9)
    w1, m, v = C.adam(w, g, np.zeros(10), np.zeros(10), 1, lr=1e-2, eps=1e-12)
    assert np.allclose(w1, w - 1e-2 * np.sign(g))
