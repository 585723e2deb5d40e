"""FP64 reference of the inversion-guess network (a project extension: the paper
has no network).  Test infrastructure: never used by the product path.

Architecture (one hidden layer of H ReLU units, scalar in and out):
    x  = (L - a) b,          y = b2 + sum_h W2_h max(W1_h x + b1_h, 0),
    mu = m + s y,            loss = mean_i (y_i - (t_i - m)/s)^2.
Weight vector layout: [a, b, m, s, W1[H], b1[H], W2[H], b2]; the gradient is taken
with respect to the trainable part [W1, b1, W2, b2].  Backpropagation is written out
from the chain rule; tests pin it against central finite differences.
"""
import numpy as np

H = 32
HDR = 4


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    a, b, m, s = w[:4]
    W1 = w[HDR:HDR + H]
    b1 = w[HDR + H:HDR + 2 * H]
    W2 = w[HDR + 2 * H:HDR + 3 * H]
    b2 = w[HDR + 3 * H]
    return a, b, m, s, W1, b1, W2, b2


def forward(w, L):
    """Network output y (normalised) and mu for inputs L (array)."""
    a, b, m, s, W1, b1, W2, b2 = unpack(w)
    x = (np.asarray(L, dtype=np.float64) - a) * b
    z = np.multiply.outer(x, W1) + b1
    y = b2 + np.maximum(z, 0.0) @ W2
    return y, m + s * y


def loss(w, L, t):
    a, b, m, s, *_ = unpack(w)
    y, _ = forward(w, L)
    tn = (np.asarray(t, dtype=np.float64) - m) / s
    return np.mean((y - tn) ** 2)


def loss_grad(w, L, t):
    """(loss, gradient over [W1, b1, W2, b2]) by backpropagation."""
    a, b, m, s, W1, b1, W2, b2 = unpack(w)
    x = (np.asarray(L, dtype=np.float64) - a) * b
    z = np.multiply.outer(x, W1) + b1              # (n, H)
    act = np.maximum(z, 0.0)
    y = b2 + act @ W2
    tn = (np.asarray(t, dtype=np.float64) - m) / s
    r = y - tn
    n = r.size
    dy = 2.0 * r / n                              # d loss / d y_i
    dz = np.outer(dy, W2) * (z > 0)               # (n, H)
    g = np.concatenate([(dz * x[:, None]).sum(0), dz.sum(0), (dy[:, None] * act).sum(0), [dy.sum()]])
    return np.mean(r * r), g


def finite_difference_grad(w, L, t, h=1e-6):
    w = np.asarray(w, dtype=np.float64).copy()
    g = np.empty(3 * H + 1)
    for j in range(3 * H + 1):
        k = HDR + j
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        g[j] = (loss(wp, L, t) - loss(wm, L, t)) / (2 * h)
    return g
