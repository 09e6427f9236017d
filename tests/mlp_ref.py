"""Plain numpy FP64 reference of the screening network (16 -> 64 -> 64 -> 1,
ReLU) and of its asymmetric squared loss, with hand-written backpropagation;
parameter layout as RSGDF_MLP_NPARAM in include/rsgdf.h."""
import numpy as np

F, H = 16, 64
OFF_MEAN, OFF_ISTD = 0, 16
OFF_W1 = 32
OFF_B1 = OFF_W1 + H * F
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
OFF_LO = OFF_B3 + 1
OFF_HI = OFF_LO + F
NPARAM = OFF_HI + F
NTRAIN = OFF_B3 + 1 - OFF_W1


def unpack(p):
    p = np.asarray(p, np.float64)
    return (p[OFF_MEAN:OFF_MEAN + F], p[OFF_ISTD:OFF_ISTD + F], p[OFF_W1:OFF_B1].reshape(H, F), p[OFF_B1:OFF_W2],
            p[OFF_W2:OFF_B2].reshape(H, H), p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def forward(p, X):
    mean, istd, W1, b1, W2, b2, W3, b3 = unpack(p)
    x = (np.asarray(X, np.float64) - mean) * istd
    a1 = x @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    return h2 @ W3 + b3, (x, a1, h1, a2, h2)


def loss(p, X, y, kappa):
    pred, _ = forward(p, X)
    e = pred - np.asarray(y, np.float64)
    w = np.where(e < 0.0, kappa, 1.0)
    return float(np.sum(w * e * e) / len(e))


def grad(p, X, y, kappa):
    """Gradient over W1, b1, W2, b2, W3, b3 in parameter order."""
    mean, istd, W1, b1, W2, b2, W3, b3 = unpack(p)
    pred, (x, a1, h1, a2, h2) = forward(p, X)
    n = len(pred)
    e = pred - np.asarray(y, np.float64)
    w = np.where(e < 0.0, kappa, 1.0)
    dy = 2.0 * w * e / n
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    d2 = np.outer(dy, W3) * (a2 > 0.0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(0)
    d1 = (d2 @ W2) * (a1 > 0.0)
    gW1 = d1.T @ x
    gb1 = d1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
