"""FP64 reference of the MLP cost model (test infrastructure only).

Network: x (F) -> h1 = relu(W1 x + b1) (64) -> h2 = relu(W2 h1 + b2) (64)
-> y = w3 . h2 + b3, loss L = mean((y - t)^2).  Parameters are one flat
array in the order W1[64][F], b1[64], W2[64][64], b2[64], w3[64], b3.
Backward pass by the chain rule written out; Adam as defined by Kingma and Ba
(2015), with bias correction.
"""
import numpy as np

H = 64


def sizes(F):
    return [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]


def num_params(F):
    return sum(int(np.prod(s)) for _, s in sizes(F))


def unpack(p, F):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shp in sizes(F):
        k = int(np.prod(shp))
        out[name] = p[o:o + k].reshape(shp)
        o += k
    return out


def pack(d, F):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in sizes(F)])


def forward(p, X):
    X = np.asarray(X, dtype=np.float64)
    F = X.shape[1]
    w = unpack(p, F)
    z1 = X @ w["W1"].T + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["w3"] + w["b3"][0]
    return y, (X, z1, h1, z2, h2)


def loss(p, X, T):
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(T, dtype=np.float64)) ** 2))


def loss_and_grad(p, X, T):
    y, (X, z1, h1, z2, h2) = forward(p, X)
    T = np.asarray(T, dtype=np.float64)
    N, F = X.shape
    w = unpack(p, F)
    r = y - T
    L = float(np.mean(r ** 2))
    dy = 2.0 * r / N                      # dL/dy
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, w["w3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ w["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return L, pack(g, F)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Returns (p, m, v) after step t (t >= 1)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
