"""FP64 reference of the scheduling cost model (test infrastructure).

MLP 4 -> 64 -> 64 -> 1 with ReLU on standardised inputs and targets:
    x = (f - mean) / std,  h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),
    y = w3 . h2 + b3,       prediction = y * ystd + ymean,
loss = mean over samples of (y - (t - ymean) / ystd)^2.  The gradient is the
chain rule written out by hand; it is pinned to central finite differences
of the loss in the tests.  Parameter layout: W1[64][4], b1[64], W2[64][64],
b2[64], w3[64], b3; norm = mean[4], std[4], ymean, ystd.
"""
import numpy as np

IN, H = 4, 64
NPARAM = H * IN + H + H * H + H + H + 1


def unpack(p):
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + H * IN].reshape(H, IN); o += H * IN
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(p, norm, feats):
    norm = np.asarray(norm, np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(p)
    x = (np.asarray(feats, np.float64).reshape(-1, IN) - norm[:4]) / norm[4:8]
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0)
    y = h2 @ w3 + b3
    return y, (x, z1, h1, z2, h2)


def predict(p, norm, feats):
    y, _ = forward(p, norm, feats)
    return y * norm[9] + norm[8]


def loss(p, norm, feats, targets):
    y, _ = forward(p, norm, feats)
    t = (np.asarray(targets, np.float64) - norm[8]) / norm[9]
    return float(np.mean((y - t) ** 2))


def loss_grad(p, norm, feats, targets):
    y, (x, z1, h1, z2, h2) = forward(p, norm, feats)
    t = (np.asarray(targets, np.float64) - norm[8]) / norm[9]
    n = y.shape[0]
    W1, b1, W2, b2, w3, b3 = unpack(p)
    dy = 2.0 * (y - t) / n                      # d loss / d y
    gw3 = h2.T @ dy
    gb3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return float(np.mean((y - t) ** 2)), g


def fd_grad(p, norm, feats, targets, idx, h=1e-6):
    p = np.asarray(p, np.float64).copy()
    out = []
    for i in idx:
        a = p.copy(); a[i] += h
        b = p.copy(); b[i] -= h
        out.append((loss(a, norm, feats, targets) - loss(b, norm, feats, targets)) / (2 * h))
    return np.array(out)
