"""Pin of the FP64 cost-model reference: its hand-written gradient against
central finite differences of its loss."""
import numpy as np

from oracle import mlp


def make(seed=0, n=257):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.NPARAM)
    norm = np.array([1.0, -2.0, 0.5, 3.0, 2.0, 0.7, 1.5, 0.9, 10.0, 3.0])
    f = rng.normal(0, 2, (n, 4)) + norm[:4]
    t = rng.normal(10, 3, n)
    return p, norm, f, t


def test_gradient_matches_finite_differences():
    p, norm, f, t = make()
    _, g = mlp.loss_grad(p, norm, f, t)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 60, replace=False), [mlp.NPARAM - 1, 0, 256, 4416, 4480]])
    fd = mlp.fd_grad(p, norm, f, t, idx)
    assert np.abs(fd - g[idx]).max() <= 1e-6 * max(1.0, np.abs(g).max())


def test_forward_shapes_and_relu():
    p, norm, f, t = make(n=5)
    y, (x, z1, h1, z2, h2) = mlp.forward(p, norm, f)
    assert y.shape == (5,) and h1.shape == (5, 64)
    assert np.all(h1 >= 0) and np.all(h2 >= 0)
    # a linear target is exactly representable: zero W2 and w3 leave b3
    q = np.zeros(mlp.NPARAM)
    q[-1] = 0.25
    assert np.allclose(mlp.predict(q, norm, f), 0.25 * norm[9] + norm[8])
