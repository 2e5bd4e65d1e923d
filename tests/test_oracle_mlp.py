"""Pin of the reference network's analytic gradients: central finite differences of its loss."""
import numpy as np

from oracle import mlp


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    widths = [5, 7, 6, 4]
    n = sum(widths[i + 1] * widths[i] + widths[i + 1] for i in range(3))
    p = rng.normal(scale=0.5, size=n)
    X = rng.normal(size=(9, 5))
    Y = rng.normal(size=(9, 4))
    g = mlp.gradients(p, widths, X, Y)
    h = 1e-6
    for i in range(n):
        e = np.zeros(n); e[i] = h
        fd = (mlp.loss(p + e, widths, X, Y) - mlp.loss(p - e, widths, X, Y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_shapes_and_linear_output():
    widths = [3, 4, 2]
    p = np.zeros(3 * 4 + 4 + 4 * 2 + 2)
    p[-2:] = [1.5, -2.0]                      # output bias only
    out = mlp.forward(p, widths, np.ones((5, 3)))[-1]
    assert out.shape == (5, 2) and np.allclose(out, [1.5, -2.0])
