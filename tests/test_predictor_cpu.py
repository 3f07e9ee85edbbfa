"""The fp64 reference perceptron used to check the device predictor is itself
checked against central finite differences of its loss."""
import numpy as np

import mlp_ref


def test_reference_gradient_matches_finite_differences():
    rng = np.random.Generator(np.random.PCG64(3))
    F, H, B = 5, 7, 40
    p = rng.normal(0, 0.7, size=H * F + 2 * H + 1)
    X = rng.normal(size=(B, F))
    t = rng.normal(size=B)
    g = mlp_ref.grad(p, X, t, F, H)
    eps = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        a, b = p.copy(), p.copy()
        a[i] += eps
        b[i] -= eps
        fd[i] = (mlp_ref.loss(a, X, t, F, H) - mlp_ref.loss(b, X, t, F, H)) / (2 * eps)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_reference_forward_by_loops():
    rng = np.random.Generator(np.random.PCG64(4))
    F, H = 3, 4
    p = rng.normal(size=H * F + 2 * H + 1)
    X = rng.normal(size=(6, F))
    W1, b1, w2, b2 = mlp_ref.unpack(p, F, H)
    want = []
    for x in X:
        acc = b2
        for j in range(H):
            z = b1[j] + sum(W1[j, f] * x[f] for f in range(F))
            acc += w2[j] * max(z, 0.0)
        want.append(acc)
    np.testing.assert_allclose(mlp_ref.forward(p, X, F, H), want, rtol=1e-12)
