"""Pins of the FP64 CPU reference MLP: backpropagated gradients against
central finite differences, and GELU against its closed form."""
import math

import numpy as np

from oracle import mlp_ref as R


def _shapes(n_in, w, depth, n_out):
    dims = [n_in] + [w] * depth + [n_out]
    return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]


def test_gelu_closed_form():
    for z in (-3.0, -0.5, 0.0, 0.7, 2.5):
        assert abs(R.gelu(np.array(z)) - 0.5 * z * (1 + math.erf(z / math.sqrt(2)))) < 1e-15
        h = 1e-6
        fd = (R.gelu(np.array(z + h)) - R.gelu(np.array(z - h))) / (2 * h)
        assert abs(R.gelu_d(np.array(z)) - fd) < 1e-8


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    shapes = _shapes(5, 7, 2, 3)
    P = sum(a * b + b for a, b in shapes)
    p = rng.normal(0, 0.5, P)
    x = rng.normal(0, 1, (6, 5))
    t = rng.normal(0, 1, (6, 3))
    L, g = R.loss_grad(p, shapes, x, t)
    assert abs(L - R.loss(p, shapes, x, t)) < 1e-15
    h = 1e-6
    fd = np.zeros(P)
    for i in range(P):
        e = np.zeros(P); e[i] = h
        fd[i] = (R.loss(p + e, shapes, x, t) - R.loss(p - e, shapes, x, t)) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-8 * (1 + np.max(np.abs(g)))
