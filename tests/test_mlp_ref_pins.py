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


def test_bf16_reference_reduces_to_the_plain_one():
    """With the rounding switched off the BF16-storage reference is the plain
    (finite-difference pinned) reference; with it on, it differs by BF16
    rounding only (relative 2^-8 at most per stored operand)."""
    rng = np.random.default_rng(3)
    shapes = _shapes(6, 16, 3, 9)
    P = sum(a * b + b for a, b in shapes)
    p = rng.normal(0, 0.4, P)
    x = rng.normal(0, 1, (20, 6))
    t = rng.normal(0, 1, (20, 9))
    L, g = R.loss_grad(p, shapes, x, t)
    L1, g1 = R.loss_grad_bf16(p, shapes, x, t, rnd=lambda a: np.asarray(a, dtype=np.float64))
    assert abs(L - L1) < 1e-15 and np.max(np.abs(g - g1)) < 1e-15
    L2, g2 = R.loss_grad_bf16(p, shapes, x, t)
    assert 0 < np.max(np.abs(g - g2)) < 0.05 * np.max(np.abs(g))
    assert np.all(R.bf16(np.array([1.0, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9])) == [1.0, 1.0, 1.0 + 2 ** -7])
