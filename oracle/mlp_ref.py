"""Plain FP64 CPU reference of the warm-start network (TEST INFRASTRUCTURE
ONLY; only tests import it).  Multilayer perceptron with exact-erf GELU
hidden layers, a linear output layer and mean-squared-error loss; gradients by
explicit backpropagation.  Parameter layout: per layer W[out][in] then b[out].
"""
import numpy as np
from scipy.special import erf


def unpack(params, shapes):
    out, off = [], 0
    for fin, fout in shapes:
        W = params[off:off + fin * fout].reshape(fout, fin); off += fin * fout
        b = params[off:off + fout]; off += fout
        out.append((W, b))
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(params, shapes, x):
    layers = unpack(np.asarray(params, dtype=np.float64), shapes)
    h = np.asarray(x, dtype=np.float64)
    zs, hs = [], [h]
    for i, (W, b) in enumerate(layers):
        z = h @ W.T + b
        zs.append(z)
        h = gelu(z) if i + 1 < len(layers) else z
        hs.append(h)
    return h, zs, hs


def loss(params, shapes, x, t):
    y, _, _ = forward(params, shapes, x)
    return np.mean((y - np.asarray(t, dtype=np.float64)) ** 2)


def loss_grad(params, shapes, x, t):
    layers = unpack(np.asarray(params, dtype=np.float64), shapes)
    y, zs, hs = forward(params, shapes, x)
    t = np.asarray(t, dtype=np.float64)
    n = y.size
    d = 2.0 * (y - t) / n
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, b = layers[i]
        gW = d.T @ hs[i]
        gb = d.sum(axis=0)
        grads[i] = (gW, gb)
        if i > 0:
            d = (d @ W) * gelu_d(zs[i - 1])
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return np.mean((y - t) ** 2), flat


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) through float32, returned as
    float64: the value the GPU keeps when it stores a BF16 operand."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def loss_grad_bf16(params, shapes, x, t, rnd=bf16):
    """The same network with the storage precision of the GPU path: the matrix
    products take BF16 operands (the input, the weights, the hidden
    activations GELU(z) and the back-propagated errors dL/dz) and accumulate
    exactly; biases, pre-activations, the loss and the bias gradients stay
    unrounded.  With rnd the identity this is loss_grad."""
    layers = unpack(np.asarray(params, dtype=np.float64), shapes)
    t = np.asarray(t, dtype=np.float64)
    Wr = [rnd(W) for W, _ in layers]
    h = rnd(np.asarray(x, dtype=np.float64))
    hs, zs = [h], []
    for i, (W, b) in enumerate(layers):
        z = h @ Wr[i].T + b
        zs.append(z)
        if i + 1 < len(layers):
            h = rnd(gelu(z))
            hs.append(h)
    y = zs[-1]
    n = y.size
    d = 2.0 * (y - t) / n          # unrounded error of the output layer
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        db_ = rnd(d)
        grads[i] = (db_.T @ hs[i], d.sum(axis=0))
        if i > 0:
            d = (db_ @ Wr[i]) * gelu_d(zs[i - 1])
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return np.mean((y - t) ** 2), flat
