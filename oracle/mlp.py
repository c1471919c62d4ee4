"""Multilayer perceptron of the learned extrapolator (oracle; test
infrastructure).

Not part of the paper: the learned extrapolator sits beside the DMD
extrapolation of Sec. 6 and is checked here from first principles.  Layers
z_l = a_l W_l + b_l, a_{l+1} = max(z_l, 0) for hidden layers, output y =
z_{L-1}; loss = mean over all outputs of (y - t)^2; back-propagation by the
chain rule; Adam as published by Kingma & Ba (2015, Algorithm 1).

quantize=True applies bfloat16 rounding (round to nearest even of the FP32
value) where the device kernels feed the matrix cores: weights, layer inputs
and pre-activation gradients entering a product.  Everything else is float64.
"""

import numpy as np


def bf16_round(x):
    """Nearest bfloat16 (ties to even) of the float32 value of x, as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    r = np.where(nan, (u >> 16) | 0x40, r).astype(np.uint32) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits_to_float(h):
    """float64 values of bfloat16 bit patterns (uint16)."""
    return (np.asarray(h, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def split_params(dims, p):
    """[(W_l, b_l)] from the flat parameter vector (W_l row-major dims[l] x dims[l+1])."""
    out, o = [], 0
    for l in range(len(dims) - 1):
        k, n = dims[l], dims[l + 1]
        W = np.asarray(p[o:o + k * n], dtype=np.float64).reshape(k, n)
        o += k * n
        b = np.asarray(p[o:o + n], dtype=np.float64)
        o += n
        out.append((W, b))
    return out


def param_count(dims):
    return sum(dims[l] * dims[l + 1] + dims[l + 1] for l in range(len(dims) - 1))


def forward(dims, p, X, quantize=True):
    """Returns (y, layer inputs a_l)."""
    q = bf16_round if quantize else (lambda v: np.asarray(v, dtype=np.float64))
    layers = split_params(dims, p)
    a = q(X)
    acts = [a]
    for l, (W, b) in enumerate(layers):
        z = a @ q(W) + b
        if l + 1 < len(layers):
            a = q(np.maximum(z, 0.0))
            acts.append(a)
        else:
            return z, acts


def loss_and_grad(dims, p, X, T, quantize=True):
    """Loss and its gradient with respect to the flat parameter vector."""
    q = bf16_round if quantize else (lambda v: np.asarray(v, dtype=np.float64))
    layers = split_params(dims, p)
    y, acts = forward(dims, p, X, quantize)
    B, n_out = y.shape
    loss = float(np.mean((y - T) ** 2))
    dz = 2.0 * (y - T) / (B * n_out)          # d loss / d z of the output layer
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        dzq = q(dz)
        grads[l] = (acts[l].T @ dzq, dz.sum(axis=0))
        if l > 0:
            dz = (dzq @ q(W).T) * (acts[l] > 0)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step number t >= 1); returns (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
