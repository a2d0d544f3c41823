"""Plain NumPy reference of the learned Newton initial guess: a multilayer
perceptron (N+2) -> 256 -> 256 -> (N+1) with ReLU hidden layers, its
mean-squared-error gradients and the Adam update.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves every cell's reaction system by Newton's method started
from the previous iterate (step S5, eq. reaction_step_numerical_methodology)
and says nothing about learned guesses; the model, its inputs and outputs
and its training are this library's extension of the hot path, so there is
no passage to follow: the definitions below are the textbook ones (dense
layers, ReLU, mean squared error, Adam with bias correction), written out
plainly.

Modes reproduce where the GPU kernels round: ``fp64`` rounds nothing;
``fp32`` rounds every GEMM operand to float32; ``bf16`` rounds every GEMM
operand (weights, activations and back-propagated errors) to bfloat16 with
round-to-nearest-even.  Products and sums are then taken in float64 here (the
GPU accumulates in float32; the tests state the tolerance this costs).

Parameters are a list of (W, b) with W of shape (fan_in, fan_out).
"""
import numpy as np


def bf16(x):
    """Round to the nearest bfloat16 (ties to even) via float32; float64 out."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64).reshape(x32.shape)


def _q(x, mode):
    if mode == "bf16":
        return bf16(x)
    if mode == "fp32":
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    return np.asarray(x, dtype=np.float64)


def forward(params, X, mode="fp64"):
    """Activations [X, h1, h2, y] (pre-rounding values of each layer)."""
    acts = [np.asarray(X, dtype=np.float64)]
    last = len(params) - 1
    h = acts[0]
    for l, (W, b) in enumerate(params):
        z = _q(h, mode) @ _q(W, mode) + np.asarray(b, dtype=np.float64)
        h = z if l == last else np.maximum(z, 0.0)
        acts.append(h)
    return acts


def loss(params, X, T, mode="fp64"):
    """Mean over the batch and the outputs of the squared error."""
    y = forward(params, X, mode)[-1]
    return float(np.mean((y - T) ** 2))


def gradients(params, X, T, mode="fp64"):
    """Back-propagation of ``loss``: list of (dW, db), and the loss."""
    acts = forward(params, X, mode)
    y = acts[-1]
    B, n_out = y.shape
    dz = 2.0 * (y - T) / (B * n_out)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        h_in = acts[l]
        dzq = _q(dz, mode)
        grads[l] = (_q(h_in, mode).T @ dzq, dz.sum(axis=0))
        if l > 0:
            dz = (dzq @ _q(W, mode).T) * (h_in > 0.0)
    return grads, float(np.mean((y - T) ** 2))


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected first and second moments) of every
    parameter array; ``t`` is the 1-based step number.  Returns new
    (params, m, v)."""
    new_p, new_m, new_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        out = []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = beta1 * mm + (1.0 - beta1) * g
            vv = beta2 * vv + (1.0 - beta2) * g * g
            mh = mm / (1.0 - beta1 ** t)
            vh = vv / (1.0 - beta2 ** t)
            out.append((p - lr * mh / (np.sqrt(vh) + eps), mm, vv))
        new_p.append((out[0][0], out[1][0]))
        new_m.append((out[0][1], out[1][1]))
        new_v.append((out[0][2], out[1][2]))
    return new_p, new_m, new_v


def pack(params):
    """Flat parameter vector in the library's order: W1, b1, W2, b2, ..."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unpack(flat, sizes):
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = flat[o:o + a * b].reshape(a, b)
        o += a * b
        bb = flat[o:o + b]
        o += b
        out.append((W, bb))
    return out
