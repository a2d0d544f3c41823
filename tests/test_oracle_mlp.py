"""Pins of the MLP oracle (learned Newton guess) against facts that do not
come from the oracle itself: central finite differences of the loss, the
least-squares optimum of a linear model, the size of Adam's first step, and
bfloat16 rounding as torch implements it."""
import numpy as np
import pytest

import synth
from oracle import mlp


def _problem(sizes, B, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    params = synth.mlp_init(sizes, seed)
    params = [(W, rng.standard_normal(W.shape[1]) * 0.1) for W, _ in params]
    X = rng.standard_normal((B, sizes[0]))
    T = rng.standard_normal((B, sizes[-1]))
    return params, X, T


def test_gradients_match_central_differences():
    sizes = [5, 7, 6, 3]
    params, X, T = _problem(sizes, 11, 1)
    grads, L = mlp.gradients(params, X, T)
    assert L == pytest.approx(mlp.loss(params, X, T), rel=1e-14)
    h = 1e-6
    rng = np.random.Generator(np.random.PCG64(2))
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            for _ in range(6):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp = mlp.loss(params, X, T)
                arr[idx] = old - h
                lm = mlp.loss(params, X, T)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx, fd, g[idx])


def test_gradient_descent_reaches_least_squares_optimum():
    """A single linear layer trained by the oracle's gradients converges to
    numpy's least-squares solution (sign and scale of the gradient)."""
    rng = np.random.Generator(np.random.PCG64(3))
    X = rng.standard_normal((200, 4))
    Wt = rng.standard_normal((4, 2))
    T = X @ Wt + 0.3 + 0.01 * rng.standard_normal((200, 2))
    params = [(np.zeros((4, 2)), np.zeros(2))]
    for _ in range(3000):
        (gW, gb), = mlp.gradients(params, X, T)[0]
        params = [(params[0][0] - 0.5 * gW, params[0][1] - 0.5 * gb)]
    A = np.hstack([X, np.ones((200, 1))])
    sol = np.linalg.lstsq(A, T, rcond=None)[0]
    np.testing.assert_allclose(params[0][0], sol[:4], atol=1e-8)
    np.testing.assert_allclose(params[0][1], sol[4], atol=1e-8)


def test_adam_first_step_moves_by_lr():
    """With zero moments, the bias-corrected first step is lr * g / (|g| +
    eps'), i.e. lr times the sign of the gradient up to eps."""
    sizes = [3, 4, 2]
    params, X, T = _problem(sizes, 5, 4)
    grads, _ = mlp.gradients(params, X, T)
    zeros = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    new, m, v = mlp.adam_step(params, grads, zeros, zeros, 1, lr=1e-3, eps=1e-12)
    for (W, b), (W1, b1), (gW, gb) in zip(params, new, grads):
        np.testing.assert_allclose(W - W1, 1e-3 * np.sign(gW), rtol=1e-6, atol=1e-12)
        np.testing.assert_allclose(b - b1, 1e-3 * np.sign(gb), rtol=1e-6, atol=1e-12)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.Generator(np.random.PCG64(5))
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.uniform(-8, 8, 4000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)


def test_modes_agree_to_their_precision():
    sizes = [11, 256, 256, 10]
    params, X, T = _problem(sizes, 64, 6)
    y64 = mlp.forward(params, X)[-1]
    y32 = mlp.forward(params, X, "fp32")[-1]
    ybf = mlp.forward(params, X, "bf16")[-1]
    s = np.abs(y64).max()
    assert np.abs(y32 - y64).max() <= 1e-5 * s
    assert np.abs(ybf - y64).max() <= 5e-2 * s
    flat = mlp.pack(params)
    back = mlp.unpack(flat, sizes)
    for (W, b), (W2, b2) in zip(params, back):
        np.testing.assert_array_equal(W, W2)
        np.testing.assert_array_equal(b, b2)
