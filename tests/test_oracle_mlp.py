"""Pins of the FP64 reference network: gradients against central finite
differences, a single linear layer against its closed-form gradient, and
Adam's first step (which moves every parameter by lr * sign(gradient))."""
import numpy as np

from oracle import mlp


def _params(sizes, rng):
    return [(rng.standard_normal((o, i)) / np.sqrt(i), 0.1 * rng.standard_normal(o))
            for i, o in zip(sizes[:-1], sizes[1:])]


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(5)
    params = _params([5, 7, 6, 3], rng)
    x, t = rng.standard_normal((9, 5)), rng.standard_normal((9, 3))
    grads = mlp.gradients(params, x, t)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
                old = arr[idx]
                arr[idx] = old + h
                lp = mlp.loss(params, x, t)
                arr[idx] = old - h
                lm = mlp.loss(params, x, t)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[idx]) < 1e-6 * max(1.0, abs(fd)), (li, idx, fd, g[idx])


def test_linear_layer_closed_form():
    rng = np.random.default_rng(6)
    W, b = rng.standard_normal((4, 3)), rng.standard_normal(4)
    x, t = rng.standard_normal((10, 3)), rng.standard_normal((10, 4))
    (gW, gb), = mlp.gradients([(W, b)], x, t)
    r = x @ W.T + b - t
    assert np.allclose(gW, r.T @ x / 10, atol=1e-13)
    assert np.allclose(gb, r.sum(0) / 10, atol=1e-13)


def test_adam_first_step_is_sign_step():
    rng = np.random.default_rng(7)
    params = _params([3, 4, 2], rng)
    x, t = rng.standard_normal((5, 3)), rng.standard_normal((5, 2))
    grads = mlp.gradients(params, x, t)
    new = mlp.adam_step(params, grads, mlp.adam_state(params), lr=1e-2, eps=1e-300)
    for (W, b), (W2, b2), (gW, gb) in zip(params, new, grads):
        assert np.allclose(W - W2, 1e-2 * np.sign(gW), atol=1e-12)
        assert np.allclose(b - b2, 1e-2 * np.sign(gb), atol=1e-12)
