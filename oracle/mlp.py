"""FP64 reference of the learned initial guess's network -- TEST
INFRASTRUCTURE ONLY (see the package docstring).

A fully connected network y = W_L relu(... relu(W_1 x + b_1) ...) + b_L with
a mean-squared-error loss 0.5 * mean over samples of |y - t|^2 summed over
outputs, its gradients by the chain rule, and one Adam step (Kingma and Ba,
2015: first and second moment estimates with bias correction).  The paper
has no network; this is the plain definition of the one the library trains
(shapes and update rule stated in the design notes), written as loops over
layers with numpy products as the only primitive.

Pins: the gradients against central finite differences of the loss, and a
one-layer network against the closed form (X^T (X W^T + b - T)) / n.
"""
from __future__ import annotations

import numpy as np


def forward(params, x):
    """params: list of (W [out][in], b [out]); x [n][in].  Returns the output
    and the list of layer inputs and pre-activations (for backward)."""
    acts, pres = [x], []
    h = x
    for i, (W, b) in enumerate(params):
        z = h @ W.T + b
        pres.append(z)
        h = np.maximum(z, 0.0) if i + 1 < len(params) else z
        acts.append(h)
    return h, acts, pres


def loss(params, x, t):
    y, _, _ = forward(params, x)
    return 0.5 * np.sum((y - t) ** 2) / len(x)


def gradients(params, x, t):
    """d loss / d (W, b) for every layer, by backpropagation."""
    y, acts, pres = forward(params, x)
    n = len(x)
    g = (y - t) / n                      # d loss / d output
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        if i + 1 < len(params):
            g = g * (pres[i] > 0)        # through relu
        grads[i] = (g.T @ acts[i], g.sum(0))
        g = g @ W                        # d loss / d layer input
    return grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; state = {'t': int, 'm': [...], 'v': [...]}."""
    state["t"] += 1
    t = state["t"]
    out = []
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, gp) in enumerate(((W, gW), (b, gb))):
            m = state["m"][2 * i + j] = beta1 * state["m"][2 * i + j] + (1 - beta1) * gp
            v = state["v"][2 * i + j] = beta2 * state["v"][2 * i + j] + (1 - beta2) * gp * gp
            mh, vh = m / (1 - beta1 ** t), v / (1 - beta2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out


def adam_state(params):
    return {"t": 0, "m": [np.zeros_like(a) for W, b in params for a in (W, b)],
            "v": [np.zeros_like(a) for W, b in params for a in (W, b)]}
