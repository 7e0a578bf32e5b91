"""FP64 multilayer perceptron of the oracle: forward pass, hand-derived
backward pass and Adam, for the learned linewidth surrogate.

The paper has no surrogate; the network is a reading fixed here:
input -> 4 hidden layers of 64 units with tanh -> linear scalar output, loss
= weighted mean squared error sum_i c_i (y_hat_i - y_i)^2 / sum_i c_i (c_i are
bootstrap counts), Adam with bias correction (Kingma & Ba, 2015):
    m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
    p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parameters are a list [W0, b0, W1, b1, ..., W4, b4] with W_l of shape
(fan_in, fan_out); the flat order used to pass them around is that list's
concatenation with each W in row-major order.

This is test infrastructure.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64
DEPTH = 4


def layer_sizes(n_in, hidden=HIDDEN, depth=DEPTH):
    return [n_in] + [hidden] * depth + [1]


def init_params(n_in, rng, hidden=HIDDEN, depth=DEPTH):
    """Glorot-uniform weights drawn from rng (in layer order), zero biases."""
    sizes = layer_sizes(n_in, hidden, depth)
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / (a + b))
        params.append(rng.uniform(-lim, lim, size=(a, b)))
        params.append(np.zeros(b))
    return params


def flatten(params):
    return np.concatenate([p.reshape(-1) for p in params])


def unflatten(flat, n_in, hidden=HIDDEN, depth=DEPTH):
    sizes = layer_sizes(n_in, hidden, depth)
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        out.append(flat[o:o + a * b].reshape(a, b))
        o += a * b
        out.append(flat[o:o + b].copy())
        o += b
    return out


def forward(params, X):
    """Returns the output (n,) and the list of layer activations."""
    acts = [X]
    h = X
    n_layers = len(params) // 2
    for l in range(n_layers):
        z = h @ params[2 * l] + params[2 * l + 1]
        h = np.tanh(z) if l < n_layers - 1 else z
        acts.append(h)
    return h[:, 0], acts


def loss_and_grad(params, X, y, c):
    """Weighted MSE and its gradient, by explicit back-propagation."""
    yh, acts = forward(params, X)
    csum = c.sum()
    r = yh - y
    loss = float(np.sum(c * r * r) / csum)
    delta = (2.0 * c * r / csum)[:, None]  # dL/dz of the output layer
    n_layers = len(params) // 2
    grads = [None] * len(params)
    for l in range(n_layers - 1, -1, -1):
        h_in = acts[l]
        grads[2 * l] = h_in.T @ delta
        grads[2 * l + 1] = delta.sum(axis=0)
        if l > 0:
            delta = (delta @ params[2 * l].T) * (1.0 - acts[l] ** 2)
    return loss, grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        for k, g in enumerate(grads):
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * g * g
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            params[k] = params[k] - self.lr * mh / (np.sqrt(vh) + self.eps)
        return params


def train(params, X, y, c, steps, lr=1e-3):
    opt = Adam(params, lr=lr)
    losses = []
    for _ in range(steps):
        loss, g = loss_and_grad(params, X, y, c)
        losses.append(loss)
        params = opt.step(params, g)
    return params, losses
