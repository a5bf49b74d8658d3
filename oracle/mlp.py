"""FP64 reference of the scheduler's cost model: a 2 x 64 hidden-layer tanh MLP.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Not a component of the paper.  The paper schedules internal tasks with an
estimated workload (W_i = N_E,i^2, Sec. III-C-2) and notes the estimate could
be replaced by a better model of the task time; this project learns that
model.  Architecture: x (F) -> tanh(W1 x + b1) (64) -> tanh(W2 . + b2) (64)
-> w3 . + b3 (1).  Loss: mean squared error on log time.  Optimiser: Adam.
Backpropagation is written out by hand so the GPU kernels can be checked
against it, and it is itself checked against central differences.
"""
from __future__ import annotations

import numpy as np

H = 64


def init_params(n_in, seed=0):
    rng = np.random.default_rng(seed)
    return dict(
        W1=rng.standard_normal((H, n_in)) / np.sqrt(n_in), b1=np.zeros(H),
        W2=rng.standard_normal((H, H)) / np.sqrt(H), b2=np.zeros(H),
        w3=rng.standard_normal(H) / np.sqrt(H), b3=np.zeros(1))


def forward(p, X):
    z1 = X @ p['W1'].T + p['b1']
    a1 = np.tanh(z1)
    z2 = a1 @ p['W2'].T + p['b2']
    a2 = np.tanh(z2)
    y = a2 @ p['w3'] + p['b3'][0]
    return y, (X, a1, a2)


def loss_and_grad(p, X, t):
    """Mean squared error 1/B sum (y - t)^2 and its gradient for every parameter."""
    y, (X, a1, a2) = forward(p, X)
    B = X.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    g = {}
    g['w3'] = a2.T @ dy
    g['b3'] = np.array([dy.sum()])
    dz2 = np.outer(dy, p['w3']) * (1.0 - a2 * a2)
    g['W2'] = dz2.T @ a1
    g['b2'] = dz2.sum(axis=0)
    dz1 = (dz2 @ p['W2']) * (1.0 - a1 * a1)
    g['W1'] = dz1.T @ X
    g['b1'] = dz1.sum(axis=0)
    return loss, g


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    state['t'] = state.get('t', 0) + 1
    t = state['t']
    for k in p:
        m = state.setdefault('m_' + k, np.zeros_like(p[k]))
        v = state.setdefault('v_' + k, np.zeros_like(p[k]))
        m[:] = b1 * m + (1 - b1) * g[k]
        v[:] = b2 * v + (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p
