"""CPU ORACLE of the learned index's stage-1 network -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the HIP library never uses it.

The paper has no learned component (its only vector representation of a
sequence is a fixed amino-acid count vector); the learned index is an
addition that may change the speed of a lookup and never its result. What
has a definition to check is its training loss and that loss's gradient:

    f(x)  = b2 + sum_j w2[j] * tanh(w1[j] * x + b1[j])        (j < H)
    loss  = (1 / n) * sum_s (f(x_s) - y_s) ** 2

with the parameter vector laid out as [w1 (H), b1 (H), w2 (H), b2]. This
module evaluates both in float64 with numpy, the gradient by the chain rule
written out term by term. It is pinned (``tests/test_mlp_oracle.py``) by
central finite differences of ``loss``, by the closed forms of the special
case w2 = 0, and by ``loss`` at a zero parameter vector. Parity of the
lookups themselves is pinned through the symmetric-deletion oracle: the
learned index must return exactly the pairs ``oracle.query_search`` returns.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 32
PARAMS = 3 * HIDDEN + 1


def split(params, hidden: int = HIDDEN):
    p = np.asarray(params, dtype=np.float64).reshape(3 * hidden + 1)
    return p[:hidden], p[hidden:2 * hidden], p[2 * hidden:3 * hidden], p[3 * hidden]


def forward(params, x, hidden: int = HIDDEN):
    """f(x) for every sample, float64."""
    w1, b1, w2, b2 = split(params, hidden)
    x = np.asarray(x, dtype=np.float64)
    return b2 + np.tanh(np.outer(x, w1) + b1) @ w2


def loss(params, x, y, hidden: int = HIDDEN) -> float:
    """Mean squared error of f against the targets, float64."""
    r = forward(params, x, hidden) - np.asarray(y, dtype=np.float64)
    return float(np.mean(r * r))


def loss_and_grad(params, x, y, hidden: int = HIDDEN):
    """(loss, gradient in the parameter layout), float64.

    With r_s = f(x_s) - y_s and h_sj = tanh(z_sj), z_sj = w1[j] x_s + b1[j]:
      d loss / d b2     = (2/n) sum_s r_s
      d loss / d w2[j]  = (2/n) sum_s r_s h_sj
      d loss / d b1[j]  = (2/n) sum_s r_s w2[j] (1 - h_sj^2)
      d loss / d w1[j]  = (2/n) sum_s r_s w2[j] (1 - h_sj^2) x_s
    """
    w1, b1, w2, b2 = split(params, hidden)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(x)
    h = np.tanh(np.outer(x, w1) + b1)          # (n, H)
    r = b2 + h @ w2 - y                         # (n,)
    g_out = 2.0 * r / n                         # d loss / d f(x_s)
    g_w2 = h.T @ g_out
    g_z = np.outer(g_out, w2) * (1.0 - h * h)   # d loss / d z_sj
    g_b1 = g_z.sum(axis=0)
    g_w1 = g_z.T @ x
    g_b2 = g_out.sum()
    grad = np.concatenate([g_w1, g_b1, g_w2, [g_b2]])
    return float(np.mean(r * r)), grad
