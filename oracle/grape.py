"""Gradient-based control optimisation of the gate fidelity, written plainly.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run this module.  It shares
no code with the HIP library.

GRAPE (Applications and outlook section): repeat
    L, dL/dc  <- the oracle's fidelity loss and control gradient at c
    c         <- c - step * dL/dc                          (gradient descent)
           or    Adam: m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
                 c <- c - step * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
and record L before every update and after the last.
"""
from __future__ import annotations

import numpy as np

from . import propagator as orc


def grape(H0, Hk, samples, h: float, order: int, V, iters: int, step: float, optimizer: str = "adam",
          b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """(optimised samples, loss history of length iters + 1)."""
    c = np.array(samples, dtype=np.float64, copy=True)
    m = np.zeros_like(c)
    v = np.zeros_like(c)
    losses = []
    for it in range(iters + 1):
        U = orc.propagate(H0, Hk, c, h, order)
        losses.append(orc.fidelity_loss(U, V))
        if it == iters:
            break
        _, g = orc.control_gradient(H0, Hk, c, h, order, orc.fidelity_grad_U(U, V))
        if optimizer == "gd":
            c = c - step * g
        else:
            t = it + 1
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            c = c - step * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return c, np.array(losses)
