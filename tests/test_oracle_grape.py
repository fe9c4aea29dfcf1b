"""Pins of the GRAPE oracle loop (oracle/grape.py): on a qubit with one sx
control and no drift every slice commutes, U = exp(-i theta sx) with
theta = h sum c, the loss is cos^2 theta and every coordinate's gradient is
-h sin 2 theta, so both optimisers reduce to a scalar recursion on theta
that the loop must follow exactly."""
import math

import numpy as np

import oracle.grape as og
import oracle.propagator as orc

SX = np.array([[0, 1], [1, 0]], dtype=complex)


def _setup(n=12, h=0.05):
    H0 = np.zeros((2, 2), complex)
    Hk = SX[None].copy()
    c = np.full((1, n), 0.3)
    return H0, Hk, c, h


def test_gd_follows_scalar_recursion():
    H0, Hk, c, h = _setup()
    n = c.shape[1]
    step = 2.0
    _, losses = og.grape(H0, Hk, c, h, 2, SX, iters=6, step=step, optimizer="gd")
    theta = h * c.sum()
    for k in range(7):
        assert abs(losses[k] - math.cos(theta) ** 2) < 1e-13, k
        theta += step * n * h * h * math.sin(2 * theta)
    assert losses[-1] < losses[0]


def test_adam_follows_scalar_recursion():
    H0, Hk, c, h = _setup()
    n = c.shape[1]
    step, b1, b2, eps = 0.05, 0.9, 0.999, 1e-8
    _, losses = og.grape(H0, Hk, c, h, 2, SX, iters=6, step=step, optimizer="adam")
    theta, m, v = h * c.sum(), 0.0, 0.0
    for k in range(7):
        assert abs(losses[k] - math.cos(theta) ** 2) < 1e-13, k
        g = -h * math.sin(2 * theta)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        t = k + 1
        theta += n * h * (-step * (m / (1 - b1 ** t)) / (math.sqrt(v / (1 - b2 ** t)) + eps))


def test_gd_decreases_a_random_problem():
    import synth
    w = synth.qubit_register(n_slices=32)
    _, losses = og.grape(w.H0, w.Hk, w.samples, w.h, 2, w.target, iters=5, step=0.5, optimizer="gd")
    assert np.all(np.diff(losses) < 0)
    assert abs(losses[0] - orc.fidelity_loss(orc.propagate(w.H0, w.Hk, w.samples, w.h, 2), w.target)) < 1e-15
