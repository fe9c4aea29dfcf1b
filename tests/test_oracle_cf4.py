"""Pins of the commutator-free fourth-order integrator in the oracle
(``order = orc.CF4``) against facts fixed by the mathematics:

* constant controls: U(T) = exp(-i H T) (scipy's Pade expm);
* commuting (diagonal) Hamiltonians with quadratic controls: U(T) =
  exp(-i integral of H), the integral in closed form (Simpson is exact on
  quadratics, so the two exponents must add up to it);
* one slice agrees with the commutator Magnus step to O(h^5) (local error
  ratio 32 per halving of h) -- a wrong order of the two factors flips the
  sign of the implied commutator and leaves O(h^3);
* global convergence slope 4 on the circularly driven qubit, whose
  rotating-frame closed form is exact;
* the control gradient against central differences and, for commuting
  Hamiltonians, against the closed-form derivative of the phases;
* trajectory end point equals the propagation; planted mistakes fail.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle.propagator as orc
import synth
from test_oracle_pins import circular_drive_exact, rand_herm

CF4 = orc.CF4


def static_error():
    rng = np.random.default_rng(51)
    d, K, n, h = 5, 2, 30, 0.07
    H0 = rand_herm(rng, d)
    Hk = np.stack([rand_herm(rng, d) for _ in range(K)])
    cv = np.array([0.4, -0.9])
    c = np.repeat(cv[:, None], 2 * n + 1, axis=1)
    ref = scipy.linalg.expm(-1j * (H0 + cv[0] * Hk[0] + cv[1] * Hk[1]) * (n * h))
    return orc.relative_frobenius(orc.propagate(H0, Hk, c, h, CF4), ref)


def commuting_quadratic_error():
    """H(t) = diag(e0) + sum_k c_k(t) diag(e_k), c_k(t) = a_k + b_k t + q_k t^2:
    phi = T e0 + sum_k (a_k T + b_k T^2/2 + q_k T^3/3) e_k."""
    rng = np.random.default_rng(52)
    d, K, n, h = 4, 2, 9, 0.13
    e0 = rng.standard_normal(d)
    ek = rng.standard_normal((K, d))
    a, b, q = rng.standard_normal(K), rng.standard_normal(K), rng.standard_normal(K)
    t = synth.sample_times(n, h, CF4)
    c = a[:, None] + b[:, None] * t[None] + q[:, None] * t[None] ** 2
    T = n * h
    phi = T * e0 + (a * T + b * T ** 2 / 2 + q * T ** 3 / 3) @ ek
    U = orc.propagate(np.diag(e0).astype(complex), np.stack([np.diag(e) for e in ek]).astype(complex), c, h, CF4)
    return float(np.max(np.abs(U - np.diag(np.exp(-1j * phi)))))


def local_ratio(seed=53):
    """err(h)/err(h/2) for one slice of CF4 against the commutator Magnus step."""
    rng = np.random.default_rng(seed)
    d = 4
    H0 = rand_herm(rng, d)
    H1 = rand_herm(rng, d)
    H2 = rand_herm(rng, d)

    def err(h):
        # smooth H(t) = H0 + sin(2t) H1 + cos(3t) H2 sampled at 0, h/2, h
        t = np.array([0.0, 0.5 * h, h])
        c = np.stack([np.sin(2 * t), np.cos(3 * t)])
        Hk = np.stack([H1, H2])
        Ucf = orc.propagate(H0, Hk, c, h, CF4)
        Um = orc.propagate(H0, Hk, c, h, 4)
        return np.linalg.norm(Ucf - Um)

    e = [err(h) for h in (0.2, 0.1, 0.05)]
    return e[0] / e[1], e[1] / e[2]


def drive_error(n):
    w = synth.circular_drive(n, CF4)
    m = w.meta
    U = orc.propagate(w.H0, w.Hk, w.samples, w.h, CF4)
    return orc.relative_frobenius(U, circular_drive_exact(m["w0"], m["w1"], m["wrf"], m["t"]))


def slope():
    ns = [16, 32, 64, 128]
    e = [drive_error(n) for n in ns]
    return -np.polyfit(np.log(ns), np.log(e), 1)[0]


def fd_gradient_error(seed=54):
    rng = np.random.default_rng(seed)
    d, K, n, h = 4, 2, 5, 0.3
    H0 = rand_herm(rng, d, 2.0)
    Hk = np.stack([rand_herm(rng, d) for _ in range(K)])
    c = rng.uniform(-1, 1, size=(K, 2 * n + 1))
    V = synth.haar_unitary(rng, d)
    U, grad = orc.control_gradient(H0, Hk, c, h, CF4, orc.fidelity_grad_U(orc.propagate(H0, Hk, c, h, CF4), V))
    eps = 1e-6
    fd = np.zeros_like(c)
    for k in range(K):
        for i in range(c.shape[1]):
            cp = c.copy(); cp[k, i] += eps
            cm = c.copy(); cm[k, i] -= eps
            fd[k, i] = (orc.fidelity_loss(orc.propagate(H0, Hk, cp, h, CF4), V)
                        - orc.fidelity_loss(orc.propagate(H0, Hk, cm, h, CF4), V)) / (2 * eps)
    return float(np.max(np.abs(grad - fd)) / np.max(np.abs(fd)))


def commuting_gradient_error():
    """Diagonal Hamiltonians: phi_a = (h/6) sum_j (A1 + 4 A2 + A3)_aa, so
    dL/dc_k[q] = (h/6) w_q sum_a (dL/dphi_a)(e_k)_a with the Simpson sample
    weights w_q = 1 at the two ends, 2 at interior slice boundaries, 4 at
    the slice midpoints."""
    rng = np.random.default_rng(55)
    d, K, n, h = 3, 2, 6, 0.17
    e0 = rng.standard_normal(d)
    ek = rng.standard_normal((K, d))
    c = rng.uniform(-1, 1, size=(K, 2 * n + 1))
    V = synth.haar_unitary(rng, d)
    wq = np.where(np.arange(2 * n + 1) % 2 == 1, 4.0, 2.0)
    wq[0] = wq[-1] = 1.0
    phi = n * h * e0 + (h / 6.0) * (ek.T @ (c @ wq))
    v = np.diag(V)
    g = np.sum(np.conj(v) * np.exp(-1j * phi))
    dL_dphi = -(2.0 / d ** 2) * np.real(np.conj(g) * (-1j) * np.conj(v) * np.exp(-1j * phi))
    ref = (h / 6.0) * (ek @ dL_dphi)[:, None] * wq[None, :]
    U = np.diag(np.exp(-1j * phi))
    _, grad = orc.control_gradient(np.diag(e0).astype(complex), np.stack([np.diag(e) for e in ek]).astype(complex),
                                   c, h, CF4, orc.fidelity_grad_U(U, V))
    return float(np.max(np.abs(grad - ref)))


def test_static_exact():
    assert static_error() < 1e-13


def test_commuting_quadratic_controls_exact():
    assert commuting_quadratic_error() < 1e-13


def test_local_agreement_with_commutator_magnus_is_fifth_order():
    r1, r2 = local_ratio()
    assert 26.0 < r1 < 38.0 and 28.0 < r2 < 36.0


def test_convergence_slope_is_four():
    assert abs(slope() - 4.0) < 0.05
    assert drive_error(4096) < 1e-11


def test_gradient_matches_central_differences():
    assert fd_gradient_error() < 1e-7


def test_gradient_commuting_closed_form():
    assert commuting_gradient_error() < 1e-13


def test_trajectory_end_point_and_unitarity():
    w = synth.random_system(4, 2, n_slices=25, h=0.05, order=CF4, tag=56)
    P = orc.trajectory(w.H0, w.Hk, w.samples, w.h, CF4)
    U = orc.propagate(w.H0, w.Hk, w.samples, w.h, CF4)
    assert P.shape == (26, 4, 4)
    assert np.max(np.abs(P[-1] - U)) < 1e-14
    assert np.max(np.abs(P[0] - np.eye(4))) == 0.0
    assert orc.unitarity_defect(U) < 1e-13


# --------------------------------------------------------- planted mistakes

def _swap_factors(H0, Hk, samples, h, start=0, stop=None):
    Gf, Gs = _orig(H0, Hk, samples, h, start, stop)
    return Gs, Gf


def _same_weights_twice(H0, Hk, samples, h, start=0, stop=None):
    Gf, _ = _orig(H0, Hk, samples, h, start, stop)
    return Gf, Gf


def _trapezoid_halves(H0, Hk, samples, h, start=0, stop=None):
    samples = np.asarray(samples, np.float64)
    n = (samples.shape[1] - 1) // 2
    stop = n if stop is None else stop
    A = orc.hamiltonian_samples(H0, Hk, samples[:, 2 * start: 2 * stop + 1])
    A1, A3 = A[0:-1:2], A[2::2]
    return (h / 4.0) * (A1 + A3), (h / 4.0) * (A1 + A3)


_orig = orc.cf4_exponents


def _pins_ok():
    try:
        return (static_error() < 1e-13 and commuting_quadratic_error() < 1e-13
                and 26.0 < local_ratio()[0] < 38.0 and abs(slope() - 4.0) < 0.05)
    except Exception:
        return False


@pytest.mark.parametrize("fn", [_swap_factors, _same_weights_twice, _trapezoid_halves])
def test_planted_mistakes_are_caught(monkeypatch, fn):
    assert _pins_ok()
    monkeypatch.setattr(orc, "cf4_exponents", fn)
    assert not _pins_ok()
