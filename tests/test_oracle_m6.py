"""Pins of the oracle's sixth-order Magnus scheme (order code 6).

The scheme (three Gauss-Legendre samples per slice, the moments a1, a2, a3,
the commutators C1, C2 and Omega; see oracle.propagator) is checked against
what fixes it independently of its own formula:

* constant H: exact, U(T) = exp(-i H T) by scipy's expm;
* commuting H(t) with controls polynomial of degree <= 5: the commutators
  vanish and the three-node Gauss rule integrates H exactly, so U(T) =
  exp(-i integral of H) in closed form; degree 6 is not integrated exactly;
* convergence slope 6 against the circular drive's closed form (the
  convergence figure's problem) and against an independent fourth-order
  reference on a random 4-level system;
* local error of one slice O(h^7) (ratio 2^7 per halving);
* planted mistakes in the scheme (a dropped commutator, a wrong sign or
  coefficient, equispaced instead of Gauss-Legendre samples) each fail a pin.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle.propagator as orc
import synth

M6 = orc.M6


def circular_exact(w0=1.0, w1=0.1, wrf=1.0, t=6.0):
    Z, X = synth.PAULI_Z, synth.PAULI_X
    return scipy.linalg.expm(-1j * wrf * t * Z / 2) @ scipy.linalg.expm(
        -1j * (((w0 - wrf) / 2) * Z + (w1 / 2) * X) * t)


def slope(ns, errs):
    return -np.polyfit(np.log(ns), np.log(errs), 1)[0]


def circular_slope():
    ns = [8, 16, 32, 64]
    errs = []
    for n in ns:
        w = synth.circular_drive(n, M6)
        errs.append(orc.relative_frobenius(orc.propagate(w.H0, w.Hk, w.samples, w.h, M6), circular_exact()))
    return slope(ns, errs), errs


def random_system_fn(d=4, seed=11):
    rng = np.random.default_rng([synth.SEED_BASE, seed])
    H0 = synth.gue(rng, d, 1.0)
    H1 = synth.gue(rng, d, 1.0)
    H2 = synth.gue(rng, d, 1.0)

    def ctrl(t):
        return np.stack([np.sin(1.3 * t + 0.2), np.cos(2.1 * t) ** 2])
    return H0, np.stack([H1, H2]), ctrl


def random_slope():
    """Slope on a random system against a fine fourth-order (midpoint-Simpson
    commutator Magnus) reference: a different integrator, so an error in the
    sixth-order formula cannot cancel."""
    H0, Hk, ctrl = random_system_fn()
    T = 3.0
    nref = 4096
    href = T / nref
    Uref = orc.propagate(H0, Hk, ctrl(synth.sample_times(nref, href, 4)), href, 4)
    ns = [8, 16, 32, 64]
    errs = []
    for n in ns:
        h = T / n
        U = orc.propagate(H0, Hk, ctrl(synth.sample_times(n, h, M6)), h, M6)
        errs.append(orc.relative_frobenius(U, Uref))
    return slope(ns, errs), errs


def static_error():
    w = synth.random_system(4, 2, n_slices=20, h=0.3, order=M6, tag=7)
    c = np.array([[0.7], [-0.4]]) * np.ones((1, w.n_samples))
    H = w.H0 + 0.7 * w.Hk[0] - 0.4 * w.Hk[1]
    U = orc.propagate(w.H0, w.Hk, c, w.h, M6)
    return orc.relative_frobenius(U, scipy.linalg.expm(-1j * H * (w.h * w.n_slices)))


def commuting_poly_error(degree):
    """Diagonal (commuting) H0, H_k; c_k(t) polynomials of the given degree."""
    rng = np.random.default_rng([synth.SEED_BASE, 77, degree])
    d = 5
    H0 = np.diag(rng.normal(size=d)).astype(np.complex128)
    Hk = np.stack([np.diag(rng.normal(size=d)).astype(np.complex128) for _ in range(2)])
    coef = rng.normal(size=(2, degree + 1))
    n, h = 7, 0.4
    T = n * h
    t = synth.sample_times(n, h, M6)
    c = np.stack([np.polyval(coef[k], t) for k in range(2)])
    U = orc.propagate(H0, Hk, c, h, M6)
    integ = [np.polyval(np.polyint(coef[k]), T) - np.polyval(np.polyint(coef[k]), 0.0) for k in range(2)]
    Hint = H0 * T + integ[0] * Hk[0] + integ[1] * Hk[1]
    return orc.relative_frobenius(U, scipy.linalg.expm(-1j * Hint))


def local_error_ratio():
    """One slice against a fine fourth-order reference of the same slice."""
    H0, Hk, ctrl = random_system_fn(seed=12)
    errs = []
    for h in (0.4, 0.2):
        U = orc.propagate(H0, Hk, ctrl(synth.sample_times(1, h, M6)), h, M6)
        nref = 2048
        Uref = orc.propagate(H0, Hk, ctrl(synth.sample_times(nref, h / nref, 4)), h / nref, 4)
        errs.append(orc.relative_frobenius(U, Uref))
    return errs[0] / errs[1]


def test_sixth_order_static_closed_form():
    assert static_error() <= 1e-13


def test_sixth_order_commuting_polynomial_exact():
    for deg in range(0, 6):
        assert commuting_poly_error(deg) <= 1e-13, deg
    # the three-node Gauss rule integrates degree 6 only approximately
    assert commuting_poly_error(6) >= 1e-9


def test_sixth_order_slope_circular_drive():
    s, errs = circular_slope()
    print("circular drive errors", errs, "slope", s)
    assert abs(s - 6.0) <= 0.15, s


def test_sixth_order_slope_random_system():
    s, errs = random_slope()
    print("random system errors", errs, "slope", s)
    assert abs(s - 6.0) <= 0.15, s


def test_sixth_order_local_error():
    r = local_error_ratio()
    print("local error ratio", r)
    assert 2 ** 6.7 <= r <= 2 ** 7.3, r


def test_sixth_order_exponent_is_hermitian():
    w = synth.random_system(6, 3, n_slices=5, h=0.2, order=M6, tag=9)
    G = orc.slice_exponents(w.H0, w.Hk, w.samples, w.h, M6)
    assert np.max(np.abs(G - np.conj(np.swapaxes(G, -1, -2)))) <= 1e-15


def _all_pins_ok():
    try:
        return (static_error() <= 1e-13 and all(commuting_poly_error(k) <= 1e-13 for k in range(6))
                and abs(circular_slope()[0] - 6.0) <= 0.15 and abs(random_slope()[0] - 6.0) <= 0.15)
    except Exception:
        return False


def _variant(drop_c2=False, sign=1.0, a3_div=12.0, a2_scale=1.0, c2_scale=1.0):
    def comm(x, y):
        return x @ y - y @ x

    def f(A1, A2, A3, h):
        B1, B2, B3 = -1j * A1, -1j * A2, -1j * A3
        r15 = math.sqrt(15.0)
        a1 = h * B2
        a2 = a2_scale * (r15 * h / 3.0) * (B3 - B1)
        a3 = (10.0 * h / 3.0) * (B3 - 2.0 * B2 + B1)
        C1 = comm(a1, a2)
        C2 = 0.0 if drop_c2 else -(c2_scale / 60.0) * comm(a1, 2.0 * a3 + C1)
        om = a1 + a3 / a3_div + sign * (1.0 / 240.0) * comm(-20.0 * a1 - a3 + C1, a2 + C2)
        return 1j * om
    return f


PLANTED = [
    ("C2 dropped", _variant(drop_c2=True)),
    ("commutator term sign flipped", _variant(sign=-1.0)),
    ("a3 / 6 instead of a3 / 12", _variant(a3_div=6.0)),
    ("a2 coefficient halved", _variant(a2_scale=0.5)),
    ("C2 coefficient doubled", _variant(c2_scale=2.0)),
]


@pytest.mark.parametrize("name,fn", PLANTED, ids=[p[0] for p in PLANTED])
def test_planted_sixth_order_mistakes_are_caught(monkeypatch, name, fn):
    assert _all_pins_ok()
    monkeypatch.setattr(orc, "magnus6_exponent", fn)
    assert not _all_pins_ok(), f"no pin caught: {name}"


def test_planted_equispaced_samples_are_caught():
    """Samples at 0, h/2, h (equispaced) instead of the Gauss-Legendre nodes
    break the scheme's order."""
    ns = [8, 16, 32, 64]
    errs = []
    for n in ns:
        w = synth.circular_drive(n, M6)
        j = np.arange(n)[:, None]
        t = ((j + np.array([0.0, 0.5, 1.0])[None, :]) * w.h).reshape(-1)
        c = np.stack([np.cos(t), np.sin(t)])
        errs.append(orc.relative_frobenius(orc.propagate(w.H0, w.Hk, c, w.h, M6), circular_exact()))
    assert abs(slope(ns, errs) - 6.0) > 0.5


def test_stored_full_size_sixth_order_reference():
    """The stored sixth-order U(T) of the d = 16 random qudit (N = 2^17,
    written by tests/golden/make_full_size.py with the oracle) is unitary and
    agrees with the stored fourth-order U(T) of the same system over the same
    span within the fourth-order scheme's own error there: that scheme needs
    N = 2^15 for 1e-6, so at 2^17 (h / 4) its error is below 1e-6 / 4^4
    = 3.9e-9; bound 1e-8."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_oracle.npz")
    with np.load(path) as z:
        U6, U4 = z["random_qudit_m6"], z["random_qudit"]
    assert np.max(np.abs(U6.conj().T @ U6 - np.eye(16))) <= 1e-11
    assert orc.relative_frobenius(U6, U4) <= 1e-8
