"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types an oracle formula: each compares the oracle with a
closed form, a different library algorithm (scipy's Pade scaling-and-squaring
expm, block-matrix Frechet identity), an invariant, or a measured convergence
order.  ``test_planted_mistakes_are_caught`` plants plausible mistakes in the
oracle (on the CPU) and checks that at least one pin fails for each.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle.propagator as orc
import synth

X, Y, Z, I2 = synth.PAULI_X, synth.PAULI_Y, synth.PAULI_Z, synth.PAULI_I


# ----------------------------------------------------------------- closed forms

def pauli_exp(a):
    """exp(-i a.sigma) = cos|a| I - i sin|a| (a.sigma)/|a| (Pauli algebra)."""
    n = math.sqrt(sum(x * x for x in a))
    s = a[0] * X + a[1] * Y + a[2] * Z
    return math.cos(n) * I2 - 1j * (math.sin(n) / n) * s


def circular_drive_exact(w0, w1, wrf, t):
    """Rotating-frame solution of the circularly driven qubit (eq. driven_hamiltonian):
    U(t) = exp(-i wrf t sz/2) exp(-i [((w0-wrf)/2) sz + (w1/2) sx] t)."""
    R = np.diag([np.exp(-0.5j * wrf * t), np.exp(0.5j * wrf * t)])
    return R @ pauli_exp((0.5 * w1 * t, 0.0, 0.5 * (w0 - wrf) * t))


def rand_herm(rng, d, scale=1.0):
    a = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    h = 0.5 * (a + a.conj().T)
    return scale * h / np.linalg.norm(h, 2)


# ------------------------------------------------------------ pin functions
# Each returns a scalar error; the tests assert bounds, and the mutation test
# checks that mutated oracles break at least one bound.

def pin_pauli():
    errs = []
    for a in [(0.3, 0, 0), (0, -1.2, 0), (0, 0, 2.5), (0.1, -0.7, 0.4), (1e-7, 2e-7, -3e-7)]:
        G = a[0] * X + a[1] * Y + a[2] * Z
        errs.append(np.max(np.abs(orc.expm_minus_i(G[None])[0] - pauli_exp(a))))
    return max(errs)


def pin_expm_scipy():
    rng = np.random.default_rng(11)
    worst = 0.0
    for d in (3, 8, 16):
        for nrm in (1e-6, 1e-3, 0.1, 1.0, 10.0, 100.0):
            G = rand_herm(rng, d, nrm)
            ref = scipy.linalg.expm(-1j * G)
            worst = max(worst, orc.relative_frobenius(orc.expm_minus_i(G[None])[0], ref))
    return worst


def pin_static():
    """Constant controls: U(T) = exp(-i H T) (eq. for a stationary Hamiltonian)."""
    rng = np.random.default_rng(5)
    d, K, n, h = 5, 2, 40, 0.05
    H0 = rand_herm(rng, d)
    Hk = np.stack([rand_herm(rng, d) for _ in range(K)])
    cvals = np.array([0.7, -0.3])
    H = H0 + cvals[0] * Hk[0] + cvals[1] * Hk[1]
    ref = scipy.linalg.expm(-1j * H * (n * h))
    worst = 0.0
    for order, ns in ((2, n), (4, 2 * n + 1)):
        c = np.repeat(cvals[:, None], ns, axis=1)
        worst = max(worst, orc.relative_frobenius(orc.propagate(H0, Hk, c, h, order), ref))
    return worst


def pin_product_order():
    """Two piecewise-constant slices: sx then sz.  U = exp(-i h sz) exp(-i h sx)."""
    h = 0.4
    Hk = np.stack([X, Z])
    c = np.array([[1.0, 0.0], [0.0, 1.0]])
    U = orc.propagate(np.zeros((2, 2), complex), Hk, c, h, 2)
    return np.max(np.abs(U - pauli_exp((0, 0, h)) @ pauli_exp((h, 0, 0))))


def drive_error(n, order):
    w = synth.circular_drive(n, order)
    U = orc.propagate(w.H0, w.Hk, w.samples, w.h, order)
    m = w.meta
    return orc.relative_frobenius(U, circular_drive_exact(m["w0"], m["w1"], m["wrf"], m["t"]))


def pin_slope(order):
    ns = [16, 32, 64, 128]
    e = [drive_error(n, order) for n in ns]
    return -np.polyfit(np.log(ns), np.log(e), 1)[0]


def pin_frechet():
    """Daleckii-Krein directional derivative vs the block-matrix identity
    expm([[A, E], [0, A]]) = [[e^A, L(A,E)], [0, e^A]] with A=-iG, E->-iE."""
    rng = np.random.default_rng(3)
    worst = 0.0
    for d, nrm in ((2, 0.5), (4, 2.0), (6, 0.01)):
        G = rand_herm(rng, d, nrm)
        G[0, 0] += 0.0  # keep Hermitian
        E = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        blk = np.zeros((2 * d, 2 * d), complex)
        blk[:d, :d] = -1j * G
        blk[d:, d:] = -1j * G
        blk[:d, d:] = -1j * E
        ref = scipy.linalg.expm(blk)[:d, d:]
        got = orc.frechet_expm_minus_i(G[None], E[None])[0]
        worst = max(worst, orc.relative_frobenius(got, ref))
    # degenerate spectrum (divided difference on the diagonal)
    G = np.diag([0.3, 0.3, -0.2]).astype(complex)
    E = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    blk = np.zeros((6, 6), complex)
    blk[:3, :3] = blk[3:, 3:] = -1j * G
    blk[:3, 3:] = -1j * E
    worst = max(worst, orc.relative_frobenius(orc.frechet_expm_minus_i(G[None], E[None])[0],
                                              scipy.linalg.expm(blk)[:3, 3:]))
    return worst


def fd_gradient_error(order, seed=7):
    """Oracle control gradient vs central differences of the fidelity loss."""
    rng = np.random.default_rng(seed)
    d, K, n, h = 4, 2, 6, 0.3
    H0 = rand_herm(rng, d, 2.0)
    Hk = np.stack([rand_herm(rng, d) for _ in range(K)])
    ns = n if order == 2 else 2 * n + 1
    c = rng.uniform(-1, 1, size=(K, ns))
    V = synth.haar_unitary(rng, d)
    U, grad = orc.control_gradient(H0, Hk, c, h, order, orc.fidelity_grad_U(orc.propagate(H0, Hk, c, h, order), V))
    eps = 1e-6
    fd = np.zeros_like(c)
    for k in range(K):
        for i in range(ns):
            cp = c.copy(); cp[k, i] += eps
            cm = c.copy(); cm[k, i] -= eps
            fd[k, i] = (orc.fidelity_loss(orc.propagate(H0, Hk, cp, h, order), V)
                        - orc.fidelity_loss(orc.propagate(H0, Hk, cm, h, order), V)) / (2 * eps)
    return float(np.max(np.abs(grad - fd)) / np.max(np.abs(fd)))


def commuting_gradient_error():
    """Diagonal (commuting) Hamiltonians: U(T)=diag(exp(-i phi)), phi_a = h sum_j H(t_j)_aa,
    so dL/dc_k[j] = h sum_a (dL/dphi_a) (H_k)_aa in closed form."""
    rng = np.random.default_rng(9)
    d, K, n, h = 4, 3, 7, 0.2
    e0 = rng.standard_normal(d)
    ek = rng.standard_normal((K, d))
    H0 = np.diag(e0).astype(complex)
    Hk = np.stack([np.diag(e) for e in ek]).astype(complex)
    c = rng.uniform(-1, 1, size=(K, n))
    V = synth.haar_unitary(rng, d)
    phi = h * (n * e0 + ek.T @ c.sum(axis=1))
    v = np.diag(V)
    g = np.sum(np.conj(v) * np.exp(-1j * phi))
    dL_dphi = -(2.0 / d ** 2) * np.real(np.conj(g) * (-1j) * np.conj(v) * np.exp(-1j * phi))
    ref = h * np.repeat((ek @ dL_dphi)[:, None], n, axis=1)
    U = np.diag(np.exp(-1j * phi))
    _, grad = orc.control_gradient(H0, Hk, c, h, 2, orc.fidelity_grad_U(U, V))
    return float(np.max(np.abs(grad - ref)))


# ------------------------------------------------------------------- tests

def test_pauli_closed_form():
    assert pin_pauli() < 1e-14


def test_expm_matches_scipy_pade_over_norm_range():
    assert pin_expm_scipy() < 2e-12


def test_static_hamiltonian_exact_solution():
    assert pin_static() < 1e-12


def test_product_order_later_slice_on_left():
    assert pin_product_order() < 1e-14


def test_circular_drive_closed_form():
    # 4th-order Magnus at 4096 slices reaches the rounding floor.
    assert drive_error(4096, 4) < 1e-11
    # second order: error ~ C h^2, matches the known constant within 5%
    e = drive_error(128, 2)
    assert 2.5e-5 < e < 3.1e-5


def test_convergence_slope_midpoint_is_two():
    assert abs(pin_slope(2) - 2.0) < 0.03


def test_convergence_slope_magnus4_is_four():
    assert abs(pin_slope(4) - 4.0) < 0.05


def test_unitarity():
    w = synth.random_qudit(n_slices=2000)
    U = orc.propagate(w.H0, w.Hk, w.samples, w.h, w.order)
    assert orc.unitarity_defect(U) < 1e-12


def test_fine_step_brute_force_dim2():
    """Driven qubit (dim 2): a 4th-order run at 16x finer slices is converged
    (doubling N again changes it by < 1e-10), and the default 2nd-order run's
    error against it shrinks 4x when its own slices are halved."""
    wf = synth.driven_qubit(n_slices=160_000, h=0.01 / 16, order=4)
    Uf = orc.propagate(wf.H0, wf.Hk, wf.samples, wf.h, 4)
    wff = synth.driven_qubit(n_slices=320_000, h=0.01 / 32, order=4)
    Uff = orc.propagate(wff.H0, wff.Hk, wff.samples, wff.h, 4)
    assert orc.relative_frobenius(Uf, Uff) < 1e-10
    assert orc.unitarity_defect(Uf) < 1e-10
    w = synth.driven_qubit(n_slices=10_000)
    e1 = orc.relative_frobenius(orc.propagate(w.H0, w.Hk, w.samples, w.h, 2), Uf)
    w2 = synth.driven_qubit(n_slices=20_000, h=0.005)
    e2 = orc.relative_frobenius(orc.propagate(w2.H0, w2.Hk, w2.samples, w2.h, 2), Uf)
    assert 3.8 < e1 / e2 < 4.2


def test_frechet_matches_block_exponential():
    assert pin_frechet() < 1e-12


@pytest.mark.parametrize("order", [2, 4])
def test_gradient_matches_central_differences(order):
    assert fd_gradient_error(order) < 1e-6


def test_gradient_commuting_closed_form():
    assert commuting_gradient_error() < 1e-13


def test_fidelity_loss_special_values():
    rng = np.random.default_rng(1)
    U = synth.haar_unitary(rng, 4)
    assert abs(orc.fidelity_loss(U, U)) < 1e-14
    assert abs(orc.fidelity_loss(U, np.exp(0.7j) * U)) < 1e-14
    # traceless relative rotation: Tr(V^H U) = 0
    V = U @ np.diag([1, -1, 1j, -1j])
    assert abs(orc.fidelity_loss(U, V) - 1.0) < 1e-14


def test_magnus_effective_controls_identity():
    """Eq. magnus_coeffs: the commutator term equals a weighted sum of the
    effective control Hamiltonians i[H0,H_k], i[H_k,H_k'] (k<k'); count 3K/2+K^2/2."""
    rng = np.random.default_rng(21)
    d, K = 6, 3
    H0 = rand_herm(rng, d)
    Hk = np.stack([rand_herm(rng, d) for _ in range(K)])
    s = rng.standard_normal((K, 3))
    h = 0.37
    A = [H0 + sum(s[k, i] * Hk[k] for k in range(K)) for i in range(3)]
    G = orc.magnus4_exponent(A[0][None], A[1][None], A[2][None], h)[0]
    basis, w = [H0], [h]
    for k in range(K):
        basis.append(Hk[k]); w.append(h / 6 * (s[k, 0] + 4 * s[k, 1] + s[k, 2]))
    for k in range(K):
        basis.append(1j * (H0 @ Hk[k] - Hk[k] @ H0)); w.append(h * h / 12 * (s[k, 2] - s[k, 0]))
    for k in range(K):
        for kk in range(k + 1, K):
            basis.append(1j * (Hk[k] @ Hk[kk] - Hk[kk] @ Hk[k]))
            w.append(h * h / 12 * (s[k, 0] * s[kk, 2] - s[k, 2] * s[kk, 0]))
    assert len(basis) - 1 == (3 * K + K * K) // 2
    for B in basis:
        assert np.max(np.abs(B - B.conj().T)) < 1e-14
    assert np.max(np.abs(G - sum(wi * Bi for wi, Bi in zip(w, basis)))) < 1e-14


# --------------------------------------------------------- mutation check

def _mut_sign(A1, A2, A3, h):
    return (h / 6.0) * (A1 + 4.0 * A2 + A3) - 1j * (h * h / 12.0) * (A1 @ A3 - A3 @ A1)


def _mut_drop_comm(A1, A2, A3, h):
    return (h / 6.0) * (A1 + 4.0 * A2 + A3)


def _mut_trapezoid(A1, A2, A3, h):
    return (h / 2.0) * (A1 + A3) + 1j * (h * h / 12.0) * (A1 @ A3 - A3 @ A1)


def _mut_expm_sign(G):
    lam, Q = np.linalg.eigh(G)
    return (Q * np.exp(1j * lam)[..., None, :]) @ np.conj(np.swapaxes(Q, -1, -2))


def _mut_expm_transpose(G):
    lam, Q = np.linalg.eigh(G)
    return (Q * np.exp(-1j * lam)[..., None, :]) @ np.swapaxes(Q, -1, -2)


def _mut_order(Us, U=None):
    d = Us.shape[-1]
    U = np.eye(d, dtype=np.complex128) if U is None else U
    for j in range(Us.shape[0]):
        U = U @ Us[j]
    return U


def _all_pins_ok():
    checks = [
        pin_pauli() < 1e-14,
        pin_expm_scipy() < 2e-12,
        pin_static() < 1e-12,
        pin_product_order() < 1e-14,
        drive_error(4096, 4) < 1e-11,
        abs(pin_slope(2) - 2.0) < 0.03,
        abs(pin_slope(4) - 4.0) < 0.05,
        fd_gradient_error(2) < 1e-6,
        fd_gradient_error(4) < 1e-6,
        commuting_gradient_error() < 1e-13,
    ]
    return all(checks)


@pytest.mark.parametrize("name,attr,fn", [
    ("commutator sign flipped", "magnus4_exponent", _mut_sign),
    ("commutator dropped", "magnus4_exponent", _mut_drop_comm),
    ("Simpson replaced by trapezoid", "magnus4_exponent", _mut_trapezoid),
    ("exponent sign flipped", "expm_minus_i", _mut_expm_sign),
    ("Q^T instead of Q^H", "expm_minus_i", _mut_expm_transpose),
    ("product order reversed", "ordered_product", _mut_order),
])
def test_planted_mistakes_are_caught(monkeypatch, name, attr, fn):
    assert _all_pins_ok()
    monkeypatch.setattr(orc, attr, fn)
    assert not _all_pins_ok(), f"no pin caught: {name}"


def test_planted_gradient_mistakes_are_caught(monkeypatch):
    orig = orc.frechet_expm_minus_i

    def transposed(G, E):
        return orig(G, np.swapaxes(E, -1, -2))

    def conj_phase(G, E):
        return np.conj(orig(G, E))

    for bad in (transposed, conj_phase):
        monkeypatch.setattr(orc, "frechet_expm_minus_i", bad)
        assert fd_gradient_error(2) > 1e-3 or fd_gradient_error(4) > 1e-3
    monkeypatch.setattr(orc, "frechet_expm_minus_i", orig)


def test_planted_sampling_mistake_is_caught():
    """Left-endpoint instead of midpoint samples drops the midpoint rule to first order."""
    ns = [16, 32, 64, 128]
    e = []
    for n in ns:
        w = synth.circular_drive(n, 2)
        t = np.arange(n) * w.h   # left endpoints
        c = np.stack([np.cos(t), np.sin(t)])
        U = orc.propagate(w.H0, w.Hk, c, w.h, 2)
        e.append(orc.relative_frobenius(U, circular_drive_exact(1.0, 0.1, 1.0, 6.0)))
    slope = -np.polyfit(np.log(ns), np.log(e), 1)[0]
    assert abs(slope - 2.0) > 0.5


def test_trajectory_static_closed_form_and_end_point():
    """Constant H: every partial product is exp(-i H t_j), from one
    eigendecomposition at each time; the last one is propagate()'s U(T)."""
    import synth
    w = synth.random_system(5, 2, n_slices=40, h=0.03, order=2, tag=21)
    c = np.repeat(np.array([[0.7], [-0.2]]), 40, axis=1)
    H = w.H0 + 0.7 * w.Hk[0] - 0.2 * w.Hk[1]
    P = orc.trajectory(w.H0, w.Hk, c, 0.03, 2)
    lam, Q = np.linalg.eigh(H)
    for j in (0, 1, 17, 40):
        ref = (Q * np.exp(-1j * lam * 0.03 * j)) @ Q.conj().T
        assert np.max(np.abs(P[j] - ref)) < 1e-13
    w4 = synth.random_system(4, 2, n_slices=33, h=0.05, order=4, tag=22)
    P4 = orc.trajectory(w4.H0, w4.Hk, w4.samples, w4.h, 4)
    assert P4.shape == (34, 4, 4)
    assert np.max(np.abs(P4[-1] - orc.propagate(w4.H0, w4.Hk, w4.samples, w4.h, 4))) < 1e-13
    assert np.allclose(P4[0], np.eye(4))


def test_trajectory_follows_circular_drive_closed_form():
    """The driven two-level system's closed-form U(t) (rotating frame) at
    every slice boundary, to the 4th-order Magnus accuracy."""
    import synth
    w = synth.circular_drive(n_slices=400, order=4)
    P = orc.trajectory(w.H0, w.Hk, w.samples, w.h, 4)
    w0, w1, wr = w.meta["w0"], w.meta["w1"], w.meta["wrf"]
    sz = np.diag([1.0, -1.0]).astype(complex)
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    for j in (0, 100, 257, 400):
        t = j * w.h
        rot = scipy.linalg.expm(-1j * wr * t * sz / 2)
        eff = scipy.linalg.expm(-1j * t * (0.5 * (w0 - wr) * sz + 0.5 * w1 * sx))
        assert np.max(np.abs(P[j] - rot @ eff)) < 1e-8
