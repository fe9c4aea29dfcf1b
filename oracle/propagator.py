"""Plain FP64 oracle of the parallel-in-time Schrodinger propagator.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run this module.  It shares
no code with the HIP library and imports nothing from it; its inputs come from
the seeded generators in ``synth`` (which hold none of the method's
arithmetic).

What it computes, written as the plain definitions (units with hbar = 1, so
U = exp(-i H t), Computational approach section):

* slice exponents G_j (Hermitian), one per slice of width h:
  - midpoint rule: G_j = h * H(t_j + h/2), with H(t) = H0 + sum_k c_k(t) H_k
    (eq. format_control; "simply set G = H dt" in the Implementation section);
  - 4th-order Magnus (Magnus integrators section, Simpson rule for Omega_1 and
    the two-point rule for Omega_2): with A1, A2, A3 the Hamiltonian at the
    start, middle and end of the slice,
        G_j = (h/6)(A1 + 4 A2 + A3) + i (h^2/12) [A1, A3].
    The commutator sign is the one that makes U = exp(-i G) the 4th-order
    step for the standard product order (later slices on the left); the
    paper prints the opposite sign, which gives 4th order only in the
    transposed, reversed-order view (our reading of that sign).
    The commutator is formed from the assembled A1, A3, never through
    effective control Hamiltonians.
  - commutator-free 4th order (the alternative the Magnus integrators
    section names for higher orders, after Alvermann and Fehske; the
    two-exponential scheme of Blanes and Moan): with M1 = integral of H
    and M2 = (1/h) integral of (t - t_mid) H over the slice, both by
    Simpson's rule on the same three samples,
        U_j = exp(-i (M1/2 + 2 M2)) exp(-i (M1/2 - 2 M2))
            = exp(-i (h/12)(-A1 + 4 A2 + 3 A3)) exp(-i (h/12)(3 A1 + 4 A2 - A3)),
    whose combined exponent is M1 + i [M1, M2] up to O(h^5), the commutator
    Magnus exponent above; no commutator of the controls is formed.
    Scheme code CF4 (= 5) in the ``order`` argument.
  - sixth-order Magnus (the higher-order Magnus integrators the Magnus
    integrators section points to, with their extra commutators; the
    three-node scheme of Blanes, Casas and Ros, BIT 2000): with the slice's
    Hamiltonian sampled at the Gauss-Legendre nodes t_j + c_i h,
    c = 1/2 - sqrt(15)/10, 1/2, 1/2 + sqrt(15)/10 (three samples per slice,
    3N in all), and A_i = -i H(t_j + c_i h) the generator of Y' = A Y,
        a1 = h A_2,  a2 = (sqrt(15) h / 3)(A_3 - A_1),
        a3 = (10 h / 3)(A_3 - 2 A_2 + A_1),
        C1 = [a1, a2],  C2 = -(1/60) [a1, 2 a3 + C1],
        Omega = a1 + a3 / 12 + (1/240) [-20 a1 - a3 + C1, a2 + C2],
    and G_j = i Omega (Hermitian), U_j = exp(Omega) = exp(-i G_j).
    Scheme code M6 (= 6) in the ``order`` argument.
* slice propagators U_j = exp(-i G_j) by Hermitian eigendecomposition:
  G = Q diag(lam) Q^H  =>  exp(-i G) = Q diag(exp(-i lam)) Q^H (the
  decomposition route of the Matrix exponential section: for Hermitian
  matrices the Schur form is diagonal).
* the ordered product U(T) = U_{N-1} ... U_1 U_0 (eq. slices), taken
  sequentially, one factor at a time.
* the gate-fidelity loss L = 1 - |Tr(V^H U)|^2 / d^2 and its gradient with
  respect to every control sample, from prefix/suffix products and the
  Frechet derivative of exp(-i G) in Daleckii-Krein form (divided differences
  of f(x) = exp(-i x) on the eigenvalues).

Everything is complex128 / float64.  Loops over slices are plain Python;
batched LAPACK (numpy.linalg.eigh) is used for the eigendecompositions.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "hamiltonian_samples",
    "CF4",
    "n_slices",
    "magnus4_exponent",
    "cf4_exponents",
    "M6",
    "GL3_NODES",
    "magnus6_exponent",
    "slice_propagators",
    "slice_exponents",
    "expm_minus_i",
    "ordered_product",
    "propagate",
    "trajectory",
    "unitarity_defect",
    "fidelity_loss",
    "fidelity_grad_U",
    "frechet_expm_minus_i",
    "control_gradient",
    "relative_frobenius",
]

_CHUNK = 8192

CF4 = 5   # scheme code of the commutator-free fourth-order integrator
M6 = 6    # scheme code of the sixth-order Magnus integrator

# Gauss-Legendre nodes of three points on [0, 1]: the sixth-order scheme's
# sample positions within a slice
GL3_NODES = (0.5 - 15.0 ** 0.5 / 10.0, 0.5, 0.5 + 15.0 ** 0.5 / 10.0)


def n_slices(order: int, n_samples: int) -> int:
    """Slices covered by n_samples samples: one sample per slice for the
    midpoint rule, three per slice for the sixth-order scheme (3N in all),
    three per slice with shared ends (2N + 1 in all) otherwise."""
    if order == 2:
        return n_samples
    if order == M6:
        return n_samples // 3
    return (n_samples - 1) // 2


def hamiltonian_samples(H0: np.ndarray, Hk: np.ndarray, samples: np.ndarray) -> np.ndarray:
    """H at every sample: H0 + sum_k c_k H_k (eq. format_control). -> [S, d, d]."""
    H0 = np.asarray(H0, dtype=np.complex128)
    Hk = np.asarray(Hk, dtype=np.complex128)
    c = np.asarray(samples, dtype=np.float64)
    out = np.broadcast_to(H0, (c.shape[1],) + H0.shape).copy()
    for k in range(Hk.shape[0]):
        out += c[k][:, None, None] * Hk[k][None]
    return out


def magnus4_exponent(A1: np.ndarray, A2: np.ndarray, A3: np.ndarray, h: float) -> np.ndarray:
    """4th-order commutator-Magnus exponent for a slice of width h.

    Omega_1 = -i * integral of H by Simpson's rule, Omega_2 = (h^2/12)[A1, A3]
    (two-point rule, eq. magnus), G = i * Omega: G = (h/6)(A1+4A2+A3) + i(h^2/12)[A1,A3].
    """
    comm = A1 @ A3 - A3 @ A1
    return (h / 6.0) * (A1 + 4.0 * A2 + A3) + 1j * (h * h / 12.0) * comm


def magnus6_exponent(A1: np.ndarray, A2: np.ndarray, A3: np.ndarray, h: float) -> np.ndarray:
    """Sixth-order Magnus exponent G (Hermitian, U = exp(-i G)) of a slice of
    width h from H at its three Gauss-Legendre nodes (A1, A2, A3 = H at
    t + c_1 h, t + c_2 h, t + c_3 h; batched over leading axes).

    The steps are those of the scheme, in the notation of the Magnus
    expansion for Y' = A Y with A = -i H: the three moments a1, a2, a3, the
    commutators C1, C2, then Omega, and G = i Omega.
    """
    def comm(x, y):
        return x @ y - y @ x
    B1, B2, B3 = -1j * A1, -1j * A2, -1j * A3
    r15 = 15.0 ** 0.5
    a1 = h * B2
    a2 = (r15 * h / 3.0) * (B3 - B1)
    a3 = (10.0 * h / 3.0) * (B3 - 2.0 * B2 + B1)
    C1 = comm(a1, a2)
    C2 = -(1.0 / 60.0) * comm(a1, 2.0 * a3 + C1)
    omega = a1 + a3 / 12.0 + (1.0 / 240.0) * comm(-20.0 * a1 - a3 + C1, a2 + C2)
    return 1j * omega


def slice_exponents(H0, Hk, samples, h: float, order: int, start: int = 0, stop: int | None = None) -> np.ndarray:
    """Hermitian slice exponents G_j for slices [start, stop)."""
    samples = np.asarray(samples, dtype=np.float64)
    if order == 2:
        n = samples.shape[1]
        stop = n if stop is None else stop
        return h * hamiltonian_samples(H0, Hk, samples[:, start:stop])
    if order == 4:
        n = (samples.shape[1] - 1) // 2
        stop = n if stop is None else stop
        A = hamiltonian_samples(H0, Hk, samples[:, 2 * start: 2 * stop + 1])
        return magnus4_exponent(A[0:-1:2], A[1::2], A[2::2], h)
    if order == M6:
        n = samples.shape[1] // 3
        stop = n if stop is None else stop
        A = hamiltonian_samples(H0, Hk, samples[:, 3 * start: 3 * stop])
        return magnus6_exponent(A[0::3], A[1::3], A[2::3], h)
    raise ValueError("order must be 2, 4 or 6")


def cf4_exponents(H0, Hk, samples, h: float, start: int = 0, stop: int | None = None):
    """(G_first, G_second) of the commutator-free 4th-order scheme for slices
    [start, stop): U_j = exp(-i G_second[j]) exp(-i G_first[j]) with
    G_first = (h/12)(3 A1 + 4 A2 - A3), G_second = (h/12)(-A1 + 4 A2 + 3 A3)."""
    samples = np.asarray(samples, dtype=np.float64)
    n = (samples.shape[1] - 1) // 2
    stop = n if stop is None else stop
    A = hamiltonian_samples(H0, Hk, samples[:, 2 * start: 2 * stop + 1])
    A1, A2, A3 = A[0:-1:2], A[1::2], A[2::2]
    return (h / 12.0) * (3.0 * A1 + 4.0 * A2 - A3), (h / 12.0) * (-A1 + 4.0 * A2 + 3.0 * A3)


def slice_propagators(H0, Hk, samples, h: float, order: int, start: int = 0, stop: int | None = None):
    """U_j for slices [start, stop): exp(-i G_j), or for CF4 the product of
    its two exponentials (the second on the left)."""
    if order == CF4:
        Gf, Gs = cf4_exponents(H0, Hk, samples, h, start, stop)
        return expm_minus_i(Gs) @ expm_minus_i(Gf)
    return expm_minus_i(slice_exponents(H0, Hk, samples, h, order, start, stop))


def expm_minus_i(G: np.ndarray) -> np.ndarray:
    """exp(-i G) for Hermitian G (batched), by eigendecomposition."""
    lam, Q = np.linalg.eigh(G)
    return (Q * np.exp(-1j * lam)[..., None, :]) @ np.conj(np.swapaxes(Q, -1, -2))


def ordered_product(Us: np.ndarray, U: np.ndarray | None = None) -> np.ndarray:
    """U <- U_j U for j = 0, 1, ... in order (later slices on the left)."""
    d = Us.shape[-1]
    U = np.eye(d, dtype=np.complex128) if U is None else U
    for j in range(Us.shape[0]):
        U = Us[j] @ U
    return U


def propagate(H0, Hk, samples, h: float, order: int, return_slices: bool = False):
    """U(T) = U_{N-1} ... U_0 with U_j = exp(-i G_j).  Optionally all U_j."""
    samples = np.asarray(samples, dtype=np.float64)
    n = n_slices(order, samples.shape[1])
    d = np.asarray(H0).shape[0]
    U = np.eye(d, dtype=np.complex128)
    slices = np.empty((n, d, d), dtype=np.complex128) if return_slices else None
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        Uj = slice_propagators(H0, Hk, samples, h, order, s, e)
        if return_slices:
            slices[s:e] = Uj
        U = ordered_product(Uj, U)
    return (U, slices) if return_slices else U


def trajectory(H0, Hk, samples, h: float, order: int) -> np.ndarray:
    """Every partial product P_j = U_{j-1} ... U_0, j = 0..N (P_0 = I,
    P_N = U(T)), taken sequentially: the time evolution at each slice
    boundary t_j = j h (eq. slices read at intermediate times)."""
    samples = np.asarray(samples, dtype=np.float64)
    n = n_slices(order, samples.shape[1])
    d = np.asarray(H0).shape[0]
    out = np.empty((n + 1, d, d), dtype=np.complex128)
    out[0] = np.eye(d)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        Uj = slice_propagators(H0, Hk, samples, h, order, s, e)
        for q in range(e - s):
            out[s + q + 1] = Uj[q] @ out[s + q]
    return out


def unitarity_defect(U: np.ndarray) -> float:
    """||U^H U - I||_F."""
    d = U.shape[-1]
    return float(np.linalg.norm(np.conj(U.T) @ U - np.eye(d)))


def relative_frobenius(A: np.ndarray, B: np.ndarray) -> float:
    """||A - B||_F / ||B||_F."""
    return float(np.linalg.norm(A - B) / np.linalg.norm(B))


def fidelity_loss(U: np.ndarray, V: np.ndarray) -> float:
    """L = 1 - |Tr(V^H U)|^2 / d^2."""
    d = U.shape[-1]
    g = np.trace(np.conj(V.T) @ U)
    return float(1.0 - abs(g) ** 2 / d ** 2)


def fidelity_grad_U(U: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Gradient of the fidelity loss in the convention dL = Re Tr(W^H dU):
    W = 2 dL/d(conj U) = -(2 g / d^2) V with g = Tr(V^H U)."""
    d = U.shape[-1]
    g = np.trace(np.conj(V.T) @ U)
    return -(2.0 * g / d ** 2) * V


def frechet_expm_minus_i(G: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Directional derivative of f(G) = exp(-i G) at Hermitian G along E.

    Daleckii-Krein: with G = Q diag(lam) Q^H,
    L_f(G, E) = Q [ (Q^H E Q) o Phi ] Q^H, Phi_ab = f[lam_a, lam_b] the divided
    difference of f, here -i exp(-i (lam_a+lam_b)/2) sinc((lam_a-lam_b)/2)
    (which is exact also on the diagonal, where it equals f'(lam_a)).
    """
    lam, Q = np.linalg.eigh(G)
    Qh = np.conj(np.swapaxes(Q, -1, -2))
    la = lam[..., :, None]
    lb = lam[..., None, :]
    phi = -1j * np.exp(-0.5j * (la + lb)) * np.sinc((la - lb) / (2.0 * np.pi))
    return Q @ ((Qh @ E @ Q) * phi) @ Qh


def control_gradient(H0, Hk, samples, h: float, order: int, W: np.ndarray):
    """dL/d samples for a real loss L(U(T)) whose gradient is W (dL = Re Tr(W^H dU)).

    With P_j = U_{j-1}...U_0, S_j = U_{N-1}...U_{j+1}:
      dL = Re sum_j Tr(W^H S_j dU_j P_j) = Re sum_j Tr(Fg_j dG_j),
      Fg_j = L_f(G_j, Lam_j),  Lam_j = P_j W^H S_j
    (cyclic trace and Tr(A L_f(G,E)) = Tr(L_f(G,A) E), f's divided differences
    being symmetric).  dG_j / d sample comes from differentiating the slice
    exponent as defined above.  Returns (U(T), grad[K, n_samples]).
    """
    H0 = np.asarray(H0, np.complex128)
    Hk = np.asarray(Hk, np.complex128)
    samples = np.asarray(samples, np.float64)
    if order == CF4:
        return _control_gradient_cf4(H0, Hk, samples, h, W)
    if order == M6:
        raise NotImplementedError("the sixth-order scheme has no gradient here")
    n = n_slices(order, samples.shape[1])
    d = H0.shape[0]
    G = slice_exponents(H0, Hk, samples, h, order)
    Us = expm_minus_i(G)
    P = np.empty_like(Us)
    acc = np.eye(d, dtype=np.complex128)
    for j in range(n):
        P[j] = acc
        acc = Us[j] @ acc
    U = acc
    S = np.empty_like(Us)
    acc = np.eye(d, dtype=np.complex128)
    for j in range(n - 1, -1, -1):
        S[j] = acc
        acc = acc @ Us[j]
    Wh = np.conj(W.T)
    Lam = P @ Wh[None] @ S
    Fg = frechet_expm_minus_i(G, Lam)
    K = Hk.shape[0]
    grad = np.zeros((K, samples.shape[1]))

    def re_tr(Fa, B):
        # Re Tr(Fa @ B) for batched Fa and one matrix B
        return np.real(np.einsum("nab,ba->n", Fa, B))

    if order == 2:
        for k in range(K):
            grad[k] = h * re_tr(Fg, Hk[k])
        return U, grad
    A = hamiltonian_samples(H0, Hk, samples)
    A1, A3 = A[0:-1:2], A[2::2]
    c2 = h * h / 12.0
    for k in range(K):
        Hkk = Hk[k]
        # d/ds0: (h/6) H_k + i c2 [H_k, A3];  d/ds2: (h/6) H_k + i c2 [A1, H_k];  d/ds1: (4h/6) H_k
        d0 = (h / 6.0) * Hkk[None] + 1j * c2 * (Hkk[None] @ A3 - A3 @ Hkk[None])
        d2 = (h / 6.0) * Hkk[None] + 1j * c2 * (A1 @ Hkk[None] - Hkk[None] @ A1)
        g0 = np.real(np.einsum("nab,nba->n", Fg, d0))
        g2 = np.real(np.einsum("nab,nba->n", Fg, d2))
        g1 = (4.0 * h / 6.0) * re_tr(Fg, Hkk)
        grad[k, 0:2 * n:2] += g0
        grad[k, 1:2 * n:2] += g1
        grad[k, 2:2 * n + 1:2] += g2
    return U, grad


def _control_gradient_cf4(H0, Hk, samples, h: float, W: np.ndarray):
    """control_gradient for CF4: the 2N exponentials in product order
    (first factor of slice j at position 2j, second at 2j + 1) take the place
    of the slices; each exponent is linear in the samples,
    dG_first/d(s0, s1, s2) = (h/12)(3, 4, -1) H_k and
    dG_second/d(s0, s1, s2) = (h/12)(-1, 4, 3) H_k."""
    n = n_slices(CF4, samples.shape[1])
    d = H0.shape[0]
    Gf, Gs = cf4_exponents(H0, Hk, samples, h)
    G = np.empty((2 * n, d, d), np.complex128)
    G[0::2] = Gf
    G[1::2] = Gs
    Us = expm_minus_i(G)
    P = np.empty_like(Us)
    acc = np.eye(d, dtype=np.complex128)
    for v in range(2 * n):
        P[v] = acc
        acc = Us[v] @ acc
    U = acc
    S = np.empty_like(Us)
    acc = np.eye(d, dtype=np.complex128)
    for v in range(2 * n - 1, -1, -1):
        S[v] = acc
        acc = acc @ Us[v]
    Lam = P @ np.conj(W.T)[None] @ S
    Fg = frechet_expm_minus_i(G, Lam)
    K = Hk.shape[0]
    grad = np.zeros((K, samples.shape[1]))
    for k in range(K):
        t = np.real(np.einsum("nab,ba->n", Fg, Hk[k]))   # Re Tr(F_v H_k)
        tf, ts = t[0::2], t[1::2]
        grad[k, 0:2 * n:2] += (h / 12.0) * (3.0 * tf - ts)
        grad[k, 1:2 * n:2] += (h / 12.0) * (4.0 * tf + 4.0 * ts)
        grad[k, 2:2 * n + 1:2] += (h / 12.0) * (-tf + 3.0 * ts)
    return U, grad
