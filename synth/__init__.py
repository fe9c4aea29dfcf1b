"""Seeded synthetic workloads for the parallel-in-time Schrodinger propagator.

This module only draws inputs: Hermitian matrices, control samples, target
unitaries.  It contains none of the propagator's arithmetic (no slice
exponents, no exponentials, no products), so both the FP64 oracle and the GPU
path may take their inputs from here.

Workloads follow the shapes of the paper's experiments: a driven two-level
system (Numerical experiments section), random dense Hamiltonians of the form
H(t) = H0 + sum_k c_k(t) H_k (eq. format_control) with a few controls, a
3-qubit register, and a mix of such systems.  Samples are laid out as the
library expects them: ``samples[k, i]`` is control k at sample i, with

* order 2 (midpoint rule): n_samples = N, sample j at t = (j + 1/2) h;
* order 4 (Simpson + commutator Magnus): n_samples = 2N + 1, sample i at
  t = i h / 2, slice j using samples 2j, 2j+1, 2j+2;
* order 6 (sixth-order Magnus): n_samples = 3N, samples 3j, 3j+1, 3j+2 at
  the Gauss-Legendre nodes t = (j + c_i) h of slice j,
  c = 1/2 - sqrt(15)/10, 1/2, 1/2 + sqrt(15)/10.

Random draws use ``numpy.random.default_rng([SEED_BASE, tag])`` in a fixed
order: H0, then H_1..H_K, then control parameters, then the target.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_BASE = 210807126

PAULI_I = np.eye(2, dtype=np.complex128)
PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PAULI_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


@dataclass
class Workload:
    """One propagation problem: U(T) for H(t) = H0 + sum_k c_k(t) H_k."""

    name: str
    dim: int
    H0: np.ndarray            # [d, d] complex128, Hermitian
    Hk: np.ndarray            # [K, d, d] complex128, Hermitian
    samples: np.ndarray       # [K, n_samples] float64
    h: float                  # slice width
    order: int                # 2 or 4
    target: Optional[np.ndarray] = None   # [d, d] unitary (gradient workload)
    meta: dict = field(default_factory=dict)

    @property
    def n_ctrl(self) -> int:
        return int(self.Hk.shape[0])

    @property
    def n_samples(self) -> int:
        return int(self.samples.shape[1])

    @property
    def n_slices(self) -> int:
        if self.order == 2:
            return self.n_samples
        if self.order == 6:
            return self.n_samples // 3
        return (self.n_samples - 1) // 2


def rng_for(tag) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, int(tag)])


def gue(rng: np.random.Generator, d: int, spectral_norm: float) -> np.ndarray:
    """GUE draw A=(X+iY)/sqrt2, H=(A+A^H)/2, rescaled to a given 2-norm."""
    a = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    h = 0.5 * (a + a.conj().T)
    nrm = float(np.max(np.abs(np.linalg.eigvalsh(h))))
    return h * (spectral_norm / nrm)


def haar_unitary(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-random unitary: QR of a complex Ginibre matrix, R's diagonal phases removed."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


GL3 = (0.5 - math.sqrt(15.0) / 10.0, 0.5, 0.5 + math.sqrt(15.0) / 10.0)


def sample_times(n_slices: int, h: float, order: int) -> np.ndarray:
    """Times at which the controls are sampled (midpoints, the half-slice
    grid, or three Gauss-Legendre nodes per slice for order 6)."""
    if order == 2:
        return (np.arange(n_slices, dtype=np.float64) + 0.5) * h
    if order == 6:
        j = np.arange(n_slices, dtype=np.float64)[:, None]
        return ((j + np.array(GL3)[None, :]) * h).reshape(-1)
    return np.arange(2 * n_slices + 1, dtype=np.float64) * (0.5 * h)


def _sinusoid_params(rng, n_ctrl, n_terms):
    f = rng.uniform(0.5, 5.0, size=(n_ctrl, n_terms))
    a = rng.normal(0.0, 0.3, size=(n_ctrl, n_terms))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(n_ctrl, n_terms))
    return a, f, phi


def _sinusoid_eval(a, f, phi, t):
    # c_k(t) = sum_i a_ki sin(2 pi f_ki t + phi_ki)
    out = np.zeros((a.shape[0], t.size))
    for i in range(a.shape[1]):
        out += a[:, i:i + 1] * np.sin(2.0 * math.pi * f[:, i:i + 1] * t[None, :] + phi[:, i:i + 1])
    return out


def kron_all(*ops) -> np.ndarray:
    out = np.array([[1.0 + 0j]])
    for o in ops:
        out = np.kron(out, o)
    return out


# --------------------------------------------------------------------------
# The five workloads.  ``n_slices`` may be reduced for tests that need the
# oracle to finish quickly; all other parameters stay fixed.
# --------------------------------------------------------------------------

def driven_qubit(n_slices: int = 10_000, h: float = 0.01, order: int = 2) -> Workload:
    """Driven two-level system, dim 2: H0=(w0/2)sz, H1=sx, c(t)=W cos(w0 t),
    w0=2pi, W=2pi*0.05; T=100 at the default N=10^4, h=0.01."""
    w0 = 2.0 * math.pi
    amp = 2.0 * math.pi * 0.05
    t = sample_times(n_slices, h, order)
    c = (amp * np.cos(w0 * t))[None, :]
    return Workload("driven_qubit_d2", 2, 0.5 * w0 * PAULI_Z, PAULI_X[None].copy(), c, h, order,
                    meta={"w0": w0, "amp": amp})


def random_qudit(n_slices: int = 2 ** 17, h: float = 1e-3, order: int = 4,
                 dim: int = 16, n_ctrl: int = 3, tag: int = 2) -> Workload:
    """Random qudit, dim 16: seeded GUE H0 and 3 controls of 2-norm 1;
    c_k(t) = sum of 4 sinusoids, f~U[0.5,5], a~N(0,0.3^2), phi~U[0,2pi);
    4th-order Magnus, N=2^17 slices of width 1e-3."""
    rng = rng_for(tag)
    H0 = gue(rng, dim, 1.0)
    Hk = np.stack([gue(rng, dim, 1.0) for _ in range(n_ctrl)])
    a, f, phi = _sinusoid_params(rng, n_ctrl, 4)
    c = _sinusoid_eval(a, f, phi, sample_times(n_slices, h, order))
    return Workload(f"random_qudit_d{dim}", dim, H0, Hk, c, h, order)


def precision_sweep(n_slices: int = 2 ** 16, h: float = 0.01, order: int = 2,
                    dim: int = 64, n_ctrl: int = 2, n_segments: int = 64, tag: int = 3) -> Workload:
    """Dim 64: GUE H0 of 2-norm 10 plus 2 GUE controls of 2-norm 1 with
    piecewise-smooth amplitudes: the full span N*h is cut into 64 equal
    segments; per segment and control c = sum of 3 sinusoids (parameters as
    the random qudit), clipped to [-1, 1], with jumps at segment boundaries.
    Segment boundaries are fixed by the full-size span (2^16 slices) so a
    reduced N samples a prefix of the same waveform."""
    rng = rng_for(tag)
    H0 = gue(rng, dim, 10.0)
    Hk = np.stack([gue(rng, dim, 1.0) for _ in range(n_ctrl)])
    a, f, phi = _sinusoid_params(rng, n_ctrl * n_segments, 3)
    a = a.reshape(n_segments, n_ctrl, 3)
    f = f.reshape(n_segments, n_ctrl, 3)
    phi = phi.reshape(n_segments, n_ctrl, 3)
    t = sample_times(n_slices, h, order)
    span = (2 ** 16) * 0.01
    seg = np.minimum((t / span * n_segments).astype(np.int64), n_segments - 1)
    c = np.zeros((n_ctrl, t.size))
    for s in np.unique(seg):
        m = seg == s
        c[:, m] = _sinusoid_eval(a[s], f[s], phi[s], t[m])
    c = np.clip(c, -1.0, 1.0)
    return Workload(f"precision_sweep_d{dim}", dim, H0, Hk, c, h, order)


def qubit_register(n_slices: int = 4096, h: float = 0.1, tag: int = 4) -> Workload:
    """3-qubit register, dim 8: H0 = J(Z1Z2+Z2Z3+Z1Z3) + sum_q (w_q/2) Z_q,
    J=2pi*0.01, w_q=2pi*{0.10,0.12,0.14}; controls (W/2){X1,Y1,X2,Y2},
    W=2pi*0.05; piecewise-constant amplitudes u~U[-1,1] (one per slice,
    midpoint rule is then exact per slice); Haar target."""
    rng = rng_for(tag)
    I, X, Y, Z = PAULI_I, PAULI_X, PAULI_Y, PAULI_Z
    J = 2.0 * math.pi * 0.01
    wq = 2.0 * math.pi * np.array([0.10, 0.12, 0.14])
    z = [kron_all(Z, I, I), kron_all(I, Z, I), kron_all(I, I, Z)]
    H0 = J * (z[0] @ z[1] + z[1] @ z[2] + z[0] @ z[2]) + sum(0.5 * wq[q] * z[q] for q in range(3))
    om = 2.0 * math.pi * 0.05
    Hk = 0.5 * om * np.stack([kron_all(X, I, I), kron_all(Y, I, I), kron_all(I, X, I), kron_all(I, Y, I)])
    c = rng.uniform(-1.0, 1.0, size=(4, n_slices))
    V = haar_unitary(rng, 8)
    return Workload("qubit_register_d8", 8, H0, Hk, c, h, 2, target=V)


def batched_instances(n_inst: int = 512, tag: int = 5, max_slices: Optional[int] = None):
    """512 uneven instances: d~U{2,4,8,16,32,64}, K~U{1..4}, H0 GUE with
    2-norm log-uniform in [1,10], H_k GUE 2-norm 1, amplitudes as the random
    qudit, N=round(10^U[3,5]), order~U{2,4}, h=0.01.  ``max_slices`` caps N
    (for quick tests) without changing any other draw."""
    rng = rng_for(tag)
    out = []
    dims = [2, 4, 8, 16, 32, 64]
    for i in range(n_inst):
        d = int(dims[rng.integers(0, 6)])
        K = int(rng.integers(1, 5))
        nrm0 = float(10.0 ** rng.uniform(0.0, 1.0))
        n = int(round(10.0 ** rng.uniform(3.0, 5.0)))
        order = int((2, 4)[rng.integers(0, 2)])
        sub = np.random.default_rng([SEED_BASE, int(tag), i])
        H0 = gue(sub, d, nrm0)
        Hk = np.stack([gue(sub, d, 1.0) for _ in range(K)])
        a, f, phi = _sinusoid_params(sub, K, 4)
        if max_slices is not None:
            n = min(n, max_slices)
        h = 0.01
        c = _sinusoid_eval(a, f, phi, sample_times(n, h, order))
        out.append(Workload(f"inst{i}_d{d}", d, H0, Hk, c, h, order))
    return out


def circular_drive(n_slices: int, order: int, t_final: float = 6.0,
                   w0: float = 1.0, w1: float = 0.1, wrf: float = 1.0) -> Workload:
    """Qubit under a circularly polarised drive (eq. driven_hamiltonian):
    H = (w0/2) sz + cos(wrf t)(w1/2) sx + sin(wrf t)(w1/2) sy, with the
    parameters of the convergence figure (w0=1, w1=0.1, wrf=1, t=6)."""
    h = t_final / n_slices
    t = sample_times(n_slices, h, order)
    c = np.stack([np.cos(wrf * t), np.sin(wrf * t)])
    Hk = 0.5 * w1 * np.stack([PAULI_X, PAULI_Y])
    return Workload("circular_drive", 2, 0.5 * w0 * PAULI_Z, Hk, c, h, order,
                    meta={"w0": w0, "w1": w1, "wrf": wrf, "t": t_final})


def random_system(dim: int, n_ctrl: int, n_slices: int, h: float, order: int, tag: int,
                  h0_norm: float = 1.0) -> Workload:
    """Generic seeded GUE system with 4-sinusoid controls (test helper)."""
    rng = np.random.default_rng([SEED_BASE, 1000 + int(tag), dim, n_ctrl])
    H0 = gue(rng, dim, h0_norm)
    Hk = np.stack([gue(rng, dim, 1.0) for _ in range(n_ctrl)]) if n_ctrl > 0 else np.zeros((0, dim, dim), np.complex128)
    a, f, phi = _sinusoid_params(rng, max(n_ctrl, 1), 4)
    c = _sinusoid_eval(a, f, phi, sample_times(n_slices, h, order))[:n_ctrl]
    return Workload(f"random_d{dim}_k{n_ctrl}", dim, H0, Hk, c, h, order)


WORKLOADS = {
    "driven_qubit": driven_qubit,
    "random_qudit": random_qudit,
    "precision_sweep": precision_sweep,
    "qubit_register": qubit_register,
}
