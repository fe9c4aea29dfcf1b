"""Error bounds of the reduced-precision paths against the FP64 oracle.

These paths have no oracle of their own (their results differ from the
exact propagator by rounding in the working precision); each result's error
against the FP64 oracle must stay inside a bound derived from the arithmetic
of a plain reduced-precision chain of slice propagators.

Relative Frobenius error of U(T) over n slices of dimension d, in the
probabilistic model of rounding (independent errors add in quadrature:
a d-term sum carries ~sqrt(d) u, n independent slice errors ~sqrt(n)):

* FP32 products (4 real products per complex product): an entry of a
  product of unitary-scale matrices is a d-term sum whose terms total at
  most 1 in magnitude (Cauchy-Schwarz over unit rows and columns), so it
  carries ~sqrt(d) u32 absolute error against entries of RMS size
  1/sqrt(d): d u32 relative error per product, u32 = 2^-24; a slice takes at
  most four products at the norms of these workloads (the planner's Taylor
  products plus the chain product), and the n slices add in quadrature:
      tol(n, d) = 4 sqrt(n) d u32;
* 3M products carry their imaginary parts on the (|Ar|+|Ai|)(|Br|+|Bi|)
  scale, up to twice the 4M bound (Higham, Accuracy and Stability of
  Numerical Algorithms, section 3.6): a factor 2;
* BF16 split (hi*hi + hi*lo + lo*hi, FP32 accumulation): a split operand
  x_hi + x_lo carries 2^-16 relative error (two 8-bit significands) and the
  dropped lo*lo term is below it; per real product that is ~sqrt(d) 2^-16
  relative in the model above; each part of a complex product is a sum of
  two real products (four-product form), or in the 3M form carries up to
  twice that, and a slice takes four complex products (4 * 2 * 2 = 16,
  which covers either form):
      tol(n, d) = 16 sqrt(n) sqrt(d) 2^-16;
* slices that need s squarings: each squaring doubles the relative error of
  the Taylor step, a factor 2^s.

A single stored slice (per-slice output in complex64) carries the error of
one slice (n = 1) plus the rounding of its entries (|U_ij| <= 1) to complex64,
u32.

The library carries each reduced-precision slice as I + E and accumulates
the chain in FP64, whose errors are far below these bounds, so they remain
upper bounds; every test prints the measured error beside its bound.
"""
from __future__ import annotations

import math

U32 = 2.0 ** -24
UBF = 2.0 ** -16

FP64, FP32, FP32_3M, BF16_SPLIT = 0, 1, 2, 3
TOL64 = 1e-10


def tol(prec: int, n: int, d: int, s: int = 0) -> float:
    """Bound on the relative Frobenius error of U(T) for precision `prec`
    over n slices of dimension d whose exponentials take s squarings."""
    if prec == FP64:
        return TOL64
    n = max(int(n), 1)
    if prec == BF16_SPLIT:
        return 16.0 * math.sqrt(n) * math.sqrt(d) * UBF * 2.0 ** s
    c3m = 2.0 if prec == FP32_3M else 1.0
    return 4.0 * math.sqrt(n) * d * U32 * c3m * 2.0 ** s


def tol_slice(prec: int, d: int, s: int = 0) -> float:
    """Bound on the max-abs error of one stored complex64 slice."""
    return tol(prec, 1, d, s) + U32


def max_squarings(pm, w, prec: int, shift: bool = False) -> int:
    """Squarings the library's planner takes for the largest slice exponent
    of workload w (1-norm from the oracle's exponents; with shift, of
    G - (tr G / d) I, as the engine of dimensions <= 4 plans).  The
    commutator-free scheme plans each of its two exponentials per slice."""
    import numpy as np

    import oracle.propagator as orc
    if w.order == orc.CF4:
        G = np.concatenate(orc.cf4_exponents(w.H0, w.Hk, w.samples, w.h))
    else:
        G = orc.slice_exponents(w.H0, w.Hk, w.samples, w.h, w.order)
    if shift:
        d = G.shape[-1]
        G = G - (np.trace(G, axis1=-2, axis2=-1) / d)[:, None, None] * np.eye(d)
    nu = float(np.max(np.sum(np.abs(G), axis=-2)))
    return pm.plan_expm(nu, prec, n_slices=w.n_slices)[1]
