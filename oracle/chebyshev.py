"""Chebyshev-series exponential of a Hermitian matrix, as the paper defines it.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run this module.  It shares
no code with the HIP library.

What it computes (Matrix exponential section):

* the truncated Chebyshev series of exp(-i G) for Hermitian G whose spectrum
  lies in [alpha, beta] (eq. chebychev_series):
      exp(-i G) ~ exp(-i (alpha+beta)/2) [a_0 I + 2 sum_{k=1}^{m} a_k T_k(X)],
      X = 2/(beta-alpha) (G - (alpha+beta)/2 I),
      a_k = (-i)^k J_k((beta-alpha)/2)      (Bessel functions of the first kind),
  evaluated by the Clenshaw recurrence of Algorithm 1:
      D_{m+2} = D_{m+1} = 0,  D_k = a_k I + 2 X D_{k+1} - D_{k+2}  (k = m..0),
      result = exp(-i (alpha+beta)/2) (D_0 - D_2);
* Lubich's truncation-error estimate (eq. error_chebychev)
      eps(m, w) = 4 (exp(1 - (w/(4m+4))^2) w/(4m+4))^(m+1),  w = beta - alpha,
  and the largest ||G|| for which eps <= u when alpha = -||G||, beta = ||G||
  (the construction of Table 1).

scipy.special.jv supplies the Bessel values (a library routine used as a
step); everything else is written out.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special


def chebyshev_coefficients(alpha: float, beta: float, m: int) -> np.ndarray:
    """a_k = (-i)^k J_k((beta - alpha)/2), k = 0..m."""
    z = 0.5 * (beta - alpha)
    k = np.arange(m + 1)
    return ((-1j) ** k) * scipy.special.jv(k, z)


def chebyshev_expm_minus_i(G: np.ndarray, alpha: float, beta: float, m: int) -> np.ndarray:
    """exp(-i G) by the degree-m Chebyshev series on [alpha, beta], Clenshaw form."""
    G = np.asarray(G, np.complex128)
    d = G.shape[0]
    eye = np.eye(d, dtype=np.complex128)
    X = (2.0 / (beta - alpha)) * (G - 0.5 * (alpha + beta) * eye)
    a = chebyshev_coefficients(alpha, beta, m)
    d1 = np.zeros((d, d), np.complex128)   # D_{k+1}
    d2 = np.zeros((d, d), np.complex128)   # D_{k+2}
    keep = None
    for k in range(m, -1, -1):
        dk = a[k] * eye + 2.0 * (X @ d1) - d2
        if k == 0:
            keep = d2                      # D_2 when D_0 is formed
        d2, d1 = d1, dk
    return np.exp(-0.5j * (alpha + beta)) * (d1 - keep)


def chebyshev_series_direct(G: np.ndarray, alpha: float, beta: float, m: int) -> np.ndarray:
    """The same truncated series summed term by term with the three-term
    recurrence T_0 = I, T_1 = X, T_{k+1} = 2 X T_k - T_{k-1} (test helper)."""
    G = np.asarray(G, np.complex128)
    d = G.shape[0]
    eye = np.eye(d, dtype=np.complex128)
    X = (2.0 / (beta - alpha)) * (G - 0.5 * (alpha + beta) * eye)
    a = chebyshev_coefficients(alpha, beta, m)
    t_prev, t = eye, X
    total = a[0] * eye
    if m >= 1:
        total = total + 2.0 * a[1] * X
    for k in range(2, m + 1):
        t_prev, t = t, 2.0 * X @ t - t_prev
        total = total + 2.0 * a[k] * t
    return np.exp(-0.5j * (alpha + beta)) * total


def lubich_error(m: int, width: float) -> float:
    """eps(m, beta - alpha) of eq. error_chebychev."""
    rho = width / (4.0 * m + 4.0)
    return 4.0 * (math.exp(1.0 - rho * rho) * rho) ** (m + 1)


def chebyshev_norm_limit(m: int, u: float) -> float:
    """Largest ||G|| with eps(m, 2 ||G||) <= u (alpha = -||G||, beta = ||G||).

    eps is increasing in rho = 2||G||/(4m+4) up to rho = 1/sqrt(2), where
    exp(1 - rho^2) rho peaks, so the root is bracketed in (0, 1/sqrt(2))."""
    lo, hi = 0.0, 1.0 / math.sqrt(2.0)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if lubich_error(m, mid * (4.0 * m + 4.0)) <= u:
            lo = mid
        else:
            hi = mid
    return lo * (4.0 * m + 4.0) / 2.0
