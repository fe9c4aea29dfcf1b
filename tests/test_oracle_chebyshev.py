"""Pins of the Chebyshev-series exponential oracle (oracle/chebyshev.py).

Each pin checks the oracle against something other than itself: the
paper's printed Table 1, a second evaluation route of the same series, the
closed form of the scalar expansion, and the exact exponential within the
truncation bound.  A planted mistake in the coefficients' phase or in the
Clenshaw return value fails one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle.chebyshev as cb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "chebyshev_table1.txt")


def _table():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                rows.append((int(line[0]), line[1], line[2]))
    return rows


def _digits_match(value: float, printed: str) -> bool:
    """value agrees with the printed number to the printed digits."""
    if "e" in printed:
        mant, exp = printed.split("e")
        dec = len(mant.split(".")[1]) if "." in mant else 0
        step = 10.0 ** (int(exp) - dec)
    else:
        dec = len(printed.split(".")[1]) if "." in printed else 0
        step = 10.0 ** (-dec)
    return abs(value - float(printed)) <= 0.5 * step + 1e-12


def test_table1_reproduced_from_lubich_bound():
    rows = _table()
    assert len(rows) == 12
    for m, f32, f64 in rows:
        assert _digits_match(cb.chebyshev_norm_limit(m, 2.0 ** -24), f32), (m, f32)
        assert _digits_match(cb.chebyshev_norm_limit(m, 2.0 ** -53), f64), (m, f64)


def _rand_herm(rng, d, spec):
    a = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    h = 0.5 * (a + a.conj().T)
    w = np.linalg.eigvalsh(h)
    return h * (spec / np.max(np.abs(w)))


@pytest.mark.parametrize("m", [1, 2, 5, 11, 25])
def test_clenshaw_equals_direct_series(m):
    rng = np.random.default_rng(m)
    G = _rand_herm(rng, 7, 1.3)
    a = cb.chebyshev_expm_minus_i(G, -1.4, 1.6, m)
    b = cb.chebyshev_series_direct(G, -1.4, 1.6, m)
    assert np.max(np.abs(a - b)) < 1e-13


def test_scalar_expansion_closed_form():
    """For 1x1 G the series is eq. chebyshev_scalar: exp(i w x) =
    a_0 + 2 sum i^k J_k(w) T_k(x), here exp(-i g) on [alpha, beta]."""
    for g, al, be in [(0.3, -1.0, 1.0), (-2.0, -2.5, 0.5), (4.0, 3.5, 4.2)]:
        val = cb.chebyshev_expm_minus_i(np.array([[g]]), al, be, 40)[0, 0]
        assert abs(val - np.exp(-1j * g)) < 1e-14
        # the same through T_k(x) = cos(k arccos x)
        x = (2 * g - al - be) / (be - al)
        a = cb.chebyshev_coefficients(al, be, 40)
        s = a[0] + 2 * sum(a[k] * math.cos(k * math.acos(x)) for k in range(1, 41))
        assert abs(np.exp(-0.5j * (al + be)) * s - np.exp(-1j * g)) < 1e-14


@pytest.mark.parametrize("m", [3, 5, 7, 9, 13, 19, 25])
def test_truncation_within_table_limit(m):
    """At ||G|| = the FP64 limit of Table 1 the series matches the exact
    exponential to about the FP64 rounding level."""
    theta = cb.chebyshev_norm_limit(m, 2.0 ** -53)
    rng = np.random.default_rng(100 + m)
    G = _rand_herm(rng, 6, theta)
    err = np.max(np.abs(cb.chebyshev_expm_minus_i(G, -theta, theta, m) - scipy.linalg.expm(-1j * G)))
    assert err <= 64 * 2.0 ** -53


def test_error_decreases_with_degree_at_fixed_norm():
    rng = np.random.default_rng(7)
    G = _rand_herm(rng, 5, 2.0)
    ex = scipy.linalg.expm(-1j * G)
    errs = [np.max(np.abs(cb.chebyshev_expm_minus_i(G, -2.0, 2.0, m) - ex)) for m in (4, 8, 12, 16)]
    assert errs[0] > errs[1] > errs[2] > errs[3] and errs[3] < 1e-10
    for m, e in zip((4, 8, 12, 16), errs):
        assert e <= 2 * cb.lubich_error(m, 4.0) + 1e-15


def test_planted_mistakes_are_caught(monkeypatch):
    G = np.array([[0.2, 0.1 - 0.3j], [0.1 + 0.3j, -0.5]])
    ref = scipy.linalg.expm(-1j * G)
    good = cb.chebyshev_expm_minus_i(G, -1.0, 1.0, 25)
    assert np.max(np.abs(good - ref)) < 1e-14
    # (+i)^k instead of (-i)^k: conjugated exponential
    orig = cb.chebyshev_coefficients
    monkeypatch.setattr(cb, "chebyshev_coefficients", lambda a, b, m: np.conj(orig(a, b, m)))
    bad = cb.chebyshev_expm_minus_i(G, -1.0, 1.0, 25)
    assert np.max(np.abs(bad - ref)) > 1e-3
