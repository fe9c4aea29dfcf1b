"""Reduced-precision paths against the FP64 oracle.

These paths have no oracle of their own; each result's error against the
FP64 oracle must stay inside a bound derived from its arithmetic:

* FP32 products: every entry of a complex product of unit-norm rows and
  columns is a d-term sum rounded at u32 = 2^-24, about four products per
  slice, and the N slice propagators' errors add up like a random walk:
      tol(N, d) = 4 sqrt(N) d u32 + 1e-6;
  3M products carry their imaginary parts on the (|Ar|+|Ai|)(|Br|+|Bi|)
  scale, twice that bound.
* BF16 split (hi*hi + hi*lo + lo*hi, FP32 accumulation): the dropped lo*lo
  term and the split residues leave ~2^-16 relative error per real product,
  and about four products per slice:
      tol(N, d) = 16 sqrt(N) sqrt(d) 2^-16 + 1e-4.
The measured errors are printed for the record.
"""
import math
import sys

import numpy as np
import pytest

import oracle.propagator as orc
import synth

pytestmark = pytest.mark.gpu


def tol(prec, n, d, pm):
    if prec == pm.PM_BF16_SPLIT:
        return 16 * math.sqrt(n) * math.sqrt(d) * 2.0 ** -16 + 1e-4
    c3m = 2.0 if prec == pm.PM_FP32_3M else 1.0
    return 4 * math.sqrt(n) * d * 2.0 ** -24 * c3m + 1e-6


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07126_amd as m
    return m


@pytest.mark.parametrize("d", [5, 16, 32, 64])
@pytest.mark.parametrize("order", [2, 4])
def test_reduced_precision_error_bounds(pm, d, order):
    n = 600 if d < 64 else 200
    w = synth.random_system(d, 2, n_slices=n, h=0.03, order=order, tag=60 + d)
    Uo, slo = orc.propagate(w.H0, w.Hk, w.samples, w.h, order, return_slices=True)
    errs = {}
    for prec in (pm.PM_FP32, pm.PM_FP32_3M, pm.PM_BF16_SPLIT):
        print(f"[case] d={d} order={order} prec={prec}", file=sys.stderr, flush=True)
        with pm.Context(0, prec) as ctx:
            ctx.set_hamiltonian(w.H0, w.Hk, order)
            U, sl = ctx.equiprop(w.samples, w.h, return_slices=True)
        e = orc.relative_frobenius(U, Uo)
        es = float(np.max(np.abs(sl - slo)))
        errs[prec] = e
        print(f"  prec={prec} U(T) rel err {e:.3e} (bound {tol(prec, n, d, pm):.3e}), slice max err {es:.2e}",
              file=sys.stderr, flush=True)
        assert e <= tol(prec, n, d, pm)
        assert es <= tol(prec, 1, d, pm) * 4
        assert orc.unitarity_defect(U) <= 10 * tol(prec, n, d, pm)
    # BF16 split carries fewer significant bits than FP32
    assert errs[pm.PM_BF16_SPLIT] >= 0.5 * errs[pm.PM_FP32]


def test_precision_sweep_workload_all_modes(pm):
    """The dim-64 precision-sweep workload at reduced N, every path."""
    w = synth.precision_sweep(n_slices=256)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 2)
    for prec in (pm.PM_FP64, pm.PM_FP32, pm.PM_FP32_3M, pm.PM_BF16_SPLIT):
        with pm.Context(0, prec) as ctx:
            ctx.set_hamiltonian(w.H0, w.Hk, 2)
            e = orc.relative_frobenius(ctx.equiprop(w.samples, w.h), Uo)
        print(f"  precision sweep prec={prec}: rel err {e:.3e}", file=sys.stderr, flush=True)
        assert e <= (1e-10 if prec == pm.PM_FP64 else tol(prec, 256, 64, pm))
