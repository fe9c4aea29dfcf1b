"""Reduced-precision paths against the FP64 oracle, within the bounds of
tests/bounds.py (derived from the arithmetic; measured errors are printed).
"""
import math
import sys

import numpy as np
import pytest

import oracle.propagator as orc
import synth
from bounds import max_squarings, tol, tol_slice

pytestmark = pytest.mark.gpu


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
        sq = max_squarings(pm, w, prec)
        print(f"  prec={prec} s={sq} U(T) rel err {e:.3e} (bound {tol(prec, n, d, sq):.3e}), "
              f"slice max err {es:.2e} (bound {tol_slice(prec, d, sq):.2e})", file=sys.stderr, flush=True)
        assert e <= tol(prec, n, d, sq)
        assert es <= tol_slice(prec, d, sq)
        # ||U^H U - I||_F <= 2 ||U - Uo||_F + O(err^2) = 2 sqrt(d) rel err
        assert orc.unitarity_defect(U) <= 2.5 * math.sqrt(d) * tol(prec, n, d, sq)
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
        assert e <= tol(prec, 256, 64, max_squarings(pm, w, prec))
