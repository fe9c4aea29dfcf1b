"""The Chebyshev-series exponential (PM_EXPM_CHEBYSHEV) against the FP64
oracle: every engine (dims 2 and 4 in the algebra of the slice exponent,
16/32/64 on MFMA, embedded dims), both orders, ragged slice counts, forced
and automatic squarings; and its error handling."""
import sys

import numpy as np
import pytest

import oracle.propagator as orc
import synth

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07126_amd as m
    return m


def run(pm, w, slices=False, force_s=-1, chunk=0):
    print(f"[case] cheb {w.name} d={w.dim} N={w.n_slices} order={w.order} force_s={force_s}",
          file=sys.stderr, flush=True)
    with pm.Context(0, pm.PM_FP64) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, w.order)
        ctx.set_expm_method(pm.PM_EXPM_CHEBYSHEV)
        if force_s >= 0:
            ctx.set_expm_policy(21, force_s)
        if chunk:
            ctx.set_chunk(chunk)
        return ctx.equiprop(w.samples, w.h, return_slices=slices)


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 16, 32, 40, 64])
def test_chebyshev_dims_orders(pm, d, order):
    for n in (1, 77):
        w = synth.random_system(d, 2, n_slices=n, h=0.07, order=order, tag=n + 3)
        U, sl = run(pm, w, slices=True)
        Uo, slo = orc.propagate(w.H0, w.Hk, w.samples, w.h, order, return_slices=True)
        assert orc.relative_frobenius(U, Uo) <= TOL64, (d, order, n)
        assert np.max(np.abs(sl - slo)) <= 1e-13, (d, order, n)


@pytest.mark.parametrize("d", [2, 4, 16, 32])
def test_chebyshev_large_norms_and_forced_squarings(pm, d):
    w = synth.random_system(d, 2, n_slices=40, h=0.9, order=2, tag=8, h0_norm=20.0)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 2)
    assert orc.relative_frobenius(run(pm, w), Uo) <= TOL64
    assert orc.relative_frobenius(run(pm, w, force_s=6), Uo) <= TOL64


def test_chebyshev_headline_workload_reduced(pm):
    w = synth.random_qudit(n_slices=4096)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 4)
    assert orc.relative_frobenius(run(pm, w), Uo) <= TOL64


def test_chebyshev_method_errors_and_gradient(pm):
    with pm.Context(0, pm.PM_FP32) as ctx:
        with pytest.raises(pm.ParamentError) as e:
            ctx.set_expm_method(pm.PM_EXPM_CHEBYSHEV)
        assert e.value.name == "PM_E_UNSUPPORTED"
    w = synth.qubit_register(n_slices=64)
    with pm.Context(0, pm.PM_FP64) as ctx:
        with pytest.raises(pm.ParamentError):
            ctx.set_expm_method(7)
        ctx.set_hamiltonian(w.H0, w.Hk, 2)
        ctx.set_expm_method(pm.PM_EXPM_CHEBYSHEV)
        # the gradient entry point keeps the Taylor series and stays exact
        loss, grad, U = ctx.fidelity_grad(w.samples, w.h, w.target)
        U2 = ctx.equiprop(w.samples, w.h)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 2)
    _, go = orc.control_gradient(w.H0, w.Hk, w.samples, w.h, 2, orc.fidelity_grad_U(Uo, w.target))
    assert np.max(np.abs(grad - go)) <= 1e-9 * np.max(np.abs(go))
    assert orc.relative_frobenius(U, Uo) <= TOL64 and orc.relative_frobenius(U2, Uo) <= TOL64
