"""The sixth-order Magnus integrator (PM_ORDER_MAGNUS6) on the HIP path
against the oracle, through the C ABI: U(T) and per-slice propagators on
every dimension class with ragged slice counts and several chain splits,
the Chebyshev exponential, slices that need squarings, the convergence
slope 6 against the circular drive's closed form, and the error paths.

Bar: FP64 U(T) relative Frobenius 1e-10, per-slice propagators 1e-13
max-abs (as for the other orders).
"""
import sys

import numpy as np
import pytest
import scipy.linalg

import oracle.propagator as orc
import synth

pytestmark = pytest.mark.gpu

M6 = orc.M6
TOL64 = 1e-10


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07126_amd as m
    assert m.PM_ORDER_MAGNUS6 == M6
    return m


def gpu_run(pm, w, chunk=0, slices=False, method=0, force_s=-1):
    say(f"[case] m6 {w.name} d={w.dim} K={w.n_ctrl} N={w.n_slices} chunk={chunk} method={method} "
        f"force_s={force_s}")
    with pm.Context(0, pm.PM_FP64) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, M6)
        if chunk:
            ctx.set_chunk(chunk)
        if method:
            ctx.set_expm_method(method)
        if force_s >= 0:
            ctx.set_expm_policy(21, force_s)
        return ctx.equiprop(w.samples, w.h, return_slices=slices)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 8, 12, 16, 17, 32, 40, 64])
def test_dims_ragged_with_slices(pm, d):
    K = 2 if d > 1 else 1
    for n in (1, 3, 77):
        w = synth.random_system(d, K, n_slices=n, h=0.09, order=M6, tag=700 + n)
        U, sl = gpu_run(pm, w, slices=True)
        Uo, slo = orc.propagate(w.H0, w.Hk, w.samples, w.h, M6, return_slices=True)
        assert orc.relative_frobenius(U, Uo) <= TOL64, (d, n)
        assert np.max(np.abs(sl - slo)) <= 1e-13, (d, n)


@pytest.mark.parametrize("d", [2, 16, 32, 64])
def test_many_slices_and_chain_splits(pm, d):
    """Thousands of slices (several tree levels), with automatic, short and
    ragged chains; no controls and eight controls."""
    n = 3000 if d < 64 else 400
    for K in (0, 3, 8):
        w = synth.random_system(d, K, n_slices=n, h=0.02, order=M6, tag=710 + K)
        Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, M6)
        for chunk in (0, 1, 37):
            assert orc.relative_frobenius(gpu_run(pm, w, chunk=chunk), Uo) <= TOL64, (d, K, chunk)


@pytest.mark.parametrize("d", [4, 16, 32])
def test_squarings_and_chebyshev(pm, d):
    """Large slice norms (automatic and forced squarings) and the Chebyshev
    exponential on sixth-order exponents."""
    w = synth.random_system(d, 2, n_slices=40, h=0.7, order=M6, tag=720, h0_norm=15.0)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, M6)
    assert orc.relative_frobenius(gpu_run(pm, w), Uo) <= TOL64
    assert orc.relative_frobenius(gpu_run(pm, w, force_s=8), Uo) <= TOL64
    assert orc.relative_frobenius(gpu_run(pm, w, method=pm.PM_EXPM_CHEBYSHEV), Uo) <= TOL64


def test_random_qudit_sixth_order(pm):
    """The d = 16 random-qudit system (three controls) sampled at the
    Gauss-Legendre nodes, 4096 slices, against the oracle."""
    w = synth.random_qudit(n_slices=4096, order=M6)
    U, sl = gpu_run(pm, w, slices=True)
    Uo, slo = orc.propagate(w.H0, w.Hk, w.samples, w.h, M6, return_slices=True)
    err = orc.relative_frobenius(U, Uo)
    say(f"  rel err {err:.3e}")
    assert err <= TOL64
    assert np.max(np.abs(sl - slo)) <= 1e-13


def test_convergence_slope_six_on_gpu(pm):
    """The circular drive (convergence figure's problem) propagated by the
    library: error against the closed form falls with slope 6 in N."""
    Z, X = synth.PAULI_Z, synth.PAULI_X
    exact = scipy.linalg.expm(-1j * 6.0 * Z / 2) @ scipy.linalg.expm(-1j * (0.0 * Z + 0.05 * X) * 6.0)
    ns = [4, 8, 16, 32]
    errs = []
    for n in ns:
        w = synth.circular_drive(n, M6)
        errs.append(orc.relative_frobenius(gpu_run(pm, w), exact))
    sl = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    say(f"  errors {['%.2e' % e for e in errs]}, slope {sl:.2f}")
    assert 5.7 <= sl <= 6.3


def test_errors(pm):
    w = synth.random_system(4, 1, n_slices=5, h=0.05, order=M6, tag=730)
    with pm.Context(0, pm.PM_FP64) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, M6)
        for bad in (w.samples[:, :-1], w.samples[:, :2]):   # not a multiple of 3 / no slice
            with pytest.raises(pm.ParamentError) as e:
                ctx.equiprop(bad, w.h)
            assert e.value.name == "PM_E_INVALID_ARG"
        with pytest.raises(pm.ParamentError) as e:
            ctx.fidelity_grad(w.samples, w.h, np.eye(4))
        assert e.value.name == "PM_E_UNSUPPORTED"
        with pytest.raises(pm.ParamentError) as e:
            ctx.trajectory(w.samples, w.h)
        assert e.value.name == "PM_E_UNSUPPORTED"
        U = ctx.equiprop(w.samples, w.h)            # context still usable
    assert orc.relative_frobenius(U, orc.propagate(w.H0, w.Hk, w.samples, w.h, M6)) <= TOL64
    for prec in (pm.PM_FP32, pm.PM_FP32_3M, pm.PM_BF16_SPLIT):
        with pm.Context(0, prec) as ctx:
            with pytest.raises(pm.ParamentError) as e:
                ctx.set_hamiltonian(w.H0, w.Hk, M6)
            assert e.value.name == "PM_E_UNSUPPORTED"
    with pm.Batch(0, 0) as b:
        with pytest.raises(pm.ParamentError) as e:
            b.set([w])
        assert e.value.name == "PM_E_UNSUPPORTED"
