"""The commutator-free fourth-order integrator (PM_ORDER_CF4) on the HIP path
against the oracle, through the C ABI: U(T) on every engine's dimensions
with ragged slice counts, reduced precisions within their derived bounds,
chain splits (odd chain lengths are rounded to whole slices), the adjoint
gradient, trajectories, batched instances mixed with the other orders,
the headline workload at full size, and the error paths.

Bars: FP64 U(T) relative Frobenius 1e-10 (as for the other orders);
gradient 1e-9 relative; trajectory 1e-12 per step times max(1, N);
reduced precisions by the bounds of the precision tests, with 2N
exponentials counted as the chained factors.
"""
import math
import sys

import numpy as np
import pytest

import oracle.propagator as orc
import synth
from bounds import max_squarings, tol

pytestmark = pytest.mark.gpu

CF4 = orc.CF4
TOL64 = 1e-10


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07126_amd as m
    assert m.PM_ORDER_CF4 == CF4
    return m


def tol_reduced(pm, prec, n_factors, d, s=0):
    """The reduced-precision bound of tests/bounds.py over the n_factors
    exponentials of the product."""
    return tol(prec, n_factors, d, s)


def gpu_U(pm, w, precision=0, chunk=0):
    say(f"[case] cf4 {w.name} d={w.dim} K={w.n_ctrl} N={w.n_slices} prec={precision} chunk={chunk}")
    with pm.Context(0, precision) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, CF4)
        if chunk:
            ctx.set_chunk(chunk)
        return ctx.equiprop(w.samples, w.h)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 8, 16, 17, 32, 40, 64])
def test_dims_ragged_fp64(pm, d):
    K = 2 if d > 1 else 1
    for n in (1, 3, 77):
        w = synth.random_system(d, K, n_slices=n, h=0.07, order=CF4, tag=300 + n)
        Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, CF4)
        assert orc.relative_frobenius(gpu_U(pm, w), Uo) <= TOL64, (d, n)


@pytest.mark.parametrize("d", [2, 4, 16, 64])
def test_many_slices_and_controls(pm, d):
    n = 1000 if d < 64 else 300
    for K in (0, 3, 8):
        w = synth.random_system(d, K, n_slices=n, h=0.02, order=CF4, tag=310 + K)
        Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, CF4)
        assert orc.relative_frobenius(gpu_U(pm, w), Uo) <= TOL64, (d, K)


@pytest.mark.parametrize("d", [3, 16, 64])
def test_reduced_precisions_within_bounds(pm, d):
    n = 400 if d < 64 else 150
    w = synth.random_system(d, 2, n_slices=n, h=0.03, order=CF4, tag=320 + d)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, CF4)
    for prec in (pm.PM_FP32, pm.PM_FP32_3M, pm.PM_BF16_SPLIT):
        e = orc.relative_frobenius(gpu_U(pm, w, prec), Uo)
        say(f"  prec={prec} rel err {e:.3e} (bound {tol_reduced(pm, prec, 2 * n, d):.3e})")
        assert e <= tol_reduced(pm, prec, 2 * n, d), (d, prec, e)


@pytest.mark.parametrize("d", [2, 16, 32])
def test_chain_split_invariance(pm, d):
    w = synth.random_system(d, 2, n_slices=301, h=0.04, order=CF4, tag=330 + d)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, CF4)
    for chunk in (1, 7, 64, 4096):
        assert orc.relative_frobenius(gpu_U(pm, w, chunk=chunk), Uo) <= TOL64, (d, chunk)


def test_full_size_random_qudit(pm):
    """The headline system (d 16, K 3, N 2^17, h 1e-3) with the commutator-free
    step, against the oracle and against the commutator Magnus step."""
    w = synth.random_qudit(order=CF4)
    U = gpu_U(pm, w)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, CF4)
    assert orc.relative_frobenius(U, Uo) <= TOL64
    w4 = synth.random_qudit(order=4)
    with pm.Context(0, pm.PM_FP64) as ctx:
        ctx.set_hamiltonian(w4.H0, w4.Hk, 4)
        U4 = ctx.equiprop(w4.samples, w4.h)
    # both are fourth-order approximations of the same U(T)
    assert orc.relative_frobenius(U, U4) <= 1e-9


@pytest.mark.parametrize("d", [2, 4, 8, 16, 32])
def test_gradient_matches_oracle(pm, d):
    for n in (1, 5, 37):
        w = synth.random_system(d, 2, n_slices=n, h=0.11, order=CF4, tag=340 + n)
        V = synth.haar_unitary(np.random.default_rng(d * 13 + n), d)
        U = orc.propagate(w.H0, w.Hk, w.samples, w.h, CF4)
        _, go = orc.control_gradient(w.H0, w.Hk, w.samples, w.h, CF4, orc.fidelity_grad_U(U, V))
        say(f"[case] cf4 grad d={d} n={n}")
        with pm.Context() as ctx:
            ctx.set_hamiltonian(w.H0, w.Hk, CF4)
            lg, gg, Ug = ctx.fidelity_grad(w.samples, w.h, V)
        assert abs(lg - orc.fidelity_loss(U, V)) <= 1e-12
        err = float(np.max(np.abs(gg - go)) / np.max(np.abs(go)))
        assert err <= 1e-9, (d, n, err)


@pytest.mark.parametrize("d", [8, 16])
def test_gradient_split_chains(pm, d):
    """Chains of 10 and 14 exponentials are split into backward parts of 5
    and 7: parts that start on the second factor of a slice."""
    w = synth.random_system(d, 2, n_slices=37, h=0.09, order=CF4, tag=345)
    V = synth.haar_unitary(np.random.default_rng(d + 99), d)
    U = orc.propagate(w.H0, w.Hk, w.samples, w.h, CF4)
    _, go = orc.control_gradient(w.H0, w.Hk, w.samples, w.h, CF4, orc.fidelity_grad_U(U, V))
    for chunk in (10, 14):
        say(f"[case] cf4 grad split d={d} chunk={chunk}")
        with pm.Context() as ctx:
            ctx.set_hamiltonian(w.H0, w.Hk, CF4)
            ctx.set_chunk(chunk)
            _, gg, _ = ctx.fidelity_grad(w.samples, w.h, V)
        err = float(np.max(np.abs(gg - go)) / np.max(np.abs(go)))
        assert err <= 1e-9, (d, chunk, err)


@pytest.mark.parametrize("d", [2, 5, 16, 32])
def test_trajectory_matches_oracle(pm, d):
    for n, chunk in ((1, 0), (40, 0), (203, 5)):
        say(f"[case] cf4 trajectory d={d} n={n} chunk={chunk}")
        w = synth.random_system(d, 2, n_slices=n, h=0.05, order=CF4, tag=350 + n)
        ref = orc.trajectory(w.H0, w.Hk, w.samples, w.h, CF4)
        with pm.Context(0, pm.PM_FP64) as ctx:
            ctx.set_hamiltonian(w.H0, w.Hk, CF4)
            if chunk:
                ctx.set_chunk(chunk)
            P = ctx.trajectory(w.samples, w.h)
        assert P.shape == ref.shape
        assert np.max(np.abs(P - ref)) <= 1e-12 * max(1, n), (d, n)


def test_batch_mixes_cf4_with_other_orders(pm):
    spec = [(2, 1, 1, CF4), (3, 2, 50, 4), (4, 1, 333, CF4), (8, 3, 200, CF4), (16, 3, 700, CF4),
            (16, 1, 16, 2), (20, 2, 99, CF4), (32, 2, 150, CF4), (64, 1, 40, CF4), (5, 0, 9, CF4)]
    ws = [synth.random_system(d, K, n_slices=n, h=0.04, order=o, tag=360 + i)
          for i, (d, K, n, o) in enumerate(spec)]
    for prec in (0, 2):
        say(f"[case] cf4 batch prec={prec}")
        with pm.Batch(0, prec) as b:
            b.set(ws)
            b.run()
            Us = b.results()
        for w, U in zip(ws, Us):
            Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, w.order)
            nf = 2 * w.n_slices if w.order == CF4 else w.n_slices
            # batch packets share one plan per step: at most the instance's largest s
            bound = TOL64 if prec == 0 else tol_reduced(pm, prec, nf, w.dim, max_squarings(pm, w, prec))
            assert orc.relative_frobenius(U, Uo) <= bound, (w.name, prec)


def test_errors(pm):
    w = synth.random_system(4, 1, n_slices=5, h=0.05, order=CF4, tag=370)
    with pm.Context(0, pm.PM_FP64) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, CF4)
        with pytest.raises(pm.ParamentError):
            ctx.equiprop(w.samples, w.h, return_slices=True)
        with pytest.raises(pm.ParamentError):
            ctx.equiprop(w.samples[:, :-1], w.h)          # even sample count
        U = ctx.equiprop(w.samples, w.h)                  # context still usable
    assert orc.relative_frobenius(U, orc.propagate(w.H0, w.Hk, w.samples, w.h, CF4)) <= TOL64
