"""Parity at the workloads' full sizes, against the oracle's stored U(T).

The oracle takes minutes on these sizes (the d = 64 precision sweep alone
about 100 s), so its results are stored by tests/golden/make_full_size.py,
which calls only the oracle on the seeded inputs of ``synth``; the inputs
are regenerated here from the same seeds.

* the random qudit (d = 16, N = 2^17, order 4) in every precision, with
  per-slice output sampled against the oracle's slice exponentials;
* the same system with the sixth-order scheme (FP64), likewise;
* the precision sweep (d = 64, N = 2^16, order 2) in every precision;
* the 512-instance batch at full N: FP64 and FP32-3M batches against the
  stored U(T) of every instance of dimension <= 16 and of the longest
  instances of dimensions 32 and 64, and every instance of both batches
  against its own single-context run.
FP64 bar: relative Frobenius error <= 1e-10.  Reduced precisions: the bounds
of tests/bounds.py.
"""
import os
import sys

import numpy as np
import pytest

import oracle.propagator as orc
import synth
from bounds import TOL64, tol, tol_slice

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_oracle.npz")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07126_amd as m
    return m


@pytest.fixture(scope="module")
def golden():
    with np.load(GOLDEN) as z:
        return {k: z[k] for k in z.files}


def propagate(pm, w, prec, slices=False):
    with pm.Context(0, prec) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, w.order)
        return ctx.equiprop(w.samples, w.h, return_slices=slices)


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_random_qudit_full_size(pm, golden, prec):
    """d = 16, N = 2^17, order 4: U(T) against the stored oracle product, and
    64 sampled slices of the per-slice output against the oracle's
    exponentials (FP64: 1e-13 max-abs; complex64 output: a single slice's
    bound)."""
    w = synth.random_qudit()
    say(f"[case] random qudit full size prec={prec}")
    U, sl = propagate(pm, w, prec, slices=True)
    err = orc.relative_frobenius(U, golden["random_qudit"])
    bound = tol(prec, w.n_slices, w.dim)
    say(f"  U(T) rel err {err:.3e} (bound {bound:.3e})")
    assert err <= bound
    assert sl.dtype == (np.complex128 if prec == 0 else np.complex64)
    rng = np.random.default_rng(1)
    js = np.sort(rng.choice(w.n_slices, 64, replace=False))
    worst = 0.0
    for j in js:
        G = orc.slice_exponents(w.H0, w.Hk, w.samples, w.h, 4, j, j + 1)
        worst = max(worst, float(np.max(np.abs(sl[j] - orc.expm_minus_i(G)[0]))))
    sbound = 1e-13 if prec == 0 else tol_slice(prec, w.dim)
    say(f"  sampled slices max-abs err {worst:.3e} (bound {sbound:.3e})")
    assert worst <= sbound


def test_random_qudit_magnus6_full_size(pm, golden):
    """d = 16, N = 2^17 with the sixth-order scheme (three Gauss-Legendre
    samples per slice, FP64): U(T) against the stored oracle product, and 64
    sampled slices against the oracle's sixth-order slice exponentials."""
    w = synth.random_qudit(order=orc.M6)
    say("[case] random qudit full size, sixth order")
    U, sl = propagate(pm, w, 0, slices=True)
    err = orc.relative_frobenius(U, golden["random_qudit_m6"])
    say(f"  U(T) rel err {err:.3e} (bound {TOL64:.1e})")
    assert err <= TOL64
    rng = np.random.default_rng(2)
    js = np.sort(rng.choice(w.n_slices, 64, replace=False))
    worst = 0.0
    for j in js:
        G = orc.slice_exponents(w.H0, w.Hk, w.samples, w.h, orc.M6, j, j + 1)
        worst = max(worst, float(np.max(np.abs(sl[j] - orc.expm_minus_i(G)[0]))))
    say(f"  sampled slices max-abs err {worst:.3e} (bound 1e-13)")
    assert worst <= 1e-13


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_precision_sweep_full_size(pm, golden, prec):
    """d = 64, N = 2^16, order 2: U(T) in every precision against the stored
    oracle product."""
    w = synth.precision_sweep()
    say(f"[case] precision sweep full size prec={prec}")
    U = propagate(pm, w, prec)
    err = orc.relative_frobenius(U, golden["precision_sweep"])
    bound = tol(prec, w.n_slices, w.dim)
    say(f"  U(T) rel err {err:.3e} (bound {bound:.3e})")
    assert err <= bound
    # ||U^H U - I||_F <= 2 ||U - Uo||_F + O(err^2) = 2 sqrt(d) rel err
    assert orc.unitarity_defect(U) <= 2.5 * np.sqrt(w.dim) * bound


def nu_bound(w) -> float:
    """Upper bound on every slice exponent's 1-norm from the inputs: the
    triangle inequality over the weights of the slice exponent (order 4: the
    Simpson weights plus the commutator weights, with
    ||i[A, B]||_1 <= 2 ||A||_1 ||B||_1)."""
    n1 = lambda A: float(np.max(np.sum(np.abs(A), axis=0)))
    a0 = n1(w.H0)
    ak = [n1(H) for H in w.Hk]
    cm = [float(np.max(np.abs(c))) for c in w.samples]
    nu = w.h * (a0 + sum(c * a for c, a in zip(cm, ak)))
    if w.order == 4:
        q = w.h ** 2 / 12.0
        nu += q * sum(2 * c * 2 * a0 * a for c, a in zip(cm, ak))
        for k in range(len(ak)):
            for l in range(k + 1, len(ak)):
                nu += q * 2 * cm[k] * cm[l] * 2 * ak[k] * ak[l]
    return nu


@pytest.fixture(scope="module")
def batch_inputs():
    return synth.batched_instances(512)


@pytest.mark.parametrize("prec", [0, 2])
def test_batch_full_size(pm, golden, batch_inputs, prec):
    """All 512 instances at full N (about 1e7 slices) in one persistent
    launch: against the stored oracle U(T) of the kept instances, and every
    instance against its own single-context run (each within the bound of
    the exact propagator, so the two within twice it)."""
    ws = batch_inputs
    say(f"[case] 512-instance batch full size prec={prec}")
    with pm.Batch(0, prec) as b:
        b.set(ws)
        say(f"  packets {b.n_packets}")
        b.run()
        Us = b.results()
    idx, offs, flat = golden["batch_index"], golden["batch_offset"], golden["batch_U"]
    worst = 0.0
    for q, i in enumerate(idx):
        w = ws[i]
        Uo = flat[offs[q]:offs[q + 1]].reshape(w.dim, w.dim)
        s = 0 if prec == 0 else pm.plan_expm(nu_bound(w), prec, n_slices=w.n_slices)[1]
        bound = tol(prec, w.n_slices, w.dim, s)
        e = orc.relative_frobenius(Us[i], Uo)
        worst = max(worst, e / bound)
        assert e <= bound, (i, w.dim, w.n_slices, w.order, e, bound)
    say(f"  {len(idx)} instances against the oracle: worst error / bound {worst:.3f}")
    worst = 0.0
    for i, w in enumerate(ws):
        Us1 = propagate(pm, w, prec)
        s = 0 if prec == 0 else pm.plan_expm(nu_bound(w), prec, n_slices=w.n_slices)[1]
        bound = 2 * tol(prec, w.n_slices, w.dim, s)
        e = orc.relative_frobenius(Us[i], Us1)
        worst = max(worst, e / bound)
        assert e <= bound, (i, w.dim, w.n_slices, w.order, e, bound)
    say(f"  512 instances against single-context runs: worst difference / bound {worst:.3f}")
