"""Adjoint gradient of the HIP path against the FP64 oracle and finite differences.

Bar: the GPU gradient matches the oracle's (prefix/suffix products and
Daleckii-Krein Frechet derivatives) to 1e-9 relative (max-abs error over
max-abs entry), and central differences of the GPU loss to 1e-6.
"""
import sys

import numpy as np
import pytest

import oracle.propagator as orc
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-9


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07126_amd as m
    return m


def oracle_grad(w, V):
    U = orc.propagate(w.H0, w.Hk, w.samples, w.h, w.order)
    _, g = orc.control_gradient(w.H0, w.Hk, w.samples, w.h, w.order, orc.fidelity_grad_U(U, V))
    return orc.fidelity_loss(U, V), g


def gpu_grad(pm, w, V, chunk=0):
    say(f"[case] grad {w.name} d={w.dim} K={w.n_ctrl} N={w.n_slices} order={w.order} chunk={chunk}")
    with pm.Context() as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, w.order)
        if chunk:
            ctx.set_chunk(chunk)
        return ctx.fidelity_grad(w.samples, w.h, V)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("d", [2, 3, 4, 5, 8, 12, 16, 17, 32, 40, 64])
def test_grad_matches_oracle(pm, d, order):
    """Every engine class of the gradient, including embedded dimensions
    that are not a multiple of four (the products sum over the k-slices the
    embedded dimension reaches: d = 5 and 12 on the D = 16 pipeline, 40 on
    D = 64)."""
    for n in (1, 5, 37):
        w = synth.random_system(d, 2, n_slices=n, h=0.11, order=order, tag=40 + n)
        V = synth.haar_unitary(np.random.default_rng(d * 7 + n), d)
        lo, go = oracle_grad(w, V)
        lg, gg, Ug = gpu_grad(pm, w, V)
        assert abs(lg - lo) <= 1e-12
        assert rel(gg, go) <= TOL, (d, order, n, rel(gg, go))


def test_grad_qubit_register_full_size(pm):
    """The 3-qubit gradient workload: N = 4096, 16384 parameters."""
    w = synth.qubit_register()
    lo, go = oracle_grad(w, w.target)
    lg, gg, _ = gpu_grad(pm, w, w.target)
    say(f"  loss {lg:.12f} (oracle {lo:.12f}), grad rel err {rel(gg, go):.2e}")
    assert abs(lg - lo) <= 1e-12
    assert rel(gg, go) <= TOL


def test_grad_random_qudit_order4(pm):
    w = synth.random_qudit(n_slices=2048)
    V = synth.haar_unitary(np.random.default_rng(3), 16)
    lo, go = oracle_grad(w, V)
    lg, gg, _ = gpu_grad(pm, w, V)
    say(f"  grad rel err {rel(gg, go):.2e}")
    assert rel(gg, go) <= TOL


def test_grad_central_differences(pm):
    """Directional and coordinate central differences of the GPU loss."""
    w = synth.random_system(8, 3, n_slices=200, h=0.05, order=4, tag=77)
    V = synth.haar_unitary(np.random.default_rng(5), 8)
    _, g, _ = gpu_grad(pm, w, V)
    rng = np.random.default_rng(1)
    eps = 1e-6
    with pm.Context() as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, 4)

        def loss(c):
            return orc.fidelity_loss(ctx.equiprop(c, w.h), V)

        for _ in range(12):
            k = int(rng.integers(0, w.n_ctrl))
            i = int(rng.integers(0, w.n_samples))
            cp = w.samples.copy(); cp[k, i] += eps
            cm = w.samples.copy(); cm[k, i] -= eps
            fd = (loss(cp) - loss(cm)) / (2 * eps)
            assert abs(fd - g[k, i]) <= 1e-6 * max(1e-3, np.max(np.abs(g)))
        v = rng.standard_normal(w.samples.shape)
        fd = (loss(w.samples + eps * v) - loss(w.samples - eps * v)) / (2 * eps)
        assert abs(fd - np.sum(g * v)) <= 1e-6 * max(abs(fd), 1e-6)


def test_grad_checkpoint_interval_invariance(pm):
    """Checkpoints every sqrt(N) slices, every slice, and the default give the
    same gradient; the same configuration twice is bitwise identical."""
    w = synth.random_system(16, 2, n_slices=1024, h=0.03, order=2, tag=12)
    V = synth.haar_unitary(np.random.default_rng(9), 16)
    _, g0, _ = gpu_grad(pm, w, V)
    for ch in (32, 1, 300):
        _, g1, _ = gpu_grad(pm, w, V, chunk=ch)
        assert rel(g1, g0) <= 1e-12, ch
    _, g2, _ = gpu_grad(pm, w, V)
    assert np.array_equal(g2, g0)


def test_contexts_on_concurrent_streams(pm):
    """Eight independent evaluations enqueued at once on four contexts with
    four streams: each equals its context's result when run alone."""
    import torch
    ws = [synth.qubit_register(n_slices=500, tag=1100 + i) for i in range(8)]
    say("[case] grad 8 evaluations on 4 streams")
    ctxs = [pm.Context() for _ in range(4)]
    try:
        for c in ctxs:
            c.set_hamiltonian(ws[0].H0, ws[0].Hk, 2)
        S = [torch.tensor(w.samples, device="cuda") for w in ws]
        W = [torch.tensor(-(2.0 / 64) * w.target, device="cuda") for w in ws]
        G = [torch.zeros_like(s) for s in S]
        alone = []
        for i, w in enumerate(ws):
            ctxs[i % 4].backward_dev(S[i], w.h, W[i], G[i])
            torch.cuda.synchronize()
            alone.append(G[i].cpu().numpy())
            G[i].zero_()
        torch.cuda.synchronize()
        streams = [torch.cuda.Stream() for _ in range(4)]
        for i, w in enumerate(ws):
            ctxs[i % 4].backward_dev(S[i], w.h, W[i], G[i], stream=streams[i % 4])
        torch.cuda.synchronize()
        for i in range(8):
            assert np.array_equal(G[i].cpu().numpy(), alone[i]), i
        # and the first against the oracle (W = dL/dU-bar of Re Tr(W^H U))
        U = orc.propagate(ws[0].H0, ws[0].Hk, ws[0].samples, ws[0].h, 2)
        _, go = orc.control_gradient(ws[0].H0, ws[0].Hk, ws[0].samples, ws[0].h, 2, -(2.0 / 64) * ws[0].target)
        assert rel(alone[0], go) <= TOL
    finally:
        for c in ctxs:
            c.close()


def test_autograd_function(pm):
    import torch
    w = synth.random_system(8, 2, n_slices=300, h=0.04, order=4, tag=21)
    V = synth.haar_unitary(np.random.default_rng(2), 8)
    with pm.Context() as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, 4)
        s = torch.tensor(w.samples, device="cuda", requires_grad=True)
        U = pm.propagate_autograd(ctx, s, w.h)
        Vt = torch.tensor(V, device="cuda")
        g = torch.trace(Vt.conj().T @ U)
        L = 1 - g.abs() ** 2 / 64
        L.backward()
        lo, go = oracle_grad(w, V)
        assert abs(L.item() - lo) <= 1e-12
        assert rel(s.grad.cpu().numpy(), go) <= TOL


def test_grad_rejects_reduced_precision(pm):
    w = synth.random_system(4, 1, n_slices=3, h=0.1, order=2, tag=1)
    with pm.Context(0, pm.PM_FP32) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, 2)
        with pytest.raises(pm.ParamentError) as e:
            ctx.fidelity_grad(w.samples, w.h, np.eye(4))
        assert e.value.name == "PM_E_UNSUPPORTED"
