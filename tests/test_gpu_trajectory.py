"""Trajectories (every partial product P_j, states P_j Psi_0, densities
P_j rho_0 P_j^H) against the oracle's sequential partial products, on both
engines' dimensions, both orders, ragged slice counts and chain splits that
exercise the checkpoint assembly across blocks; and the error paths."""
import sys

import numpy as np
import pytest

import oracle.propagator as orc
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07126_amd as m
    return m


def _ctx(pm, w, chunk=0):
    ctx = pm.Context(0, pm.PM_FP64)
    ctx.set_hamiltonian(w.H0, w.Hk, w.order)
    if chunk:
        ctx.set_chunk(chunk)
    return ctx


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("d", [1, 2, 3, 5, 8, 12, 16, 20, 32, 45, 64])
def test_propagator_trajectory(pm, d, order):
    for n, chunk in ((1, 0), (77, 0), (203, 5)):
        print(f"[case] trajectory d={d} order={order} n={n} chunk={chunk}", file=sys.stderr, flush=True)
        w = synth.random_system(d, 2, n_slices=n, h=0.05, order=order, tag=40 + n)
        ref = orc.trajectory(w.H0, w.Hk, w.samples, w.h, order)
        with _ctx(pm, w, chunk) as ctx:
            P = ctx.trajectory(w.samples, w.h)
        assert P.shape == ref.shape
        err = np.max(np.abs(P - ref), axis=(1, 2))
        assert np.max(err) <= TOL * max(1, n), (d, order, n, np.argmax(err), np.max(err))


@pytest.mark.parametrize("d", [2, 8, 16, 33])
def test_state_and_density_trajectories(pm, d):
    w = synth.random_system(d, 3, n_slices=150, h=0.04, order=4, tag=50 + d)
    ref = orc.trajectory(w.H0, w.Hk, w.samples, w.h, 4)
    rng = np.random.default_rng(d)
    nv = min(3, d)
    psi = rng.standard_normal((d, nv)) + 1j * rng.standard_normal((d, nv))
    a = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    rho = a @ a.conj().T
    rho /= np.trace(rho).real
    with _ctx(pm, w, chunk=7) as ctx:
        S = ctx.trajectory(w.samples, w.h, pm.PM_TRAJ_STATES, psi)
        R = ctx.trajectory(w.samples, w.h, pm.PM_TRAJ_DENSITY, rho)
    assert S.shape == (151, d, nv) and R.shape == (151, d, d)
    assert np.max(np.abs(S - ref @ psi)) <= 1e-11
    Rref = ref @ rho @ np.conj(np.swapaxes(ref, 1, 2))
    assert np.max(np.abs(R - Rref)) <= 1e-11
    assert np.max(np.abs(np.trace(R, axis1=1, axis2=2) - 1.0)) <= 1e-11


def test_trajectory_end_point_matches_propagation_and_errors(pm):
    w = synth.random_qudit(n_slices=5000)
    with pm.Context(0, pm.PM_FP64) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, w.order)
        P = ctx.trajectory(w.samples, w.h)
        U = ctx.equiprop(w.samples, w.h)
        assert np.max(np.abs(P[-1] - U)) <= 1e-12
        assert np.allclose(P[0], np.eye(16))
        import torch
        s = torch.from_numpy(w.samples).cuda()
        out = torch.empty((5001, 16, 16), dtype=torch.complex128, device="cuda")
        with pytest.raises(pm.ParamentError):
            ctx.trajectory_dev(s, w.h, out, kind=9)
        with pytest.raises(pm.ParamentError):   # states need x0
            ctx.trajectory_dev(s, w.h, out, kind=pm.PM_TRAJ_STATES)
    with pm.Context(0, pm.PM_FP32) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, w.order)
        with pytest.raises(pm.ParamentError) as e:
            ctx.trajectory(w.samples, w.h)
        assert e.value.name == "PM_E_UNSUPPORTED"
