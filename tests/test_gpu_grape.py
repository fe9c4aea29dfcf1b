"""The device GRAPE loop (pm_grape_dev) against the oracle loop: the loss
history and the optimised controls of both optimisers on the 3-qubit
register, and the single-qubit closed form; errors."""
import math
import sys

import numpy as np
import pytest

import oracle.grape as og
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07126_amd as m
    return m


@pytest.mark.parametrize("opt,step", [("gd", 0.5), ("adam", 0.05)])
def test_grape_matches_oracle_loop(pm, opt, step):
    import torch
    print(f"[case] grape {opt}", file=sys.stderr, flush=True)
    w = synth.qubit_register(n_slices=96)
    c_ref, l_ref = og.grape(w.H0, w.Hk, w.samples, w.h, 2, w.target, iters=8, step=step, optimizer=opt)
    with pm.Context(0, pm.PM_FP64) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, 2)
        s = torch.from_numpy(w.samples.copy()).cuda()
        V = torch.from_numpy(np.ascontiguousarray(w.target)).cuda()
        loss = ctx.grape_dev(s, w.h, V, 8, step, pm.PM_OPT_GD if opt == "gd" else pm.PM_OPT_ADAM)
        torch.cuda.synchronize()
        l_gpu, c_gpu = loss.cpu().numpy(), s.cpu().numpy()
    assert np.max(np.abs(l_gpu - l_ref)) <= 1e-10
    assert np.max(np.abs(c_gpu - c_ref)) <= 1e-8 * max(1.0, np.max(np.abs(c_ref)))
    assert l_gpu[-1] < l_gpu[0]


def test_grape_single_qubit_closed_form(pm):
    import torch
    n, h, step = 40, 0.02, 3.0
    H0 = np.zeros((2, 2), complex)
    SX = np.array([[0, 1], [1, 0]], dtype=complex)
    with pm.Context(0, pm.PM_FP64) as ctx:
        ctx.set_hamiltonian(H0, SX[None], 2)
        s = torch.full((1, n), 0.25, dtype=torch.float64, device="cuda")
        V = torch.from_numpy(SX.copy()).cuda()
        loss = ctx.grape_dev(s, h, V, 5, step, pm.PM_OPT_GD).cpu().numpy()
        with pytest.raises(pm.ParamentError):
            ctx.grape_dev(s, h, V, 5, -1.0, pm.PM_OPT_GD)
        with pytest.raises(pm.ParamentError):
            ctx.grape_dev(s, h, V, 5, 1.0, 7)
    theta = h * 0.25 * n
    for k in range(6):
        assert abs(loss[k] - math.cos(theta) ** 2) < 1e-12
        theta += step * n * h * h * math.sin(2 * theta)
