"""Device-workspace planning under a limit (pm_workspace_plan, host-only):
the chain length a call takes so that its workspace fits, and the refusal
(PM_E_OOM) when even one chain does not.  No GPU is touched."""
import pytest

pm = pytest.importorskip("paper_2108_07126_amd")

FP64, FP32 = 0, 1


def plan(d, K, order, prec, n_samples, kind, limit=0):
    return pm.workspace_plan(d, K, order, prec, n_samples, kind, limit)


@pytest.mark.parametrize("d,K,order,n,kind", [
    (16, 3, 4, 2 ** 18 + 1, pm.PM_WORK_PROPAGATE),     # the random qudit
    (64, 2, 2, 2 ** 16, pm.PM_WORK_PROPAGATE),         # the dim-64 sweep
    (2, 1, 2, 2 ** 20, pm.PM_WORK_PROPAGATE),          # the small-dimension engine
    (8, 4, 2, 4096, pm.PM_WORK_GRADIENT),              # the qubit register's gradient
    (16, 3, 4, 2 ** 14 + 1, pm.PM_WORK_TRAJECTORY),
    (32, 2, 5, 2 ** 13 + 1, pm.PM_WORK_GRADIENT),      # commutator-free: 2N exponentials
])
def test_limit_lengthens_chains_until_the_workspace_fits(d, K, order, n, kind):
    c0, b0 = plan(d, K, order, FP64, n, kind)
    assert plan(d, K, order, FP64, n, kind, limit=b0) == (c0, b0)       # fits as is
    last_c = c0
    for frac in (0.7, 0.5, 0.3, 0.15):
        lim = int(b0 * frac)
        try:
            c, b = plan(d, K, order, FP64, n, kind, limit=lim)
        except pm.ParamentError as e:
            assert e.name == "PM_E_OOM"
            break
        assert b <= lim and c > c0 and c >= last_c
        last_c = c
    if order == 5:
        assert last_c % 2 == 0     # chains start at slice boundaries


@pytest.mark.parametrize("kind", [pm.PM_WORK_PROPAGATE, pm.PM_WORK_GRADIENT, pm.PM_WORK_TRAJECTORY])
def test_refusal_below_one_chain(kind):
    """One chain still needs its tree slack, U(T), its checkpoint and (for
    the gradient) every slice's weight gradients: a limit below that is
    refused with PM_E_OOM, one at it is met by a single chain."""
    n = 4096
    c0, b0 = plan(8, 4, 2, FP64, n, kind)
    lo, hi = 1, b0
    # smallest limit that fits (bytes decrease monotonically in the chain length)
    while lo < hi:
        mid = (lo + hi) // 2
        try:
            plan(8, 4, 2, FP64, n, kind, limit=mid)
            hi = mid
        except pm.ParamentError as e:
            assert e.name == "PM_E_OOM"
            lo = mid + 1
    c, b = plan(8, 4, 2, FP64, n, kind, limit=lo)
    assert b == lo and c >= c0
    with pytest.raises(pm.ParamentError) as e:
        plan(8, 4, 2, FP64, n, kind, limit=lo - 1)
    assert e.value.name == "PM_E_OOM"
    if kind == pm.PM_WORK_GRADIENT:
        assert b >= n * (1 + 4) * 8          # the weight gradients alone


def test_gradient_kinds_need_fp64_and_known_orders():
    with pytest.raises(pm.ParamentError) as e:
        plan(8, 4, 2, FP32, 4096, pm.PM_WORK_GRADIENT)
    assert e.value.name == "PM_E_UNSUPPORTED"
    with pytest.raises(pm.ParamentError) as e:
        plan(8, 4, pm.PM_ORDER_MAGNUS6, FP64, 3 * 4096, pm.PM_WORK_TRAJECTORY)
    assert e.value.name == "PM_E_UNSUPPORTED"
    with pytest.raises(pm.ParamentError) as e:
        plan(8, 4, 2, FP64, 4096, 7)
    assert e.value.name == "PM_E_INVALID_ARG"
    with pytest.raises(pm.ParamentError) as e:
        plan(8, 4, 4, FP64, 4096, pm.PM_WORK_PROPAGATE)   # order 4 needs 2N + 1 samples
    assert e.value.name == "PM_E_INVALID_ARG"
    c, b = plan(8, 4, pm.PM_ORDER_MAGNUS6, FP64, 3 * 4096, pm.PM_WORK_PROPAGATE)
    assert c >= 1 and b > 0
