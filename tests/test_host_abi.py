"""CPU tests of the library's host side: ABI exports, the Hermitian basis and
slice weights of the expand step, Taylor thresholds and the (m, s) planner.
No GPU is touched."""
import math
import os
import re

import numpy as np
import pytest
import scipy.linalg

import oracle.propagator as orc
import synth

pm = pytest.importorskip("paper_2108_07126_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    syms = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            syms |= set(re.findall(r"\b(pm_[a-z0-9_]+)\s*\(", txt))
    return syms


def test_library_exports_every_declared_symbol():
    syms = header_symbols()
    assert len(syms) >= 14
    for s in sorted(syms):
        assert hasattr(pm._lib, s), s
    # the binding declares a signature for each one
    assert syms == set(pm.SIGNATURES), syms ^ set(pm.SIGNATURES)


def test_status_strings():
    for i, name in enumerate(pm.STATUS):
        assert pm._lib.pm_status_string(i).decode() == name


def test_basis_count_matches_effective_control_count():
    for K in range(0, 9):
        assert pm.basis_count(K, 2) == 1 + K
        # 3K/2 + K^2/2 effective controls besides H0 (eq. magnus_coeffs)
        assert pm.basis_count(K, 4) - 1 == (3 * K + K * K) // 2
    assert pm.basis_count(9, 2) == -1
    assert pm.basis_count(2, 3) == -1
    for K in range(0, 9):   # the commutator-free scheme forms no commutators
        assert pm.basis_count(K, pm.PM_ORDER_CF4) == 1 + K


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("d,K", [(2, 1), (5, 3), (16, 3), (8, 4)])
def test_expand_matches_oracle_slice_exponents(order, d, K):
    """sum_m w_{j,m} B_m (host basis and weights) equals the oracle's directly
    assembled exponent (commutator formed from A1, A3) to rounding."""
    w = synth.random_system(d, K, n_slices=7, h=0.05, order=order, tag=d * 10 + K)
    B, norms = pm.build_basis_host(w.H0, w.Hk, order)
    assert B.shape[0] == pm.basis_count(K, order)
    for m in range(B.shape[0]):
        assert np.max(np.abs(B[m] - B[m].conj().T)) == 0.0
        assert abs(norms[m] - np.max(np.sum(np.abs(B[m]), axis=0))) < 1e-13 * max(1, norms[m])
    Gref = orc.slice_exponents(w.H0, w.Hk, w.samples, w.h, order)
    for j in range(w.n_slices):
        wt = pm.slice_weights_host(w.samples, w.h, order, j)
        G = np.tensordot(wt, B, axes=1)
        assert np.max(np.abs(G - Gref[j])) < 1e-14 * max(1.0, np.max(np.abs(Gref[j])))


@pytest.mark.parametrize("d,K", [(2, 1), (5, 3), (8, 4)])
def test_cf4_expand_matches_oracle_exponents(d, K):
    """CF4: the weights of exponent 2j (2j + 1) on the basis H0, H_k give the
    oracle's first (second) factor exponent of slice j."""
    cf4 = pm.PM_ORDER_CF4
    w = synth.random_system(d, K, n_slices=6, h=0.07, order=cf4, tag=d * 10 + K + 500)
    B, _ = pm.build_basis_host(w.H0, w.Hk, cf4)
    assert B.shape[0] == 1 + K
    Gf, Gs = orc.cf4_exponents(w.H0, w.Hk, w.samples, w.h)
    for j in range(w.n_slices):
        for f, Gref in ((0, Gf[j]), (1, Gs[j])):
            G = np.tensordot(pm.slice_weights_host(w.samples, w.h, cf4, 2 * j + f), B, axes=1)
            assert np.max(np.abs(G - Gref)) < 1e-14 * max(1.0, np.max(np.abs(Gref)))
    with pytest.raises(pm.ParamentError):
        pm.slice_weights_host(w.samples, w.h, cf4, 2 * w.n_slices)


def test_non_hermitian_rejected():
    H0 = np.array([[1.0, 0.5], [0.4, -1.0]], complex)
    with pytest.raises(pm.ParamentError) as e:
        pm.build_basis_host(H0, np.zeros((0, 2, 2)), 2)
    assert e.value.name == "PM_E_NOT_HERMITIAN"
    H0 = np.array([[1.0, np.nan], [np.nan, -1.0]], complex)
    with pytest.raises(pm.ParamentError):
        pm.build_basis_host(H0, np.zeros((0, 2, 2)), 2)


def test_bad_arguments_rejected():
    with pytest.raises(pm.ParamentError):
        pm.slice_weights_host(np.zeros((1, 4)), 0.1, 4, 0)  # order 4 needs an odd count
    with pytest.raises(pm.ParamentError):
        pm.taylor_theta(0)
    with pytest.raises(pm.ParamentError):
        pm.plan_expm(-1.0)


def _taylor(X, m):
    T = np.eye(X.shape[0], dtype=complex)
    P = np.eye(X.shape[0], dtype=complex)
    for k in range(1, m + 1):
        P = P @ X / k
        T = T + P
    return T


@pytest.mark.parametrize("prec,u,n", [(pm.PM_FP64, 2.0 ** -53, 1), (pm.PM_FP32, 2.0 ** -24, 1),
                                      (pm.PM_BF16_SPLIT, 2.0 ** -16, 1), (pm.PM_FP32, 2.0 ** -32, 2 ** 16),
                                      (pm.PM_FP64, 2.0 ** -53, 2 ** 16)])
def test_taylor_theta_bounds_truncation(prec, u, n):
    """FP64: theta_m makes the remainder bound equal 2^-53.  Reduced modes:
    the bound relative to theta equals u/sqrt(N).  The true truncation error
    of exp(X) - T_m(X) at ||X||_1 = theta_m (X skew-Hermitian) stays below
    the bound."""
    rng = np.random.default_rng(4)
    prev = 0.0
    relative = prec != pm.PM_FP64
    for m in range(1, 22):
        th = pm.taylor_theta(m, prec, n)
        assert th > prev
        prev = th
        bound = th ** (m + 1) / math.factorial(m + 1) / (1 - th / (m + 2))
        target = u * th if relative else u
        assert abs(bound - target) < 1e-6 * target
        if 3 <= m <= 15:
            A = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
            G = 0.5 * (A + A.conj().T)
            G *= th / np.max(np.sum(np.abs(G), axis=0))
            X = -1j * G
            err = np.linalg.norm(scipy.linalg.expm(X) - _taylor(X, m), 1)
            assert err <= 1.5 * target + 64 * 2.0 ** -53


def _cost(m):
    return 0 if m <= 1 else (1 if m == 2 else m // 2 + 1)


@pytest.mark.parametrize("prec", [pm.PM_FP64, pm.PM_FP32, pm.PM_BF16_SPLIT])
@pytest.mark.parametrize("n", [1, 4096, 2 ** 17])
def test_planner_is_feasible_and_optimal(prec, n):
    th = {m: pm.taylor_theta(m, prec, n) for m in range(1, 22)}
    for nu in [0.0, 1e-9, 3e-4, 0.0043, 0.0346, 0.195, 0.43, 1.0, 3.7, 40.0, 1e4]:
        m, s = pm.plan_expm(nu, prec, n_slices=n)
        assert nu / 2 ** s <= th[m]
        # brute force over all feasible (m', s')
        best = min(_cost(mm) + ss for ss in range(0, 40) for mm in th if nu / 2 ** ss <= th[mm])
        assert _cost(m) + s == best
    # tie goes to the smaller s
    m, s = pm.plan_expm(0.0043, pm.PM_FP64)
    assert (m, s) == (5, 0)


def test_create_without_device_reports_device_error():
    import ctypes
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    h = ctypes.c_void_p()
    st = pm._lib.pm_create(ctypes.byref(h), 0, pm.PM_FP64)
    if has_gpu:
        assert st == 0
        pm._lib.pm_destroy(h)
    else:
        assert pm.STATUS[st] == "PM_E_DEVICE"
        assert "no HIP device" in pm._lib.pm_last_error(None).decode()
        st = pm._lib.pm_batch_create(ctypes.byref(h), 0, pm.PM_FP32)
        assert pm.STATUS[st] == "PM_E_DEVICE"
        assert "no HIP device" in pm._lib.pm_batch_last_error(None).decode()
    assert pm.STATUS[pm._lib.pm_create(ctypes.byref(h), 0, 7)] == "PM_E_INVALID_ARG"
    assert "precision" in pm._lib.pm_last_error(None).decode()


def test_tuning_set_validation(tmp_path):
    """pm_tuning_set accepts the documented keys and classes only; the table
    loader applies well-formed lines and skips the rest."""
    lib = pm._lib
    assert lib.pm_tuning_set(b"chains", 16, 0, 0) == 0
    assert lib.pm_tuning_set(b"chains", 8, 0, 128) == 1
    assert lib.pm_tuning_set(b"chains", 16, 4, 128) == 1
    assert lib.pm_tuning_set(b"chains", 16, 0, -1) == 1
    assert lib.pm_tuning_set(b"batch_chunk", 2, 0, 32) == 1
    assert lib.pm_tuning_set(b"batch_chunk", 32, 1, 0) == 0
    assert lib.pm_tuning_set(b"unknown", 16, 0, 1) == 1
    t = tmp_path / "tuning.txt"
    t.write_text("# comment\nchains 16 0 0\nbatch_chunk 64 2 0  # default\nchains 7 0 5\nbad line\n")
    assert pm.load_tuning(str(t)) == 2
    pm.load_tuning()  # restore the shipped table, if any


def test_chebyshev_thresholds_reproduce_table1():
    """The library's Chebyshev limits (its own solver of Lubich's estimate)
    against the values printed in the paper's Table 1."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "chebyshev_table1.txt")
    rows = [l.split("#", 1)[0].split() for l in open(path)]
    rows = [r for r in rows if r]
    assert len(rows) == 12
    for m, f32, f64 in rows:
        for printed, prec in ((f32, pm.PM_FP32), (f64, pm.PM_FP64)):
            mant = printed.split("e")[0]
            dec = len(mant.split(".")[1]) if "." in mant else 0
            scale = 10.0 ** (int(printed.split("e")[1]) - dec) if "e" in printed else 10.0 ** (-dec)
            assert abs(pm.chebyshev_theta(int(m), prec) - float(printed)) <= 0.5 * scale + 1e-12, (m, printed)


def split_products(m):
    """Products of the even/odd split Chebyshev evaluation of degree m:
    Y = 2X^2 - I, T_2(Y)..T_{m/2}(Y), and X times the odd sum."""
    return 0 if m <= 1 else (1 if m == 2 else m // 2 + 1)


@pytest.mark.parametrize("prec", [pm.PM_FP64, pm.PM_FP32])
def test_chebyshev_planner_is_feasible_and_optimal(prec):
    th = {m: pm.chebyshev_theta(m, prec) for m in range(1, 26)}
    cost = lambda mm, ss: split_products(mm) + ss
    for nu in [0.0, 1e-9, 3e-4, 0.0043, 0.0346, 0.195, 0.43, 1.0, 3.7, 40.0, 1e4]:
        m, s = pm.plan_chebyshev(nu, prec)
        assert nu / 2 ** s <= th[m]
        feas = [(mm, ss) for ss in range(0, 40) for mm in th if nu / 2 ** ss <= th[mm]]
        best = min(cost(mm, ss) for mm, ss in feas)
        assert cost(m, s) == best
        # ties go to the smaller s, then to the smaller degree
        assert s == min(ss for mm, ss in feas if cost(mm, ss) == best)
        assert m == min(mm for mm, ss in feas if cost(mm, ss) == best and ss == s)
    m, s = pm.plan_chebyshev(0.3, prec, force_s=3)
    assert s == 3 and m == min(mm for mm in th if 0.3 / 8 <= th[mm])
    with pytest.raises(pm.ParamentError):
        pm.plan_chebyshev(1.0, prec, max_degree=26)


@pytest.mark.parametrize("d,K", [(2, 1), (5, 3), (16, 3), (8, 0)])
def test_m6_moment_weights_and_exponent(d, K):
    """Sixth order: the three weight rows of a slice on the basis {H0, H_k}
    give the scheme's moments P1 = h A2, P2 = (sqrt(15) h/3)(A3 - A1),
    P3 = (10 h/3)(A3 - 2 A2 + A1) of the oracle's Hamiltonian samples, and
    the Hermitian form the device evaluates,
    G = P1 + P3/12 - (i/240)[-20 P1 - P3 + R1, P2 + R2] with
    R1 = -i[P1, P2], R2 = (i/60)[P1, 2 P3 + R1], is the oracle's exponent."""
    m6 = pm.PM_ORDER_MAGNUS6
    w = synth.random_system(d, K, n_slices=5, h=0.2, order=m6, tag=d * 10 + K + 600)
    assert pm.basis_count(K, m6) == 1 + K
    B, _ = pm.build_basis_host(w.H0, w.Hk, m6)
    A = orc.hamiltonian_samples(w.H0, w.Hk, w.samples)
    Gref = orc.slice_exponents(w.H0, w.Hk, w.samples, w.h, m6)
    h, r15 = w.h, math.sqrt(15.0)
    for j in range(w.n_slices):
        a1, a2, a3 = A[3 * j], A[3 * j + 1], A[3 * j + 2]
        wt = pm.slice_weights_host(w.samples, w.h, m6, j)
        assert wt.shape == (3, 1 + K)
        P = [np.tensordot(wt[q], B, axes=1) for q in range(3)]
        ref = [h * a2, (r15 * h / 3) * (a3 - a1), (10 * h / 3) * (a3 - 2 * a2 + a1)]
        for q in range(3):
            assert np.max(np.abs(P[q] - ref[q])) < 1e-14 * max(1.0, np.max(np.abs(ref[q])))
        comm = lambda x, y: x @ y - y @ x
        R1 = -1j * comm(P[0], P[1])
        R2 = (1j / 60) * comm(P[0], 2 * P[2] + R1)
        G = P[0] + P[2] / 12 - (1j / 240) * comm(-20 * P[0] - P[2] + R1, P[1] + R2)
        assert np.max(np.abs(G - Gref[j])) < 1e-14 * max(1.0, np.max(np.abs(Gref[j])))


def test_m6_sample_count_rules():
    """Order 6 takes 3N samples: the weight helper refuses other counts."""
    m6 = pm.PM_ORDER_MAGNUS6
    c = np.zeros((1, 7))
    with pytest.raises(pm.ParamentError):
        pm.slice_weights_host(c, 0.1, m6, 0)
    assert pm.slice_weights_host(np.zeros((1, 6)), 0.1, m6, 1).shape == (3, 2)
    with pytest.raises(pm.ParamentError):
        pm.slice_weights_host(np.zeros((1, 6)), 0.1, m6, 2)
    assert pm.n_slices(9, m6) == 3
