"""Parity of the HIP path with the FP64 oracle, through the C ABI.

FP64 bar: relative Frobenius error of U(T) <= 1e-10, per-slice propagators
within 1e-13 max-abs.  FP32 (complex64) paths: the bounds of tests/bounds.py,
derived from the arithmetic.
"""
import math
import sys

import numpy as np
import pytest
import scipy.linalg

import oracle.propagator as orc
import synth

pytestmark = pytest.mark.gpu

from bounds import FP32, FP32_3M, TOL64, U32, max_squarings, tol, tol_slice


def tol32(n, d, s=0):
    return tol(FP32, n, d, s)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07126_amd as m
    return m


def run(pm, w, precision=0, slices=False, chunk=0, force_s=-1, max_deg=21):
    say(f"[case] {w.name} d={w.dim} K={w.n_ctrl} N={w.n_slices} order={w.order} prec={precision} "
        f"chunk={chunk} force_s={force_s}")
    with pm.Context(0, precision) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, w.order)
        if chunk:
            ctx.set_chunk(chunk)
        if force_s >= 0 or max_deg != 21:
            ctx.set_expm_policy(max_deg, force_s)
        return ctx.equiprop(w.samples, w.h, return_slices=slices)


def test_driven_qubit_full_size_fp64(pm):
    w = synth.driven_qubit()
    U, sl = run(pm, w, slices=True)
    Uo, slo = orc.propagate(w.H0, w.Hk, w.samples, w.h, w.order, return_slices=True)
    assert orc.relative_frobenius(U, Uo) <= TOL64
    assert np.max(np.abs(sl - slo)) <= 1e-13


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 8, 12, 16, 17, 32, 40, 64])
def test_dims_orders_ragged_fp64(pm, d, order):
    K = 2 if d > 1 else 1
    for n in (1, 3, 77):
        w = synth.random_system(d, K, n_slices=n, h=0.07, order=order, tag=n)
        U, sl = run(pm, w, slices=True)
        Uo, slo = orc.propagate(w.H0, w.Hk, w.samples, w.h, order, return_slices=True)
        assert orc.relative_frobenius(U, Uo) <= TOL64, (d, order, n)
        assert np.max(np.abs(sl - slo)) <= 1e-13, (d, order, n)


@pytest.mark.parametrize("d", [2, 4, 16, 32, 64])
def test_dims_many_slices_fp64_and_fp32(pm, d):
    n = 1000 if d < 64 else 300
    w = synth.random_system(d, 3, n_slices=n, h=0.02, order=4, tag=5)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 4)
    assert orc.relative_frobenius(run(pm, w), Uo) <= TOL64
    e32 = orc.relative_frobenius(run(pm, w, precision=pm.PM_FP32), Uo)
    say(f"  fp32 rel err {e32:.3e} (bound {tol32(n, d):.3e})")
    assert e32 <= tol32(n, d)


def test_random_qudit_reduced_fp64_fp32(pm):
    w = synth.random_qudit(n_slices=4096)
    U, sl = run(pm, w, slices=True)
    Uo, slo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 4, return_slices=True)
    assert orc.relative_frobenius(U, Uo) <= TOL64
    assert np.max(np.abs(sl - slo)) <= 1e-13
    U32v, sl32 = run(pm, w, precision=pm.PM_FP32, slices=True)
    assert sl32.dtype == np.complex64
    assert orc.relative_frobenius(U32v, Uo) <= tol32(4096, 16)
    assert np.max(np.abs(sl32 - slo)) <= tol_slice(FP32, 16)


def test_precision_sweep_reduced(pm):
    w = synth.precision_sweep(n_slices=512)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 2)
    assert orc.relative_frobenius(run(pm, w), Uo) <= TOL64
    e32 = orc.relative_frobenius(run(pm, w, precision=pm.PM_FP32), Uo)
    say(f"  d=64 fp32 rel err {e32:.3e}")
    assert e32 <= tol32(512, 64)


def test_qubit_register_fp64(pm):
    w = synth.qubit_register()
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 2)
    assert orc.relative_frobenius(run(pm, w), Uo) <= TOL64


@pytest.mark.parametrize("d", [2, 16])
def test_static_hamiltonian_exact(pm, d):
    """Constant controls: U(T) = exp(-i H T) by scipy's Pade expm."""
    w = synth.random_system(d, 2, n_slices=500, h=0.01, order=2, tag=9)
    c = np.repeat(np.array([[0.4], [-0.9]]), 500, axis=1)
    H = w.H0 + 0.4 * w.Hk[0] - 0.9 * w.Hk[1]
    with pm.Context() as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, 2)
        U = ctx.equiprop(c, 0.01)
    assert orc.relative_frobenius(U, scipy.linalg.expm(-1j * H * 5.0)) <= TOL64


@pytest.mark.parametrize("d", [2, 4, 16, 32])
def test_forced_and_large_norm_squarings(pm, d):
    w = synth.random_system(d, 2, n_slices=50, h=0.9, order=2, tag=3, h0_norm=20.0)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 2)
    assert orc.relative_frobenius(run(pm, w), Uo) <= TOL64          # auto: s > 0
    assert orc.relative_frobenius(run(pm, w, force_s=9), Uo) <= TOL64
    e32 = orc.relative_frobenius(run(pm, w, precision=pm.PM_FP32), Uo)
    s32 = max_squarings(pm, w, FP32, shift=d <= 4)
    say(f"  fp32 s={s32} rel err {e32:.3e} (bound {tol32(50, d, s32):.3e})")
    assert e32 <= tol32(50, d, s32)


@pytest.mark.parametrize("d", [2, 16, 32])
def test_chunking_and_tree_shape_invariance(pm, d):
    """Chain lengths 1 (pure tree), ragged and large give the same U(T); the
    same configuration twice is bitwise identical."""
    # dimensions <= 4 take chains in whole units of 1024 slices
    w = synth.random_system(d, 2, n_slices=9333 if d <= 4 else 1333, h=0.03, order=2, tag=4)
    ref = run(pm, w, chunk=1024 if d <= 4 else 7)
    for ch in ((2048, 3072, 10240) if d <= 4 else (1, 64, 1333)):
        U = run(pm, w, chunk=ch)
        assert orc.relative_frobenius(U, ref) <= 1e-13
    again = run(pm, w, chunk=1024 if d <= 4 else 7)
    assert np.array_equal(again, ref)


@pytest.mark.parametrize("d", [2, 4, 5, 8, 16, 32, 64])
def test_largest_basis_order4(pm, d):
    """Eight controls with 4th-order Magnus: 45 basis matrices (the largest
    basis; past the LDS copy on the MFMA engines, the last commutator pairs
    in the weight recipe), FP64 and FP32-3M against the oracle."""
    n = 60 if d == 64 else 200
    w = synth.random_system(d, 8, n_slices=n, h=0.02, order=4, tag=90 + d)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 4)
    assert orc.relative_frobenius(run(pm, w), Uo) <= TOL64, d
    e = orc.relative_frobenius(run(pm, w, precision=pm.PM_FP32_3M), Uo)
    assert e <= tol(FP32_3M, n, d, max_squarings(pm, w, FP32_3M, shift=d <= 4)), (d, e)


@pytest.mark.parametrize("d", [1, 2])
def test_small_dims_per_slice_default_chains(pm, d):
    """Per-slice output on dimensions 1 and 2 at the default decomposition
    (one chain per resident wave, not the U(T)-only tuned count): about a
    million slices with a ragged last chain, every slice and U(T) against
    the oracle in FP64 and FP32."""
    w = synth.random_system(d, 1, n_slices=(1 << 20) + 777, h=0.01, order=2, tag=90 + d)
    Uo, slo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 2, return_slices=True)
    U, sl = run(pm, w, slices=True)
    assert orc.relative_frobenius(U, Uo) <= TOL64
    assert np.max(np.abs(sl - slo)) <= 1e-13
    U32v, sl32 = run(pm, w, precision=pm.PM_FP32, slices=True)
    assert sl32.dtype == np.complex64
    assert orc.relative_frobenius(U32v, Uo) <= tol32(w.n_slices, d)
    assert np.max(np.abs(sl32 - slo)) <= tol_slice(FP32, d)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_small_dims_deep_tree(pm, d):
    """The small-dimension engine with about 150 leaves (three levels of the
    fan-in-8 tree, a ragged last group and a ragged last chain) against the
    oracle, and against a shallower split of the same slices."""
    w = synth.random_system(d, 2, n_slices=600_001, h=0.01, order=2, tag=70 + d)
    Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 2)
    U = run(pm, w, chunk=1024)
    assert orc.relative_frobenius(U, Uo) <= TOL64
    assert orc.relative_frobenius(run(pm, w, chunk=32768), U) <= 1e-12


def test_state_machine_and_errors(pm):
    with pm.Context() as ctx:
        with pytest.raises(pm.ParamentError) as e:
            ctx.dim, ctx.order = 2, 2
            ctx.equiprop(np.zeros((1, 4)), 0.1)
        assert e.value.name == "PM_E_NOT_READY"
        with pytest.raises(pm.ParamentError) as e:
            ctx.set_hamiltonian(np.array([[0, 1], [0, 0]], complex), np.zeros((0, 2, 2)), 2)
        assert e.value.name == "PM_E_NOT_HERMITIAN"
        ctx.set_hamiltonian(synth.PAULI_Z, synth.PAULI_X[None], 4)
        for bad in (np.zeros((1, 4)), np.zeros((1, 1))):
            with pytest.raises(pm.ParamentError) as e:
                ctx.equiprop(bad, 0.1)
            assert e.value.name == "PM_E_INVALID_ARG"
        with pytest.raises(pm.ParamentError):
            ctx.equiprop(np.zeros((1, 5)), -0.1)
        with pytest.raises(pm.ParamentError):
            ctx.equiprop(np.full((1, 5), np.nan), 0.1)
        for bad in (-2, 101):
            with pytest.raises(pm.ParamentError) as e:
                ctx.set_chain_skew(bad)
            assert e.value.name == "PM_E_INVALID_ARG"
        ctx.set_chain_skew(-1)
        # still usable
        U = ctx.equiprop(np.zeros((1, 5)), 0.1)
        assert orc.relative_frobenius(U, scipy.linalg.expm(-1j * synth.PAULI_Z * 0.2)) <= TOL64
        with pytest.raises(pm.ParamentError) as e:
            ctx.set_hamiltonian(np.eye(65, dtype=complex), np.zeros((0, 65, 65)), 2)
        assert e.value.name == "PM_E_INVALID_ARG"


def test_device_entry_point_matches_host(pm):
    import torch
    w = synth.random_system(16, 3, n_slices=999, h=0.02, order=4, tag=8)
    with pm.Context() as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, 4)
        Uh, slh = ctx.equiprop(w.samples, w.h, return_slices=True)
        s = torch.from_numpy(w.samples).cuda()
        U = torch.zeros((16, 16), dtype=torch.complex128, device="cuda")
        sl = torch.zeros((999, 16, 16), dtype=torch.complex128, device="cuda")
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            ctx.equiprop_dev(s, w.h, U, sl)
        st.synchronize()
        assert np.array_equal(U.cpu().numpy(), Uh)
        assert np.array_equal(sl.cpu().numpy(), slh)


def test_launch_shape_reports_decomposition(pm):
    """pm_launch_shape reports the chunking a propagation uses: explicit
    chunks are honoured, chains cover every slice once, leaves never exceed
    chains, and the propagation at that shape is still exact."""
    w = synth.random_qudit(n_slices=1000)
    with pm.Context(0, pm.PM_FP64) as ctx:
        ctx.set_hamiltonian(w.H0, w.Hk, w.order)
        c, n, l = ctx.launch_shape(w.n_samples)
        assert c >= 1 and n == -(-1000 // c) and 1 <= l <= n
        ctx.set_chunk(7)
        c, n, l = ctx.launch_shape(w.n_samples)
        assert (c, n) == (7, 143) and l == 36
        U = ctx.equiprop(w.samples, w.h)
    assert orc.relative_frobenius(U, orc.propagate(w.H0, w.Hk, w.samples, w.h, w.order)) <= TOL64


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("case", ["large_trace", "near_degenerate"])
def test_small_dims_shift_and_degenerate_spectra(pm, d, case):
    """Dims <= 4 exponentiate G - (tr G / D) I in the algebra of its powers
    and restore the phase: a large trace (phase far from 1 per slice) and a
    nearly scalar H (clustered eigenvalues) must both stay at FP64 parity,
    in U(T) and in every slice."""
    w = synth.random_system(d, 2, n_slices=301, h=0.05, order=4, tag=11)
    H0 = w.H0 + 37.0 * np.eye(d) if case == "large_trace" else 3.0 * np.eye(d) + 1e-9 * w.H0
    Hk = w.Hk if case == "large_trace" else 1e-9 * w.Hk
    with pm.Context(0, pm.PM_FP64) as ctx:
        ctx.set_hamiltonian(H0, Hk, 4)
        U, sl = ctx.equiprop(w.samples, w.h, return_slices=True)
    Uo, slo = orc.propagate(H0, Hk, w.samples, w.h, 4, return_slices=True)
    assert orc.relative_frobenius(U, Uo) <= TOL64
    assert np.max(np.abs(sl - slo)) <= 1e-13
    with pm.Context(0, pm.PM_FP32) as ctx:
        ctx.set_hamiltonian(H0, Hk, 4)
        U32v = ctx.equiprop(w.samples, w.h)
    class _W:   # the shifted system the engine of dimensions <= 4 plans on
        pass
    ww = _W()
    ww.H0, ww.Hk, ww.samples, ww.h, ww.order, ww.n_slices = H0, Hk, w.samples, w.h, 4, w.n_slices
    s32 = max_squarings(pm, ww, FP32, shift=True)
    e32 = orc.relative_frobenius(U32v, Uo)
    say(f"  fp32 s={s32} rel err {e32:.3e} (bound {tol32(301, d, s32):.3e})")
    assert e32 <= tol32(301, d, s32)


def assoc_bound(n):
    """Two associations of one product of n unitary FP64 factors differ by
    their rounding, a random walk of about sqrt(n) unit roundoffs (margin 64):
    a slice left out or taken twice would differ by O(h)."""
    return 64 * math.sqrt(n) * 2.0 ** -53


@pytest.mark.parametrize("case", ["fp64_order4", "fp32_3m_order2", "fp64_cf4", "fp64_pairs_d8", "fp64_magnus6",
                                  "fp64_chebyshev"])
def test_uneven_chains(pm, case):
    """A 16-wide-tile launch of exactly two blocks of four chains per compute
    unit gives the first-dispatched blocks' chains more slices
    (pm_set_chain_skew).  Equal chains, the automatic skew and 60 % all
    exponentiate every slice once (per-slice output identical), give the same
    U(T) to rounding, and match the oracle."""
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    chains, chunk = 2 * n_cu * 4, 6
    prec = FP32_3M if case == "fp32_3m_order2" else 0
    d = 8 if case == "fp64_pairs_d8" else 16
    order = {"fp64_order4": 4, "fp32_3m_order2": 2, "fp64_cf4": orc.CF4, "fp64_pairs_d8": 2,
             "fp64_magnus6": orc.M6, "fp64_chebyshev": 4}[case]
    n = chains * chunk // (2 if order == orc.CF4 else 1)   # CF4: two exponentials per slice
    w = synth.random_system(d, 3, n_slices=n, h=0.02, order=order, tag=77)
    slices = order not in (orc.CF4, orc.M6)
    out = {}
    for skew in (0, -1, 60):
        say(f"[case] uneven chains {case} d={d} N={n} chunk={chunk} skew={skew}")
        with pm.Context(0, prec) as ctx:
            ctx.set_hamiltonian(w.H0, w.Hk, order)
            if case == "fp64_chebyshev":
                ctx.set_expm_method(pm.PM_EXPM_CHEBYSHEV)
            ctx.set_chunk(chunk)
            ctx.set_chain_skew(skew)
            assert ctx.launch_shape(w.n_samples)[1:] == (chains, chains // 4)
            out[skew] = ctx.equiprop(w.samples, w.h, return_slices=slices)
    ref = out[0]
    if slices:
        Uo, slo = orc.propagate(w.H0, w.Hk, w.samples, w.h, order, return_slices=True)
    else:
        Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, order)
    for skew, res in out.items():
        U, sl = res if slices else (res, None)
        if prec == 0:
            assert orc.relative_frobenius(U, Uo) <= TOL64, skew
            assert orc.relative_frobenius(U, ref[0] if slices else ref) <= assoc_bound(n), skew
        else:
            assert orc.relative_frobenius(U, Uo) <= tol(FP32_3M, n, d), skew
        if slices:
            # a slice's exponential does not depend on its chain (slice pairs:
            # the tile's plan covers both slices of a pair, so rounding may differ)
            if case == "fp64_pairs_d8":
                assert np.max(np.abs(sl - ref[1])) <= 1e-14, skew
            else:
                assert np.array_equal(sl, ref[1]), skew
            assert np.max(np.abs(sl - slo)) <= (1e-13 if prec == 0 else tol_slice(FP32_3M, d)), skew


@pytest.mark.parametrize("d", [2, 4])
def test_uneven_chains_small_dims(pm, d):
    """The small-dimension engine at two blocks of four one-chain waves per
    compute unit: uneven chains (in whole units of 1024 slices) exponentiate
    every slice once and give the oracle's U(T)."""
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    chains, chunk = 2 * n_cu * 4, 2048
    n = chains * chunk - 777                 # a ragged last chain
    w = synth.random_system(d, 2, n_slices=n, h=0.004, order=2, tag=78)
    out = {}
    for skew in (0, -1, 60):
        say(f"[case] uneven chains small d={d} N={n} chunk={chunk} skew={skew}")
        with pm.Context(0, 0) as ctx:
            ctx.set_hamiltonian(w.H0, w.Hk, 2)
            ctx.set_chunk(chunk)
            ctx.set_chain_skew(skew)
            assert ctx.launch_shape(w.n_samples)[1:] == (chains, chains // 4)
            out[skew] = ctx.equiprop(w.samples, w.h, return_slices=True)
    Uo, slo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 2, return_slices=True)
    for skew, (U, sl) in out.items():
        assert np.array_equal(sl, out[0][1]), skew
        assert orc.relative_frobenius(U, out[0][0]) <= assoc_bound(n), skew
        assert orc.relative_frobenius(U, Uo) <= TOL64, skew
    assert np.max(np.abs(out[-1][1] - slo)) <= 1e-13


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_small_dims_sample_block_edges(pm, d):
    """Order 2 on the small-dimension engine where its sample blocks meet
    their edges: no controls (nothing is loaded), a single slice (one sample
    per control, read where it is used), and lengths that end inside a
    block, on the last sample of a 16-byte piece (N = 3, 17, 1001) and on a
    whole piece (N = 2); every slice and U(T) against the oracle, in FP64
    and FP32."""
    for K in (0, 1, 2):
        for n in (1, 2, 3, 17, 1001):
            w = synth.random_system(d, K, n_slices=n, h=0.05, order=2, tag=300 + n)
            Uo, slo = orc.propagate(w.H0, w.Hk, w.samples, w.h, 2, return_slices=True)
            U, sl = run(pm, w, slices=True)
            assert orc.relative_frobenius(U, Uo) <= TOL64, (K, n)
            assert np.max(np.abs(sl - slo)) <= 1e-13, (K, n)
            U32v, sl32 = run(pm, w, precision=pm.PM_FP32, slices=True)
            sq = max_squarings(pm, w, pm.PM_FP32, shift=True)
            assert orc.relative_frobenius(U32v, Uo) <= tol32(n, d, sq), (K, n)
            assert np.max(np.abs(sl32 - slo)) <= tol_slice(FP32, d, sq), (K, n)
