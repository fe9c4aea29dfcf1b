"""Benchmark of the parallel-in-time propagator on one MI355X.

Workload: the random-qudit system (dim 16, 3 GUE controls, 4 sinusoids per
control, N = 2^17 slices of width 1e-3, 4th-order commutator Magnus).  One
*step* is one full propagation of that workload (expand, plan, exponentiate
every slice, chain products and tree to U(T)) with the samples already
resident in HBM, through the C ABI's device entry point.

Prints ONE JSON line.  Besides the headline (FP64 steps/s = slices/s), the
line carries the roofline of the propagation kernel (timed with HIP events on
the launch stream), the oracle's CPU rate, and one object per leg:
  precisions   every precision mode on the headline workload
  slices       the headline workload with every U_j written to HBM
  d64          the dim-64 precision sweep (2^16 slices), every mode, MFMA roofline
  small        dims 2, 4 and 8 with per-slice output (HBM roofline)
  chebyshev    the paper's Chebyshev-series exponential (FP64) on the headline
               and dim-64 workloads, beside the Taylor series
  trajectory   every partial product U(t_j) of the headline workload (FP64)
  grad         fidelity-gradient evals/s on the 3-qubit register
  batch        512 uneven instances in one graph-captured launch
  cpu          the oracle's rate and every mode's error against it
  fixed_error  smallest N reaching a target U(T) error, FP64 vs mixed, on
               the headline and the dim-64 systems (stored oracle references)
``--legs`` picks a subset (default: all); ``--legs copy`` adds a plain
1 GiB device copy, the calibration kernel for the HBM byte counters.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "steps/sec at fixed U(T) error, FP64 vs mixed precision; fidelity-grad evals/sec"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
PEAK = {"fp64": PEAK_FP64_TFLOPS, "fp32": PEAK_FP32_TFLOPS, "fp32_3m": PEAK_FP32_TFLOPS,
        "bf16_split": PEAK_BF16_TFLOPS}
# HBM bytes per launch of the headline kernel come from the FETCH_SIZE /
# WRITE_SIZE passes summarised in this profile, whose pin block records the
# per-dispatch counters, their copy-kernel scale factors and the sha256 of
# the kernel's sources at the time; the traffic is reported only while the
# sources still hash to that value.
TRAFFIC_SOURCES = ["engine_mfma.hip", "mfma_kernel.h", "mfma_tiles.h", "mfma_tree.h", "engine_common.h", "pm_internal.h"]
TRAFFIC_PROFILE = "profiles/propagate_d16_random_qudit_traffic.md"
LEGS = ["precisions", "slices", "d64", "small", "chebyshev", "cf4", "trajectory", "grad", "grape", "batch", "cpu",
        "fixed_error", "magnus6"]


def taylor_products(m: int) -> int:
    return 0 if m <= 1 else (1 if m == 2 else m // 2 + 1)


def engine_dim(d: int) -> int:
    return d if d <= 4 else (16 if d <= 16 else (32 if d <= 32 else 64))


def algorithmic_flops(pm, w, precision, n_leaves: int) -> float:
    """Flops the kernel's algorithm needs for one propagation: per slice
    8 d^3 per complex product over the Taylor products (Y powers and G S'),
    the s squarings and the chain product, plus 4 M d^2 for the expand; the
    tree adds (n_leaves - 1) products.  (m, s) per slice come from the
    library's planner on ||G_j||_1."""
    D = engine_dim(w.dim)
    B, _ = pm.build_basis_host(w.H0, w.Hk, w.order)
    M = B.shape[0]
    n = w.n_slices
    S = w.samples
    h = w.h
    # weights of every slice on the basis (same formulas as the expand step)
    Wt = np.zeros((n, M))
    Wt[:, 0] = h
    K = w.n_ctrl
    if w.order == 2:
        Wt[:, 1:1 + K] = h * S.T
    else:
        s0, s1, s2 = S[:, 0:2 * n:2], S[:, 1:2 * n:2], S[:, 2:2 * n + 1:2]
        Wt[:, 1:1 + K] = (h / 6) * (s0 + 4 * s1 + s2).T
        Wt[:, 1 + K:1 + 2 * K] = (h * h / 12) * (s2 - s0).T
        q = 1 + 2 * K
        for a in range(K):
            for b in range(a + 1, K):
                Wt[:, q] = (h * h / 12) * (s0[a] * s2[b] - s2[a] * s0[b])
                q += 1
    prods = 0
    for c0 in range(0, n, 8192):
        G = np.tensordot(Wt[c0:c0 + 8192], B, axes=1)
        nu = np.max(np.sum(np.abs(G), axis=1), axis=1)
        for x in nu:
            m, s = pm.plan_expm(float(x), precision, n_slices=n)
            prods += taylor_products(m) + s + 1
    prods += n_leaves - 1
    return 8.0 * D ** 3 * prods + 4.0 * M * D * D * n


def issued_mfma_flops(pm, w, precision, n_leaves: int) -> float:
    """MFMA flops the kernel issues for one propagation of w on the 16/32/64
    engines: FP64 and 3M products are three real D x D x D products (6 D^3
    flops per complex product), FP32 4M products four (8 D^3), BF16-split
    products four real products of three BF16 terms each (24 D^3); the
    expand and the plan run on the vector ALU and are not counted."""
    per = {0: 6.0, 1: 8.0, 2: 6.0, 3: 24.0}[precision]
    alg = algorithmic_flops(pm, w, precision, n_leaves)
    D = engine_dim(w.dim)
    B, _ = pm.build_basis_host(w.H0, w.Hk, w.order)
    expand = 4.0 * B.shape[0] * D * D * w.n_slices
    return (alg - expand) / 8.0 * per


def traffic_pin(path: str = TRAFFIC_PROFILE) -> dict:
    """key: value lines of the profile's pin block (<!-- pin ... -->)."""
    pin = {}
    try:
        with open(os.path.join(ROOT, path)) as f:
            txt = f.read()
    except OSError:
        return pin
    if "<!-- pin" not in txt:
        return pin
    block = txt.split("<!-- pin", 1)[1].split("-->", 1)[0]
    for line in block.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            pin[k.strip()] = v.strip()
    return pin


def sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2108_07126_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def headline_traffic():
    pin = traffic_pin()
    try:
        if pin.get("sources_sha256") != sources_sha256():
            return None
        return 1024.0 * (float(pin["fetch_scale"]) * float(pin["fetch_kib_per_dispatch"]) +
                         float(pin["write_scale"]) * float(pin["write_kib_per_dispatch"]))
    except (KeyError, ValueError):
        return None


def time_launches(fn, steps: int, warmup: int):
    """Run fn() warmup+steps times; HIP events (torch's current stream, which
    is the launch stream) around each timed call.  Returns (wall ms/step,
    mean event ms per launch)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    per = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    return wall, per


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return os.cpu_count() or 1


def mode_list(pm):
    return [("fp64", pm.PM_FP64), ("fp32", pm.PM_FP32), ("fp32_3m", pm.PM_FP32_3M),
            ("bf16_split", pm.PM_BF16_SPLIT)]


def flops_of(pm, ctx, w, precision) -> float:
    _, chains, _ = ctx.launch_shape(w.n_samples)
    return algorithmic_flops(pm, w, precision, chains)


def leg_d64(pm, torch, dev, args, out):
    """The dim-64 precision sweep: GUE H0 of norm 10 + 2 controls, 2^16
    slices, midpoint rule; every mode against its own MFMA peak."""
    import synth
    w = synth.precision_sweep()
    s_dev = torch.from_numpy(w.samples).to(dev)
    res = {"workload": "precision_sweep_d64_K2_N65536_h1e-2_midpoint"}
    Ug = {}
    for name, prec in mode_list(pm):
        ctx = pm.Context(0, prec)
        ctx.set_hamiltonian(w.H0, w.Hk, w.order)
        U = torch.zeros((64, 64), dtype=torch.complex128, device=dev)
        wall, k = time_launches(lambda: ctx.equiprop_dev(s_dev, w.h, U), max(3, args.steps // 4), 2)
        fl = flops_of(pm, ctx, w, prec)
        ach = fl / (k * 1e-3) / 1e12
        iss = issued_mfma_flops(pm, w, prec, ctx.launch_shape(w.n_samples)[1])
        res[name] = {"steps_per_s": w.n_slices / (wall * 1e-3), "ms_per_step": wall, "kernel_ms": k,
                     "algorithmic_flop_per_launch": fl, "achieved_tflops": ach, "peak_tflops": PEAK[name],
                     "frac": ach / PEAK[name], "issued_mfma_flop_per_launch": iss,
                     "issued_mfma_frac": iss / (k * 1e-3) / 1e12 / PEAK[name],
                     "launch_shape": list(ctx.launch_shape(w.n_samples))}
        Ug[name] = U.cpu().numpy()
        ctx.close()
    out["d64"] = res
    return w, Ug


def batch_flops(pm, ws, precision, sample: int = 128) -> float:
    """Algorithmic flops of a batch at each instance's own dimension d:
    per slice 8 d^3 per complex product (Taylor products, squarings, chain)
    plus 4 M d^2 for the expand, the planner's (m, s) on `sample` evenly
    spaced slices of each instance scaled to its N (orders 2 and 4)."""
    total = 0.0
    for w in ws:
        B, _ = pm.build_basis_host(w.H0, w.Hk, w.order)
        M, d, n, K, h = B.shape[0], w.dim, w.n_slices, w.n_ctrl, w.h
        idx = np.unique(np.linspace(0, n - 1, min(n, sample)).astype(np.int64))
        Wt = np.zeros((idx.size, M))
        Wt[:, 0] = h
        S = w.samples
        if K:
            if w.order == 2:
                Wt[:, 1:1 + K] = h * S[:, idx].T
            else:
                s0, s1, s2 = S[:, 2 * idx], S[:, 2 * idx + 1], S[:, 2 * idx + 2]
                Wt[:, 1:1 + K] = (h / 6) * (s0 + 4 * s1 + s2).T
                Wt[:, 1 + K:1 + 2 * K] = (h * h / 12) * (s2 - s0).T
                q = 1 + 2 * K
                for a in range(K):
                    for b in range(a + 1, K):
                        Wt[:, q] = (h * h / 12) * (s0[a] * s2[b] - s2[a] * s0[b])
                        q += 1
        G = np.tensordot(Wt, B, axes=1)
        nu = np.max(np.sum(np.abs(G), axis=1), axis=1)
        prods = 0
        for x in nu:
            m, s_ = pm.plan_expm(float(x), precision, n_slices=n)
            prods += taylor_products(m) + s_ + 1
        total += (8.0 * d ** 3 * prods + 4.0 * M * d * d * idx.size) * (n / idx.size)
    return total


def sampled_flops(pm, w, precision, sample: int = 65536) -> float:
    """Algorithmic flops of a propagation at the user dimension d: per slice
    8 d^3 per complex product (Taylor products, squarings, chain) plus
    4 M d^2 for the expand, the planner's (m, s) taken on the first `sample`
    slices' ||G_j||_1 and scaled to all N (order-2 workloads)."""
    B, _ = pm.build_basis_host(w.H0, w.Hk, w.order)
    M, d, n = B.shape[0], w.dim, w.n_slices
    ns = min(n, sample)
    Wt = np.zeros((ns, M))
    Wt[:, 0] = w.h
    Wt[:, 1:1 + w.n_ctrl] = w.h * w.samples[:, :ns].T
    G = np.tensordot(Wt, B, axes=1)
    nu = np.max(np.sum(np.abs(G), axis=1), axis=1)
    prods = 0
    for x in nu:
        m, s_ = pm.plan_expm(float(x), precision, n_slices=n)
        prods += taylor_products(m) + s_ + 1
    return (8.0 * d ** 3 * prods + 4.0 * M * d * d * ns) * (n / ns)


def leg_small(pm, torch, dev, args, out):
    """Dims 2, 4 and 8 with every U_j written out.  Algorithmic bytes per
    slice = the slice's control samples (8 B each) + its propagator (d^2
    complex entries, 16 B in FP64 and 8 B otherwise); algorithmic flops from
    sampled_flops.  The roofline time is the larger of bytes / 8 TB/s and
    flops / the precision's vector/MFMA peak: dims 2 and 4 sit at or below
    the FP64 ridge (9.8 flop/B), dim 8 far above it (compute-bound)."""
    import synth
    cases = [("driven_qubit_d2_N2^26", synth.driven_qubit(n_slices=2 ** 26, h=0.01)),
             ("random_d4_K2_N2^24", synth.random_system(4, 2, n_slices=2 ** 24, h=0.01, order=2, tag=40)),
             ("qubit_register_d8_K4_N2^22", synth.qubit_register(n_slices=2 ** 22))]
    res = {}
    for label, w in cases:
        d, N = w.dim, w.n_slices
        s_dev = torch.from_numpy(w.samples).to(dev)
        row = {}
        for name, prec in (("fp64", pm.PM_FP64), ("fp32", pm.PM_FP32)):
            ctx = pm.Context(0, prec)
            ctx.set_hamiltonian(w.H0, w.Hk, w.order)
            U = torch.zeros((d, d), dtype=torch.complex128, device=dev)
            ct = torch.complex128 if prec == pm.PM_FP64 else torch.complex64
            sl = torch.empty((N, d, d), dtype=ct, device=dev)
            wall, k = time_launches(lambda: ctx.equiprop_dev(s_dev, w.h, U, sl), 5, 2)
            _, k_nos = time_launches(lambda: ctx.equiprop_dev(s_dev, w.h, U), 5, 2)
            nbytes = w.samples.size * 8 + N * d * d * (16 if prec == pm.PM_FP64 else 8)
            gbs = nbytes / (k * 1e-3) / 1e9
            flops = sampled_flops(pm, w, prec)
            peak = PEAK_FP64_TFLOPS if prec == pm.PM_FP64 else PEAK_FP32_TFLOPS
            t_roof = max(nbytes / (PEAK_HBM_GBS * 1e9), flops / (peak * 1e12)) * 1e3
            row[name] = {"steps_per_s": N / (wall * 1e-3), "kernel_ms": k, "kernel_ms_without_slices": k_nos,
                         "algorithmic_bytes": nbytes, "achieved_gbs": gbs, "frac_hbm": gbs / PEAK_HBM_GBS,
                         "algorithmic_flops": flops, "flop_per_byte": flops / nbytes,
                         "bound": ("hbm" if nbytes / (PEAK_HBM_GBS * 1e9) >= flops / (peak * 1e12)
                                   else ("alu" if d <= 4 else "mfma")),
                         "roofline_ms": t_roof, "frac_roofline": t_roof / k}
            del sl
            ctx.close()
        res[label] = row
    out["small"] = res


def leg_chebyshev(pm, torch, dev, args, out):
    """FP64 propagation with the Chebyshev series (Clenshaw, Table-1
    degrees) on the headline and dim-64 workloads."""
    import synth
    res = {}
    for label, w in (("random_qudit_d16_N2^17", synth.random_qudit()),
                     ("precision_sweep_d64_N2^16", synth.precision_sweep())):
        s_dev = torch.from_numpy(w.samples).to(dev)
        U = torch.zeros((w.dim, w.dim), dtype=torch.complex128, device=dev)
        row = {}
        for name, method in (("taylor", pm.PM_EXPM_TAYLOR), ("chebyshev", pm.PM_EXPM_CHEBYSHEV)):
            ctx = pm.Context(0, pm.PM_FP64)
            ctx.set_hamiltonian(w.H0, w.Hk, w.order)
            ctx.set_expm_method(method)
            steps = max(3, args.steps // (4 if w.dim == 64 else 1))
            _, k = time_launches(lambda: ctx.equiprop_dev(s_dev, w.h, U), steps, 2)
            row[name] = {"kernel_ms": k, "steps_per_s": w.n_slices / (k * 1e-3)}
            row[name + "_U"] = U.cpu().numpy()
            ctx.close()
        row["chebyshev_over_taylor_time"] = row["chebyshev"]["kernel_ms"] / row["taylor"]["kernel_ms"]
        res[label] = row
    out["chebyshev"] = res


def leg_cf4(pm, torch, dev, args, out):
    """FP64 propagation with the commutator-free fourth-order step against
    the commutator Magnus step at equal N on the headline system (3
    controls) and on the same system with 8 controls, where the commutator
    basis grows to 45 matrices against 9."""
    import synth
    res = {}
    for K in (3, 8):
        row = {}
        for name, order in (("magnus4", 4), ("cf4", pm.PM_ORDER_CF4)):
            w = synth.random_qudit(order=order, n_ctrl=K)
            s_dev = torch.from_numpy(w.samples).to(dev)
            U = torch.zeros((w.dim, w.dim), dtype=torch.complex128, device=dev)
            ctx = pm.Context(0, pm.PM_FP64)
            ctx.set_hamiltonian(w.H0, w.Hk, order)
            _, k = time_launches(lambda: ctx.equiprop_dev(s_dev, w.h, U), max(3, args.steps), 2)
            row[name] = {"kernel_ms": k, "steps_per_s": w.n_slices / (k * 1e-3),
                         "basis": pm.basis_count(K, order)}
            row[name + "_U"] = U.cpu().numpy()
            ctx.close()
        row["rel_diff"] = float(np.linalg.norm(row["cf4_U"] - row["magnus4_U"]) / np.linalg.norm(row["magnus4_U"]))
        del row["cf4_U"], row["magnus4_U"]
        row["cf4_over_magnus4_time"] = row["cf4"]["kernel_ms"] / row["magnus4"]["kernel_ms"]
        res[f"random_qudit_d16_K{K}_N2^17"] = row
    out["cf4"] = res


def leg_trajectory(pm, torch, dev, args, out):
    """All N+1 partial products of the headline workload (4 KiB each)."""
    import synth
    w = synth.random_qudit()
    s_dev = torch.from_numpy(w.samples).to(dev)
    ctx = pm.Context(0, pm.PM_FP64)
    ctx.set_hamiltonian(w.H0, w.Hk, w.order)
    P = torch.empty((w.n_slices + 1, 16, 16), dtype=torch.complex128, device=dev)
    wall, k = time_launches(lambda: ctx.trajectory_dev(s_dev, w.h, P), max(3, args.steps // 2), 2)
    out["trajectory"] = {"workload": "random_qudit_d16_N2^17, propagators", "ms": k,
                         "steps_per_s": w.n_slices / (k * 1e-3), "out_bytes": P.numel() * 16,
                         "out_gbs": P.numel() * 16 / (k * 1e-3) / 1e9}
    ctx.close()


GRAD_STREAMS = 4


def leg_grad_independent(pm, torch, dev, synth, n: int = 64):
    """n independent gradient evaluations of the 3-qubit register (other
    controls and targets), spread round-robin over GRAD_STREAMS contexts with
    a stream each, so that the short, latency-bound launches of different
    evaluations overlap.  W of each is dL/dU-bar of its own fidelity loss at
    its controls.  Wall clock over whole rounds of n evaluations."""
    ws = [synth.qubit_register(tag=1000 + i) for i in range(n)]
    ctxs = []
    for _ in range(GRAD_STREAMS):
        c = pm.Context(0, pm.PM_FP64)
        c.set_hamiltonian(ws[0].H0, ws[0].Hk, 2)
        ctxs.append(c)
    S, W = [], []
    for w in ws:
        U = ctxs[0].equiprop(w.samples, w.h)
        g = np.trace(w.target.conj().T @ U)
        S.append(torch.from_numpy(w.samples).to(dev))
        W.append(torch.from_numpy(-(2 * g / 64) * w.target).to(dev))
    G = [torch.zeros_like(s) for s in S]
    streams = [torch.cuda.Stream() for _ in range(GRAD_STREAMS)]

    def run():
        for i, w in enumerate(ws):
            k = i % GRAD_STREAMS
            ctxs[k].backward_dev(S[i], w.h, W[i], G[i], stream=streams[k])
    for _ in range(2):
        run()
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    for c in ctxs:
        c.close()
    return {"evaluations": n, "streams": GRAD_STREAMS, "ms_per_round": t * 1e3, "evals_per_s": n / t}


GOLDEN = os.path.join(ROOT, "tests", "golden", "full_size_oracle.npz")


def rel_frobenius(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def leg_fixed_error(pm, torch, dev, modes):
    """Steps/s at a fixed U(T) error, FP64 against the reduced precisions.

    For each workload the span T stays fixed and N = 2^n slices of width
    T / N are propagated in every mode; the error of U(T) is taken against
    the oracle's U(T) over the same span, stored by
    tests/golden/make_full_size.py: at the random qudit's own N (2^17,
    order 4), and for the dim-64 sweep at eight times its N (2^19, midpoint
    rule; its own 2^16 slices carry a discretisation error of about 2e-3,
    so its targets are 1e-2 and 1e-3 instead of the qudit's 1e-4 and 1e-6).
    N is searched only up to a quarter of the reference's N, where the
    reference's own discretisation error is below 1/4^p of the measured one
    (p the order), so the measured errors are the coarse runs' own.  For each
    target the smallest N meeting it is reported with its kernel time (HIP
    events on the launch stream) and wall time, and the FP64 / mode
    kernel-time ratio at the target: the speed-up of the mode at equal
    accuracy."""
    import synth
    if not os.path.exists(GOLDEN):
        return {"skipped": "no stored oracle reference"}
    with np.load(GOLDEN) as z:
        refs = {k: z[k] for k in ("random_qudit", "precision_sweep_fine") if k in z.files}
    # (label, reference key, workload at N slices of width h, reference N, span, order, targets, search)
    cases = [("random_qudit_d16_K3_magnus4", "random_qudit",
              lambda n, h: synth.random_qudit(n_slices=n, h=h), 2 ** 17, 2 ** 17 * 1e-3, 4, (1e-4, 1e-6),
              range(9, 16)),
             ("precision_sweep_d64_K2_midpoint", "precision_sweep_fine",
              lambda n, h: synth.precision_sweep(n_slices=n, h=h), 2 ** 19, 2 ** 16 * 1e-2, 2, (1e-2, 1e-3),
              range(12, 18))]
    res = {}
    for label, key, make, n_ref, T, slope, targets, search in cases:
        if key not in refs:
            res[label] = {"skipped": "no stored oracle reference"}
            continue
        row = {"reference": f"oracle U(T) at N = {n_ref} (order {slope}), searched N <= {n_ref // 4}: the "
                            f"reference's own discretisation error is at most 1/{4 ** slope} of the "
                            f"measured error there", "span_T": T, "targets": list(targets)}
        curves = {}
        for name, prec in modes:
            ctx = pm.Context(0, prec)
            w0 = make(2 ** search.start, T / 2 ** search.start)
            ctx.set_hamiltonian(w0.H0, w0.Hk, w0.order)
            cur = {}
            for n in search:
                nn = 2 ** n
                wn = make(nn, T / nn)
                sd = torch.from_numpy(wn.samples).to(dev)
                Ud = torch.zeros((wn.dim, wn.dim), dtype=torch.complex128, device=dev)
                wall, kms = time_launches(lambda: ctx.equiprop_dev(sd, wn.h, Ud), 5, 2)
                cur[nn] = {"err": rel_frobenius(Ud.cpu().numpy(), refs[key]), "ms": wall, "kernel_ms": kms}
            ctx.close()
            curves[name] = cur
            row[name] = {str(k): v for k, v in cur.items()}
        summ = {}
        for eps in targets:
            base = None
            for name, _ in modes:
                ok = [k for k, v in curves[name].items() if v["err"] <= eps]
                if not ok:
                    summ[f"{name}_eps_{eps:.0e}"] = None
                    continue
                k = min(ok)
                v = curves[name][k]
                e = {"n_slices": k, "kernel_ms": v["kernel_ms"], "ms": v["ms"],
                     "steps_per_s": k / (v["kernel_ms"] * 1e-3)}
                if name == "fp64":
                    base = v["kernel_ms"]
                elif base is not None:
                    e["fp64_over_mode_kernel_time"] = base / v["kernel_ms"]
                summ[f"{name}_eps_{eps:.0e}"] = e
        row["summary"] = summ
        res[label] = row
    return res


def leg_magnus6(pm, torch, dev):
    """The sixth-order Magnus scheme (three Gauss-Legendre samples per slice)
    against the fourth-order step on the random qudit (d = 16, 3 controls)
    over its fixed span T = 2^17 * 1e-3, in FP64.  N = 2^n slices of width
    T / N; the error of U(T) is taken against the oracle's sixth-order U(T)
    at N = 2^17, stored by tests/golden/make_full_size.py.  Targets are met
    only at N <= 2^15, where the reference's own discretisation error is at
    most 1/4^6 of the sixth-order run's.  For each target: the smallest N
    reaching it with either scheme, its kernel time (HIP events on the
    launch stream), and the fourth- over sixth-order time at equal accuracy.
    At N = 2^17 both schemes' cost per slice, and the sixth-order run's
    difference from the oracle at the same N (a full-size parity figure)."""
    import synth
    if not os.path.exists(GOLDEN):
        return {"skipped": "no stored oracle reference"}
    with np.load(GOLDEN) as z:
        if "random_qudit_m6" not in z.files:
            return {"skipped": "no stored oracle reference"}
        ref = z["random_qudit_m6"]
    full = 2 ** 17
    T = full * 1e-3
    targets = (1e-4, 1e-6, 1e-8)
    orders = (("magnus4", 4), ("magnus6", pm.PM_ORDER_MAGNUS6))
    res = {"workload": "random_qudit_d16_K3, span T = 131.072", "span_T": T, "targets": list(targets),
           "reference": f"oracle U(T), sixth order, N = {full}; targets searched at N <= {full // 4}"}
    curves = {}
    for name, order in orders:
        w0 = synth.random_qudit(n_slices=2 ** 9, h=T / 2 ** 9, order=order)
        ctx = pm.Context(0, pm.PM_FP64)
        ctx.set_hamiltonian(w0.H0, w0.Hk, order)
        cur = {}
        for n in list(range(9, 16)) + [17]:
            nn = 2 ** n
            wn = synth.random_qudit(n_slices=nn, h=T / nn, order=order)
            sd = torch.from_numpy(wn.samples).to(dev)
            Ud = torch.zeros((wn.dim, wn.dim), dtype=torch.complex128, device=dev)
            _, kms = time_launches(lambda: ctx.equiprop_dev(sd, wn.h, Ud), 5, 2)
            cur[nn] = {"err": rel_frobenius(Ud.cpu().numpy(), ref), "kernel_ms": kms}
        ctx.close()
        curves[name] = cur
        res[name] = {str(k): v for k, v in cur.items()}
    summ = {}
    for eps in targets:
        row = {}
        for name, _ in orders:
            ok = [k for k, v in curves[name].items() if k <= full // 4 and v["err"] <= eps]
            row[name] = {"n_slices": min(ok), "kernel_ms": curves[name][min(ok)]["kernel_ms"]} if ok else None
        if row["magnus4"] and row["magnus6"]:
            row["magnus4_over_magnus6_kernel_time"] = row["magnus4"]["kernel_ms"] / row["magnus6"]["kernel_ms"]
        summ[f"eps_{eps:.0e}"] = row
    res["summary"] = summ
    res["ns_per_slice_at_2^17"] = {name: curves[name][full]["kernel_ms"] / full * 1e6 for name, _ in orders}
    res["magnus6_rel_err_vs_oracle_at_2^17"] = curves["magnus6"][full]["err"]
    return res


def leg_copy(torch, dev, out):
    """A plain device copy of 1 GiB (reads 1 GiB, writes 1 GiB): the
    calibration kernel for the FETCH_SIZE / WRITE_SIZE counters."""
    a = torch.empty(2 ** 27, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    wall, k = time_launches(lambda: b.copy_(a), 5, 2)
    out["copy"] = {"bytes_read": a.numel() * 8, "bytes_written": a.numel() * 8, "kernel_ms": k,
                   "gbs": 2 * a.numel() * 8 / (k * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--legs", default="all",
                    help="comma list from " + ",".join(LEGS) + ",copy (default: all but copy)")
    ap.add_argument("--skip-cpu", action="store_true", help="leave out the oracle CPU baseline")
    ap.add_argument("--skip-fixed-error", action="store_true")
    ap.add_argument("--skip-batch", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the time axis would shard across GPUs with one gather of block products).",
              file=sys.stderr)
        sys.exit(2)
    legs = set(LEGS) if args.legs == "all" else set(x for x in args.legs.split(",") if x)
    unknown = legs - set(LEGS) - {"copy"}
    if unknown:
        print(f"unknown legs: {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)
    if args.skip_cpu:
        legs.discard("cpu")
    if args.skip_fixed_error:
        legs.discard("fixed_error")
    if args.skip_batch:
        legs.discard("batch")

    import torch
    import paper_2108_07126_amd as pm
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    w = synth.random_qudit()
    N = w.n_slices
    d = w.dim
    s_dev = torch.from_numpy(w.samples).to(dev)

    modes = mode_list(pm) if "precisions" in legs else mode_list(pm)[:1]
    ctxs, timing, Ug, flops = {}, {}, {}, {}
    for name, prec in modes:
        ctx = pm.Context(0, prec)
        ctx.set_hamiltonian(w.H0, w.Hk, w.order)
        U = torch.zeros((d, d), dtype=torch.complex128, device=dev)
        steps = args.steps if name == "fp64" else max(5, args.steps // 2)
        timing[name] = time_launches(lambda: ctx.equiprop_dev(s_dev, w.h, U), steps, args.warmup)
        Ug[name] = U.cpu().numpy()
        ctxs[name] = ctx
        flops[name] = flops_of(pm, ctx, w, prec)
    wall64, k64 = timing["fp64"]
    chunk, chains, leaves = ctxs["fp64"].launch_shape(w.n_samples)
    ach64 = flops["fp64"] / (k64 * 1e-3) / 1e12
    issued64 = issued_mfma_flops(pm, w, pm.PM_FP64, chains)

    out = {
        "metric": METRIC,
        "value": N / (wall64 * 1e-3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "random_qudit_d16_K3_N131072_h1e-3_magnus4", "dim": d, "n_ctrl": w.n_ctrl,
                   "n_slices": N, "order": 4, "dt": w.h, "output": "U(T)", "chunk": chunk, "chains": chains,
                   "leaves": leaves},
        "roofline": {"bound": "mfma", "achieved": ach64, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach64 / PEAK_FP64_TFLOPS, "traffic": headline_traffic(),
                     "traffic_unit": "bytes per launch", "traffic_profile": TRAFFIC_PROFILE,
                     "algorithmic_bytes_per_launch": w.samples.size * 8 + d * d * 16,
                     "kernel": "propagate_mfma<double,16,4,true,0,false,false,false>", "kernel_ms": k64,
                     "algorithmic_flop_per_launch": flops["fp64"],
                     "frac_basis": "algorithmic flops: 8 d^3 per complex product",
                     "issued_mfma_flop_per_launch": issued64,
                     "issued_mfma_frac": issued64 / (k64 * 1e-3) / 1e12 / PEAK_FP64_TFLOPS},
    }
    if "precisions" in legs:
        out["precisions"] = {name: {"steps_per_s": N / (timing[name][0] * 1e-3), "ms_per_step": timing[name][0],
                                    "kernel_ms": timing[name][1],
                                    "achieved_tflops": flops[name] / (timing[name][1] * 1e-3) / 1e12,
                                    "peak_tflops": PEAK[name]}
                             for name, _ in modes}

    if "slices" in legs:
        # per-slice output: 512 MiB of complex128 propagators per step
        sl = torch.empty((N, d, d), dtype=torch.complex128, device=dev)
        U64 = torch.zeros((d, d), dtype=torch.complex128, device=dev)
        wall64s, k64s = time_launches(lambda: ctxs["fp64"].equiprop_dev(s_dev, w.h, U64, sl),
                                      max(5, args.steps // 2), 2)
        del sl
        out["fp64_with_slices"] = {"steps_per_s": N / (wall64s * 1e-3), "kernel_ms": k64s,
                                   "slice_bytes": N * d * d * 16,
                                   "hbm_write_gbs": N * d * d * 16 / (k64s * 1e-3) / 1e9}

    w64 = Ug64 = None
    if "d64" in legs:
        w64, Ug64 = leg_d64(pm, torch, dev, args, out)
    if "small" in legs:
        leg_small(pm, torch, dev, args, out)
    if "copy" in legs:
        leg_copy(torch, dev, out)
    if "chebyshev" in legs:
        leg_chebyshev(pm, torch, dev, args, out)
    if "cf4" in legs:
        leg_cf4(pm, torch, dev, args, out)
    if "trajectory" in legs:
        leg_trajectory(pm, torch, dev, args, out)

    wg = None
    if "grad" in legs:
        # adjoint gradient: fidelity-grad evals/s on the 3-qubit register workload
        wg = synth.qubit_register()
        cg = pm.Context(0, pm.PM_FP64)
        cg.set_hamiltonian(wg.H0, wg.Hk, 2)
        sg = torch.from_numpy(wg.samples).to(dev)
        Wt = torch.zeros((8, 8), dtype=torch.complex128, device=dev)
        gt = torch.zeros_like(sg)
        Ut = torch.zeros((8, 8), dtype=torch.complex128, device=dev)
        loss, grad_h, Uh = cg.fidelity_grad(wg.samples, wg.h, wg.target)   # host entry point (also warms up)
        g_tr = np.trace(wg.target.conj().T @ Uh)
        Wt.copy_(torch.from_numpy(-(2 * g_tr / 64) * wg.target))
        wall_g, k_g = time_launches(lambda: cg.backward_dev(sg, wg.h, Wt, gt, Ut), max(5, args.steps), 2)
        out["grad"] = {"workload": "qubit_register_d8_K4_N4096", "evals_per_s": 1e3 / wall_g,
                       "ms_per_eval": wall_g, "gpu_ms_per_eval": k_g, "params": int(wg.samples.size),
                       "loss": loss}
        out["grad"]["x64"] = leg_grad_independent(pm, torch, dev, synth)

    if "grape" in legs:
        # the whole optimisation loop on the device: forward, loss, adjoint, Adam update
        wq = synth.qubit_register()
        cq = pm.Context(0, pm.PM_FP64)
        cq.set_hamiltonian(wq.H0, wq.Hk, 2)
        s0 = torch.from_numpy(wq.samples).to(dev)
        sq = s0.clone()
        Vq = torch.from_numpy(np.ascontiguousarray(wq.target)).to(dev)
        iters = 20
        lq = torch.empty(iters + 1, dtype=torch.float64, device=dev)

        def grape_run():
            sq.copy_(s0)
            cq.grape_dev(sq, wq.h, Vq, iters, 0.05, pm.PM_OPT_ADAM, lq)
        wall_q, k_q = time_launches(grape_run, 3, 1)
        lh = lq.cpu().numpy()
        out["grape"] = {"workload": "qubit_register_d8_K4_N4096, Adam", "iters": iters,
                        "ms_per_iter": wall_q / iters, "iters_per_s": iters / (wall_q * 1e-3),
                        "loss_first": float(lh[0]), "loss_last": float(lh[-1])}
        cq.close()

    if "batch" in legs:
        # batched uneven instances: one persistent, graph-captured launch
        ws = synth.batched_instances()
        nsl = int(sum(x.n_slices for x in ws))
        bt = pm.Batch(0, pm.PM_FP32_3M)
        t0 = time.perf_counter()
        bt.set(ws)
        t_set = time.perf_counter() - t0
        wall_b, k_b = time_launches(lambda: bt.run(torch.cuda.current_stream()), 3, 1)
        fl = batch_flops(pm, ws, pm.PM_FP32_3M)
        out["batch"] = {"workload": "512 uneven instances (d 2..64, K 1..4, N 1e3..1e5, orders 2/4)",
                        "precision": "fp32_3m", "slices": nsl, "packets": bt.n_packets, "ms_per_run": wall_b,
                        "kernel_ms": k_b, "steps_per_s": nsl / (wall_b * 1e-3), "set_s": t_set,
                        "algorithmic_flops": fl, "achieved_tflops": fl / (k_b * 1e-3) / 1e12,
                        "frac_fp32_peak": fl / (k_b * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}
        bt.close()

    Uo = None
    if "cpu" in legs:
        import oracle.propagator as orc
        t0 = time.perf_counter()
        Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, w.order)
        dt_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": N / dt_cpu, "unit": "steps/s", "cores": blas_threads(), "kind": "oracle",
                               "sample": f"the whole workload ({N} slices, one run, {dt_cpu:.1f} s)",
                               "host_nproc": os.cpu_count(), "host_cpu": host_cpu_model()}
        out["error_vs_oracle"] = {name: orc.relative_frobenius(Ug[name], Uo) for name, _ in modes}
        if "chebyshev" in out:
            row = out["chebyshev"]["random_qudit_d16_N2^17"]
            out["error_vs_oracle"]["fp64_chebyshev"] = orc.relative_frobenius(row["chebyshev_U"], Uo)
        if wg is not None:
            _, go = orc.control_gradient(wg.H0, wg.Hk, wg.samples, wg.h, 2,
                                         orc.fidelity_grad_U(orc.propagate(wg.H0, wg.Hk, wg.samples, wg.h, 2),
                                                             wg.target))
            out["grad"]["rel_err_vs_oracle"] = float(np.max(np.abs(grad_h - go)) / np.max(np.abs(go)))
        if w64 is not None:
            # dim 64: error of U(T) on a bounded prefix (the oracle needs about
            # 1.5 ms per slice at this size on the host)
            n_pre = 4096
            wp = synth.precision_sweep(n_slices=n_pre)
            Uo64 = orc.propagate(wp.H0, wp.Hk, wp.samples, wp.h, wp.order)
            e64 = {}
            for name, prec in mode_list(pm):
                with pm.Context(0, prec) as ctx:
                    ctx.set_hamiltonian(wp.H0, wp.Hk, wp.order)
                    e64[name] = orc.relative_frobenius(ctx.equiprop(wp.samples, wp.h), Uo64)
            out["d64"]["error_vs_oracle_first_4096_slices"] = e64

    if "fixed_error" in legs:
        out["fixed_error"] = leg_fixed_error(pm, torch, dev, modes)
    if "magnus6" in legs:
        out["magnus6"] = leg_magnus6(pm, torch, dev)

    if "chebyshev" in out:
        for row in out["chebyshev"].values():
            row.pop("taylor_U", None)
            row.pop("chebyshev_U", None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
