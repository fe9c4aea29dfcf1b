"""Benchmark of the parallel-in-time propagator on one MI355X.

Workload: the random-qudit system (dim 16, 3 GUE controls, 4 sinusoids per
control, N = 2^17 slices of width 1e-3, 4th-order commutator Magnus).  One
*step* is one full propagation of that workload (expand, plan, exponentiate
every slice, chain products and tree to U(T)) with the samples already
resident in HBM, through the C ABI's device entry point.

Prints ONE JSON line.  Besides the headline (FP64 steps/s = slices/s), the
line carries the roofline of the propagation kernel (timed with HIP events on
the launch stream), the oracle's CPU rate, the FP32 path's rate and error,
the fixed-error comparison FP64 vs FP32, and a per-slice-output variant.
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


def taylor_products(m: int) -> int:
    return 0 if m <= 1 else (1 if m == 2 else m // 2 + 1)


def algorithmic_flops(pm, w, precision, n_leaves: int) -> float:
    """Flops the kernel's algorithm needs for one propagation: per slice
    8 d^3 per complex product over the Taylor products (Y powers and G S'),
    the s squarings and the chain product, plus 4 M d^2 for the expand; the
    tree adds (n_leaves - 1) products.  (m, s) per slice come from the
    library's planner on ||G_j||_1."""
    d = w.dim
    D = 16 if 4 < d <= 16 else (32 if 16 < d <= 32 else (64 if d > 32 else d))
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
            m, s = pm.plan_expm(float(x), 0 if precision == 0 else 1, n_slices=n)
            prods += taylor_products(m) + s + 1
    prods += n_leaves - 1
    return 8.0 * D ** 3 * prods + 4.0 * M * D * D * n


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


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return os.cpu_count() or 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--skip-cpu", action="store_true", help="leave out the oracle CPU baseline")
    ap.add_argument("--skip-fixed-error", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the time axis would shard across GPUs with one gather of block products).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2108_07126_amd as pm
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    w = synth.random_qudit()
    N = w.n_slices
    d = w.dim
    s_dev = torch.from_numpy(w.samples).to(dev)

    def make(precision):
        ctx = pm.Context(0, precision)
        ctx.set_hamiltonian(w.H0, w.Hk, w.order)
        return ctx

    ctx64 = make(pm.PM_FP64)
    U64 = torch.zeros((d, d), dtype=torch.complex128, device=dev)
    wall64, k64 = time_launches(lambda: ctx64.equiprop_dev(s_dev, w.h, U64), args.steps, args.warmup)
    Ug64 = U64.cpu().numpy()

    ctx32 = make(pm.PM_FP32)
    U32 = torch.zeros((d, d), dtype=torch.complex128, device=dev)
    wall32, k32 = time_launches(lambda: ctx32.equiprop_dev(s_dev, w.h, U32), args.steps, args.warmup)
    Ug32 = U32.cpu().numpy()

    # per-slice output variant (a4): 512 MiB of complex128 propagators per step
    sl = torch.empty((N, d, d), dtype=torch.complex128, device=dev)
    wall64s, k64s = time_launches(lambda: ctx64.equiprop_dev(s_dev, w.h, U64, sl), max(5, args.steps // 2), 2)
    del sl

    # leaves used by the automatic chunking (same rule as the library)
    resident = 256 * 8
    chunk = max(1, math.ceil(N / (2 * resident)))
    leaves = math.ceil(N / chunk)
    flops64 = algorithmic_flops(pm, w, 0, leaves)
    flops32 = algorithmic_flops(pm, w, 1, leaves)
    ach64 = flops64 / (k64 * 1e-3) / 1e12

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
                   "n_slices": N, "order": 4, "dt": w.h, "output": "U(T)", "chunk": chunk, "leaves": leaves},
        "roofline": {"bound": "mfma", "achieved": ach64, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach64 / PEAK_FP64_TFLOPS, "traffic": None,
                     "kernel": "propagate_mfma<double,16,4>", "kernel_ms": k64,
                     "algorithmic_flop_per_launch": flops64},
        "fp32": {"steps_per_s": N / (wall32 * 1e-3), "ms_per_step": wall32, "kernel_ms": k32,
                 "achieved_tflops": flops32 / (k32 * 1e-3) / 1e12, "peak_tflops": PEAK_FP32_TFLOPS},
        "fp64_with_slices": {"steps_per_s": N / (wall64s * 1e-3), "kernel_ms": k64s,
                             "slice_bytes": N * d * d * 16,
                             "hbm_write_gbs": N * d * d * 16 / (k64s * 1e-3) / 1e9},
        "grad": None,
    }

    Uo = None
    if not args.skip_cpu:
        import oracle.propagator as orc
        t0 = time.perf_counter()
        Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, w.order)
        dt_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": N / dt_cpu, "unit": "steps/s", "cores": blas_threads(), "kind": "oracle",
                               "sample": f"the whole workload ({N} slices, one run, {dt_cpu:.1f} s)"}
        out["error_vs_oracle"] = {"fp64": orc.relative_frobenius(Ug64, Uo), "fp32": orc.relative_frobenius(Ug32, Uo)}

    if not args.skip_fixed_error and Uo is not None:
        import oracle.propagator as orc
        # same T, coarser slicing: smallest N=2^n meeting each target error
        T = N * w.h
        res = {}
        for name, ctx in (("fp64", ctx64), ("fp32", ctx32)):
            errs = {}
            for n in range(8, 18):
                nn = 2 ** n
                wn = synth.random_qudit(n_slices=nn, h=T / nn)
                sd = torch.from_numpy(wn.samples).to(dev)
                Ud = torch.zeros((d, d), dtype=torch.complex128, device=dev)
                wall, _ = time_launches(lambda: ctx.equiprop_dev(sd, wn.h, Ud), 5, 2)
                errs[nn] = (orc.relative_frobenius(Ud.cpu().numpy(), Uo), wall)
            res[name] = {str(k): {"err": v[0], "ms": v[1]} for k, v in errs.items()}
            for eps in (1e-4, 1e-6):
                ok = [k for k, v in errs.items() if v[0] <= eps]
                key = f"eps_{eps:.0e}"
                if ok:
                    k = min(ok)
                    res.setdefault("summary", {})[f"{name}_{key}"] = {
                        "n_slices": k, "ms": errs[k][1], "steps_per_s": k / (errs[k][1] * 1e-3)}
                else:
                    res.setdefault("summary", {})[f"{name}_{key}"] = None
        out["fixed_error"] = res

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
