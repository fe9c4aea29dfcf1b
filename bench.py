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
    ap.add_argument("--skip-batch", action="store_true")
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

    modes = [("fp64", pm.PM_FP64), ("fp32", pm.PM_FP32), ("fp32_3m", pm.PM_FP32_3M),
             ("bf16_split", pm.PM_BF16_SPLIT)]
    ctxs, timing, Ug = {}, {}, {}
    for name, prec in modes:
        ctx = make(prec)
        U = torch.zeros((d, d), dtype=torch.complex128, device=dev)
        steps = args.steps if name == "fp64" else max(5, args.steps // 2)
        timing[name] = time_launches(lambda: ctx.equiprop_dev(s_dev, w.h, U), steps, args.warmup)
        Ug[name] = U.cpu().numpy()
        ctxs[name] = ctx
    wall64, k64 = timing["fp64"]

    # per-slice output variant: 512 MiB of complex128 propagators per step
    sl = torch.empty((N, d, d), dtype=torch.complex128, device=dev)
    U64 = torch.zeros((d, d), dtype=torch.complex128, device=dev)
    wall64s, k64s = time_launches(lambda: ctxs["fp64"].equiprop_dev(s_dev, w.h, U64, sl),
                                  max(5, args.steps // 2), 2)
    del sl

    # leaves used by the automatic chunking (same rule as the library)
    chunk = max(1, math.ceil(N / (256 * 8)))
    leaves = math.ceil(N / chunk)
    flops = {name: algorithmic_flops(pm, w, 0 if name == "fp64" else 1, leaves) for name, _ in modes}
    ach64 = flops["fp64"] / (k64 * 1e-3) / 1e12

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
                     "kernel": "propagate_mfma<double,16,4,true,0>", "kernel_ms": k64,
                     "algorithmic_flop_per_launch": flops["fp64"]},
        "precisions": {name: {"steps_per_s": N / (timing[name][0] * 1e-3), "ms_per_step": timing[name][0],
                              "kernel_ms": timing[name][1],
                              "achieved_tflops": flops[name] / (timing[name][1] * 1e-3) / 1e12}
                       for name, _ in modes},
        "fp64_with_slices": {"steps_per_s": N / (wall64s * 1e-3), "kernel_ms": k64s,
                             "slice_bytes": N * d * d * 16,
                             "hbm_write_gbs": N * d * d * 16 / (k64s * 1e-3) / 1e9},
    }

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
    out["grad"] = {"workload": "qubit_register_d8_K4_N4096", "evals_per_s": 1e3 / wall_g, "ms_per_eval": wall_g,
                   "gpu_ms_per_eval": k_g, "params": int(wg.samples.size), "loss": loss}

    # batched uneven instances: one persistent, graph-captured launch
    if not args.skip_batch:
        ws = synth.batched_instances()
        nsl = int(sum(x.n_slices for x in ws))
        bt = pm.Batch(0, pm.PM_FP32_3M)
        t0 = time.perf_counter()
        bt.set(ws)
        t_set = time.perf_counter() - t0
        wall_b, k_b = time_launches(lambda: bt.run(torch.cuda.current_stream()), 3, 1)
        out["batch"] = {"workload": "512 uneven instances (d 2..64, K 1..4, N 1e3..1e5, orders 2/4)",
                        "precision": "fp32_3m", "slices": nsl, "packets": bt.n_packets, "ms_per_run": wall_b,
                        "steps_per_s": nsl / (wall_b * 1e-3), "set_s": t_set}
        bt.close()

    Uo = None
    if not args.skip_cpu:
        import oracle.propagator as orc
        t0 = time.perf_counter()
        Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, w.order)
        dt_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": N / dt_cpu, "unit": "steps/s", "cores": blas_threads(), "kind": "oracle",
                               "sample": f"the whole workload ({N} slices, one run, {dt_cpu:.1f} s)"}
        out["error_vs_oracle"] = {name: orc.relative_frobenius(Ug[name], Uo) for name, _ in modes}
        _, go = orc.control_gradient(wg.H0, wg.Hk, wg.samples, wg.h, 2,
                                     orc.fidelity_grad_U(orc.propagate(wg.H0, wg.Hk, wg.samples, wg.h, 2), wg.target))
        out["grad"]["rel_err_vs_oracle"] = float(np.max(np.abs(grad_h - go)) / np.max(np.abs(go)))

    if not args.skip_fixed_error and Uo is not None:
        import oracle.propagator as orc
        # same T, coarser slicing: smallest N=2^n meeting each target error
        T = N * w.h
        res = {"reference": "oracle at the workload's own N (2^17 slices)"}
        summ = {}
        for name, _ in modes:
            errs = {}
            for n in range(8, 18):
                nn = 2 ** n
                wn = synth.random_qudit(n_slices=nn, h=T / nn)
                sd = torch.from_numpy(wn.samples).to(dev)
                Ud = torch.zeros((d, d), dtype=torch.complex128, device=dev)
                wall, _ = time_launches(lambda: ctxs[name].equiprop_dev(sd, wn.h, Ud), 5, 2)
                errs[nn] = (orc.relative_frobenius(Ud.cpu().numpy(), Uo), wall)
            res[name] = {str(k): {"err": v[0], "ms": v[1]} for k, v in errs.items()}
            for eps in (1e-4, 1e-6):
                ok = [k for k, v in errs.items() if v[0] <= eps]
                summ[f"{name}_eps_{eps:.0e}"] = ({"n_slices": min(ok), "ms": errs[min(ok)][1],
                                                  "steps_per_s": min(ok) / (errs[min(ok)][1] * 1e-3)}
                                                 if ok else None)
        res["summary"] = summ
        out["fixed_error"] = res

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
