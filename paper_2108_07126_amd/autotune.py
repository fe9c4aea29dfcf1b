"""Autotuner: measures candidate chain lengths on the GPU and writes the
table ``tuning.txt`` that the binding applies at import.

For every engine class and precision the propagation kernel is timed on a
synthetic workload of that dimension for several target chain counts; for
the batched engine the chain length per dimension class is timed on a slice
of the 512-instance workload.  Run on the target GPU:

    python -m paper_2108_07126_amd.autotune [--quick]
"""
from __future__ import annotations

import argparse
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _time(fn, reps=8, warm=2):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_propagation(pm, synth, quick):
    import torch
    rows = []
    # sizes in the throughput regime of each class (the small dimensions are
    # cheap per slice, so they are tuned on long runs)
    classes = [(2, 2 ** 24), (4, 2 ** 22), (16, 2 ** 17), (32, 2 ** 15), (64, 2 ** 13)]
    targets = [512, 1024, 2048, 4096, 8192] if not quick else [1024, 2048, 4096]
    for D, N in classes:
        w = synth.random_system(D, 3, n_slices=N, h=1e-3, order=4, tag=D)
        s = torch.from_numpy(w.samples).cuda()
        U = torch.zeros((D, D), dtype=torch.complex128, device="cuda")
        precs = [0, 1] if D <= 4 else [0, 1, 2, 3]
        for prec in precs:
            ctx = pm.Context(0, prec)
            ctx.set_hamiltonian(w.H0, w.Hk, 4)
            best = None
            for t in targets:
                unit = 256 if D <= 4 else 1   # the engines' chunk units
                chunk = max(unit, unit * math.ceil(N / t / unit))
                ctx.set_chunk(chunk)
                ms = _time(lambda: ctx.equiprop_dev(s, w.h, U))
                print(f"propagate D={D} prec={prec} chains={t} chunk={chunk}: {ms:.3f} ms", flush=True)
                if best is None or ms < best[0]:
                    best = (ms, t)
            rows.append(("chains", D, prec, best[1]))
            ctx.close()
    return rows


def tune_batch(pm, synth, quick):
    import torch
    rows = []
    ws = synth.batched_instances(n_inst=96 if quick else 192, max_slices=20000)
    for prec in ([2] if quick else [0, 1, 2, 3]):
        best_cfg = {16: 64, 32: 32, 64: 16}
        for D in (64, 32, 16):
            best = None
            for ch in (8, 16, 32, 64, 128):
                b = pm.Batch(0, prec)
                for dc, c in best_cfg.items():
                    b.set_chunk(dc, c)
                b.set_chunk(D, ch)
                b.set(ws)
                ms = _time(lambda: b.run(torch.cuda.current_stream()), reps=3, warm=1)
                b.close()
                print(f"batch prec={prec} class={D} chunk={ch}: {ms:.2f} ms", flush=True)
                if best is None or ms < best[0]:
                    best = (ms, ch)
            best_cfg[D] = best[1]
        for D, ch in best_cfg.items():
            rows.append(("batch_chunk", D, prec, ch))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.txt"))
    args = ap.parse_args()
    import paper_2108_07126_amd as pm
    import synth
    rows = tune_propagation(pm, synth, args.quick) + tune_batch(pm, synth, args.quick)
    with open(args.out, "w") as f:
        f.write("# written by paper_2108_07126_amd.autotune on the target GPU\n")
        f.write("# key dim_class precision value\n")
        for key, dc, prec, val in rows:
            f.write(f"{key} {dc} {prec} {val}\n")
    print(f"wrote {args.out} ({len(rows)} entries)", flush=True)


if __name__ == "__main__":
    main()
