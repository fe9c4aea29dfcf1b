"""Write the oracle's U(T) for the full-size workloads to full_size_oracle.npz.

The full-size parity tests compare the library with these values; the
oracle needs minutes for them (the d = 64 precision sweep alone takes about
100 s), far too long to recompute inside a GPU test run.  Every value here
is computed by the oracle (``oracle.propagator.propagate``: eigendecomposition
per slice and the sequential product) on the seeded inputs of ``synth``;
nothing comes from the library.

Contents:
  random_qudit      U(T) of the d = 16 random qudit at N = 2^17 (order 4)
  random_qudit_m6   U(T) of the same system with the sixth-order scheme at
                    N = 2^17 (its three Gauss-Legendre samples per slice; the
                    reference of the sixth- against fourth-order comparison)
  precision_sweep   U(T) of the d = 64 precision sweep at N = 2^16 (order 2)
  precision_sweep_fine
                    U(T) of the same system over the same span at N = 2^19
                    (the reference of the fixed-error comparison at d = 64)
  batch_index       instance indices of the 512-instance batch that are kept:
                    every instance of dimension <= 16, the two longest of
                    dimension 32 and of dimension 64 with order 2, and the
                    longest of each with order 4
  batch_offset      start of each kept instance's U(T) in batch_U (complex
                    entries), one more entry for the end
  batch_U           the kept instances' U(T), concatenated row-major

Run:  python tests/golden/make_full_size.py   (about 6 minutes on 8 cores)

The fine reference takes the oracle's steps in the oracle's order -- the
slice propagators of each 8192-slice block by eigendecomposition
(``slice_propagators``, computed for several blocks at once in worker
processes), multiplied in sequence into U (``ordered_product``), exactly
the blocks and products of ``propagate``.
"""
from __future__ import annotations

import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle.propagator as orc  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "full_size_oracle.npz")


def batch_selection(insts) -> list[int]:
    """Indices of the batch instances whose U(T) is stored."""
    keep = [i for i, w in enumerate(insts) if w.dim <= 16]
    for d in (32, 64):
        for order, count in ((2, 2), (4, 1)):
            cand = sorted((w.n_slices, i) for i, w in enumerate(insts) if w.dim == d and w.order == order)
            keep += [i for _, i in cand[-count:]]
    return sorted(keep)


_INSTS = None


def _job(key):
    global _INSTS
    t0 = time.time()
    if key == "random_qudit":
        w = synth.random_qudit()
    elif key == "random_qudit_m6":
        w = synth.random_qudit(order=orc.M6)
    elif key == "precision_sweep":
        w = synth.precision_sweep()
    else:
        if _INSTS is None:
            _INSTS = synth.batched_instances(512)
        w = _INSTS[int(key)]
    U = orc.propagate(w.H0, w.Hk, w.samples, w.h, w.order)
    return key, U, time.time() - t0


FINE_N = 2 ** 19
BLOCK = 8192


def _fine_block(rng):
    s, e = rng
    w = synth.precision_sweep(n_slices=FINE_N, h=2 ** 16 * 0.01 / FINE_N)
    return orc.slice_propagators(w.H0, w.Hk, w.samples, w.h, w.order, s, e)


def fine_reference(ex) -> np.ndarray:
    """U(T) of the d = 64 sweep at 2^18 slices: blocks of slice propagators
    from the pool (at most eight in flight), multiplied in order."""
    U = np.eye(64, dtype=np.complex128)
    starts = list(range(0, FINE_N, BLOCK))
    futs, nxt = {}, 0
    for i in range(len(starts)):
        while nxt < len(starts) and nxt < i + 8:
            futs[nxt] = ex.submit(_fine_block, (starts[nxt], min(FINE_N, starts[nxt] + BLOCK)))
            nxt += 1
        U = orc.ordered_product(futs.pop(i).result(), U)
    return U


def main() -> None:
    insts = synth.batched_instances(512)
    sel = batch_selection(insts)
    # longest jobs first so the pool drains evenly
    jobs = ["precision_sweep", "random_qudit", "random_qudit_m6"] + [str(i) for i in sel]
    jobs.sort(key=lambda k: -(2 ** 16 * 64 ** 3 if k == "precision_sweep" else
                              2 ** 17 * 16 ** 3 if k.startswith("random_qudit") else
                              insts[int(k)].n_slices * insts[int(k)].dim ** 3))
    res = {}
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        for key, U, dt in ex.map(_job, jobs):
            res[key] = U
            if dt > 5:
                print(f"{key}: {dt:.1f} s", flush=True)
        t0 = time.time()
        res["precision_sweep_fine"] = fine_reference(ex)
        print(f"precision_sweep_fine: {time.time() - t0:.1f} s", flush=True)
    offs = [0]
    flat = []
    for i in sel:
        flat.append(res[str(i)].reshape(-1))
        offs.append(offs[-1] + flat[-1].size)
    np.savez_compressed(OUT, random_qudit=res["random_qudit"], random_qudit_m6=res["random_qudit_m6"],
                        precision_sweep=res["precision_sweep"],
                        precision_sweep_fine=res["precision_sweep_fine"],
                        batch_index=np.array(sel, np.int64), batch_offset=np.array(offs, np.int64),
                        batch_U=np.concatenate(flat))
    print(f"wrote {OUT}: {len(sel)} batch instances", flush=True)


if __name__ == "__main__":
    main()
