"""Batched uneven instances in one persistent, graph-captured launch."""
import math
import sys

import numpy as np
import pytest

import oracle.propagator as orc
import synth
from bounds import max_squarings, tol

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07126_amd as m
    return m


def mixed_instances():
    spec = [(2, 1, 1, 2), (3, 2, 50, 4), (4, 1, 333, 2), (5, 3, 17, 4), (8, 4, 1000, 2), (12, 2, 64, 4),
            (16, 3, 1500, 4), (16, 1, 16, 2), (17, 2, 200, 2), (24, 1, 99, 4), (32, 2, 400, 2), (40, 3, 61, 4),
            (64, 1, 150, 2), (64, 2, 33, 4), (2, 2, 2000, 4), (8, 0, 10, 2)]
    out = []
    for i, (d, K, n, order) in enumerate(spec):
        out.append(synth.random_system(d, K, n_slices=n, h=0.04, order=order, tag=200 + i))
    return out


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_batch_matches_oracle(pm, prec):
    ws = mixed_instances()
    say(f"[case] batch of {len(ws)} mixed instances prec={prec}")
    with pm.Batch(0, prec) as b:
        b.set(ws)
        b.run()
        Us = b.results()
    worst = 0.0
    for w, U in zip(ws, Us):
        Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, w.order)
        e = orc.relative_frobenius(U, Uo)
        # packets share one plan per step: at most the instance's largest s
        s = 0 if prec == 0 else max_squarings(pm, w, prec)
        worst = max(worst, e / tol(prec, w.n_slices, w.dim, s))
        assert e <= tol(prec, w.n_slices, w.dim, s), (w.name, w.n_slices, e)
    say(f"  worst error / bound {worst:.3f}")


def test_batch_equals_standalone_fp64(pm):
    ws = mixed_instances()[:8]
    with pm.Batch(0, 0) as b:
        b.set(ws)
        b.run()
        Us = b.results()
    for w, U in zip(ws, Us):
        with pm.Context(0, 0) as c:
            c.set_hamiltonian(w.H0, w.Hk, w.order)
            assert orc.relative_frobenius(U, c.equiprop(w.samples, w.h)) <= 1e-12


def test_batch_graph_replays(pm):
    """The captured graph replayed several times with eager work between the
    replays; every replay matches the first bit for bit."""
    import torch
    ws = mixed_instances()
    with pm.Batch(0, 2) as b:
        b.set(ws)
        b.run()
        ref = b.results()
        x = torch.randn(512, 512, device="cuda")
        for r in range(4):
            y = (x @ x).sum()
            torch.cuda.synchronize()
            b.run()
            got = b.results()
            for a, c in zip(ref, got):
                assert np.array_equal(a, c), r
            assert torch.isfinite(y)


def test_batch_chunk_tuning_invariance(pm):
    ws = mixed_instances()
    res = []
    for ch in ((16, 8), (32, 4), (64, 4)), ((16, 200), (32, 100), (64, 50)):
        with pm.Batch(0, 0) as b:
            for dc, c in ch:
                b.set_chunk(dc, c)
            b.set(ws)
            b.run()
            res.append(b.results())
    for a, c in zip(*res):
        assert orc.relative_frobenius(a, c) <= 1e-12


def test_batch_workload_reduced(pm):
    """The 512-instance workload's first 96 instances with N capped at 3000."""
    ws = synth.batched_instances(n_inst=96, max_slices=3000)
    with pm.Batch(0, pm.PM_FP32_3M) as b:
        b.set(ws)
        b.run()
        Us = b.results()
        say(f"  packets {b.n_packets}")
    worst = 0.0
    for w, U in zip(ws, Us):
        Uo = orc.propagate(w.H0, w.Hk, w.samples, w.h, w.order)
        e = orc.relative_frobenius(U, Uo)
        worst = max(worst, e)
        assert e <= tol(2, w.n_slices, w.dim, max_squarings(pm, w, 2)), (w.name, e)
    say(f"  worst rel err {worst:.3e}")


def test_batch_errors(pm):
    w = synth.random_system(4, 1, n_slices=4, h=0.1, order=2, tag=1)
    with pm.Batch(0, 0) as b:
        with pytest.raises(pm.ParamentError):
            b.run()
        bad = synth.random_system(4, 1, n_slices=4, h=0.1, order=4, tag=1)
        bad.samples = bad.samples[:, :4]
        with pytest.raises(pm.ParamentError):
            b.set([w, bad])
        b.set([w])
        b.run()
        assert orc.relative_frobenius(b.results()[0], orc.propagate(w.H0, w.Hk, w.samples, w.h, 2)) <= 1e-10
