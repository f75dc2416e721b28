"""A context whose per-call scratch comes from a caller's device buffer (the
arena of qsv_create): shot runs and mixed batches give the results of a
context that allocates its own scratch, bit for bit (an arena context runs a
batch's tile-pass requests itself, after the persistent launch, instead of on
a fork), and an arena too small for one shot is rejected with an error."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _same(a, b):
    assert np.array_equal(a.creg, b.creg)
    assert np.array_equal(a.record, b.record)
    assert np.array_equal(a.record_prob, b.record_prob)
    assert np.array_equal(a.n_events, b.n_events)
    assert np.array_equal(a.shot_status, b.shot_status)


def test_arena_context_equals_allocating_context():
    import torch
    from paper_2604_11599_amd import Context
    buf = torch.empty(768 << 20, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    ar = Context(0, arena=buf.data_ptr(), arena_bytes=buf.numel())
    ref = Context(0)
    try:
        srcs = [W.c3_program(3, n=15), W.c1_program(seed=4), W.c3_program(21, n=13, layers=3),
                W.random_dynamic_program(9, 11, n_ops=40, final_measure=True)]
        pa = [ar.load(s) for s in srcs]
        pr = [ref.load(s) for s in srcs]
        for k in range(2):
            say("arena shots, program", k)
            _same(pa[k].run_shots(70, seed=5 + k), pr[k].run_shots(70, seed=5 + k))
        shots = (64, 24, 12, 9)   # the first (15 qubits, 64 shots) takes the tile passes
        ra = ar.run_batch([{"prog": p, "shots": n, "seed": 40 + i} for i, (p, n) in enumerate(zip(pa, shots))])
        rr = ref.run_batch([{"prog": p, "shots": n, "seed": 40 + i} for i, (p, n) in enumerate(zip(pr, shots))])
        say("arena batch")
        for a, b in zip(ra, rr):
            _same(a, b)
    finally:
        ar.close()
        ref.close()
        del buf


def test_arena_too_small_for_one_shot_is_rejected():
    import torch
    from paper_2604_11599_amd import Context, QsvError
    buf = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    ar = Context(0, arena=buf.data_ptr(), arena_bytes=buf.numel())
    try:
        prog = ar.load(W.c3_program(3, n=18))   # one shot's state alone is 4 MiB
        with pytest.raises(QsvError, match="arena"):
            prog.run_shots(4, seed=1)
    finally:
        ar.close()
        del buf
