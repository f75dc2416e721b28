"""GPU parity of the persistent batch path (qsv_run_batch) against the oracle.

Mixed widths (resident states up to 12 qubits, HBM-slot states of 13..20
qubits, a wider request that falls back to qsv_run_shots), uneven trajectory
lengths, forced records, the shared deterministic prefix of 13..20-qubit
requests with several shots, the tile-pass route of 13..20-qubit requests with
at least 64 shots, and the independence of a request's results from the rest
of its batch.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import sim

pytestmark = pytest.mark.gpu
PROB_TOL = 1e-12
TIE = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_11599_amd import Context
    c = Context(0)
    yield c
    c.close()


def _check(src, res, n_shots, seed, shot_offset=0, forced=None):
    bits = res.bits()
    skipped = 0
    for s in range(n_shots):
        f = None if forced is None else list(forced[s])
        o = sim.run_shot(src, seed=seed, shot=shot_offset + s, forced=f)
        if forced is None and any(abs(e[3] - e[4]) < TIE for e in o.events):
            skipped += 1
            continue
        assert res.shot_status[s] == o.status
        assert list(bits[s]) == o.cbits, f"shot {s}"
        assert list(res.record[s, :len(o.record)]) == o.record
        assert res.n_events[s] == len(o.events)
        assert abs(res.record_prob[s] - o.record_prob) < PROB_TOL
    assert skipped <= max(1, n_shots // 10)


def test_batch_mixed_widths_match_oracle(ctx):
    srcs = [W.random_dynamic_program(500 + n, n, n_ops=50, final_measure=(n % 2 == 0))
            for n in (1, 2, 3, 5, 8, 11, 12, 13, 14, 16, 18)]
    srcs += [W.c1_program(7), W.c3_program(8, n=14, layers=3), W.conditional_reset_program("plus"),
             W.rus_program(1.7, 6)]
    progs = [ctx.load(s) for s in srcs]
    reqs = [{"prog": p, "shots": 6 + 3 * (i % 3), "seed": 100 + i, "shot_offset": 7 * i}
            for i, p in enumerate(progs)]
    say("batch of", len(reqs), "requests")
    res = ctx.run_batch(reqs)
    for src, rq, r in zip(srcs, reqs, res):
        say("check", src.splitlines()[3], rq["shots"])
        _check(src, r, rq["shots"], rq["seed"], rq["shot_offset"])


def test_batch_forced_records(ctx):
    srcs = [W.random_dynamic_program(900 + n, n, n_ops=40, final_measure=True) for n in (6, 13, 15)]
    reqs, forced = [], []
    for i, src in enumerate(srcs):
        o = [sim.run_shot(src, seed=3, shot=s) for s in range(4)]
        width = max(1, max(len(x.record) for x in o))
        f = np.zeros((4, width), dtype=np.uint8)
        for s, x in enumerate(o):
            f[s, :len(x.record)] = x.record
        forced.append(f)
        reqs.append({"prog": ctx.load(src), "shots": 4, "seed": 3, "forced": f})
    res = ctx.run_batch(reqs)
    for src, f, r in zip(srcs, forced, res):
        _check(src, r, 4, 3, forced=f)


def test_batch_alone_equals_in_mix(ctx):
    a = ctx.load(W.c3_program(11, n=14, layers=4))
    others = [ctx.load(W.random_dynamic_program(40 + n, n, n_ops=60)) for n in (4, 9, 12, 15, 17)]
    alone = ctx.run_batch([{"prog": a, "shots": 32, "seed": 9}])[0]
    mix = ctx.run_batch([{"prog": p, "shots": 20, "seed": k} for k, p in enumerate(others)]
                        + [{"prog": a, "shots": 32, "seed": 9}])[-1]
    assert np.array_equal(alone.creg, mix.creg)
    assert np.array_equal(alone.record, mix.record)
    assert np.array_equal(alone.record_prob, mix.record_prob)
    assert np.array_equal(alone.n_events, mix.n_events)


def test_batch_wide_request_falls_back(ctx):
    src = ("OPENQASM 3.0; qubit[21] q; bit[3] c; h q[0]; cx q[0], q[20]; ry(0.7) q[13]; "
           "c[0] = measure q[20]; if (c[0]) x q[5]; c[1] = measure q[5]; c[2] = measure q[13];")
    small = W.random_dynamic_program(77, 5, n_ops=20)
    res = ctx.run_batch([{"prog": ctx.load(src), "shots": 5, "seed": 2},
                         {"prog": ctx.load(small), "shots": 5, "seed": 4}])
    _check(src, res[0], 5, 2)
    _check(small, res[1], 5, 4)


def test_batch_c3_with_mix_sampled(ctx):
    # the batching workload at reduced shot counts: every request checked against the oracle
    main = W.c3_program(3, n=16)
    mix = W.c3_mix(seed=33, count=4)
    reqs = [{"prog": ctx.load(main), "shots": 12, "seed": 1}]
    reqs += [{"prog": ctx.load(m), "shots": 3, "seed": 50 + k} for k, m in enumerate(mix)]
    res = ctx.run_batch(reqs)
    _check(main, res[0], 12, 1)
    for k, (m, r) in enumerate(zip(mix, res[1:])):
        _check(m, r, 3, 50 + k)


def test_batch_prefix_keeps_assigned_bits(ctx):
    """A streamed (13..20-qubit) request with 2..63 shots runs its deterministic
    prefix once; bits assigned in that prefix, before the first measurement,
    must reach every shot (one shot takes no prefix: both agree with the
    oracle)."""
    src = ("OPENQASM 3.0; qubit[14] q; bit[3] c; c = 2; h q[0]; ry(0.4) q[9]; cx q[0], q[13]; "
           "c[0] = measure q[0]; if (c == 2) x q[1]; if (c == 3) ry(0.3) q[2]; c[2] = measure q[1];")
    prog = ctx.load(src)
    for shots in (8, 1):
        res = ctx.run_batch([{"prog": prog, "shots": shots, "seed": 12}])[0]
        _check(src, res, shots, 12)
        bits = res.bits()
        assert np.all(bits[:, 1] == 1) and np.all(bits[:, 2] == 1 - bits[:, 0])
    lo = ctx.load(W.logic_program(5, 14, assign=True))
    res = ctx.run_batch([{"prog": lo, "shots": 10, "seed": 3}])[0]
    _check(W.logic_program(5, 14, assign=True), res, 10, 3)


def test_batch_many_shot_route_matches_oracle(ctx):
    """13..20-qubit requests with at least 64 shots leave the persistent launch
    and run on the tile passes with shared trajectories inside qsv_run_batch:
    every shot against the oracle, beside persistent requests of the batch."""
    main = W.c3_program(3, n=16)
    other = W.random_dynamic_program(321, 14, n_ops=50, final_measure=True)
    small = W.c1_program(7)
    reqs = [{"prog": ctx.load(main), "shots": 64, "seed": 5, "shot_offset": 100},
            {"prog": ctx.load(other), "shots": 96, "seed": 6},
            {"prog": ctx.load(small), "shots": 16, "seed": 7}]
    say("batch with two >= 64-shot streamed requests")
    res = ctx.run_batch(reqs)
    _check(main, res[0], 64, 5, 100)
    _check(other, res[1], 96, 6)
    _check(small, res[2], 16, 7)


def _same(a, b):
    assert np.array_equal(a.creg, b.creg)
    assert np.array_equal(a.record, b.record)
    assert np.array_equal(a.record_prob, b.record_prob)
    assert np.array_equal(a.n_events, b.n_events)
    assert np.array_equal(a.shot_status, b.shot_status)


def test_batch_overlapped_route_equals_separate_runs():
    """With persistent and tile-pass requests in one batch (an 18-qubit request
    takes the tile passes at any shot count), the tile-pass ones run on the
    context's batch forks, one host thread each, overlapping the persistent
    launch: repeated batches (the forks reused) give the results of the same
    requests run separately, the forks' launches are counted in the context's
    profile, and a forked context (which runs them after the launch on itself)
    gives the same results; the 18-qubit request agrees with the oracle."""
    from paper_2604_11599_amd import Context
    c = Context(0, profile=True)
    try:
        big1 = c.load(W.c3_program(3, n=16))
        big2 = c.load(W.random_dynamic_program(322, 15, n_ops=40, final_measure=True))
        wide_src = W.c3_program(77, n=18, layers=3)     # 18 qubits: the tile passes at any shot count
        wide = c.load(wide_src)
        smalls = [c.load(W.c3_program(20 + k, n=n, layers=3)) for k, n in enumerate((8, 12, 14, 17))]
        reqs = [{"prog": big1, "shots": 80, "seed": 3}, {"prog": big2, "shots": 64, "seed": 4, "shot_offset": 7},
                {"prog": wide, "shots": 6, "seed": 8}]
        reqs += [{"prog": p, "shots": 10, "seed": 30 + k} for k, p in enumerate(smalls)]
        sep_big = [big1.run_shots(80, seed=3, share=True), big2.run_shots(64, seed=4, shot_offset=7, share=True),
                   wide.run_shots(6, seed=8, share=True)]
        sep_small = c.run_batch(reqs[3:])
        for rep in range(3):
            say(f"overlapped batch, repetition {rep}")
            c.profile_reset()
            res = c.run_batch(reqs)
            prof = c.profile()
            for a, b in zip(res[:3], sep_big):
                _same(a, b)
            for a, b in zip(res[3:], sep_small):
                _same(a, b)
            assert prof["persistent_launches"] >= 1 and prof["pass_launches"] >= 1
        f = c.fork()
        say("same batch on a forked context")
        res_f = f.run_batch(reqs)
        for a, b in zip(res_f, res):
            _same(a, b)
        _check(W.random_dynamic_program(322, 15, n_ops=40, final_measure=True), res[1], 64, 4, 7)
        _check(wide_src, res[2], 6, 8)
    finally:
        c.close()


def test_batch_streamed_states_on_narrower_tiles(ctx):
    """Streamed (13..20-qubit) requests in the persistent launch whose plans
    use 11- and 10-bit tiles (fewer threads per tile than the workgroup has):
    every shot against the oracle, and equal to the default 12-bit plan."""
    src = W.random_dynamic_program(401, 15, n_ops=60, final_measure=True)
    base = ctx.run_batch([{"prog": ctx.load(src), "shots": 6, "seed": 9}])[0]
    _check(src, base, 6, 9)
    for tb in (11, 10):
        prog = ctx.load(src)
        prog.replan(tb, 4, 0.5)
        res = ctx.run_batch([{"prog": prog, "shots": 6, "seed": 9}])[0]
        _check(src, res, 6, 9)
