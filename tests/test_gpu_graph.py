"""Captured launch sequences (QSV_RUN_GRAPH) against the uncaptured calls.

A graph is captured by the first call of a shape and replayed by later calls
with other seeds, shot offsets, parameters and forced outcomes; every replay
must give results bit-identical to the eager call with the same inputs, with
eager work (other programs, other shapes) run between the replays, and the
eager results themselves agree with the oracle elsewhere in the suite.
"""
import numpy as np
import pytest

import workloads as W
from oracle import sim

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_11599_amd import Context
    c = Context(0)
    yield c
    c.close()


def _same(a, b, state=False):
    assert np.array_equal(a.creg, b.creg)
    assert np.array_equal(a.record, b.record)
    assert np.array_equal(a.n_events, b.n_events)
    assert np.array_equal(a.record_prob, b.record_prob)
    assert np.array_equal(a.shot_status, b.shot_status)
    if state:
        assert np.array_equal(a.state, b.state)


def test_replays_equal_eager_calls(ctx):
    c1 = ctx.load(W.c1_program(seed=1))
    other = ctx.load(W.random_dynamic_program(31, 13, n_ops=50, final_measure=True))
    for k, seed in enumerate((5, 6, 7, 8)):
        g = c1.run_shots(1000, seed=seed, shot_offset=100 * k, graph=True)
        e = c1.run_shots(1000, seed=seed, shot_offset=100 * k)
        _same(g, e)
        # eager work of another program and shape between the replays
        _same(other.run_shots(9, seed=seed, graph=True), other.run_shots(9, seed=seed))
    # the replayed results are the oracle's for a few shots
    for s in range(3):
        o = sim.run_shot(W.c1_program(seed=1), seed=8, shot=300 + s)
        if any(abs(ev[3] - ev[4]) < 1e-12 for ev in o.events):
            continue
        assert list(g.bits()[s]) == o.cbits


def test_replays_with_state_forced_noise_and_dense_passes(ctx):
    # all-dense 12-bit passes on the matrix cores, the 4-qubit site and branches
    src = W.c2_program(seed=2, n=14, layers=10, final_measure=False)
    p = ctx.load(src)
    for seed in (1, 2, 3):
        _same(p.run_shots(8, seed=seed, state_out=True, graph=True), p.run_shots(8, seed=seed, state_out=True),
              state=True)
    f = np.array([[0, 1, 0, 1]] * 8, dtype=np.uint8)
    g = np.array([[1, 1, 0, 0]] * 8, dtype=np.uint8)
    _same(p.run_shots(8, seed=4, forced=f, graph=True), p.run_shots(8, seed=4, forced=f))
    _same(p.run_shots(8, seed=4, forced=g, graph=True), p.run_shots(8, seed=4, forced=g))
    # complex64 and readout/reset errors are part of the captured shape
    q = ctx.load(W.c1_program(seed=3))
    for seed in (9, 10):
        _same(q.run_shots(200, seed=seed, complex64=True, readout_error=0.05, reset_error=0.02, graph=True),
              q.run_shots(200, seed=seed, complex64=True, readout_error=0.05, reset_error=0.02))


def test_parameters_rebound_per_replay_and_sharing_ignores_the_flag(ctx):
    src = W.param_program(3, 12, 60, 8) + "bit[12] f;\nf = measure q;\n"
    p = ctx.load(src)
    rng = np.random.default_rng(2)
    for _ in range(3):
        th = rng.uniform(-3, 3, 8)
        _same(p.run_shots(64, theta=th, seed=3, graph=True), p.run_shots(64, theta=th, seed=3))
    c3 = ctx.load(W.c3_program(seed=3, n=14, layers=4))
    _same(c3.run_shots(64, seed=2, share=True, graph=True), c3.run_shots(64, seed=2))
