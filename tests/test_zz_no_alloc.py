"""qsv_run_shots_noalloc against qsv_run_shots.

The no-allocation entry point carves every device buffer it needs from the
library's fixed per-device scratch array instead of allocating; its results
must be bit-identical to qsv_run_shots on the same inputs (same kernels, same
Philox streams). Calls come in a row, each later one with a smaller input, so
every call after the first runs on the array as the previous call left it.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert np.array_equal(a.creg, b.creg)
    assert np.array_equal(a.record, b.record)
    assert np.array_equal(a.n_events, b.n_events)
    assert np.array_equal(a.record_prob, b.record_prob)
    assert np.array_equal(a.shot_status, b.shot_status)


def test_noalloc_matches_run_shots():
    from paper_2604_11599_amd import Context, QsvError
    from paper_2604_11599_amd import _abi as A
    ctx = Context(0)
    try:
        # 16 qubits, 1 MiB per shot: 600 shots run in about ten batches of the array
        rus = ctx.load(W.c3_program(seed=3, n=16))
        _same(rus.run_shots(600, seed=5, noalloc=True), rus.run_shots(600, seed=5))
        # smaller input next, with the state of shot 0
        c1 = ctx.load(W.c1_program(seed=1))
        a = c1.run_shots(100, seed=6, state_out=True, noalloc=True)
        b = c1.run_shots(100, seed=6, state_out=True)
        _same(a, b)
        assert np.array_equal(a.state, b.state)
        # shared trajectories, forced records and a complex64 state through the array
        f = np.array([[1, 0, 1]] * 40, dtype=np.uint8)
        _same(c1.run_shots(40, seed=7, forced=f, share=True, noalloc=True),
              c1.run_shots(40, seed=7, forced=f, share=True))
        _same(rus.run_shots(30, seed=8, complex64=True, noalloc=True),
              rus.run_shots(30, seed=8, complex64=True))
        # a 20-qubit shot (16 MiB): three shots per batch
        wide = ctx.load(W.random_dynamic_program(2020, 20, n_ops=40, final_measure=True))
        _same(wide.run_shots(7, seed=9, noalloc=True), wide.run_shots(7, seed=9))
        # a 23-qubit shot (128 MiB) does not fit: a clear error, nothing run
        big = ctx.load("OPENQASM 3.0;\nqubit[23] q;\nbit b;\nh q[0];\nb = measure q[0];\n")
        with pytest.raises(QsvError) as err:
            big.run_shots(1, noalloc=True)
        assert err.value.status == A.QSV_ERR_LIMIT
        # the context still works afterwards on both entry points
        _same(c1.run_shots(5, seed=10, noalloc=True), c1.run_shots(5, seed=10))
    finally:
        ctx.close()
