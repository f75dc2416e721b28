"""GPU parity of depolarizing noise as trajectories (programs loaded with
noise slots, run with qsv_run_opts.depolarizing), through the C ABI.

Each shot's Paulis come from counters of its own (statement, loop ordinals,
application, operand), so every shot equals the oracle's shot with the same
seed and index: records bit for bit (away from a draw within 1e-12 of its
threshold), the trajectory probability to 1e-12 and shot 0's amplitudes to
1e-10, on the gate-list path, on 12-bit all-dense passes (per-shot matrices
composed per shot, on the matrix cores) and in complex64 (within the
single-precision tie band). A rate of 0 reproduces the noiseless program.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import sim

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_11599_amd import Context
    c = Context(0)
    yield c
    c.close()


def _check(ctx, src, p, shots, seed, band=1e-12, amp_tol=1e-10, complex64=False):
    prog = ctx.load(src, noise=True)
    r = prog.run_shots(shots, seed=seed, depolarizing=p, state_out=True, complex64=complex64)
    bits = r.bits()
    checked = 0
    for s in range(shots):
        o = sim.run_shot(src, seed=seed, shot=s, depolarizing=p)
        if any(abs(e[3] - e[4]) < band for e in o.events):
            continue
        assert list(bits[s]) == o.cbits, (s, list(bits[s]), o.cbits)
        assert list(r.record[s][:len(o.record)]) == o.record
        tol = 4e-5 * o.record_prob if complex64 else 1e-12
        assert abs(r.record_prob[s] - o.record_prob) <= tol
        if s == 0:
            assert np.max(np.abs(r.state - o.psi.reshape(-1))) < amp_tol
        checked += 1
    assert checked >= shots // 2
    return r


@pytest.mark.parametrize("seed", range(6))
def test_noisy_random_dynamic_programs_match_oracle(ctx, seed):
    n = 3 + 2 * seed
    say("noisy random dynamic program", seed, n, "qubits")
    _check(ctx, W.random_dynamic_program(300 + seed, n, n_ops=50, final_measure=True), 0.1, 10, seed=seed)


def test_noisy_c1_and_dense_matrix_core_passes_match_oracle(ctx):
    """C1 (10 qubits, register phases) and the headline program at 14 qubits,
    whose passes are all dense on 12-bit tiles: the noise slots enter the
    composed 16x16 products, composed per shot."""
    _check(ctx, W.c1_program(seed=3), 0.02, 12, seed=4)
    from paper_2604_11599_amd import lower
    from paper_2604_11599_amd.api import plan_inspect
    src = W.c2_program(seed=2, n=14, layers=8)
    st = plan_inspect(lower(src, noise=True), 0)
    say("c2 14q noisy plan:", st.n_passes, "passes", st.n_dense_phases, "dense phases")
    assert st.n_dense_phases > 0
    _check(ctx, src, 0.01, 6, seed=5)


def test_low_rate_takes_clean_phases_and_matches_oracle(ctx):
    """At a low rate most (shot, dense phase) pairs draw no Pauli: those take
    the phase's matrix composed once from the set without Paulis, the others
    are composed for their shot. Shots with and without draws match the
    oracle (bits, record probabilities, shot 0's amplitudes)."""
    _check(ctx, W.c1_program(seed=9), 0.002, 40, seed=13)
    _check(ctx, W.c2_program(seed=2, n=14, layers=8), 0.002, 8, seed=14)


def test_noisy_complex64_matches_oracle_outside_the_tie_band(ctx):
    _check(ctx, W.c1_program(seed=6), 0.03, 16, seed=7, band=1e-4, amp_tol=2e-5, complex64=True)


def test_zero_rate_equals_the_noiseless_program(ctx):
    src = W.random_dynamic_program(77, 9, n_ops=60, final_measure=True)
    a = ctx.load(src, noise=True).run_shots(40, seed=3, depolarizing=0.0)
    b = ctx.load(src).run_shots(40, seed=3)
    assert np.array_equal(a.creg, b.creg) and np.array_equal(a.record, b.record)
    assert np.max(np.abs(a.record_prob - b.record_prob)) < 1e-15


def test_noisy_graph_replays_equal_eager_calls(ctx):
    prog = ctx.load(W.c1_program(seed=8), noise=True)
    for seed in (1, 2, 3):
        g = prog.run_shots(64, seed=seed, depolarizing=0.05, graph=True)
        e = prog.run_shots(64, seed=seed, depolarizing=0.05)
        assert np.array_equal(g.creg, e.creg) and np.array_equal(g.record_prob, e.record_prob)


def test_noisy_conditional_reset_rate(ctx):
    """The paper's conditional reset (|+>, measure, X if 1, measure) under
    depolarizing noise: only the Pauli after the conditional X can flip the
    final bit, so it is 1 with probability (1/2)(2p/3) = p/3."""
    src = ('OPENQASM 3.0;\ninclude "stdgates.inc";\nqubit[1] q;\nbit c;\nbit f;\n'
           'h q[0];\nc = measure q[0];\nif (c == 1) x q[0];\nf = measure q[0];\n')
    p, n = 0.03, 10000
    r = ctx.load(src, noise=True).run_shots(n, seed=11, depolarizing=p)
    ones = float(np.mean(r.bits()[:, 1]))
    assert abs(ones - p / 3) < 4.5 * np.sqrt(p / 3 * (1 - p / 3) / n)
    for s in range(20):
        assert list(r.bits()[s]) == sim.run_shot(src, seed=11, shot=s, depolarizing=p).cbits


def test_noise_rejections(ctx):
    from paper_2604_11599_amd import QsvError
    plain = ctx.load(W.c1_program(seed=1))
    with pytest.raises(QsvError):
        plain.run_shots(4, depolarizing=0.1)           # no noise slots
    noisy = ctx.load(W.c1_program(seed=1), noise=True)
    with pytest.raises(QsvError):
        noisy.run_shots(4, depolarizing=1.5)           # rate out of range
    with pytest.raises(QsvError):
        ctx.run_batch([{"prog": noisy, "shots": 4, "seed": 1}])
