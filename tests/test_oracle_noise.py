"""Pins of the oracle's readout and reset errors against the Philox words
(whose generator is pinned to the Random123 known-answer vectors) and against
closed forms: a readout error flips the recorded bit when the word after the
outcome's word is below the rate; a reset error flips the reset qubit the
same way. With both rates zero nothing changes."""
import numpy as np

import workloads as W
from oracle import philox, sim

H = 'OPENQASM 3.0;\ninclude "stdgates.inc";\n'


def _u(seed, shot, event):
    return philox.word_to_uniform(philox.event_word(seed, shot, event))


def test_readout_error_flips_the_recorded_bit_on_its_own_word():
    src = H + "qubit[1] q;\nbit c;\nc = measure q;\n"
    e, flips = 0.2, 0
    for shot in range(3000):
        it = sim.run_shot(src, seed=7, shot=shot, readout_error=e)
        flip = _u(7, shot, 1) < e
        assert it.cbits == [int(flip)] and it.record == [int(flip)]
        assert it.words_drawn == 2 and it.record_prob == 1.0
        flips += flip
    assert abs(flips / 3000 - e) < 4 * np.sqrt(e * (1 - e) / 3000)


def test_noisy_conditional_reset_closed_form():
    """The conditional reset of the paper's dynamic-circuit tests under readout
    noise: the final record is 1 exactly when one of the two readouts flipped,
    so it is 1 with probability 2 e (1 - e)."""
    src = H + "qubit[1] q;\nbit c;\nbit f;\nh q[0];\nc = measure q[0];\nif (c == 1) x q[0];\nf = measure q[0];\n"
    e, ones = 0.1, 0
    for shot in range(3000):
        it = sim.run_shot(src, seed=3, shot=shot, readout_error=e)
        expect = int(_u(3, shot, 1) < e) ^ int(_u(3, shot, 3) < e)
        assert it.cbits[1] == expect
        ones += expect
    p = 2 * e * (1 - e)
    assert abs(ones / 3000 - p) < 4 * np.sqrt(p * (1 - p) / 3000)


def test_reset_error_flips_the_qubit_on_its_own_word():
    src = H + "qubit[1] q;\nbit f;\nx q[0];\nreset q[0];\nf = measure q[0];\n"
    for shot in range(500):
        it = sim.run_shot(src, seed=11, shot=shot, reset_error=0.3)
        assert it.cbits == [int(_u(11, shot, 1) < 0.3)]
        assert it.words_drawn == 3


def test_zero_rates_change_nothing():
    src = W.c1_program(4)
    for shot in range(5):
        a = sim.run_shot(src, seed=2, shot=shot)
        b = sim.run_shot(src, seed=2, shot=shot, readout_error=0.0, reset_error=0.0)
        assert a.cbits == b.cbits and a.record == b.record and np.array_equal(a.psi, b.psi)
        assert a.words_drawn == len(a.events)
