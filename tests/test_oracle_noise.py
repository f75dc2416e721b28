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


# ---------------------------------------------------------------------------
# Depolarizing noise as trajectories: after each application of a gate
# statement, each of its qubits takes X, Y or Z with probability p/3 each.
# ---------------------------------------------------------------------------
def _p1(src, p, shots, seed=11):
    return sum(sim.run_shot(src, seed=seed, shot=s, depolarizing=p).cbits[0] for s in range(shots)) / shots


def _close(got, want, shots):
    assert abs(got - want) < 4.5 * np.sqrt(want * (1 - want) / shots) + 1e-12, (got, want)


def test_depolarizing_flip_rates_closed_forms():
    """X and Y flip a computational-basis qubit, Z does not, so one noisy gate
    flips it with probability q = 2p/3 and two independent ones with 2 q (1 - q).
    Two statements, two iterations of one loop statement and the two qubits of
    a broadcast draw independently; a custom gate call draws once after its
    whole body (x x = identity inside)."""
    p, n = 0.3, 4000
    q = 2 * p / 3
    two = 2 * q * (1 - q)
    _close(_p1(H + "qubit[1] q;\nbit c;\nx q[0];\nx q[0];\nc = measure q[0];\n", p, n), two, n)
    _close(_p1(H + "qubit[1] q;\nbit c;\nfor int i in [0:1] { x q[0]; }\nc = measure q[0];\n", p, n), two, n)
    _close(_p1(H + "qubit[1] q;\nbit c;\nid q[0];\nc = measure q[0];\n", p, n), q, n)
    _close(_p1(H + "gate g a { x a; x a; }\nqubit[1] q;\nbit c;\ng q[0];\nc = measure q[0];\n", p, n), q, n)
    # broadcast: both qubits of `x q;` flip independently: parity of the two measured bits
    src = H + "qubit[2] q;\nbit[2] c;\nx q;\nc = measure q;\n"
    par = sum(sum(sim.run_shot(src, seed=5, shot=s, depolarizing=p).cbits) % 2 for s in range(n)) / n
    _close(par, two, n)


def _rho_exact(gates, p, nq):
    """Exact density matrix: each gate's unitary, then the depolarizing channel
    rho -> (1 - p) rho + p/3 (X rho X + Y rho Y + Z rho Z) on each of its qubits."""
    from oracle import gates as G
    dim = 1 << nq
    rho = np.zeros((dim, dim), complex)
    rho[0, 0] = 1.0

    def op(m, qs):
        full = np.zeros((dim, dim), complex)
        for col in range(dim):
            v = np.zeros(dim, complex)
            v[col] = 1.0
            e = sim.TensorEngine(nq)
            e.psi = v.copy()
            e.apply(m, qs)
            full[:, col] = e.psi
        return full

    paulis = [G.gate_matrix(k, [])[0] for k in ("x", "y", "z")]
    for name, angles, qs in gates:
        U = op(G.gate_matrix(name, angles)[0], qs)
        rho = U @ rho @ U.conj().T
        for q in qs:
            rho = (1 - p) * rho + sum(op(P, [q]) @ rho @ op(P, [q]).conj().T for P in paulis) * (p / 3)
    return rho


def test_depolarizing_trajectory_average_equals_the_channel():
    """The average of |psi><psi| over trajectories equals the exact channel on
    a 3-qubit circuit with one- and two-qubit gates, a loop and a broadcast
    (element-wise within 5 standard errors of a bounded average)."""
    p, n = 0.25, 6000
    src = (H + "qubit[3] q;\nh q[0];\ncx q[0], q[1];\nfor int i in [0:1] { rx(0.7) q[2]; cz q[1], q[2]; }\n"
           "ry(0.4) q;\ncp(0.9) q[2], q[0];\n")
    gates = [("h", [], [0]), ("cx", [], [0, 1])]
    gates += [("rx", [0.7], [2]), ("cz", [], [1, 2])] * 2
    gates += [("ry", [0.4], [k]) for k in range(3)] + [("cp", [0.9], [2, 0])]
    want = _rho_exact(gates, p, 3)
    acc = np.zeros((8, 8), complex)
    for s in range(n):
        psi = sim.run_shot(src, seed=21, shot=s, depolarizing=p).psi.reshape(-1)
        acc += np.outer(psi, psi.conj())
    got = acc / n
    assert np.max(np.abs(got - want)) < 5 / np.sqrt(n)
    # and the noiseless state is far from it (the test sees the noise)
    ideal = sim.final_state(src).reshape(-1)
    assert np.max(np.abs(np.outer(ideal, ideal.conj()) - want)) > 0.1


def test_depolarizing_draws_leave_the_event_stream_alone():
    """Noise words have their own counters: where noise cannot change the
    outcome probabilities (a Pauli keeps |+> at 1/2, 1/2), the outcome, the
    trajectory probability and the words drawn are those of the noiseless run."""
    src = H + "qubit[2] q;\nbit[2] c;\nh q[0];\nx q[1];\nc[0] = measure q[0];\nc[1] = measure q[1];\n"
    for s in range(200):
        a = sim.run_shot(src, seed=9, shot=s, depolarizing=0.5)
        b = sim.run_shot(src, seed=9, shot=s)
        assert a.cbits[0] == b.cbits[0] and a.words_drawn == b.words_drawn == 2
        assert a.record_prob == b.record_prob
        assert all(e[4] in (0, 1) for e in a.noise_events)
