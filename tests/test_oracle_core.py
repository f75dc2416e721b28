"""Pins of the CPU oracle against published values, closed forms and brute force.

None of these tests use the GPU library: they establish that the oracle itself
is right before anything is compared with it.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import brute, gates as G, philox, sim
from oracle.qasm import QasmSyntaxError, parse

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Philox
# ---------------------------------------------------------------------------
def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(x, 16) for x in line.split()]
                rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_philox_known_answers(ctr, key, out):
    assert philox.philox4x64(ctr, key) == out


@pytest.mark.parametrize("seed,shot", [(0, 0), (1, 7), (2 ** 63 + 5, 12345), (42, 2 ** 40)])
def test_philox_stream_matches_numpy(seed, shot):
    ref = np.random.Philox(key=np.array([seed, shot], dtype=np.uint64)).random_raw(23)
    s = philox.ShotStream(seed, shot)
    got = [s.next_word() for _ in range(23)]
    assert got == [int(x) for x in ref]
    assert [philox.event_word(seed, shot, e) for e in range(23)] == got


def test_uniform_mapping():
    assert philox.word_to_uniform(0) == 0.0
    assert philox.word_to_uniform(2 ** 64 - 1) == 1.0 - 2.0 ** -53
    assert philox.word_to_uniform(1 << 63) == 0.5


# ---------------------------------------------------------------------------
# Gate matrices
# ---------------------------------------------------------------------------
ANGLES = [0.0, 0.3, 1.1, math.pi / 2, math.pi, 2.5, 4.0, -1.7]


def test_gates_unitary():
    rng = np.random.default_rng(0)
    for name in list(G.ONE_QUBIT) + list(G.TWO_QUBIT):
        npar = (G.ONE_QUBIT.get(name) or G.TWO_QUBIT.get(name))[0]
        for _ in range(3):
            m, _ = G.gate_matrix(name, list(rng.uniform(-7, 7, npar)))
            assert np.allclose(m.conj().T @ m, np.eye(m.shape[0]), atol=1e-15), name


def test_gate_identities():
    pi = math.pi
    assert np.allclose(G.u_gate(pi, 0, pi), G.X, atol=1e-15)
    assert np.allclose(G.u_gate(pi / 2, 0, pi), G.H, atol=1e-15)
    assert np.allclose(G.rx(pi), -1j * G.X, atol=1e-15)
    assert np.allclose(G.ry(pi), -1j * G.Y, atol=1e-15)
    assert np.allclose(G.H @ G.Z @ G.H, G.X, atol=1e-15)
    assert np.allclose(G.S @ G.S, G.Z) and np.allclose(G.T @ G.T, G.S)
    assert np.allclose(G.SX @ G.SX, G.X, atol=1e-15)
    cx = G.controlled(G.X)
    assert np.allclose(cx @ cx, np.eye(4))
    for t in ANGLES:
        assert np.allclose(G.rz(t), np.exp(-0.5j * t) * G.phase(t), atol=1e-15)
        assert np.allclose(G.rx(t), G.u_gate(t, -pi / 2, pi / 2), atol=1e-15)
        assert np.allclose(G.ry(t), G.u_gate(t, 0, 0), atol=1e-15)
        # rotation gates are exponentials of Pauli generators
        for r, p in ((G.rx, G.X), (G.ry, G.Y), (G.rz, G.Z)):
            assert np.allclose(r(t), math.cos(t / 2) * np.eye(2) - 1j * math.sin(t / 2) * p, atol=1e-15)
    # U = RZ(phi) RY(theta) RZ(lambda) up to the global phase e^{i(phi+lambda)/2}
    th, ph, la = 0.7, 1.9, -2.3
    assert np.allclose(G.u_gate(th, ph, la), np.exp(0.5j * (ph + la)) * G.rz(ph) @ G.ry(th) @ G.rz(la))


def test_gate_derivatives_match_finite_differences():
    h = 1e-6
    for name, npar in [("rx", 1), ("ry", 1), ("rz", 1), ("p", 1), ("U", 3), ("u2", 2), ("cp", 1),
                       ("crx", 1), ("cry", 1), ("crz", 1)]:
        for base in ([0.4, -1.3, 2.2], [3.0, 0.1, -0.5]):
            a = base[:npar]
            for k in range(npar):
                ap, am = list(a), list(a)
                ap[k] += h
                am[k] -= h
                fd = (G.gate_matrix(name, ap)[0] - G.gate_matrix(name, am)[0]) / (2 * h)
                assert np.allclose(G.gate_derivative(name, a, k), fd, atol=1e-9), (name, k)


# ---------------------------------------------------------------------------
# Parser
# ---------------------------------------------------------------------------
def test_parser_constructs():
    ast = parse('OPENQASM 3.0; include "stdgates.inc"; input array[float[64], 3] th; '
                'qubit[3] q; bit[2] c; const float[64] k = pi/4; '
                'gate g(a) x, y { rx(a) x; cx x, y; } '
                'g(th[0] * 2 + k) q[0], q[1]; c[0] = measure q[0]; measure q[1] -> c[1]; '
                'if (c == 0b11) { x q[2]; } else h q[2]; '
                'for uint i in [0:2] { reset q[i]; if (c[1]) break; } barrier q;')
    kinds = [st[0] for st in ast]
    assert kinds == ["input", "qubit", "bit", "const", "gatedef", "gate", "measure", "measure",
                     "if", "for", "barrier"]
    assert ast[8][1] == ("cbin", "==", ("cref", ("ref", "c", None)), ("cnum", 3))
    with pytest.raises(QasmSyntaxError):
        parse("qubit[2] q; while (c == 0) { x q[0]; }")


def test_parameter_binding_and_custom_gates():
    src = W.hea2_program()
    for a, b in [(0.3, 1.2), (-2.0, 0.5)]:
        psi = sim.final_state(src, [a, b])
        ref = np.kron(G.ry(b), G.ry(a)) @ np.array([1, 0, 0, 0], dtype=complex)
        ref = G.controlled(G.X) @ ref
        assert np.allclose(psi, ref, atol=1e-15)
    src2 = ('OPENQASM 3.0; input float[64] t; qubit[2] q; gate my(a) x, y { ry(a) x; cx x, y; } '
            'my(2 * t - 0.5) q[0], q[1];')
    psi = sim.final_state(src2, [0.8])
    ref = G.controlled(G.X) @ np.kron(np.eye(2), G.ry(1.1)) @ np.array([1, 0, 0, 0], dtype=complex)
    assert np.allclose(psi, ref, atol=1e-15)


# ---------------------------------------------------------------------------
# Oracle vs dense brute force (independent state arithmetic)
# ---------------------------------------------------------------------------
def _both(src, seed, shot, forced=None):
    a = sim.Interpreter(sim.Program(src), engine_cls=sim.TensorEngine).run(seed, shot, forced)
    b = sim.Interpreter(sim.Program(src), engine_cls=brute.DenseEngine).run(seed, shot, forced)
    return a, b


@pytest.mark.parametrize("seed", range(12))
def test_oracle_matches_brute_force_random_dynamic(seed):
    n = 2 + seed % 5
    src = W.random_dynamic_program(seed, n, n_ops=30, final_measure=False)
    for shot in range(3):
        a, b = _both(src, 100 + seed, shot)
        assert a.record == b.record and a.cbits == b.cbits
        assert abs(a.record_prob - b.record_prob) < 1e-12
        assert np.max(np.abs(a.psi - b.psi)) < 1e-13
        assert abs(np.linalg.norm(a.psi) - 1.0) < 1e-12


def test_two_qubit_operand_order_brute_force():
    # explicit construction vs Kronecker products for adjacent operands
    for m in (G.controlled(G.X), G.controlled(G.ry(0.7)), G.SWAP):
        f = brute.full_operator(m, [0, 1], 3)
        assert np.allclose(f, np.kron(np.eye(2), m))
        # reversed operands: conjugate by SWAP
        f2 = brute.full_operator(m, [1, 0], 2)
        assert np.allclose(f2, G.SWAP @ m @ G.SWAP)
    # CX(control=2, target=0) on |100> (index 4) -> |101> (index 5)
    it = sim.run_shot('qubit[3] q; x q[2]; cx q[2], q[0];')
    assert abs(it.psi[5] - 1) < 1e-15


# ---------------------------------------------------------------------------
# Closed forms from the paper's validation suites
# ---------------------------------------------------------------------------
def test_bell_and_ghz():
    for n in (2, 3, 5):
        src = ("qubit[%d] q; bit[%d] c; h q[0];" % (n, n)
               + "".join(f"cx q[{i}], q[{i + 1}];" for i in range(n - 1)) + "c = measure q;")
        outs = set()
        for shot in range(64):
            it = sim.run_shot(src, seed=9, shot=shot)
            assert len(set(it.record)) == 1           # all outcomes equal the first
            assert abs(it.record_prob - 0.5) < 1e-15
            assert it.events[0][4] == pytest.approx(0.5, abs=1e-15)
            outs.add(it.record[0])
        assert outs == {0, 1}


@pytest.mark.parametrize("prep", ["plus", "minus"])
def test_conditional_reset_always_zero(prep):
    src = W.conditional_reset_program(prep)
    res = sim.run_shots(src, 10000, seed=7)
    assert all(r["cbits"][1] == 0 for r in res)       # f[0] is |0> in every shot
    first = [r["cbits"][0] for r in res]
    assert 4700 < sum(first) < 5300                   # the mid-circuit outcome is a fair coin


def test_teleportation_returns_to_zero():
    rng = np.random.default_rng(3)
    for _ in range(4):
        a, b, c = rng.uniform(0, 2 * math.pi, 3)
        src = W.teleport_program(a, b, c)
        for rec in range(4):
            it = sim.run_shot(src, forced=[rec & 1, rec >> 1])
            assert abs(it.record_prob - 0.25) < 1e-13
            psi = it.psi.reshape(2, 2, 2)               # axes q2, q1, q0
            assert np.sum(np.abs(psi[1]) ** 2) < 1e-26  # target qubit back in |0>


def test_if_else_branch_states():
    th = 1.234
    src = W.if_else_program(th)
    for m in (0, 1):
        it = sim.run_shot(src, forced=[m])
        assert abs(it.record_prob - 0.5) < 1e-15
        psi = it.psi.reshape(2, 2)   # [b1, b0]
        if m == 1:
            expect = np.array([math.cos(th / 2), -1j * math.sin(th / 2)])
        else:
            expect = np.array([np.exp(-0.5j * th), 0])
        assert np.allclose(psi[:, m], expect, atol=1e-15)
        assert np.allclose(psi[:, 1 - m], 0)


def test_multibit_predicate():
    for bits in range(16):
        it = sim.run_shot(W.multibit_predicate_program(bits))
        assert sum(b << i for i, b in enumerate(it.cbits)) == bits
        target = (it.psi.reshape(2, 16)[1] != 0).any()
        assert target == (bits == 0b1010)


def test_repeat_until_success_trip_counts():
    from scipy import stats
    phi, K, shots = 2.1, 8, 4000
    s = math.cos(phi / 2) ** 2
    res = sim.run_shots(W.rus_program(phi, K), shots, seed=11)
    trips = np.array([len(r["record"]) for r in res])
    expect = np.array([(1 - s) ** (k - 1) * s for k in range(1, K)] + [(1 - s) ** (K - 1)])
    obs = np.bincount(trips, minlength=K + 1)[1:]
    exp = expect * shots
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    assert stats.chisquare(o, e).pvalue > 0.01
    # a loop that ended by break has last outcome 0; one that ran out has all ones
    for r, t in zip(res, trips):
        assert r["record"][:-1] == [1] * (t - 1)
        assert r["record"][-1] == 0 or t == K


def test_qft_of_basis_states():
    n = 5
    for x in (0, 1, 6, 19, 31):
        psi = sim.final_state(W.qft_program(n, x))
        k = np.arange(1 << n)
        expect = np.exp(2j * math.pi * x * k / (1 << n)) / math.sqrt(1 << n)
        assert np.allclose(psi, expect, atol=1e-14)


def test_bernstein_vazirani():
    for n, secret in [(4, 0b1011), (7, 0b1100101), (3, 0)]:
        it = sim.run_shot(W.bv_program(secret, n), seed=5)
        assert sum(b << i for i, b in enumerate(it.cbits)) == secret
        assert abs(it.record_prob - 1.0) < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_random_clifford_equal_magnitudes(seed):
    n = 2 + seed * 3 % 9
    psi = sim.final_state(W.random_clifford_program(seed, n, 10 + 15 * seed))
    p = np.abs(psi) ** 2
    nz = p[p > 1e-12]
    r = math.log2(len(nz))
    assert r == int(r)
    assert np.allclose(nz, 2.0 ** -r, atol=1e-13)


def test_c1_forced_records_partition_unity():
    src = W.c1_program(1, final_measure=False)
    total = 0.0
    for rec in range(8):
        it = sim.run_shot(src, forced=[(rec >> i) & 1 for i in range(3)])
        assert it.status == sim.STATUS_OK
        assert it.cbits == [(rec >> i) & 1 for i in range(3)]
        assert abs(np.linalg.norm(it.psi) - 1) < 1e-12
        total += it.record_prob
    assert abs(total - 1.0) < 1e-13


def test_forced_zero_probability_aborts():
    it = sim.run_shot("qubit[1] q; bit c; c = measure q[0]; x q[0];", forced=[1])
    assert it.status == sim.STATUS_FORCED_ZERO_PROB
    assert it.record == []


def test_sampled_records_chi_square():
    from scipy import stats
    src = W.c1_program(1, final_measure=False)
    probs = np.array([sim.run_shot(src, forced=[(r >> i) & 1 for i in range(3)]).record_prob
                      for r in range(8)])
    shots = 1500
    res = sim.run_shots(src, shots, seed=21)
    obs = np.bincount([sum(b << i for i, b in enumerate(r["record"])) for r in res], minlength=8)
    exp = probs * shots
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    assert stats.chisquare(o, e).pvalue > 0.01


def test_reset_on_entangled_qubit_brute_force():
    src = "qubit[3] q; h q[0]; cx q[0], q[1]; ry(0.9) q[2]; cx q[2], q[0]; reset q[0];"
    for shot in range(8):
        a, b = _both(src, 3, shot)
        assert np.max(np.abs(a.psi - b.psi)) < 1e-14
        assert np.sum(np.abs(a.psi.reshape(-1, 2)[:, 1]) ** 2) < 1e-28   # q0 is |0>


# ---------------------------------------------------------------------------
# Expectation values and gradients
# ---------------------------------------------------------------------------
def test_expval_closed_forms():
    src = W.hea2_program()
    zz = np.array([[3, 3]], dtype=np.uint8)
    for a, b in [(0.1, 0.2), (1.3, -2.2), (3.0, 0.7)]:
        assert abs(sim.expval(src, [a, b], [1.0], zz) - math.cos(b)) < 1e-14
    src1 = "input float[64] t; qubit[1] q; ry(t) q[0];"
    for t in (0.3, 2.0, -1.0):
        assert abs(sim.expval(src1, [t], [1.0], [[3]]) - math.cos(t)) < 1e-15
        assert abs(sim.expval(src1, [t], [1.0], [[1]]) - math.sin(t)) < 1e-15
        assert abs(sim.expval(src1, [t], [1.0], [[2]])) < 1e-15


def test_gradient_closed_form_and_routes_agree():
    src = W.hea2_program()
    zz = np.array([[3, 3]], dtype=np.uint8)
    a, b = 0.4, 1.1
    e, g_adj = sim.grad_adjoint(src, [a, b], [1.0], zz)
    g_ps = sim.grad_param_shift(src, [a, b], [1.0], zz)
    assert abs(e - math.cos(b)) < 1e-14
    assert np.allclose(g_adj, [0.0, -math.sin(b)], atol=1e-14)
    assert np.allclose(g_ps, g_adj, atol=1e-13)


def test_gradient_small_ansatz_three_routes():
    n, layers = 4, 2
    src = W.c4_ansatz(n, layers)
    coeffs, codes = W.c4_hamiltonian(seed=8, n=n, terms=6)
    theta = W.c4_thetas(seed=9, batch=1, n_params=2 * n * layers)[0]
    e, g_adj = sim.grad_adjoint(src, theta, coeffs, codes)
    g_ps = sim.grad_param_shift(src, theta, coeffs, codes)
    assert abs(e - sim.expval(src, theta, coeffs, codes)) < 1e-13
    assert np.max(np.abs(g_adj - g_ps)) < 1e-12
    h = 1e-5
    fd = np.array([(sim.expval(src, theta + h * np.eye(len(theta))[k], coeffs, codes)
                    - sim.expval(src, theta - h * np.eye(len(theta))[k], coeffs, codes)) / (2 * h)
                   for k in range(len(theta))])
    assert np.max(np.abs(fd - g_adj)) < 1e-7


def test_expval_rejects_dynamic_programs():
    with pytest.raises(sim.OracleError):
        sim.expval(W.if_else_program(0.3), [], [1.0], [[3, 0]])
