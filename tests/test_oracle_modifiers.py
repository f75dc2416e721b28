"""Pins of the oracle's gate modifiers (inv @, pow(k) @, ctrl @, negctrl @),
against facts that do not go through the modifier code: unitarity (a gate
followed by its inverse restores any state), the named controlled gates,
closed forms of integer powers, basis-state truth tables and finite
differences of the oracle's own energies."""
import itertools
import math

import numpy as np
import pytest

from oracle import sim

H = 'OPENQASM 3.0;\ninclude "stdgates.inc";\n'
PREP = "h q[0];\nry(0.37) q[1];\ncx q[1], q[2];\nrz(1.1) q[2];\nU(0.4, 1.3, -0.6) q[0];\n"


def state(body, n=3):
    return sim.final_state(H + f"qubit[{n}] q;\n" + body)


ONE = ["id", "x", "y", "z", "h", "s", "sdg", "t", "tdg", "sx", "sxdg", "rx(0.8)", "ry(-1.2)", "rz(2.1)",
       "p(0.55)", "U(0.3, -0.9, 1.7)", "u2(0.2, -1.4)"]
TWO = ["cx", "cy", "cz", "ch", "swap", "cp(0.9)", "crx(-0.4)", "cry(1.3)", "crz(0.6)"]


@pytest.mark.parametrize("g", ONE + TWO)
def test_gate_then_inverse_restores_the_state(g):
    ops = "q[1]" if g in ONE else "q[2], q[0]"
    psi0 = state(PREP)
    psi = state(PREP + f"{g} {ops};\ninv @ {g} {ops};\n")
    assert np.max(np.abs(psi - psi0)) < 1e-13
    # pow(-1) is the inverse too
    psi = state(PREP + f"{g} {ops};\npow(-1) @ {g} {ops};\n")
    assert np.max(np.abs(psi - psi0)) < 1e-13


@pytest.mark.parametrize("one,two", [("x", "cx"), ("y", "cy"), ("z", "cz"), ("h", "ch"), ("rx(0.7)", "crx(0.7)"),
                                     ("ry(-0.3)", "cry(-0.3)"), ("rz(1.9)", "crz(1.9)"), ("p(2.2)", "cp(2.2)")])
def test_ctrl_matches_the_named_controlled_gate(one, two):
    a = state(PREP + f"ctrl @ {one} q[2], q[1];\n")
    b = state(PREP + f"{two} q[2], q[1];\n")
    assert np.max(np.abs(a - b)) < 1e-14


def test_negctrl_is_x_conjugated_ctrl():
    a = state(PREP + "negctrl @ ry(0.9) q[0], q[2];\n")
    b = state(PREP + "x q[0];\ncry(0.9) q[0], q[2];\nx q[0];\n")
    assert np.max(np.abs(a - b)) < 1e-14


def test_integer_powers_closed_forms():
    for pw, g, ref in [("pow(2)", "s", "z"), ("pow(2)", "sx", "x"), ("pow(-1)", "t", "tdg"), ("pow(4)", "t", "z"),
                       ("pow(3)", "rx(0.2)", "rx(0.6000000000000001)"), ("pow(0)", "h", "id")]:
        a = state(PREP + f"{pw} @ {g} q[1];\n")
        b = state(PREP + f"{ref} q[1];\n")
        assert np.max(np.abs(a - b)) < 1e-14, (pw, g)


def test_toffoli_truth_table():
    for bits in itertools.product((0, 1), repeat=3):
        prep = "".join(f"x q[{i}];\n" for i, b in enumerate(bits) if b)
        psi = state(prep + "ctrl @ ctrl @ x q[0], q[1], q[2];\n")
        out = list(bits)
        if bits[0] and bits[1]:
            out[2] ^= 1
        idx = sum(b << i for i, b in enumerate(out))
        assert abs(abs(psi[idx]) - 1.0) < 1e-15


def test_modifiers_on_gate_definitions():
    gdef = "gate two(a) u, v { h u; crz(a) u, v; ry(a / 2) v; }\n"
    psi0 = state(gdef + PREP)
    psi = state(gdef + PREP + "two(0.8) q[0], q[2];\ninv @ two(0.8) q[0], q[2];\n")
    assert np.max(np.abs(psi - psi0)) < 1e-13
    gdef1 = "gate rot(a) u { rx(a) u; rz(2 * a) u; }\n"
    a = state(gdef1 + PREP + "ctrl @ rot(0.5) q[1], q[0];\n")
    b = state(gdef1 + PREP + "crx(0.5) q[1], q[0];\ncrz(1.0) q[1], q[0];\n")
    assert np.max(np.abs(a - b)) < 1e-14


def test_gradient_through_modifiers_matches_finite_differences():
    src = (H + "input array[float[64], 3] t;\nqubit[2] q;\nh q[0];\ninv @ rx(t[0]) q[1];\n"
           "ctrl @ U(t[1], 0.3, t[2]) q[0], q[1];\nnegctrl @ ry(2 * t[0]) q[1], q[0];\npow(2) @ rz(t[2]) q[1];\n")
    coeffs = [0.7, -1.3, 0.4]
    codes = np.array([[3, 3], [1, 0], [2, 1]], dtype=np.uint8)
    th = np.array([0.4, -1.1, 0.8])
    e, g = sim.grad_adjoint(src, th, coeffs, codes)
    h = 1e-6
    for k in range(3):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (sim.expval(src, tp, coeffs, codes) - sim.expval(src, tm, coeffs, codes)) / (2 * h)
        assert abs(fd - g[k]) < 1e-8
    assert abs(e - sim.expval(src, th, coeffs, codes)) < 1e-14
