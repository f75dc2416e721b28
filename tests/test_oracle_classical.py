"""Oracle pins for classical integer expressions and variables (OpenQASM 3
classical types in the symbol table, Methodology, parsing and semantic
analysis; feed-forward on computed values, Methodology, transpiling dynamic
control flow).

Register values are prepared in qubits and measured, so the oracle reads them
as it reads any measured bits; results are compared with numpy's own 64-bit
and 8-bit two's-complement integer arithmetic (np.int64, np.uint8), and with
Python booleans for conditions. Precedence is checked against explicitly
parenthesised Python expressions (C and Python disagree on & versus ==)."""
import itertools

import numpy as np
import pytest

from oracle import sim

HEAD = ('OPENQASM 3.0;\ninclude "stdgates.inc";\nqubit[7] q;\nbit[3] c;\nbit[3] d;\nbit t;\n'
        'int[16] x;\nuint[8] u;\nint[4] y;\n')
X0 = 7        # first bit of x in the flat classical array (c, d, t come first)
U0, Y0 = 23, 31


def _prep(a, b):
    lines = [f"x q[{i}];" for i in range(3) if (a >> i) & 1]
    lines += [f"x q[{3 + i}];" for i in range(3) if (b >> i) & 1]
    lines += [f"c[{i}] = measure q[{i}];" for i in range(3)]
    lines += [f"d[{i}] = measure q[{3 + i}];" for i in range(3)]
    return "\n".join(lines) + "\n"


def _bits(o, off, width):
    return sum(o.cbits[off + i] << i for i in range(width))


def _np_op(op, a, b):
    a, b = np.int64(a), np.int64(b)
    with np.errstate(all="ignore"):
        if op == "/":
            return 0 if b == 0 else int(np.fix(np.float64(a) / np.float64(b)))
        if op == "%":
            return 0 if b == 0 else int(np.fmod(a, b))
        return int({"+": a + b, "-": a - b, "*": a * b, "&": a & b, "|": a | b, "^": a ^ b,
                    "<<": a << b, ">>": a >> b}[op])


@pytest.mark.parametrize("op", ["+", "-", "*", "/", "%", "&", "|", "^", "<<", ">>"])
def test_binary_operators_against_numpy_int64(op):
    for a, b in itertools.product(range(8), repeat=2):
        o = sim.run_shot(HEAD + _prep(a, b) + f"x = c {op} d;\n", seed=1)
        want = _np_op(op, a, b) & 0xFFFF
        assert _bits(o, X0, 16) == want, (op, a, b)


@pytest.mark.parametrize("op", ["==", "!=", "<", ">", "<=", ">="])
def test_register_versus_register_comparisons(op):
    py = {"==": lambda a, b: a == b, "!=": lambda a, b: a != b, "<": lambda a, b: a < b,
          ">": lambda a, b: a > b, "<=": lambda a, b: a <= b, ">=": lambda a, b: a >= b}[op]
    for a, b in itertools.product(range(8), repeat=2):
        o = sim.run_shot(HEAD + _prep(a, b) + f"if (c {op} d) x q[6];\nt = measure q[6];\n", seed=1)
        assert o.cbits[6] == int(py(a, b)), (op, a, b)


def test_signed_variables_and_wrapping():
    # int[4] y = -3 stores 0b1101 and reads back as -3
    o = sim.run_shot(HEAD + "y = -3;\nx = y * 2;\nu = 250;\nu += 10;\n", seed=1)
    assert _bits(o, Y0, 4) == 0b1101
    assert _bits(o, X0, 16) == (int(np.int64(-3) * np.int64(2)) & 0xFFFF)
    with np.errstate(all="ignore"):
        assert _bits(o, U0, 8) == int(np.uint8(250) + np.uint8(10))
    # 64-bit wrap-around of intermediate results
    src = HEAD + "int[64] w = 9223372036854775807;\nw += 1;\nx = w == -9223372036854775807 - 1;\n"
    o = sim.run_shot(src, seed=1)
    with np.errstate(all="ignore"):
        big = np.int64(9223372036854775807) + np.int64(1)
    assert _bits(o, X0, 16) == int(big == np.int64(-9223372036854775807 - 1))
    w0 = 35
    assert _bits(o, w0, 64) == int(big) & 0xFFFFFFFFFFFFFFFF


def test_precedence_and_unary_operators():
    cases = [("(c & 3) == d", lambda a, b: (a & 3) == b), ("c & 3 == d", lambda a, b: a & int(3 == b)),
             ("c + d * 2 > 7", lambda a, b: a + b * 2 > 7), ("c << 1 | d", lambda a, b: (a << 1) | b),
             ("!c == 1 || d == 2", lambda a, b: (not a == 1) or b == 2),
             ("~c & 7 != d", lambda a, b: (~a) & int(7 != b)),
             ("-c + d >= 0 && c ^ d", lambda a, b: (-a + b >= 0) and (a ^ b) != 0)]
    for expr, fn in cases:
        for a, b in itertools.product(range(8), repeat=2):
            o = sim.run_shot(HEAD + _prep(a, b) + f"if ({expr}) x q[6];\nt = measure q[6];\n", seed=1)
            assert o.cbits[6] == int(bool(fn(a, b))), (expr, a, b)


def test_shift_and_division_edge_readings():
    o = sim.run_shot(HEAD + "x = 5 << 70;\nu = 200 >> 64;\ny = -1;\nint[16] z = y >> 99;\n", seed=1)
    assert _bits(o, X0, 16) == 0 and _bits(o, U0, 8) == 0
    assert _bits(o, 35, 16) == 0xFFFF                     # -1 >> 99 keeps the sign
    o = sim.run_shot(HEAD + "x = 7 / 0;\nu = 7 % 0;\ny = -7 / 2;\n", seed=1)
    assert _bits(o, X0, 16) == 0 and _bits(o, U0, 8) == 0 and _bits(o, Y0, 4) == (-3 & 0xF)


def test_variables_steer_feed_forward_and_count_in_loops():
    """A counter incremented in a bounded loop on measured outcomes, then a
    branch on the count: the classical value follows the measured bits."""
    src = ('OPENQASM 3.0;\ninclude "stdgates.inc";\nqubit[4] q;\nbit[3] c;\nbit f;\nuint[4] n = 0;\n'
           'for uint i in [0:2] { h q[i]; c[i] = measure q[i]; if (c[i]) n += 1; }\n'
           'if (n >= 2) x q[3];\nf = measure q[3];\n')
    for s in range(24):
        o = sim.run_shot(src, seed=3, shot=s)
        k = sum(o.cbits[:3])
        assert sum(o.cbits[4 + i] << i for i in range(4)) == k
        assert o.cbits[3] == int(k >= 2)
