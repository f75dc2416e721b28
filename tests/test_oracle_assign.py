"""Oracle pins for classical assignment (OpenQASM 3 classical bits; the
paper's feed-forward, Methodology, Transpiling Dynamic Control Flow): every
assignment of the measured bits, prepared deterministically, against Python
integers and booleans."""
import itertools

import pytest

from oracle import sim

HEAD = 'OPENQASM 3.0;\ninclude "stdgates.inc";\nconst int k = 6;\nqubit[4] q;\nbit[3] c;\nbit[3] d;\nbit t;\n'


def _prep(bits):
    lines = [f"x q[{i}];" for i, v in enumerate(bits) if v]
    lines += [f"c[{i}] = measure q[{i}];" for i in range(3)]
    return "\n".join(lines) + "\n"


def _val(bits):
    return sum(b << i for i, b in enumerate(bits))


BIT_CASES = [
    ("c[2] = c[0] && c[1];", lambda a, b, e: (a, b, int(a and b))),
    ("c[0] = !c[0];", lambda a, b, e: (1 - a, b, e)),
    ("c[1] = c[0] || c == 4;", lambda a, b, e: (a, int(a or _val((a, b, e)) == 4), e)),
    ("c[0] = !c[0] && c[1];", lambda a, b, e: (int((not a) and b), b, e)),   # the right side reads c[0] first
    ("c[2] = c[0];", lambda a, b, e: (a, b, a)),
    ("c[1] = c >= 3;", lambda a, b, e: (a, int(_val((a, b, e)) >= 3), e)),
]


@pytest.mark.parametrize("stmt,fn", BIT_CASES)
def test_bit_assignment_truth_table(stmt, fn):
    for bits in itertools.product((0, 1), repeat=3):
        o = sim.run_shot(HEAD + _prep(bits) + stmt + "\n", seed=1)
        assert tuple(o.cbits[:3]) == fn(*bits), (stmt, bits)


def test_register_assignment_and_copy():
    for bits in itertools.product((0, 1), repeat=3):
        o = sim.run_shot(HEAD + _prep(bits) + "d = c;\nc = 5;\n", seed=1)
        assert o.cbits[3:6] == list(bits) and o.cbits[:3] == [1, 0, 1]
    o = sim.run_shot(HEAD + "c = k;\nd[1] = 1;\nd[2] = 0;\n", seed=1)
    assert o.cbits[:3] == [0, 1, 1] and o.cbits[3:6] == [0, 1, 0]
    o = sim.run_shot(HEAD + "c = 0b011;\n", seed=1)
    assert o.cbits[:3] == [1, 1, 0]


def test_assigned_bits_drive_feed_forward():
    """A computed bit steers a later if: x on q[3] exactly when c[0] xor c[1]."""
    for bits in itertools.product((0, 1), repeat=3):
        src = (HEAD + _prep(bits) + "c[2] = c[0] && !c[1] || !c[0] && c[1];\n"
               "if (c[2]) x q[3];\nt = measure q[3];\n")
        o = sim.run_shot(src, seed=1)
        assert o.cbits[6] == bits[0] ^ bits[1] and o.cbits[2] == bits[0] ^ bits[1]
