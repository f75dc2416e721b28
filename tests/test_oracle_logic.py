"""Oracle pins for `&&`, `||` and `!` in if conditions (OpenQASM 3 logical
operators; the paper's multi-bit predicates, Methodology, Transpiling Dynamic
Control Flow): every assignment of three measured bits, prepared
deterministically, against Python's own boolean operators; `&&` binds tighter
than `||`; the condition is read once, when the if executes."""
import itertools

import pytest

from oracle import sim

HEAD = 'OPENQASM 3.0;\ninclude "stdgates.inc";\nqubit[5] q;\nbit[3] c;\nbit t;\nbit e;\n'

# condition text and the same condition as a Python function of (c0, c1, c2)
CASES = [
    ("c[0] && c[1]", lambda a, b, d: a and b),
    ("c[0] || c[1]", lambda a, b, d: a or b),
    ("c[0] || c[1] && c[2]", lambda a, b, d: a or (b and d)),
    ("(c[0] || c[1]) && c[2]", lambda a, b, d: (a or b) and d),
    ("!c[0] && c[1] || c[2]", lambda a, b, d: ((not a) and b) or d),
    ("!(c[0] || c[1]) && c[2]", lambda a, b, d: (not (a or b)) and d),
    ("c == 5 || c[1] && !c[2]", lambda a, b, d: (a + 2 * b + 4 * d) == 5 or (b and not d)),
    ("(c[0] || c[1]) && (c[1] || c[2])", lambda a, b, d: (a or b) and (b or d)),
    ("c[0] && c[1] && c[2] || !c[0] && !c[1]", lambda a, b, d: (a and b and d) or (not a and not b)),
    ("c >= 3 && c != 6 || c[1] == 0 && c < 2", lambda a, b, d: (3 <= a + 2 * b + 4 * d != 6) or
     (b == 0 and a + 2 * b + 4 * d < 2)),
]


def _prep(bits):
    lines = [f"x q[{i}];" for i, v in enumerate(bits) if v]
    lines += [f"c[{i}] = measure q[{i}];" for i in range(3)]
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("cond,fn", CASES)
def test_logical_conditions_truth_table(cond, fn):
    for bits in itertools.product((0, 1), repeat=3):
        src = HEAD + _prep(bits) + f"if ({cond}) x q[3]; else x q[4];\nt = measure q[3];\ne = measure q[4];\n"
        o = sim.run_shot(src, seed=1)
        want = bool(fn(*bits))
        assert o.cbits[3] == int(want) and o.cbits[4] == int(not want), (cond, bits)


def test_condition_is_read_when_the_if_executes():
    """The body overwrites a bit the condition tested; the else branch does not
    run and the condition is not re-read."""
    src = HEAD + _prep((1, 1, 0)) + ("if (c[0] && c[1]) { x q[1]; c[1] = measure q[1]; } else x q[4];\n"
                                     "t = measure q[3];\ne = measure q[4];\n")
    o = sim.run_shot(src, seed=2)
    assert o.cbits[:3] == [1, 0, 0] and o.cbits[4] == 0
