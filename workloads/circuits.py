"""OpenQASM 3 program generators (text only; no simulation arithmetic).

Shapes follow the workloads the paper validates (Experiments, benchmark suites):
random static circuits, conditional reset, teleportation, if/else branching,
multi-bit predicates, bounded repeat-until-success loops and a hardware-efficient
VQE ansatz with runtime ``input`` parameters, scaled to the sizes of the five
benchmark configurations:

  C1  10 qubits, 20 layers of U3-on-every-qubit + 5 CX on a random perfect
      matching; after layers 5, 10, 15 a measure -> if (c[i]==1) x -> reset site;
      final measure-all.
  C2  28 qubits, 40 brickwork layers (U3 on all, CX(2j,2j+1) on even layers,
      CX(2j+1,2j+2) on odd layers); a 4-qubit measure into bit[4] c;
      if (c == 0b1010) { 3 random gates }; if (c[0]) rx else rz; measure-all.
  C3  16 qubits, 12 random layers, then a repeat-until-success loop of at most
      8 iterations (measure the ancilla, break on 0, otherwise reset it and
      reapply a fixed 2-layer random block); measure-all.
  C4  20-qubit hardware-efficient ansatz: 6 layers of RY(theta), RZ(theta) on
      every qubit and a CX ladder (240 parameters), with a random 60-term
      2-local Pauli Hamiltonian.
"""
import math

import numpy as np

HEADER = 'OPENQASM 3.0;\ninclude "stdgates.inc";\n'
TWO_PI = 2.0 * math.pi


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _ang(x):
    return repr(float(x))


def _u3(rng, q, reg="q"):
    a = rng.random(3) * TWO_PI
    return f"U({_ang(a[0])}, {_ang(a[1])}, {_ang(a[2])}) {reg}[{q}];"


def _matching(rng, n, count):
    perm = rng.permutation(n)
    return [(int(perm[2 * k]), int(perm[2 * k + 1])) for k in range(count)]


def _layer(rng, n, n_cx, reg="q"):
    lines = [_u3(rng, q, reg) for q in range(n)]
    lines += [f"cx {reg}[{a}], {reg}[{b}];" for a, b in _matching(rng, n, n_cx)]
    return lines


# ---------------------------------------------------------------------------
# Benchmark configurations
# ---------------------------------------------------------------------------
def c1_program(seed=1, n=10, layers=20, sites=(5, 10, 15), final_measure=True):
    rng = _rng(seed)
    lines = [HEADER, f"qubit[{n}] q;", f"bit[{len(sites)}] c;"]
    if final_measure:
        lines.append(f"bit[{n}] f;")
    k = 0
    for layer in range(1, layers + 1):
        lines += _layer(rng, n, n // 2)
        if layer in sites:
            m = int(rng.integers(n))
            r = int(rng.integers(n - 1))
            r = r if r < m else r + 1
            lines += [f"c[{k}] = measure q[{m}];", f"if (c[{k}] == 1) x q[{r}];", f"reset q[{m}];"]
            k += 1
    if final_measure:
        lines.append("f = measure q;")
    return "\n".join(lines) + "\n"


def _brickwork_layer(rng, n, layer, reg="q", offset=0, width=None):
    width = n if width is None else width
    lines = [_u3(rng, offset + q, reg) for q in range(width)]
    start = 0 if layer % 2 == 0 else 1
    for a in range(start, width - 1, 2):
        lines.append(f"cx {reg}[{offset + a}], {reg}[{offset + a + 1}];")
    return lines


def brickwork_program(seed=2, n=28, layers=40, final_measure=False):
    """Plain brickwork: U3 on every qubit, then CX on alternating neighbour pairs."""
    rng = _rng(seed)
    lines = [HEADER, f"qubit[{n}] q;"]
    if final_measure:
        lines.append(f"bit[{n}] f;")
    for layer in range(layers):
        lines += _brickwork_layer(rng, n, layer)
    if final_measure:
        lines.append("f = measure q;")
    return "\n".join(lines) + "\n"


def c2_program(seed=2, n=28, layers=40, n_measure=4, final_measure=True, pattern=0b1010):
    rng = _rng(seed)
    lines = [HEADER, f"qubit[{n}] q;", f"bit[{n_measure}] c;"]
    if final_measure:
        lines.append(f"bit[{n}] f;")
    for layer in range(layers):
        lines += _brickwork_layer(rng, n, layer)
    mq = [int(x) for x in rng.choice(n, size=n_measure, replace=False)]
    for i, q in enumerate(mq):
        lines.append(f"c[{i}] = measure q[{q}];")
    block = []
    for _ in range(3):
        if rng.random() < 0.5:
            block.append(_u3(rng, int(rng.integers(n))))
        else:
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            block.append(f"cx q[{a}], q[{b}];")
    lines.append(f"if (c == {pattern}) {{ " + " ".join(block) + " }")
    r = int(rng.integers(n))
    th = rng.random() * TWO_PI
    lines.append(f"if (c[0]) rx({_ang(th)}) q[{r}]; else rz({_ang(th)}) q[{r}];")
    if final_measure:
        lines.append("f = measure q;")
    return "\n".join(lines) + "\n"


def c3_program(seed=3, n=16, layers=12, max_iter=8, final_measure=True):
    rng = _rng(seed)
    a = int(rng.integers(n))
    lines = [HEADER, f"qubit[{n}] q;", "bit b;"]
    if final_measure:
        lines.append(f"bit[{n}] f;")
    for _ in range(layers):
        lines += _layer(rng, n, n // 2)
    block = _layer(rng, n, n // 2) + _layer(rng, n, n // 2)
    lines.append(f"for uint i in [0:{max_iter - 1}] {{")
    lines.append(f"  b = measure q[{a}];")
    lines.append("  if (b == 0) break;")
    lines.append(f"  reset q[{a}];")
    lines += ["  " + s for s in block]
    lines.append("}")
    if final_measure:
        lines.append("f = measure q;")
    return "\n".join(lines) + "\n"


def c3_mix(seed=33, count=256, n_lo=12, n_hi=18):
    """Distinct circuits of the C3 structure with 12..18 qubits, each with its own seed."""
    rng = _rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        out.append(c3_program(seed=int(rng.integers(1 << 62)), n=n))
    return out


def c4_ansatz(n=20, layers=6):
    """Hardware-efficient ansatz: per layer RY(theta) then RZ(theta) on every qubit,
    then CX(i, i+1) for i = 0..n-2. theta[l*2n + q] feeds RY, theta[l*2n + n + q] RZ."""
    p = 2 * n * layers
    lines = [HEADER, f"input array[float[64], {p}] theta;", f"qubit[{n}] q;"]
    for layer in range(layers):
        base = 2 * n * layer
        lines += [f"ry(theta[{base + q}]) q[{q}];" for q in range(n)]
        lines += [f"rz(theta[{base + n + q}]) q[{q}];" for q in range(n)]
        lines += [f"cx q[{q}], q[{q + 1}];" for q in range(n - 1)]
    return "\n".join(lines) + "\n"


def c4_hamiltonian(seed=4, n=20, terms=60):
    """Random 2-local Pauli sum: each term on 2 distinct uniform qubits with Paulis
    uniform over {X, Y, Z} (codes 1, 2, 3) and a N(0, 1) coefficient."""
    rng = _rng(seed)
    coeffs = rng.standard_normal(terms)
    codes = np.zeros((terms, n), dtype=np.uint8)
    for t in range(terms):
        a, b = rng.choice(n, size=2, replace=False)
        codes[t, a] = rng.integers(1, 4)
        codes[t, b] = rng.integers(1, 4)
    return coeffs, codes


def c4_thetas(seed=44, batch=64, n_params=240):
    rng = _rng(seed)
    return rng.uniform(-math.pi, math.pi, size=(batch, n_params))


# ---------------------------------------------------------------------------
# Property workloads at full width
# ---------------------------------------------------------------------------
def separable_brickwork(seed=5, n=28, blocks=4, layers=40):
    """Brickwork whose CX gates never cross block boundaries, so the final state is
    a tensor product of independent blocks. Returns (full_program, block_programs,
    block_offsets); block b acts on qubits [offset_b, offset_b + width_b)."""
    rng = _rng(seed)
    width = n // blocks
    offs = [b * width for b in range(blocks)]
    widths = [width] * (blocks - 1) + [n - width * (blocks - 1)]
    full = [HEADER, f"qubit[{n}] q;"]
    parts = [[HEADER, f"qubit[{w}] q;"] for w in widths]
    for layer in range(layers):
        for b in range(blocks):
            brng = np.random.Generator(np.random.PCG64(int(rng.integers(1 << 62))))
            local = _brickwork_layer(brng, widths[b], layer, width=widths[b])
            parts[b] += local
            full += [_shift_qubits(s, offs[b]) for s in local]
    return ("\n".join(full) + "\n", ["\n".join(p) + "\n" for p in parts], offs)


def _shift_qubits(line, off):
    import re
    return re.sub(r"q\[(\d+)\]", lambda m: f"q[{int(m.group(1)) + off}]", line)


def mirror_program(seed=6, n=28, layers=40):
    """Brickwork U followed by its exact inverse U^dag; the result is |0...0>."""
    rng = _rng(seed)
    fwd = []
    for layer in range(layers):
        fwd.append(_brickwork_layer(rng, n, layer))
    lines = [HEADER, f"qubit[{n}] q;"]
    for layer in fwd:
        lines += layer
    for layer in reversed(fwd):
        for s in reversed(layer):
            lines.append(_inverse_line(s))
    return "\n".join(lines) + "\n"


def _inverse_line(s):
    # U(a, b, c)^dag = U(-a, -c, -b); cx is self-inverse.
    if s.startswith("U("):
        inside, rest = s[2:].split(")", 1)
        a, b, c = (float(x) for x in inside.split(","))
        return f"U({_ang(-a)}, {_ang(-c)}, {_ang(-b)}){rest}"
    return s


# ---------------------------------------------------------------------------
# Random dynamic programs for parity at small sizes
# ---------------------------------------------------------------------------
_ONE_Q_FIXED = ["x", "y", "z", "h", "s", "sdg", "t", "tdg", "sx", "id"]
_ONE_Q_PARAM = {"rx": 1, "ry": 1, "rz": 1, "p": 1, "U": 3, "u2": 2}
_TWO_Q_FIXED = ["cx", "cy", "cz", "swap", "ch"]
_TWO_Q_PARAM = {"cp": 1, "crx": 1, "cry": 1, "crz": 1}


def _random_gate(rng, n):
    r = rng.random()
    if r < 0.25:
        return f"{_ONE_Q_FIXED[int(rng.integers(len(_ONE_Q_FIXED)))]} q[{int(rng.integers(n))}];"
    if r < 0.6 or n < 2:
        name = list(_ONE_Q_PARAM)[int(rng.integers(len(_ONE_Q_PARAM)))]
        args = ", ".join(_ang(x) for x in rng.random(_ONE_Q_PARAM[name]) * TWO_PI)
        return f"{name}({args}) q[{int(rng.integers(n))}];"
    a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
    if r < 0.85:
        return f"{_TWO_Q_FIXED[int(rng.integers(len(_TWO_Q_FIXED)))]} q[{a}], q[{b}];"
    name = list(_TWO_Q_PARAM)[int(rng.integers(len(_TWO_Q_PARAM)))]
    return f"{name}({_ang(rng.random() * TWO_PI)}) q[{a}], q[{b}];"


def random_dynamic_program(seed, n, n_ops=40, n_bits=4, p_dynamic=0.25, final_measure=True,
                           allow_loops=True):
    """Random gates interleaved with measure / reset / if-else / bounded loops."""
    rng = _rng(seed)
    lines = [HEADER, f"qubit[{n}] q;", f"bit[{n_bits}] c;"]
    if final_measure:
        lines.append(f"bit[{n}] f;")
    depth = 0

    def emit_block(count, in_loop):
        out = []
        for _ in range(count):
            r = rng.random()
            if r < 1.0 - p_dynamic:
                out.append(_random_gate(rng, n))
                continue
            r = rng.random()
            if r < 0.35:
                out.append(f"c[{int(rng.integers(n_bits))}] = measure q[{int(rng.integers(n))}];")
            elif r < 0.5:
                out.append(f"reset q[{int(rng.integers(n))}];")
            elif r < 0.8 or not allow_loops or depth > 0:
                body = [_random_gate(rng, n) for _ in range(int(rng.integers(1, 4)))]
                other = [_random_gate(rng, n) for _ in range(int(rng.integers(0, 3)))]
                if rng.random() < 0.5:
                    cond = f"c[{int(rng.integers(n_bits))}] == {int(rng.integers(2))}"
                else:
                    cond = f"c == {int(rng.integers(1 << n_bits))}"
                s = f"if ({cond}) {{ " + " ".join(body) + " }"
                if other:
                    s += " else { " + " ".join(other) + " }"
                out.append(s)
            else:
                k = int(rng.integers(1, 4))
                bit = int(rng.integers(n_bits))
                inner = [f"c[{bit}] = measure q[{int(rng.integers(n))}];",
                         f"if (c[{bit}] == {int(rng.integers(2))}) break;"]
                inner += [_random_gate(rng, n) for _ in range(int(rng.integers(1, 4)))]
                out.append(f"for uint i in [0:{k - 1}] {{ " + " ".join(inner) + " }")
        return out

    lines += emit_block(n_ops, False)
    if final_measure:
        lines.append("f = measure q;")
    return "\n".join(lines) + "\n"


def _random_logic_cond(rng, n_bits, depth):
    """A random condition over c[0..n_bits-1] with !, && and || (nested to `depth`)."""
    if depth == 0 or rng.random() < 0.3:
        r = rng.random()
        if r < 0.4:
            atom = f"c[{int(rng.integers(n_bits))}]"
        elif r < 0.7:
            atom = f"c[{int(rng.integers(n_bits))}] == {int(rng.integers(2))}"
        else:
            atom = f"c {['==', '!=', '<', '>='][int(rng.integers(4))]} {int(rng.integers(1 << n_bits))}"
        if rng.random() < 0.25:
            return f"!({atom})"
        return f"({atom})" if rng.random() < 0.5 else atom
    op = "&&" if rng.random() < 0.5 else "||"
    a = _random_logic_cond(rng, n_bits, depth - 1)
    b = _random_logic_cond(rng, n_bits, depth - 1)
    s = f"{a} {op} {b}"
    return f"!({s})" if rng.random() < 0.2 else f"({s})" if rng.random() < 0.5 else s


def logic_program(seed, n, n_ops=30, n_bits=3, final_measure=True, assign=False):
    """Random gates, measurements into c[0..n_bits-1] and if / if-else blocks
    whose conditions combine bit tests and comparisons with !, && and ||.
    assign: also classical assignments (a condition into one bit, an integer
    into the register)."""
    rng = _rng(seed)
    lines = [HEADER, f"qubit[{n}] q;", f"bit[{n_bits}] c;"]
    if final_measure:
        lines.append(f"bit[{n}] f;")
    for i in range(n_bits):
        lines.append(f"h q[{i % n}];")
        lines.append(f"c[{i}] = measure q[{i % n}];")
    for _ in range(n_ops):
        r = rng.random()
        if r < 0.6:
            lines.append(_random_gate(rng, n))
        elif r < 0.75:
            lines.append(f"c[{int(rng.integers(n_bits))}] = measure q[{int(rng.integers(n))}];")
        elif assign and r < 0.85:
            if rng.random() < 0.8:
                lines.append(f"c[{int(rng.integers(n_bits))}] = {_random_logic_cond(rng, n_bits, 2)};")
            else:
                lines.append(f"c = {int(rng.integers(1 << n_bits))};")
        else:
            body = [_random_gate(rng, n) for _ in range(int(rng.integers(1, 4)))]
            s = f"if ({_random_logic_cond(rng, n_bits, 2)}) {{ " + " ".join(body) + " }"
            if rng.random() < 0.5:
                s += " else { " + " ".join(_random_gate(rng, n) for _ in range(int(rng.integers(1, 3)))) + " }"
            lines.append(s)
    if final_measure:
        lines.append("f = measure q;")
    return "\n".join(lines) + "\n"


def random_clifford_program(seed, n, n_gates):
    """Random H / S / CX circuit (a stabilizer state at the end)."""
    rng = _rng(seed)
    lines = [HEADER, f"qubit[{n}] q;"]
    for _ in range(n_gates):
        r = rng.random()
        if r < 0.35 or n < 2:
            lines.append(f"h q[{int(rng.integers(n))}];")
        elif r < 0.6:
            lines.append(f"s q[{int(rng.integers(n))}];")
        else:
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            lines.append(f"cx q[{a}], q[{b}];")
    return "\n".join(lines) + "\n"


# ---------------------------------------------------------------------------
# Small protocols from the paper's validation suites
# ---------------------------------------------------------------------------
def conditional_reset_program(prep="minus"):
    """Prepare |+> (h) or |-> (x; h), measure, and apply x when the outcome is 1."""
    prep_lines = "h q[0];" if prep == "plus" else "x q[0];\nh q[0];"
    return (HEADER + "qubit[1] q;\nbit[1] c;\nbit[1] f;\n" + prep_lines + "\n"
            "c[0] = measure q[0];\nif (c[0] == 1) x q[0];\nf[0] = measure q[0];\n")


def teleport_program(alpha, beta, gamma):
    """Teleport U(alpha, beta, gamma)|0> from q[0] to q[2]; then undo U on q[2]."""
    return (HEADER + "qubit[3] q;\nbit[2] c;\n"
            f"U({_ang(alpha)}, {_ang(beta)}, {_ang(gamma)}) q[0];\n"
            "h q[1];\ncx q[1], q[2];\ncx q[0], q[1];\nh q[0];\n"
            "c[0] = measure q[0];\nc[1] = measure q[1];\n"
            "if (c[1] == 1) x q[2];\nif (c[0] == 1) z q[2];\n"
            f"U({_ang(-alpha)}, {_ang(-gamma)}, {_ang(-beta)}) q[2];\n")


def if_else_program(theta):
    return (HEADER + "qubit[2] q;\nbit[1] c;\nh q[0];\nc[0] = measure q[0];\n"
            f"if (c[0]) rx({_ang(theta)}) q[1]; else rz({_ang(theta)}) q[1];\n")


def multibit_predicate_program(bits, pattern=0b1010):
    """Prepare |bits> with x gates on 4 data qubits, measure them into bit[4] c and
    flip a fifth qubit iff c == pattern."""
    xs = "".join(f"x q[{i}];\n" for i in range(4) if (bits >> i) & 1)
    return (HEADER + "qubit[5] q;\nbit[4] c;\n" + xs
            + "for uint i in [0:3] { c[i] = measure q[i]; }\n"
            + f"if (c == {pattern}) {{ x q[4]; }}\n")


def rus_program(phi, max_iter=8):
    """Repeat-until-success: rotate the ancilla by RY(phi), measure it, stop on
    outcome 0, otherwise reset it and try again (at most max_iter tries)."""
    return (HEADER + "qubit[1] q;\nbit b;\n"
            f"for uint i in [0:{max_iter - 1}] {{\n"
            f"  ry({_ang(phi)}) q[0];\n  b = measure q[0];\n"
            "  if (b == 0) break;\n  reset q[0];\n}\n")


def qft_program(n, x):
    """Prepare basis state |x> and apply the quantum Fourier transform."""
    lines = [HEADER, f"qubit[{n}] q;"]
    lines += [f"x q[{i}];" for i in range(n) if (x >> i) & 1]
    for j in reversed(range(n)):
        lines.append(f"h q[{j}];")
        for k in reversed(range(j)):
            lines.append(f"cp(pi / {2 ** (j - k)}) q[{k}], q[{j}];")
    for i in range(n // 2):
        lines.append(f"swap q[{i}], q[{n - 1 - i}];")
    return "\n".join(lines) + "\n"


def bv_program(secret, n):
    """Bernstein-Vazirani on n data qubits plus one ancilla (qubit n)."""
    lines = [HEADER, f"qubit[{n + 1}] q;", f"bit[{n}] c;", f"x q[{n}];"]
    lines += [f"h q[{i}];" for i in range(n + 1)]
    lines += [f"cx q[{i}], q[{n}];" for i in range(n) if (secret >> i) & 1]
    lines += [f"h q[{i}];" for i in range(n)]
    lines += [f"c[{i}] = measure q[{i}];" for i in range(n)]
    return "\n".join(lines) + "\n"


def hea2_program():
    """Two-qubit ansatz RY(a) q0, RY(b) q1, CX(0,1) with runtime inputs a, b."""
    return (HEADER + "input float[64] a;\ninput float[64] b;\nqubit[2] q;\n"
            "ry(a) q[0];\nry(b) q[1];\ncx q[0], q[1];\n")


def param_program(seed, n, n_gates, n_params):
    """Random parameterised unitary circuit over `n_params` runtime inputs t[k]:
    U, rx, ry, rz, p, crx, cry, crz, cp with angles t[k], 2 * t[k], t[k] + 0.3
    or -t[k], mixed with h, cx, swap and sx on uniform random qubits."""
    rng = _rng(seed)
    lines = [HEADER, f"input array[float[64], {n_params}] t;", f"qubit[{n}] q;"]

    def ang():
        k = int(rng.integers(n_params))
        return (f"t[{k}]", f"2 * t[{k}]", f"t[{k}] + 0.3", f"-t[{k}]")[int(rng.integers(4))]

    for _ in range(n_gates):
        kind = int(rng.integers(13))
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        if kind == 0:
            lines.append(f"U({ang()}, {ang()}, {ang()}) q[{a}];")
        elif kind <= 4:
            lines.append(f"{('rx', 'ry', 'rz', 'p')[kind - 1]}({ang()}) q[{a}];")
        elif kind <= 8:
            lines.append(f"{('crx', 'cry', 'crz', 'cp')[kind - 5]}({ang()}) q[{a}], q[{b}];")
        elif kind <= 10:
            lines.append(f"{('cx', 'swap')[kind - 9]} q[{a}], q[{b}];")
        else:
            lines.append(f"{('h', 'sx')[kind - 11]} q[{a}];")
    return "\n".join(lines) + "\n"



def modifier_program(seed, n, n_gates, final_measure=True):
    """Random circuit of gate calls under gate modifiers: inv @, pow(k) @ (k in
    -2..3), ctrl @ and negctrl @ (one control) on one-qubit gates, inv @ on
    two-qubit gates and on a gate definition, mixed with plain gates."""
    rng = _rng(seed)
    one = ["x", "y", "z", "h", "s", "sdg", "t", "tdg", "sx", "sxdg", "rx", "ry", "rz", "p", "U", "u2"]
    two = ["cx", "cz", "cp", "crx", "cry", "swap"]
    lines = [HEADER, "gate blk(a) u, v { h u; crz(a) u, v; ry(0.5 * a) v; }", f"qubit[{n}] q;"]
    if final_measure:
        lines.append(f"bit[{n}] f;")

    def call(name):
        if name in ("rx", "ry", "rz", "p", "cp", "crx", "cry"):
            return f"{name}({_ang(rng.random() * TWO_PI)})"
        if name == "U":
            a = rng.random(3) * TWO_PI
            return f"U({_ang(a[0])}, {_ang(a[1])}, {_ang(a[2])})"
        if name == "u2":
            a = rng.random(2) * TWO_PI
            return f"u2({_ang(a[0])}, {_ang(a[1])})"
        return name

    for _ in range(n_gates):
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        r = rng.random()
        if r < 0.3:
            lines.append(f"{call(str(rng.choice(one)))} q[{a}];")
        elif r < 0.5:
            mod = ["ctrl", "negctrl"][int(rng.integers(2))]
            inner = "inv @ " if rng.random() < 0.3 else ""
            lines.append(f"{mod} @ {inner}{call(str(rng.choice(one)))} q[{a}], q[{b}];")
        elif r < 0.7:
            k = int(rng.integers(-2, 4))
            lines.append(f"pow({k}) @ {call(str(rng.choice(one)))} q[{a}];")
        elif r < 0.85:
            lines.append(f"inv @ {call(str(rng.choice(two)))} q[{a}], q[{b}];")
        else:
            lines.append(f"inv @ blk({_ang(rng.random() * TWO_PI)}) q[{a}], q[{b}];")
    if final_measure:
        lines.append("f = measure q;")
    return "\n".join(lines) + "\n"
