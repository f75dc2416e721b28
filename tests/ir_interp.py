"""Test-only interpreter of the lowered instruction stream.

Executes the guarded stream the product's lowering emits, with the oracle's
gate matrices and tensor engine, so that lowering can be compared with the
oracle's direct walk of the syntax tree on the CPU.
"""
import math

from oracle import gates as G
from oracle.philox import ShotStream, noise_word, word_to_uniform
from oracle.sim import TensorEngine

OP_GATE, OP_MEASURE, OP_RESET, OP_SETF, OP_CLRF, OP_SETB, OP_CLRB, OP_CSTORE, OP_NOISE = 1, 2, 3, 4, 5, 6, 7, 8, 9
CMP_TRUE, CMP_EXPR = 6, 7
M64 = (1 << 64) - 1


def _s64(v):
    v &= M64
    return v - (1 << 64) if v >> 63 else v


def run_code(code, pc, bits):
    """The postfix classical-expression code of the lowered stream, from pc to
    its end op (0), on Python integers wrapped to signed 64 bits."""
    st = []
    while True:
        c = code[pc]
        op = int(c["op"])
        pc += 1
        if op == 0:
            return st[-1]
        if op == 1:
            st.append(int(c["imm"]))
            continue
        if op == 2:
            w, lo = int(c["width"]), int(c["lo"])
            v = sum(bits[lo + i] << i for i in range(w))
            if int(c["sgn"]) and v >> (w - 1):
                v -= 1 << w
            st.append(_s64(v))
            continue
        if op in (3, 4, 5):
            a = st.pop()
            st.append(_s64(-a) if op == 3 else _s64(~a) if op == 4 else int(a == 0))
            continue
        b, a = st.pop(), st.pop()
        if op == 9 or op == 10:
            if b == 0:
                r = 0
            else:
                q = abs(a) // abs(b)
                q = q if (a < 0) == (b < 0) else -q
                r = q if op == 9 else a - q * b
        elif op == 14:
            r = a << b if 0 <= b < 64 else 0
        elif op == 15:
            r = a >> b if 0 <= b < 64 else (-1 if a < 0 else 0)
        else:
            r = {6: a + b, 7: a - b, 8: a * b, 11: a & b, 12: a | b, 13: a ^ b, 16: int(a == b), 17: int(a != b),
                 18: int(a < b), 19: int(a > b), 20: int(a <= b), 21: int(a >= b), 22: int(a != 0 and b != 0),
                 23: int(a != 0 or b != 0)}[op]
        st.append(_s64(r))


KIND_NAMES = ["id", "x", "y", "z", "h", "s", "sdg", "t", "tdg", "sx", "sxdg", "rx", "ry", "rz", "p", "U",
              "cx", "cy", "cz", "ch", "swap", "cp", "crx", "cry", "crz"]
N_ANGLES = {"rx": 1, "ry": 1, "rz": 1, "p": 1, "U": 3, "cp": 1, "crx": 1, "cry": 1, "crz": 1}


def eval_pred(p, bits, code=None):
    lo, width, value, cmp = int(p["lo"]), int(p["width"]), int(p["value"]), int(p["cmp"])
    if cmp == CMP_TRUE:
        return True
    if cmp == CMP_EXPR:
        return run_code(code, value, bits) != 0
    v = sum(bits[lo + i] << i for i in range(width))
    return [v == value, v != value, v < value, v > value, v <= value, v >= value][cmp]


def run(lp, theta=(), seed=0, shot=0, forced=None, depolarizing=0.0):
    eng = TensorEngine(lp.n_qubits)
    bits = [0] * lp.n_clbits
    flags = 0
    stream = ShotStream(seed, shot)
    record, nmeas = [], 0
    forced = list(forced or [])
    code = getattr(lp, "code", None)
    for ins in lp.instr:
        op, guard = int(ins["op"]), int(ins["guard"])
        active = (flags & guard) == guard
        if op == OP_SETF:
            v = active and eval_pred(lp.pred[int(ins["pred"])], bits, code)
            f = int(ins["flag"])
            flags = (flags & ~(1 << f)) | (int(v) << f)
            continue
        if not active:
            continue
        if op == OP_CLRF:
            flags &= ~(1 << int(ins["flag"]))
        elif op in (OP_SETB, OP_CLRB):
            bits[int(ins["cbit"])] = 1 if op == OP_SETB else 0
        elif op == OP_NOISE:
            if depolarizing > 0.0:
                c = [int(x) for x in lp.noise[int(ins["pred"])]["ctr"]]
                u = word_to_uniform(noise_word(seed, shot, *c))
                if u < depolarizing:
                    name = "x" if u < depolarizing / 3 else ("y" if u < 2 * depolarizing / 3 else "z")
                    eng.apply(G.gate_matrix(name, [])[0], [int(ins["q0"])])
        elif op == OP_CSTORE:
            v = run_code(code, int(ins["pred"]), bits)
            for i in range(int(ins["flag"])):
                bits[int(ins["cbit"]) + i] = (v >> i) & 1
        elif op == OP_GATE:
            name = KIND_NAMES[int(ins["kind"])]
            angles = []
            for k in range(N_ANGLES.get(name, 0)):
                a = float(ins["offset"][k])
                par = int(ins["param"][k])
                if par != 0xFFFFFFFF:
                    if par >= lp.n_params:  # a derived parameter: a combination of inputs
                        v = sum(float(e["coef"]) * float(theta[int(e["in"])]) for e in lp.lin
                                if int(e["out"]) == par - lp.n_params)
                    else:
                        v = float(theta[par])
                    a += float(ins["scale"][k]) * v
                angles.append(a)
            m, nq = G.gate_matrix(name, angles)
            qs = [int(ins["q0"])] + ([int(ins["q1"])] if nq == 2 else [])
            eng.apply(m, qs)
        else:
            q = int(ins["q0"])
            p0, p1 = eng.probs(q)
            u = stream.next_uniform()
            if op == OP_MEASURE and nmeas < len(forced):
                m = forced[nmeas]
            else:
                m = 0 if u < p0 / (p0 + p1) else 1
            eng.collapse(q, m, p0 if m == 0 else p1)
            if op == OP_MEASURE:
                nmeas += 1
                record.append(m)
                if int(ins["cbit"]) != 0xFFFFFFFF:
                    bits[int(ins["cbit"])] = m
            elif m == 1:
                eng.flip(q)
    return eng.psi, bits, record


_ = math
