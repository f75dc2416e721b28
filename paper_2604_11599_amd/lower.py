"""Lowering of the OpenQASM 3 syntax tree to libqsv's guarded instruction stream.

Follows the paper's translation scheme (Methodology): standard gates map one
to one onto gate instructions; an ``if`` becomes a predicate evaluated at run
time on the measured bits, guarding its body instead of expanding both
branches statically; ``input`` variables become runtime parameter slots, so a
program is lowered and loaded once and run with many parameter vectors.

Symbol handling (Methodology, parsing and semantic analysis):
  * compile-time constants and loop variables are folded to numbers;
  * ``input`` parameters become slots of one flat theta vector (declaration
    order, arrays contiguous); a gate angle is affine in them:
    angle = scale * theta[slot] + offset, where an angle that combines several
    inputs reads a derived parameter (a linear combination of inputs the
    device forms from theta before binding);
  * classical bits of all ``bit`` registers and classical variables (``uint[n]``,
    ``int[n]``, ``bool``) form one flat array in declaration order; a register's
    value is sum_i c[i] 2^i (two's complement for ``int`` variables).

Control flow becomes flags (64 per shot) and guard masks:
  if (p) A else B   ->  SETF t <- p ; SETF e <- !p ; A guarded by t ; B guarded by e
  for i in [a:b] S  ->  SETF l <- true ; S unrolled for each i, guarded by l
  break / continue  ->  CLRF l / CLRF c (under the enclosing guards)
  if (p && q) A     ->  SETF t1 <- p ; SETF f1 <- !p ; SETF t2 <- q (guarded by t1) ;
                        SETF f2 <- !q (guarded by t1) ; A guarded by t1, t2
  `||` mirrors `&&` (q is tested where p fails); a condition with several ways
  to hold gets its body once per way, under disjoint guards.
  c = v / d = c     ->  SETB / CLRB per bit (v an integer; d = c copies c's bits)
  c[i] = cond       ->  the guards of cond, then SETB i under each guard where
                        it holds and CLRB i under each where it fails
  x = <expression>  ->  CSTORE: the device evaluates the expression's postfix
                        code on the shot's classical bits (64-bit two's
                        complement) and stores its low bits
  if (<expression>) ->  a predicate on the expression's code where the
                        condition is not a register compared with a constant
Custom ``gate`` definitions are inlined.
"""
import collections
import math

import numpy as np

from . import frontend as F

# instruction ops, gate kinds and predicate comparisons of include/qsv.h
OP_GATE, OP_MEASURE, OP_RESET, OP_SETF, OP_CLRF, OP_SETB, OP_CLRB, OP_CSTORE, OP_NOISE = 1, 2, 3, 4, 5, 6, 7, 8, 9
# classical expression ops of include/qsv.h (QSV_C_*)
(C_END, C_IMM, C_BITS, C_NEG, C_NOT, C_LNOT, C_ADD, C_SUB, C_MUL, C_DIV, C_MOD, C_AND, C_OR, C_XOR, C_SHL, C_SHR,
 C_EQ, C_NE, C_LT, C_GT, C_LE, C_GE, C_LAND, C_LOR) = range(24)
_C_UNARY = {"-": C_NEG, "~": C_NOT, "!": C_LNOT}
_C_BINARY = {"+": C_ADD, "-": C_SUB, "*": C_MUL, "/": C_DIV, "%": C_MOD, "&": C_AND, "|": C_OR, "^": C_XOR,
             "<<": C_SHL, ">>": C_SHR, "==": C_EQ, "!=": C_NE, "<": C_LT, ">": C_GT, "<=": C_LE, ">=": C_GE,
             "&&": C_LAND, "||": C_LOR}
C_STACK = 16
_BOOLEAN_OPS = ("==", "!=", "<", ">", "<=", ">=", "&&", "||")


def _i64(v):
    """v as a signed 64-bit two's-complement value."""
    v = int(v) & 0xFFFFFFFFFFFFFFFF
    return v - (1 << 64) if v >= 1 << 63 else v


def _fold_unary(op, a):
    return {"-": _i64(-a), "~": _i64(~a), "!": int(a == 0)}[op]


def _fold_binary(op, a, b):
    """The device's 64-bit classical arithmetic on two constants."""
    if op in ("/", "%"):
        if b == 0:
            return 0
        q = abs(a) // abs(b)
        if (a < 0) != (b < 0):
            q = -q
        return _i64(q if op == "/" else a - q * b)
    if op == "<<":
        return _i64(a << b) if 0 <= b < 64 else 0
    if op == ">>":
        return a >> b if 0 <= b < 64 else (-1 if a < 0 else 0)
    table = {"+": lambda: a + b, "-": lambda: a - b, "*": lambda: a * b, "&": lambda: a & b,
             "|": lambda: a | b, "^": lambda: a ^ b, "==": lambda: a == b, "!=": lambda: a != b,
             "<": lambda: a < b, ">": lambda: a > b, "<=": lambda: a <= b, ">=": lambda: a >= b,
             "&&": lambda: a != 0 and b != 0, "||": lambda: a != 0 or b != 0}
    return _i64(int(table[op]()))
(G_ID, G_X, G_Y, G_Z, G_H, G_S, G_SDG, G_T, G_TDG, G_SX, G_SXDG, G_RX, G_RY, G_RZ, G_P, G_U,
 G_CX, G_CY, G_CZ, G_CH, G_SWAP, G_CP, G_CRX, G_CRY, G_CRZ) = range(25)
CMP_EQ, CMP_NE, CMP_LT, CMP_GT, CMP_LE, CMP_GE, CMP_TRUE = range(7)
NONE32 = 0xFFFFFFFF
MAX_QUBITS = 34
MAX_INSTRUCTIONS = 20_000_000

INSTR_DTYPE = np.dtype({
    "names": ["op", "kind", "reserved", "q0", "q1", "cbit", "pred", "flag", "guard", "param",
              "reserved2", "scale", "offset"],
    "formats": [np.uint8, np.uint8, np.uint16, np.uint32, np.uint32, np.uint32, np.uint32, np.uint32,
                np.uint64, (np.uint32, 3), np.uint32, (np.float64, 3), (np.float64, 3)],
    "offsets": [0, 1, 2, 4, 8, 12, 16, 20, 24, 32, 44, 48, 72],
    "itemsize": 96})
PRED_DTYPE = np.dtype({"names": ["lo", "width", "value", "cmp", "reserved"],
                       "formats": [np.uint32, np.uint32, np.uint64, np.uint32, np.uint32],
                       "offsets": [0, 4, 8, 16, 20], "itemsize": 24})
CMP_EXPR = 7
LIN_DTYPE = np.dtype({"names": ["out", "in", "coef"], "formats": [np.uint32, np.uint32, np.float64],
                      "offsets": [0, 4, 8], "itemsize": 16})
# qsv_noise: the first three Philox counter words of one depolarizing draw
NOISE_DTYPE = np.dtype({"names": ["ctr"], "formats": [(np.uint64, 3)], "offsets": [0], "itemsize": 24})
COP_DTYPE = np.dtype({"names": ["op", "sgn", "width", "lo", "imm"],
                      "formats": [np.uint8, np.uint8, np.uint16, np.uint32, np.int64],
                      "offsets": [0, 1, 2, 4, 8], "itemsize": 16})

# name -> (kind, qubits, angles); u2 is U with theta fixed to pi/2
_GATES = {
    "id": (G_ID, 1, 0), "x": (G_X, 1, 0), "y": (G_Y, 1, 0), "z": (G_Z, 1, 0), "h": (G_H, 1, 0),
    "s": (G_S, 1, 0), "sdg": (G_SDG, 1, 0), "t": (G_T, 1, 0), "tdg": (G_TDG, 1, 0),
    "sx": (G_SX, 1, 0), "sxdg": (G_SXDG, 1, 0),
    "rx": (G_RX, 1, 1), "ry": (G_RY, 1, 1), "rz": (G_RZ, 1, 1),
    "p": (G_P, 1, 1), "phase": (G_P, 1, 1), "u1": (G_P, 1, 1),
    "u": (G_U, 1, 3), "U": (G_U, 1, 3), "u3": (G_U, 1, 3), "u2": (G_U, 1, 2),
    "cx": (G_CX, 2, 0), "CX": (G_CX, 2, 0), "cnot": (G_CX, 2, 0), "cy": (G_CY, 2, 0),
    "cz": (G_CZ, 2, 0), "ch": (G_CH, 2, 0), "swap": (G_SWAP, 2, 0),
    "cp": (G_CP, 2, 1), "cphase": (G_CP, 2, 1), "crx": (G_CRX, 2, 1), "cry": (G_CRY, 2, 1),
    "crz": (G_CRZ, 2, 1),
}
_NAMED_CONSTANTS = {"pi": math.pi, "π": math.pi, "tau": 2.0 * math.pi, "τ": 2.0 * math.pi,
                    "euler": math.e, "ℇ": math.e}
_NEGATE = {CMP_EQ: CMP_NE, CMP_NE: CMP_EQ, CMP_LT: CMP_GE, CMP_GE: CMP_LT, CMP_GT: CMP_LE,
           CMP_LE: CMP_GT}
_CMP = {"==": CMP_EQ, "!=": CMP_NE, "<": CMP_LT, ">": CMP_GT, "<=": CMP_LE, ">=": CMP_GE}


class Affine:
    """c + sum_k coef_k * theta[k] (only affine dependence on parameters is representable)."""

    __slots__ = ("c", "terms")

    def __init__(self, c=0.0, terms=None):
        self.c = c
        self.terms = terms or {}

    def is_const(self):
        return not self.terms

    def __repr__(self):
        return f"Affine({self.c}, {self.terms})"


def _aff_scale(a, s):
    return Affine(a.c * s, {k: v * s for k, v in a.terms.items()})


def _aff_sum(*parts):
    """sum of (coefficient, Affine) pairs"""
    c, terms = 0.0, {}
    for s, a in parts:
        c += s * a.c
        for k, v in a.terms.items():
            terms[k] = terms.get(k, 0.0) + s * v
    return Affine(c, terms)


# Gate modifiers lower to standard gates. Inverses of the standard gates:
_SELF_INVERSE = {"id", "x", "y", "z", "h", "cx", "CX", "cnot", "cy", "cz", "ch", "swap"}
_INVERSE_NAME = {"s": "sdg", "sdg": "s", "t": "tdg", "tdg": "t", "sx": "sxdg", "sxdg": "sx"}
_NEGATED_ANGLE = {"rx", "ry", "rz", "p", "phase", "u1", "cp", "cphase", "crx", "cry", "crz"}
# a single control on a one-qubit gate
_CONTROLLED = {"x": "cx", "y": "cy", "z": "cz", "h": "ch", "rx": "crx", "ry": "cry", "rz": "crz",
               "p": "cp", "phase": "cp", "u1": "cp"}
_CONTROLLED_PHASE = {"s": math.pi / 2.0, "sdg": -math.pi / 2.0, "t": math.pi / 4.0, "tdg": -math.pi / 4.0}


def _inverse(g):
    """The inverse of one standard gate (name, angles, qubits)."""
    name, a, qs = g
    if name in _SELF_INVERSE:
        return g
    if name in _INVERSE_NAME:
        return (_INVERSE_NAME[name], a, qs)
    if name in _NEGATED_ANGLE:
        return (name, [_aff_scale(a[0], -1.0)], qs)
    if name in ("u", "U", "u3"):  # U(t, p, l)^dag = U(-t, -l, -p)
        return ("U", [_aff_scale(a[0], -1.0), _aff_scale(a[2], -1.0), _aff_scale(a[1], -1.0)], qs)
    if name == "u2":
        return ("U", [Affine(-math.pi / 2.0), _aff_scale(a[1], -1.0), _aff_scale(a[0], -1.0)], qs)
    raise F.QasmError(f"no inverse for gate {name}")


def _two_qubit_parts(g):
    """A two-qubit standard gate as one-qubit gates and CX, exactly (no global
    phase): CZ = H CX H, CY = S CX S^dag, CH = RY(pi/4) CX RY(-pi/4) on the
    target (X RY(pi/2) = H), controlled RY/RZ(t) = R(t/2) CX R(-t/2) CX on the
    target (X R(a) X = R(-a)), CRX = H CRZ H, CP(l) = P(l/2) on the control
    and P(l/2) CX P(-l/2) CX on the target, SWAP = three CX."""
    name, a, (c, t) = g
    half, neg_half = (_aff_scale(a[0], 0.5), _aff_scale(a[0], -0.5)) if a else (None, None)
    if name in ("cx", "CX", "cnot"):
        return [("cx", [], [c, t])]
    if name == "cz":
        return [("h", [], [t]), ("cx", [], [c, t]), ("h", [], [t])]
    if name == "cy":
        return [("sdg", [], [t]), ("cx", [], [c, t]), ("s", [], [t])]
    if name == "ch":
        return [("ry", [Affine(math.pi / 4.0)], [t]), ("cx", [], [c, t]), ("ry", [Affine(-math.pi / 4.0)], [t])]
    if name == "swap":
        return [("cx", [], [c, t]), ("cx", [], [t, c]), ("cx", [], [c, t])]
    if name in ("cry", "crz"):
        r = name[1:]  # "ry" / "rz"
        return [(r, [half], [t]), ("cx", [], [c, t]), (r, [neg_half], [t]), ("cx", [], [c, t])]
    if name == "crx":
        return ([("h", [], [t])] + _two_qubit_parts(("crz", a, [c, t])) + [("h", [], [t])])
    if name in ("cp", "cphase"):
        return [("p", [half], [c]), ("p", [half], [t]), ("cx", [], [c, t]), ("p", [neg_half], [t]),
                ("cx", [], [c, t])]
    raise F.QasmError(f"no decomposition for gate {name}")


def _toffoli(c1, c2, t):
    """CCX from one-qubit gates and six CX (the standard exact circuit: H on
    the target, T / T^dag phases, and a final CX / phase correction on the
    controls)."""
    return [("h", [], [t]), ("cx", [], [c2, t]), ("tdg", [], [t]), ("cx", [], [c1, t]), ("t", [], [t]),
            ("cx", [], [c2, t]), ("tdg", [], [t]), ("cx", [], [c1, t]), ("t", [], [c2]), ("t", [], [t]),
            ("h", [], [t]), ("cx", [], [c1, c2]), ("t", [], [c1]), ("tdg", [], [c2]), ("cx", [], [c1, c2])]


def _controlled_seq(seq, c):
    """A sequence of standard gates with one more control qubit c: one-qubit
    gates by their controlled forms, two-qubit gates through their CX
    decomposition, each controlled CX as a Toffoli."""
    out = []
    for g in seq:
        if len(g[2]) == 1:
            out += _controlled(g, c)
            continue
        for part in _two_qubit_parts(g):
            out += _toffoli(c, *part[2]) if part[0] == "cx" else _controlled(part, c)
    return out


def _expand_controls(chain):
    """ctrl(k) @ / negctrl(k) @ as k single controls (they take the leading operands in order)."""
    out = []
    for kind, v in chain:
        if kind in ("ctrl", "negctrl"):
            if v < 1:
                raise F.QasmError(f"{kind}({v}) @ needs at least one control")
            out += [(kind, 1)] * v
        else:
            out.append((kind, v))
    return out


def _controlled(g, c):
    """Standard gates applying |0><0| (x) I + |1><1| (x) g with control qubit c,
    for a one-qubit standard gate g."""
    name, a, qs = g
    t = qs[0]
    if name == "id":
        return []
    if name in _CONTROLLED:
        return [(_CONTROLLED[name], a, [c, t])]
    if name in _CONTROLLED_PHASE:
        return [("cp", [Affine(_CONTROLLED_PHASE[name])], [c, t])]
    if name in ("sx", "sxdg"):  # SX = e^{i pi/4} RX(pi/2): the phase moves to the control
        sgn = 1.0 if name == "sx" else -1.0
        return [("p", [Affine(sgn * math.pi / 4.0)], [c]), ("crx", [Affine(sgn * math.pi / 2.0)], [c, t])]
    if name in ("u", "U", "u3", "u2"):
        th, ph, la = (a if name != "u2" else [Affine(math.pi / 2.0)] + list(a))
        return [("p", [_aff_sum((0.5, la), (0.5, ph))], [c]),
                ("p", [_aff_sum((0.5, la), (-0.5, ph))], [t]),
                ("cx", [], [c, t]),
                ("U", [_aff_scale(th, -0.5), Affine(0.0), _aff_sum((-0.5, ph), (-0.5, la))], [t]),
                ("cx", [], [c, t]),
                ("U", [_aff_scale(th, 0.5), ph, Affine(0.0)], [t])]
    raise F.QasmError(f"ctrl @ {name} is not supported")


def _aff_add(a, b, sign):
    terms = dict(a.terms)
    for k, v in b.terms.items():
        terms[k] = terms.get(k, 0.0) + sign * v
    return Affine(a.c + sign * b.c if sign > 0 else a.c - b.c, {k: v for k, v in terms.items()})


class LoweredProgram:
    """The flat instruction stream plus the symbol layout it was lowered with."""

    def __init__(self, n_qubits, n_clbits, n_params, instr, pred, qregs, cregs, inputs, code=None, lin=None,
                 n_derived=0, noise=None):
        self.n_qubits, self.n_clbits, self.n_params = n_qubits, n_clbits, n_params
        self.instr, self.pred = instr, pred
        self.code = np.zeros(0, COP_DTYPE) if code is None else code
        self.lin = np.zeros(0, LIN_DTYPE) if lin is None else lin
        self.n_derived = n_derived
        self.noise = np.zeros(0, NOISE_DTYPE) if noise is None else noise
        self.qregs, self.cregs, self.inputs = qregs, cregs, inputs

    @property
    def is_unitary(self):
        return bool(np.all(self.instr["op"] == OP_GATE)) if len(self.instr) else True

    @property
    def n_measure(self):
        return int(np.sum(self.instr["op"] == OP_MEASURE))


class _LoopCtx:
    def __init__(self, brk, cont):
        self.brk, self.cont = brk, cont


class _Lowerer:
    def __init__(self, noise=False):
        self.with_noise = noise     # emit a depolarizing slot per operand after each gate application
        self.noise = []             # (sid, loop code, 64 j + k) of each slot
        self.loop_ords = []         # iteration ordinal of each enclosing for loop, outermost first
        self.rows = []
        self.preds, self.pred_ids = [], {}
        self.code = []              # classical expression code (postfix), expressions end with C_END
        self.derived, self.derived_ids = [], {}  # derived parameters: sorted ((slot, coef), ...)
        self.qregs, self.cregs, self.inputs = {}, {}, {}
        self.csigned = {}           # classical register or variable -> read as two's complement
        self.consts, self.gatedefs = {}, {}
        self.nq = self.nc = self.npar = 0
        # free flags, least recently released first: consecutive ifs take
        # different flags, so the planner can move an if's flag updates over
        # the gates of the if before it (gates whose guards read other flags)
        self.free = collections.deque(range(64))

    # -- flags --
    def _alloc(self):
        if not self.free:
            raise F.QasmError("control flow nested too deeply (more than 64 live flags)")
        return self.free.popleft()

    def _release(self, f):
        self.free.append(f)

    # -- emission --
    def _emit(self, op, guard, kind=0, q0=NONE32, q1=NONE32, cbit=NONE32, pred=NONE32, flag=0,
              angles=()):
        if len(self.rows) >= MAX_INSTRUCTIONS:
            raise F.QasmError("program unrolls to too many instructions")
        param, scale, offset = [NONE32] * 3, [0.0] * 3, [0.0] * 3
        for k, a in enumerate(angles):
            offset[k] = float(a.c)
            terms = {s_: float(c) for s_, c in a.terms.items() if c != 0.0}
            if len(terms) > 1:
                key = tuple(sorted(terms.items()))
                if key not in self.derived_ids:
                    self.derived_ids[key] = len(self.derived)
                    self.derived.append(key)
                param[k], scale[k] = self.npar + self.derived_ids[key], 1.0
            for slot, coef in terms.items() if len(terms) == 1 else ():
                param[k], scale[k] = slot, coef
        self.rows.append((op, kind, 0, q0, q1, cbit, pred, flag, guard, tuple(param), 0,
                          tuple(scale), tuple(offset)))

    def _pred(self, lo, width, value, cmp):
        key = (lo, width, value, cmp)
        if key not in self.pred_ids:
            self.pred_ids[key] = len(self.preds)
            self.preds.append((lo, width, value, cmp, 0))
        return self.pred_ids[key]

    # -- expressions --
    def value(self, e, env):
        if isinstance(e, F.Num):
            return Affine(e.value)
        if isinstance(e, F.Name):
            if e.ident in env:
                v = env[e.ident]
                if isinstance(v, Affine):
                    return v
                if isinstance(v, (int, float)):
                    return Affine(v)
                raise F.QasmError(f"{e.ident} is a qubit, not a value")
            if e.ident in self.consts:
                return self.consts[e.ident]
            if e.ident in _NAMED_CONSTANTS:
                return Affine(_NAMED_CONSTANTS[e.ident])
            if e.ident in self.inputs:
                off, size, scalar = self.inputs[e.ident]
                if not scalar:
                    raise F.QasmError(f"input array {e.ident} needs an index")
                return Affine(0.0, {off: 1.0})
            raise F.QasmError(f"undefined name {e.ident}")
        if isinstance(e, F.Subscript):
            if e.ident not in self.inputs:
                raise F.QasmError(f"{e.ident} cannot be indexed in an expression")
            off, size, scalar = self.inputs[e.ident]
            i = self.const_int(e.index, env)
            if not 0 <= i < size:
                raise F.QasmError(f"index {i} out of range for {e.ident}")
            return Affine(0.0, {off + i: 1.0})
        if isinstance(e, F.Unary):
            a = self.value(e.arg, env)
            return Affine(-a.c, {k: -v for k, v in a.terms.items()})
        if isinstance(e, F.Binary):
            a, b = self.value(e.lhs, env), self.value(e.rhs, env)
            if e.op == "+":
                return _aff_add(a, b, +1)
            if e.op == "-":
                return _aff_add(a, b, -1)
            if e.op == "*":
                if a.is_const():
                    return Affine(a.c * b.c, {k: a.c * v for k, v in b.terms.items()})
                if b.is_const():
                    return Affine(a.c * b.c, {k: v * b.c for k, v in a.terms.items()})
                raise F.QasmError("product of two parameter-dependent values is not affine")
            if e.op == "/":
                if not b.is_const():
                    raise F.QasmError("division by a parameter-dependent value is not affine")
                return Affine(a.c / b.c, {k: v / b.c for k, v in a.terms.items()})
            if not (a.is_const() and b.is_const()):
                raise F.QasmError(f"operator {e.op} needs constant operands")
            return Affine(a.c % b.c if e.op == "%" else a.c ** b.c)
        if isinstance(e, F.Call):
            a = self.value(e.args[0], env)
            if not a.is_const():
                raise F.QasmError(f"{e.fn} of a parameter-dependent value is not affine")
            fn = {"sin": math.sin, "cos": math.cos, "tan": math.tan, "exp": math.exp, "ln": math.log,
                  "sqrt": math.sqrt, "arcsin": math.asin, "arccos": math.acos, "arctan": math.atan}[e.fn]
            return Affine(fn(a.c))
        raise F.QasmError(f"unsupported expression {e!r}")

    def const_int(self, e, env):
        a = self.value(e, env)
        if not a.is_const():
            raise F.QasmError("expected a compile-time integer")
        v = a.c
        if float(v) != float(int(round(v))):
            raise F.QasmError(f"expected an integer, got {v}")
        return int(round(v))

    # -- operands --
    def qubits(self, opd, env):
        if opd.reg in env and isinstance(env[opd.reg], tuple) and env[opd.reg][0] == "q":
            if opd.index is not None:
                raise F.QasmError("gate arguments cannot be indexed")
            return [env[opd.reg][1]]
        if opd.reg not in self.qregs:
            raise F.QasmError(f"unknown qubit register {opd.reg}")
        off, size = self.qregs[opd.reg]
        if opd.index is None:
            return list(range(off, off + size))
        i = self.const_int(opd.index, env)
        if not 0 <= i < size:
            raise F.QasmError(f"qubit index {i} out of range for {opd.reg}")
        return [off + i]

    def clbits(self, opd, env):
        if opd.reg not in self.cregs:
            raise F.QasmError(f"unknown classical register {opd.reg}")
        off, size = self.cregs[opd.reg]
        if opd.index is None:
            return list(range(off, off + size))
        i = self.const_int(opd.index, env)
        if not 0 <= i < size:
            raise F.QasmError(f"bit index {i} out of range for {opd.reg}")
        return [off + i]

    # -- classical expressions --
    def cfold(self, e, env):
        """The value of a classical expression that reads no classical bits
        (numbers, constants, loop variables), else None."""
        if isinstance(e, F.CNum):
            return _i64(e.value)
        if isinstance(e, F.CRef):
            o = e.operand
            if o.reg in self.cregs:
                return None
            if o.index is not None:
                raise F.QasmError(f"{o.reg} cannot be indexed in a classical expression")
            return _i64(self.const_int(F.Name(o.reg), env))
        if isinstance(e, F.CUn):
            a = self.cfold(e.arg, env)
            return None if a is None else _fold_unary(e.op, a)
        a, b = self.cfold(e.lhs, env), self.cfold(e.rhs, env)
        return None if a is None or b is None else _fold_binary(e.op, a, b)

    def cread(self, opd, env):
        """(first bit, width, signed) of a register, variable or bit read in an expression."""
        bits = self.clbits(opd, env)
        if len(bits) > 64:
            raise F.QasmError("classical values hold at most 64 bits")
        if any(b != bits[0] + i for i, b in enumerate(bits)):
            raise F.QasmError("classical bits must be contiguous")
        return bits[0], len(bits), opd.index is None and self.csigned.get(opd.reg, False)

    def ccode(self, e, env):
        """Appends e's postfix code; returns where it starts."""
        start = len(self.code)
        depth = self._cgen(e, env, 0)
        if depth > C_STACK:
            raise F.QasmError(f"classical expression needs a stack deeper than {C_STACK}")
        self.code.append((C_END, 0, 0, 0, 0))
        return start

    def _cgen(self, e, env, depth):
        """Emits e; returns the deepest stack it uses (depth values below it)."""
        v = self.cfold(e, env)
        if v is not None:
            self.code.append((C_IMM, 0, 0, 0, v))
            return depth + 1
        if isinstance(e, F.CRef):
            lo, width, signed = self.cread(e.operand, env)
            self.code.append((C_BITS, int(signed), width, lo, 0))
            return depth + 1
        if isinstance(e, F.CUn):
            d = self._cgen(e.arg, env, depth)
            self.code.append((_C_UNARY[e.op], 0, 0, 0, 0))
            return d
        d1 = self._cgen(e.lhs, env, depth)
        d2 = self._cgen(e.rhs, env, depth + 1)
        self.code.append((_C_BINARY[e.op], 0, 0, 0, 0))
        return max(d1, d2)

    # -- conditions --
    def leaf(self, e, env):
        """(lo, width, value, cmp) when the device can test e as a plain
        predicate: an unsigned register, variable or bit of at most 63 bits,
        alone (nonzero) or compared with a constant in 0..2^63-1; else None."""
        if isinstance(e, F.CRef) and e.operand.reg in self.cregs:
            lo, width, signed = self.cread(e.operand, env)
            return (lo, width, 0, CMP_NE) if width <= 63 else None
        if isinstance(e, F.CBin) and e.op in _CMP and isinstance(e.lhs, F.CRef) and e.lhs.operand.reg in self.cregs:
            lo, width, signed = self.cread(e.lhs.operand, env)
            v = self.cfold(e.rhs, env)
            if signed or width > 63 or v is None or v < 0:
                return None
            return lo, width, v, _CMP[e.op]
        return None

    def simple(self, e, env):
        """e as one predicate (a leaf under any number of `!`), or None."""
        if isinstance(e, F.CUn) and e.op == "!":
            r = self.simple(e.arg, env)
            return None if r is None else (r[0], r[1], r[2], _NEGATE[r[3]])
        return self.leaf(e, env)

    def cond_guards(self, c, env, guard, flags):
        """Guards (lists of masks) under `guard` where c holds and where it fails.
        The masks of each list are disjoint and together cover exactly those
        shots; every flag they use is set by a SETF emitted here, in order."""
        if isinstance(c, F.CUn) and c.op == "!":
            yes, no = self.cond_guards(c.arg, env, guard, flags)
            return no, yes
        if isinstance(c, F.CBin) and c.op in ("&&", "||"):
            yes_l, no_l = self.cond_guards(c.lhs, env, guard, flags)
            # "and" needs the right side only where the left holds, "or" only where it fails
            rest = yes_l if c.op == "&&" else no_l
            yes, no = ([], list(no_l)) if c.op == "&&" else (list(yes_l), [])
            for g in rest:
                y, n = self.cond_guards(c.rhs, env, g, flags)
                yes += y
                no += n
            return yes, no
        lf = self.leaf(c, env)
        if lf is not None:
            p_yes = self._pred(*lf)
            p_no = self._pred(lf[0], lf[1], lf[2], _NEGATE[lf[3]])
        else:
            # computed on the device: predicates on the expression and on its negation
            p_yes = self._pred(0, 0, self.ccode(c, env), CMP_EXPR)
            p_no = self._pred(0, 0, self.ccode(F.CUn("!", c), env), CMP_EXPR)
        ft, ff = self._alloc(), self._alloc()
        flags += [ft, ff]
        self._emit(OP_SETF, guard, pred=p_yes, flag=ft)
        self._emit(OP_SETF, guard, pred=p_no, flag=ff)
        return [guard | (1 << ft)], [guard | (1 << ff)]

    def assign(self, st, env, guard):
        """Classical assignment: the target takes the low bits of the right
        side's 64-bit two's-complement value. Constants become set/clear-bit
        instructions, a register copy of equal width a per-bit copy, one bit
        from a condition the condition's guards; anything else is evaluated on
        the device (CSTORE). Every read of the right side happens before the
        first bit is written."""
        bits = self.clbits(st.target, env)
        e = st.expr
        v = self.cfold(e, env)
        if v is not None:
            for i, b in enumerate(bits):
                self._emit(OP_SETB if (v >> i) & 1 else OP_CLRB, guard, cbit=b)
            return
        if isinstance(e, F.CRef) and e.operand.reg in self.cregs:
            src = self.clbits(e.operand, env)
            if src == bits:
                return
            if len(src) == len(bits) and not set(src) & set(bits):
                # distinct registers do not overlap: each bit is read and written in turn
                for s_, b in zip(src, bits):
                    f = self._alloc()
                    self._emit(OP_SETF, guard, pred=self._pred(s_, 1, 0, _CMP["!="]), flag=f)
                    self._emit(OP_CLRB, guard, cbit=b)
                    self._emit(OP_SETB, guard | (1 << f), cbit=b)
                    self._release(f)
                return
        boolean = (isinstance(e, F.CBin) and e.op in _BOOLEAN_OPS) or (isinstance(e, F.CUn) and e.op == "!")
        if len(bits) == 1 and (boolean or isinstance(e, F.CRef)):
            flags = []
            yes, no = self.cond_guards(e, env, guard, flags)
            for g in yes:
                self._emit(OP_SETB, g, cbit=bits[0])
            for g in no:
                self._emit(OP_CLRB, g, cbit=bits[0])
            for f in reversed(flags):
                self._release(f)
            return
        if any(b != bits[0] + i for i, b in enumerate(bits)) or len(bits) > 64:
            raise F.QasmError("an assigned value needs at most 64 contiguous bits")
        self._emit(OP_CSTORE, guard, cbit=bits[0], pred=self.ccode(e, env), flag=len(bits))

    # -- statements --
    def program(self, stmts):
        body = []
        for st in stmts:
            if isinstance(st, F.Declare):
                table = self.qregs if st.kind == "qubit" else self.cregs
                if st.name in table:
                    raise F.QasmError(f"{st.name} declared twice")
                size = 1 if st.size is None else st.size
                if st.kind == "qubit":
                    table[st.name] = (self.nq, size)
                    self.nq += size
                else:
                    # bit registers and classical variables share the flat array
                    table[st.name] = (self.nc, size)
                    self.csigned[st.name] = st.kind == "int"
                    self.nc += size
            elif isinstance(st, F.InputDecl):
                size = 1 if st.size is None else st.size
                self.inputs[st.name] = (self.npar, size, st.size is None)
                self.npar += size
            elif isinstance(st, F.ConstDecl):
                self.consts[st.name] = self.value(st.value, {})
            elif isinstance(st, F.GateDef):
                self.gatedefs[st.name] = st
            else:
                body.append(st)
        if self.nq < 1:
            raise F.QasmError("program declares no qubits")
        if self.nq > MAX_QUBITS:
            raise F.QasmError(f"{self.nq} qubits exceed the {MAX_QUBITS}-qubit limit of one GPU")
        self.block(body, {}, 0, None)

    def block(self, body, env, guard, loop):
        for st in body:
            self.statement(st, env, guard, loop)

    def statement(self, st, env, guard, loop):
        if isinstance(st, F.GateCall):
            self.gate(st, env, guard)
        elif isinstance(st, F.Measure):
            qs = self.qubits(st.qubits, env)
            cs = self.clbits(st.target, env) if st.target is not None else [NONE32] * len(qs)
            if len(qs) != len(cs):
                raise F.QasmError("measure: register sizes differ")
            for q, c in zip(qs, cs):
                self._emit(OP_MEASURE, guard, q0=q, cbit=c)
        elif isinstance(st, F.Reset):
            for q in self.qubits(st.qubits, env):
                self._emit(OP_RESET, guard, q0=q)
        elif isinstance(st, F.Assign):
            self.assign(st, env, guard)
        elif isinstance(st, F.IfStmt) and self.simple(st.cond, env) is None:
            # `&&` / `||` or a computed condition: disjoint guards (one per way
            # it can hold, one per way it can fail), each a flag set when the if
            # executes; a body is emitted once under each of its guards
            flags = []
            yes, no = self.cond_guards(st.cond, env, guard, flags)
            for g in yes:
                self.block(st.then_body, env, g, loop)
            if st.else_body:
                for g in no:
                    self.block(st.else_body, env, g, loop)
            for f in reversed(flags):
                self._release(f)
        elif isinstance(st, F.IfStmt):
            lo, width, value, cmp = self.simple(st.cond, env)
            ft = self._alloc()
            self._emit(OP_SETF, guard, pred=self._pred(lo, width, value, cmp), flag=ft)
            fe = None
            if st.else_body:
                fe = self._alloc()
                self._emit(OP_SETF, guard, pred=self._pred(lo, width, value, _NEGATE[cmp]), flag=fe)
            self.block(st.then_body, env, guard | (1 << ft), loop)
            if fe is not None:
                self.block(st.else_body, env, guard | (1 << fe), loop)
                self._release(fe)
            self._release(ft)
        elif isinstance(st, F.ForStmt):
            self.for_loop(st, env, guard)
        elif isinstance(st, F.Break):
            if loop is None:
                raise F.QasmError("break outside a loop")
            self._emit(OP_CLRF, guard, flag=loop.brk)
        elif isinstance(st, F.Continue):
            if loop is None:
                raise F.QasmError("continue outside a loop")
            self._emit(OP_CLRF, guard, flag=loop.cont)
        elif isinstance(st, (F.Declare, F.InputDecl, F.GateDef, F.ConstDecl)):
            raise F.QasmError("declarations are only allowed at the top level")
        else:
            raise F.QasmError(f"unsupported statement {type(st).__name__}")

    def for_loop(self, st, env, guard):
        a, step, b = (self.const_int(x, env) for x in (st.start, st.step, st.stop))
        if step == 0:
            raise F.QasmError("for loop with a zero step")
        values = list(range(a, b + 1, step)) if step > 0 else list(range(a, b - 1, step))
        has_brk, has_cont = _contains(st.body, F.Break), _contains(st.body, F.Continue)
        fb = self._alloc() if has_brk else None
        fc = self._alloc() if has_cont else None
        g = guard
        if fb is not None:
            self._emit(OP_SETF, guard, pred=self._pred(0, 0, 0, CMP_TRUE), flag=fb)
            g |= 1 << fb
        self.loop_ords.append(0)
        for ordinal, v in enumerate(values):
            inner = dict(env)
            inner[st.var] = v
            gi = g
            if fc is not None:
                self._emit(OP_SETF, g, pred=self._pred(0, 0, 0, CMP_TRUE), flag=fc)
                gi |= 1 << fc
            self.loop_ords[-1] = ordinal
            self.block(st.body, inner, gi, _LoopCtx(fb, fc))
        self.loop_ords.pop()
        for f in (fc, fb):
            if f is not None:
                self._release(f)

    def gate(self, st, env, guard):
        angles = [self.value(a, env) for a in st.args]
        lists = [self.qubits(o, env) for o in st.operands]
        width = max(len(x) for x in lists)
        if any(len(x) not in (1, width) for x in lists):
            raise F.QasmError(f"gate {st.name}: register operands of different sizes")
        for j in range(width):
            qs = [x[j] if len(x) > 1 else x[0] for x in lists]
            if len(set(qs)) != len(qs):
                raise F.QasmError(f"gate {st.name}: a qubit appears twice")
            if st.mods:
                chain = []
                for kind, arg in st.mods:
                    v = 1 if arg is None else self.const_int(arg, env)
                    if kind == "pow" and arg is None:
                        raise F.QasmError("pow @ needs an exponent")
                    chain.append((kind, v))
                for name, a, q in self.modified(_expand_controls(chain), st.name, angles, qs):
                    self.apply(name, a, q, guard)
            else:
                self.apply(st.name, angles, qs, guard)
            if self.with_noise and st.sid is not None:
                self.noise_slots(st.sid, j, qs, guard)

    def noise_slots(self, sid, j, qs, guard):
        """After application j of gate statement sid: one depolarizing slot per
        operand k, whose draw has counter (sid, loop code, 64 j + k, 1); the
        loop code is sum_d ordinal_d * 2**(16 d) over the enclosing loops."""
        if len(self.loop_ords) > 4 or any(o >= 1 << 16 for o in self.loop_ords) or len(qs) > 64:
            raise F.QasmError("noise slots support at most 4 nested loops of at most 65536 iterations "
                              "and 64 operands")
        code = sum(o << (16 * d) for d, o in enumerate(self.loop_ords))
        for k, q in enumerate(qs):
            self.noise.append((sid, code, 64 * j + k))
            self._emit(OP_NOISE, guard, q0=q, pred=len(self.noise) - 1)

    def standard_gates(self, name, angles, qs):
        """The standard gates (name, angles, qubits) a gate call applies, in order."""
        if name not in self.gatedefs:
            if name not in _GATES:
                raise F.QasmError(f"unknown gate {name}")
            return [(name, list(angles), list(qs))]
        d = self.gatedefs[name]
        if len(d.params) != len(angles) or len(d.qargs) != len(qs):
            raise F.QasmError(f"gate {name}: wrong number of arguments")
        env = {p: a for p, a in zip(d.params, angles)}
        env.update({qa: ("q", q) for qa, q in zip(d.qargs, qs)})
        out = []
        for st in d.body:
            if not isinstance(st, F.GateCall):
                raise F.QasmError(f"gate {name}: only gate calls may appear in a gate body")
            a = [self.value(x, env) for x in st.args]
            q = [self.qubits(o, env)[0] for o in st.operands]
            if st.mods:
                chain = [(k, 1 if v is None else self.const_int(v, env)) for k, v in st.mods]
                out += self.modified(_expand_controls(chain), st.name, a, q)
            else:
                out += self.standard_gates(st.name, a, q)
        return out

    def modified(self, chain, name, angles, qs):
        """Standard gates of a modified gate call; chain lists the modifiers
        outermost first (controls take the leading operands)."""
        if not chain:
            return self.standard_gates(name, angles, qs)
        kind, v = chain[0]
        if kind == "inv":
            return [_inverse(g) for g in reversed(self.modified(chain[1:], name, angles, qs))]
        if kind == "pow":
            seq = self.modified(chain[1:], name, angles, qs)
            if v < 0:
                seq = [_inverse(g) for g in reversed(seq)]
            return seq * abs(v)
        if len(qs) < 2:
            raise F.QasmError(f"{kind} @ {name}: the controls leave no operand for the gate")
        c = qs[0]
        out = [("x", [], [c])] if kind == "negctrl" else []
        out += _controlled_seq(self.modified(chain[1:], name, angles, qs[1:]), c)
        if kind == "negctrl":
            out.append(("x", [], [c]))
        return out

    def apply(self, name, angles, qs, guard):
        if name in self.gatedefs:
            d = self.gatedefs[name]
            if len(d.params) != len(angles) or len(d.qargs) != len(qs):
                raise F.QasmError(f"gate {name}: wrong number of arguments")
            env = {p: a for p, a in zip(d.params, angles)}
            env.update({qa: ("q", q) for qa, q in zip(d.qargs, qs)})
            for st in d.body:
                if not isinstance(st, F.GateCall):
                    raise F.QasmError(f"gate {name}: only gate calls may appear in a gate body")
                self.gate(st, env, guard)
            return
        if name not in _GATES:
            raise F.QasmError(f"unknown gate {name}")
        kind, nq, na = _GATES[name]
        if len(qs) != nq:
            raise F.QasmError(f"gate {name} acts on {nq} qubit(s)")
        if len(angles) != na:
            raise F.QasmError(f"gate {name} takes {na} parameter(s)")
        if name == "u2":
            angles = [Affine(math.pi / 2.0)] + angles
        self._emit(OP_GATE, guard, kind=kind, q0=qs[0], q1=qs[1] if nq == 2 else NONE32, angles=angles)

    def result(self):
        instr = np.array(self.rows, dtype=INSTR_DTYPE) if self.rows else np.zeros(0, INSTR_DTYPE)
        pred = np.array(self.preds, dtype=PRED_DTYPE) if self.preds else np.zeros(0, PRED_DTYPE)
        code = np.array(self.code, dtype=COP_DTYPE) if self.code else np.zeros(0, COP_DTYPE)
        lin = [(k, slot, coef) for k, terms in enumerate(self.derived) for slot, coef in terms]
        lin = np.array(lin, dtype=LIN_DTYPE) if lin else np.zeros(0, LIN_DTYPE)
        noise = np.zeros(len(self.noise), NOISE_DTYPE)
        if self.noise:
            noise["ctr"] = np.array(self.noise, dtype=np.uint64)
        return LoweredProgram(self.nq, self.nc, self.npar, instr, pred, dict(self.qregs),
                              dict(self.cregs), dict(self.inputs), code, lin, len(self.derived), noise)


def _contains(body, cls):
    for st in body:
        if isinstance(st, cls):
            return True
        if isinstance(st, F.IfStmt) and (_contains(st.then_body, cls) or _contains(st.else_body, cls)):
            return True
    return False


def lower(source, noise=False):
    """OpenQASM 3 text (or a parsed statement list) -> LoweredProgram. With
    noise, every application of a gate statement is followed by one
    depolarizing slot (QSV_OP_NOISE) per qubit it acts on; the slots act only
    in calls with a positive depolarizing rate."""
    stmts = F.parse(source) if isinstance(source, str) else source
    lw = _Lowerer(noise)
    lw.program(stmts)
    return lw.result()
