"""Plain complex128 state-vector interpreter for OpenQASM 3 dynamic circuits.

TEST INFRASTRUCTURE ONLY. This is the oracle the GPU path is checked against.
Only tests, the smoke check and the benchmark's CPU-baseline leg may use it;
it shares no code with the product library and imports nothing from it.

It walks the oracle's own AST (``oracle.qasm``) statement by statement, the way
the paper's visitor walks the pyqasm AST (Methodology, kernel generation via
the AST visitor), but instead of emitting backend calls it executes them on a
dense state vector:

  * state: psi in C^(2^n), starting at |0...0> (the dynamic tests start every
    qubit in |0>, Experiments, dynamic circuit validation); index i = sum_q b_q 2^q;
  * gate: the matrix of the named gate applied to its operands (standard gates
    map one-to-one onto backend gates, Methodology, kernel generation);
  * measure q -> c[j]: p1 = sum |psi_i|^2 over b_q = 1, p0 likewise, N = p0 + p1,
    u from the shot's Philox stream, outcome 0 iff u < p0/N, collapse onto the
    outcome and renormalise by 1/sqrt(p_m) (mid-circuit measurement with
    feed-forward, Background, dynamic circuit testing; conditional-reset figure);
  * reset q: the same measurement (one draw, never forced, not recorded in the
    measurement record), then X if the outcome was 1;
  * if/else on a classical bit or a whole register compared with an integer
    (register value sum_i c[i] 2^i), decided per shot from the bits measured so
    far (Methodology, transpiling dynamic control flow: the body runs only
    when the predicate holds at run time);
  * for i in [a:b] (inclusive bounds) with break/continue: bounded loops;
  * input parameters: runtime values bound per call, compile-once/run-many
    (Background, parameter passing and VQE; Methodology, runtime parameters).

The state arithmetic sits in an "engine" object so that ``oracle.brute`` can run
the same walk on dense 2^n x 2^n operators and projectors as a cross-check.
"""
import math

import numpy as np

from . import gates as G
from .philox import ShotStream, noise_word, word_to_uniform
from .qasm import CONSTANTS, parse

# A forced outcome whose probability (relative to the current norm) is below
# this threshold aborts the shot: the collapse would divide by ~0.
FORCED_ZERO_PROB = 2.0 ** -60

STATUS_OK = 0
STATUS_FORCED_ZERO_PROB = -6


class OracleError(ValueError):
    pass


class _Break(Exception):
    pass


class _Continue(Exception):
    pass


class _Abort(Exception):
    pass


class Lin:
    """A real value together with its partial derivatives w.r.t. the input parameters."""

    __slots__ = ("v", "d")

    def __init__(self, v, d=None):
        self.v = float(v)
        self.d = d or {}

    @staticmethod
    def lift(x):
        return x if isinstance(x, Lin) else Lin(x)

    def _combine(self, o, fv, fa, fb):
        o = Lin.lift(o)
        d = {}
        for k, g in self.d.items():
            d[k] = d.get(k, 0.0) + fa * g
        for k, g in o.d.items():
            d[k] = d.get(k, 0.0) + fb * g
        return Lin(fv, d)

    def __add__(self, o):
        o = Lin.lift(o)
        return self._combine(o, self.v + o.v, 1.0, 1.0)

    def __sub__(self, o):
        o = Lin.lift(o)
        return self._combine(o, self.v - o.v, 1.0, -1.0)

    def __mul__(self, o):
        o = Lin.lift(o)
        return self._combine(o, self.v * o.v, o.v, self.v)

    def __truediv__(self, o):
        o = Lin.lift(o)
        return self._combine(o, self.v / o.v, 1.0 / o.v, -self.v / (o.v * o.v))

    def __neg__(self):
        return Lin(-self.v, {k: -g for k, g in self.d.items()})

    def __radd__(self, o):
        return Lin.lift(o) + self

    def __rsub__(self, o):
        return Lin.lift(o) - self

    def __rmul__(self, o):
        return Lin.lift(o) * self

    def __rtruediv__(self, o):
        return Lin.lift(o) / self

    def apply(self, f, df):
        return Lin(f(self.v), {k: df(self.v) * g for k, g in self.d.items()})


_FUNCS = {
    "sin": (math.sin, math.cos), "cos": (math.cos, lambda x: -math.sin(x)),
    "tan": (math.tan, lambda x: 1.0 / math.cos(x) ** 2), "exp": (math.exp, math.exp),
    "sqrt": (math.sqrt, lambda x: 0.5 / math.sqrt(x)), "ln": (math.log, lambda x: 1.0 / x),
    "arccos": (math.acos, lambda x: -1.0 / math.sqrt(1 - x * x)),
    "arcsin": (math.asin, lambda x: 1.0 / math.sqrt(1 - x * x)),
    "arctan": (math.atan, lambda x: 1.0 / (1 + x * x)),
}


# --------------------------------------------------------------------------
# State engine: tensor reshapes on the 2^n vector.
# --------------------------------------------------------------------------
class TensorEngine:
    """Applies k-qubit matrices by viewing psi as an n-way tensor of 2s."""

    def __init__(self, n):
        self.n = n
        self.psi = np.zeros(1 << n, dtype=np.complex128)
        self.psi[0] = 1.0

    def apply(self, m, qubits):
        n, k = self.n, len(qubits)
        t = self.psi.reshape((2,) * n)          # axis a holds qubit n-1-a
        axes = [n - 1 - q for q in reversed(qubits)]
        t = np.moveaxis(t, axes, list(range(k)))  # leading axes: q_{k-1} ... q_0
        shape = t.shape
        t = (m @ t.reshape(1 << k, -1)).reshape(shape)
        self.psi = np.moveaxis(t, list(range(k)), axes).reshape(-1).copy()

    def probs(self, q):
        v = self.psi.reshape(-1, 2, 1 << q)
        p0 = float(np.sum(np.abs(v[:, 0, :]) ** 2))
        p1 = float(np.sum(np.abs(v[:, 1, :]) ** 2))
        return p0, p1

    def collapse(self, q, m, p_m):
        v = self.psi.reshape(-1, 2, 1 << q)
        v[:, 1 - m, :] = 0.0
        v[:, m, :] *= 1.0 / math.sqrt(p_m)

    def flip(self, q):
        v = self.psi.reshape(-1, 2, 1 << q)
        self.psi = v[:, ::-1, :].reshape(-1).copy()


# --------------------------------------------------------------------------
# Program analysis: registers, inputs, constants, gate definitions.
# --------------------------------------------------------------------------
class Program:
    def __init__(self, source):
        self.ast = parse(source) if isinstance(source, str) else source
        self.qregs, self.cregs, self.inputs = {}, {}, {}
        self.signed = {}  # classical register or variable name -> read as two's complement
        self.consts, self.gatedefs = {}, {}
        self.n_qubits = self.n_clbits = self.n_params = 0
        self.body = []
        for st in self.ast:
            kind = st[0]
            if kind == "qubit":
                size = 1 if st[2] is None else st[2]
                self.qregs[st[1]] = (self.n_qubits, size, st[2] is None)
                self.n_qubits += size
            elif kind == "bit":
                size = 1 if st[2] is None else st[2]
                self.cregs[st[1]] = (self.n_clbits, size, st[2] is None)
                self.signed[st[1]] = False
                self.n_clbits += size
            elif kind == "var":
                # classical integer variables are bits too, in declaration order
                self.cregs[st[1]] = (self.n_clbits, st[2], False)
                self.signed[st[1]] = st[3]
                self.n_clbits += st[2]
            elif kind == "input":
                size = 1 if st[2] is None else st[2]
                self.inputs[st[1]] = (self.n_params, size, st[2] is None)
                self.n_params += size
            elif kind == "gatedef":
                self.gatedefs[st[1]] = st
            else:
                self.body.append(st)
        self._consts_pending = [st for st in self.body if st[0] == "const"]
        self.body = [st for st in self.body if st[0] != "const"]
        if self.n_qubits < 1:
            raise OracleError("program declares no qubits")
        self.is_unitary = not _has_nonunitary(self.body, self.gatedefs)


def _has_nonunitary(body, gatedefs):
    for st in body:
        if st[0] in ("measure", "reset", "if", "break", "continue"):
            return True
        if st[0] == "for" and _has_nonunitary(st[5], gatedefs):
            return True
    return False


# --------------------------------------------------------------------------
# Gate modifiers, by definition on matrices (operand i = bit i of the local
# index). A chain [(kind, value)] lists modifiers outermost first; they are
# applied innermost first. With a derivative dm of the base matrix, returns
# the derivative of the modified matrix as well.
#   inv:        M^dag                        d(M^dag) = (dM)^dag
#   pow(k):     M^k (k < 0: (M^dag)^|k|)     product rule
#   ctrl(n):    M where the n new leading operands are all 1, identity elsewhere
#   negctrl(n): the same where they are all 0
# --------------------------------------------------------------------------
def _controlled(m, n, on_one, fill):
    """The matrix of m with n controls as the first operands; `fill` is the
    value of the uncontrolled diagonal (1 for a matrix, 0 for a derivative)."""
    d = m.shape[0]
    big = np.zeros((d << n, d << n), dtype=np.complex128)
    if fill:
        np.fill_diagonal(big, fill)
    c = (1 << n) - 1 if on_one else 0
    for a in range(d):
        for b in range(d):
            big[(a << n) | c, (b << n) | c] = m[a, b]
    return big


def modify(chain, m, dm):
    for kind, v in reversed(list(chain)):
        if kind == "inv":
            m = m.conj().T
            dm = None if dm is None else dm.conj().T
        elif kind == "pow":
            base, dbase = (m, dm) if v >= 0 else (m.conj().T, None if dm is None else dm.conj().T)
            k = abs(v)
            pm = np.eye(m.shape[0], dtype=np.complex128)
            pd = None if dm is None else np.zeros_like(m)
            for _ in range(k):
                if pd is not None:
                    pd = pd @ base + pm @ dbase
                pm = pm @ base
            m, dm = pm, pd
        else:
            on_one = kind == "ctrl"
            m = _controlled(m, v, on_one, 1.0)
            dm = None if dm is None else _controlled(dm, v, on_one, 0.0)
    return m, dm


# --------------------------------------------------------------------------
# The tree-walking interpreter.
# --------------------------------------------------------------------------
class Interpreter:
    def __init__(self, program, theta=None, engine_cls=TensorEngine, with_derivs=False):
        self.prog = program if isinstance(program, Program) else Program(program)
        p = self.prog
        theta = np.zeros(0) if theta is None else np.asarray(theta, dtype=np.float64).reshape(-1)
        if theta.size != p.n_params:
            raise OracleError(f"program takes {p.n_params} parameters, got {theta.size}")
        self.theta = theta
        self.with_derivs = with_derivs
        self.engine_cls = engine_cls
        self.consts = {}
        for st in p._consts_pending:
            self.consts[st[1]] = self.eval(st[2], {})
        # per-gate angle overrides: {(gate_occurrence, angle_slot): delta}
        self.shift = {}
        self.tape = None

    # -- expressions --
    def eval(self, e, env):
        k = e[0]
        if k == "num":
            return Lin(e[1]) if self.with_derivs else float(e[1])
        if k == "id":
            name = e[1]
            if name in env:
                return env[name]
            if name in self.consts:
                return self.consts[name]
            if name in CONSTANTS:
                return Lin(CONSTANTS[name]) if self.with_derivs else CONSTANTS[name]
            if name in self.prog.inputs:
                off, size, scalar = self.prog.inputs[name]
                if not scalar:
                    raise OracleError(f"array input {name} used without index")
                return self._param(off)
            raise OracleError(f"unknown identifier {name}")
        if k == "index":
            name = e[1]
            idx = int(round(_val(self.eval(e[2], env))))
            if name in self.prog.inputs:
                off, size, scalar = self.prog.inputs[name]
                if not 0 <= idx < size:
                    raise OracleError(f"index {idx} out of range for {name}")
                return self._param(off + idx)
            raise OracleError(f"cannot index {name} in an expression")
        if k == "neg":
            return -self.eval(e[1], env)
        if k == "bin":
            a, b = self.eval(e[2], env), self.eval(e[3], env)
            op = e[1]
            if op == "+":
                return a + b
            if op == "-":
                return a - b
            if op == "*":
                return a * b
            if op == "/":
                return a / b
            if op == "%":
                return _val(a) % _val(b)
            if op == "**":
                return _val(a) ** _val(b)
        if k == "call":
            f, df = _FUNCS[e[1]]
            a = self.eval(e[2][0], env)
            return a.apply(f, df) if isinstance(a, Lin) else f(a)
        raise OracleError(f"bad expression {e}")

    def _param(self, k):
        v = float(self.theta[k])
        return Lin(v, {k: 1.0}) if self.with_derivs else v

    # -- operands --
    def qubits_of(self, ref, env):
        name, idx = ref[1], ref[2]
        if name in env and isinstance(env[name], tuple) and env[name][0] == "qubit":
            return [env[name][1]]
        if name not in self.prog.qregs:
            raise OracleError(f"unknown qubit register {name}")
        off, size, _ = self.prog.qregs[name]
        if idx is None:
            return list(range(off, off + size))
        i = int(round(_val(self.eval(idx, env))))
        if not 0 <= i < size:
            raise OracleError(f"qubit index {i} out of range for {name}")
        return [off + i]

    def clbits_of(self, ref, env):
        name, idx = ref[1], ref[2]
        if name not in self.prog.cregs:
            raise OracleError(f"unknown classical register {name}")
        off, size, _ = self.prog.cregs[name]
        if idx is None:
            return list(range(off, off + size))
        i = int(round(_val(self.eval(idx, env))))
        if not 0 <= i < size:
            raise OracleError(f"bit index {i} out of range for {name}")
        return [off + i]

    # -- running one shot --
    def run(self, seed=0, shot=0, forced=None, first_event=0, readout_error=0.0, reset_error=0.0,
            depolarizing=0.0):
        """first_event: index in the shot's Philox stream of the first word this
        program draws (0 for a whole program; a program that is one independent
        block of a larger product-state program starts where the draws of the
        blocks measured before it end).
        readout_error: after a measurement's outcome is drawn (the state keeps
        it), the next word u flips the recorded bit when u < readout_error.
        reset_error: after a reset, the next word u flips the qubit when
        u < reset_error. Either draw happens only when its rate is positive.
        depolarizing: after every application of a gate statement, each of its
        qubits independently takes X, Y or Z with probability p/3 each (the
        single-qubit depolarizing channel as a quantum trajectory); the draws
        come from their own counters (noise_word), not from the event stream."""
        p = self.prog
        self.readout_error = float(readout_error)
        self.reset_error = float(reset_error)
        self.depolarizing = float(depolarizing)
        self.seed, self.shot = int(seed), int(shot)
        self.loop_ords = []      # iteration ordinal of each enclosing for loop, outermost first
        self.noise_events = []   # (sid, loop code, application, operand, qubit, pauli)
        self.first_event = int(first_event)
        self.eng = self.engine_cls(p.n_qubits)
        self.cbits = [0] * p.n_clbits
        self.stream = ShotStream(seed, shot)
        self.stream.event = int(first_event)
        self.record, self.events = [], []
        self.record_prob = 1.0
        self.forced = list(forced) if forced is not None else []
        self.n_measures = 0
        self.gate_count = 0
        self.status = STATUS_OK
        try:
            self.exec_body(p.body, {})
        except _Abort:
            pass
        except (_Break, _Continue):
            raise OracleError("break/continue outside a loop")
        return self

    def exec_body(self, body, env):
        for st in body:
            self.exec_stmt(st, env)

    def exec_stmt(self, st, env):
        k = st[0]
        if k == "gate":
            self.exec_gate(st, env)
        elif k == "measure":
            qs = self.qubits_of(st[1], env)
            cs = self.clbits_of(st[2], env) if st[2] is not None else [None] * len(qs)
            if len(qs) != len(cs):
                raise OracleError("measure operand sizes differ")
            for q, c in zip(qs, cs):
                self.measure(q, c)
        elif k == "reset":
            for q in self.qubits_of(st[1], env):
                self.reset(q)
        elif k == "assign":
            self.assign(st[1], st[2], env)
        elif k == "barrier":
            pass
        elif k == "if":
            if self.cond(st[1], env):
                self.exec_body(st[2], env)
            else:
                self.exec_body(st[3], env)
        elif k == "for":
            a = int(round(_val(self.eval(st[2], env))))
            step = int(round(_val(self.eval(st[3], env))))
            b = int(round(_val(self.eval(st[4], env))))
            if step == 0:
                raise OracleError("for loop with zero step")
            i = a
            self.loop_ords.append(0)
            try:
                while (i <= b) if step > 0 else (i >= b):
                    inner = dict(env)
                    inner[st[1]] = Lin(i) if self.with_derivs else float(i)
                    try:
                        self.exec_body(st[5], inner)
                    except _Break:
                        break
                    except _Continue:
                        pass
                    i += step
                    self.loop_ords[-1] += 1
            finally:
                self.loop_ords.pop()
        elif k == "break":
            raise _Break()
        elif k == "continue":
            raise _Continue()
        else:
            raise OracleError(f"unsupported statement {k}")

    def cond(self, c, env):
        """An if condition: the classical expression read when the if executes, true iff nonzero."""
        return self.ceval(c, env) != 0

    def ceval(self, e, env):
        """Classical integer expression in 64-bit two's complement: every
        intermediate result wraps to a signed 64-bit value; comparisons and
        logical operators give 0 or 1; division truncates toward zero and
        x / 0 = x % 0 = 0; a shift by a count outside 0..63 gives 0 (a right
        shift of a negative value then gives -1); right shifts are arithmetic.
        A register, a variable or a bit reads its bits as an unsigned integer,
        or as two's complement for int variables; a constant or loop variable
        reads its value."""
        k = e[0]
        if k == "cnum":
            return _wrap64(e[1])
        if k == "cref":
            ref = e[1]
            name = ref[1]
            if name in self.prog.cregs:
                bits = self.clbits_of(ref, env)
                v = sum(self.cbits[b] << i for i, b in enumerate(bits))
                if self.prog.signed.get(name) and ref[2] is None and v >> (len(bits) - 1):
                    v -= 1 << len(bits)
                return _wrap64(v)
            if ref[2] is not None:
                raise OracleError(f"cannot index {name} in a classical expression")
            return _wrap64(int(round(_val(self.eval(("id", name), env)))))
        if k == "cun":
            a = self.ceval(e[2], env)
            return {"!": int(a == 0), "~": _wrap64(~a), "-": _wrap64(-a)}[e[1]]
        op, a, b = e[1], self.ceval(e[2], env), self.ceval(e[3], env)
        if op in ("+", "-", "*", "&", "|", "^"):
            return _wrap64({"+": a + b, "-": a - b, "*": a * b, "&": a & b, "|": a | b, "^": a ^ b}[op])
        if op in ("/", "%"):
            if b == 0:
                return 0
            q = abs(a) // abs(b) * (1 if (a < 0) == (b < 0) else -1)
            return _wrap64(q if op == "/" else a - q * b)
        if op == "<<":
            return _wrap64(a << b) if 0 <= b < 64 else 0
        if op == ">>":
            return a >> b if 0 <= b < 64 else (-1 if a < 0 else 0)
        if op in ("==", "!=", "<", ">", "<=", ">="):
            return int({"==": a == b, "!=": a != b, "<": a < b, ">": a > b, "<=": a <= b, ">=": a >= b}[op])
        if op == "&&":
            return int(a != 0 and b != 0)
        if op == "||":
            return int(a != 0 or b != 0)
        raise OracleError(f"bad classical expression {e}")

    def assign(self, target, rhs, env):
        """Classical assignment (OpenQASM 3): the target bit, register or
        variable takes the low bits of the right side's 64-bit two's-complement
        value (bit i of the target <- bit i of the value). The right side is
        read completely before any bit is written."""
        bits = self.clbits_of(target, env)
        value = self.ceval(rhs, env)
        for i, b in enumerate(bits):
            self.cbits[b] = (value >> i) & 1

    def reg_value(self, ref, env):
        bits = self.clbits_of(ref, env)
        return sum(self.cbits[b] << i for i, b in enumerate(bits))

    def exec_gate(self, st, env):
        name, args, qrefs = st[1], st[2], st[3]
        mods = st[4] if len(st) > 4 else ()
        angles = [self.eval(a, env) for a in args]
        operand_lists = [self.qubits_of(r, env) for r in qrefs]
        width = max(len(o) for o in operand_lists)
        for o in operand_lists:
            if len(o) not in (1, width):
                raise OracleError(f"gate {name}: register operands of different sizes")
        for j in range(width):
            qs = [o[j] if len(o) > 1 else o[0] for o in operand_lists]
            if len(set(qs)) != len(qs):
                raise OracleError(f"gate {name}: repeated qubit operand")
            if mods:
                self.apply_modified(mods, name, angles, qs, env)
            else:
                self.apply_named(name, angles, qs, env)
            sid = st[5] if len(st) > 5 else None
            if sid is not None and getattr(self, "depolarizing", 0.0) > 0.0:
                self.depolarize(sid, j, qs)

    def loop_code(self):
        """sum_d ordinal_d * 2**(16 d) over the enclosing for loops (outermost d = 0)."""
        if len(self.loop_ords) > 4 or any(o >= 1 << 16 for o in self.loop_ords):
            raise OracleError("noise draws support at most 4 nested loops of at most 65536 iterations")
        return sum(o << (16 * d) for d, o in enumerate(self.loop_ords))

    def depolarize(self, sid, j, qs):
        """One draw per qubit of application j of gate statement sid: the word
        noise_word(seed, shot, (sid, loop code, 64 j + k)) for operand k; with
        u = (word >> 11) 2**-53 the qubit takes X if u < p/3, Y if u < 2p/3, Z if
        u < p, nothing otherwise."""
        if len(qs) > 64:
            raise OracleError("noise draws support at most 64 operands")
        code, p = self.loop_code(), self.depolarizing
        for k, q in enumerate(qs):
            u = word_to_uniform(noise_word(self.seed, self.shot, sid, code, 64 * j + k))
            if u >= p:
                continue
            pauli = "x" if u < p / 3.0 else ("y" if u < 2.0 * p / 3.0 else "z")
            self.noise_events.append((sid, code, j, k, q, pauli))
            self.eng.apply(G.gate_matrix(pauli, [])[0], [q])

    def mod_controls(self, mods, env):
        """[(kind, n_controls or power)] of a modifier chain, outermost first."""
        out = []
        for kind, arg in mods:
            v = 1 if arg is None else int(round(_val(self.eval(arg, env))))
            if kind in ("ctrl", "negctrl") and v < 1:
                raise OracleError(f"{kind} needs at least one control")
            if kind == "pow" and arg is None:
                raise OracleError("pow needs an exponent")
            out.append((kind, v))
        return out

    def base_unitary(self, name, vals, k):
        """Matrix of a standard gate, or of a gate definition (its body applied
        to each basis state of k qubits), with numeric angles."""
        if G.is_standard(name):
            m, nq = G.gate_matrix(name, vals)
            return m, nq
        if name not in self.prog.gatedefs:
            raise OracleError(f"unknown gate {name}")
        _, _, params, qargs, body = self.prog.gatedefs[name]
        if len(params) != len(vals):
            raise OracleError(f"gate {name}: wrong number of arguments")
        nq = len(qargs)
        sub = Interpreter.__new__(Interpreter)
        sub.__dict__.update(self.__dict__)
        sub.tape = None
        sub.shift = {}
        sub.gate_count = 0
        m = np.zeros((1 << nq, 1 << nq), dtype=np.complex128)
        inner = {p: float(v) for p, v in zip(params, vals)}
        inner.update({qa: ("qubit", i) for i, qa in enumerate(qargs)})
        for c in range(1 << nq):
            sub.eng = TensorEngine(nq)
            sub.eng.psi = np.zeros(1 << nq, dtype=np.complex128)
            sub.eng.psi[c] = 1.0
            sub.exec_body(body, inner)
            m[:, c] = sub.eng.psi
        return m, nq

    def apply_modified(self, mods, name, angles, qs, env):
        chain = self.mod_controls(mods, env)
        g = self.gate_count
        self.gate_count += 1
        vals = [_val(a) for a in angles]
        for j in range(len(vals)):
            if (g, j) in self.shift:
                vals[j] += self.shift[(g, j)]
        m, k = self.base_unitary(name, vals, None)
        nctl = sum(v for kind, v in chain if kind in ("ctrl", "negctrl"))
        if k + nctl != len(qs):
            raise OracleError(f"modified gate {name} takes {k + nctl} qubits, got {len(qs)}")
        mm, _ = modify(chain, m, None)
        if self.tape is not None:
            derivs = [a.d if isinstance(a, Lin) else {} for a in angles]
            if any(derivs) and not G.is_standard(name):
                raise OracleError("gradients through a modified gate definition are not supported")
            self.tape.append((name, vals, qs, derivs, tuple(chain)))
        self.eng.apply(mm, qs)

    def apply_named(self, name, angles, qs, env):
        if name in self.prog.gatedefs:
            _, _, params, qargs, body = self.prog.gatedefs[name]
            if len(params) != len(angles) or len(qargs) != len(qs):
                raise OracleError(f"gate {name}: wrong number of arguments")
            inner = {p: a for p, a in zip(params, angles)}
            inner.update({qa: ("qubit", q) for qa, q in zip(qargs, qs)})
            self.exec_body(body, inner)
            return
        if not G.is_standard(name):
            raise OracleError(f"unknown gate {name}")
        g = self.gate_count
        self.gate_count += 1
        vals = [_val(a) for a in angles]
        for j in range(len(vals)):
            if (g, j) in self.shift:
                vals[j] += self.shift[(g, j)]
        m, nq = G.gate_matrix(name, vals)
        if nq != len(qs):
            raise OracleError(f"gate {name} takes {nq} qubits, got {len(qs)}")
        if self.tape is not None:
            derivs = [a.d if isinstance(a, Lin) else {} for a in angles]
            self.tape.append((name, vals, qs, derivs, ()))
        self.eng.apply(m, qs)

    # -- non-unitary events --
    def _draw_outcome(self, q, forced_value):
        p0, p1 = self.eng.probs(q)
        norm = p0 + p1
        u = self.stream.next_uniform()          # every event consumes one word
        if forced_value is None:
            m = 0 if u < p0 / norm else 1
        else:
            m = int(forced_value)
            if (p0 if m == 0 else p1) / norm < FORCED_ZERO_PROB:
                self.status = STATUS_FORCED_ZERO_PROB
                raise _Abort()
        p_m = p0 if m == 0 else p1
        self.eng.collapse(q, m, p_m)
        self.record_prob *= p_m / norm
        return m, u, p0 / norm

    def measure(self, q, c):
        forced_value = None
        if self.n_measures < len(self.forced):
            forced_value = self.forced[self.n_measures]
        m, u, p0n = self._draw_outcome(q, forced_value)
        self.n_measures += 1
        self.events.append(("measure", q, m, u, p0n))
        r = m
        if self.readout_error > 0.0 and self.stream.next_uniform() < self.readout_error:
            r = 1 - m
        self.record.append(r)
        if c is not None:
            self.cbits[c] = r

    def reset(self, q):
        m, u, p0n = self._draw_outcome(q, None)
        self.events.append(("reset", q, m, u, p0n))
        if m == 1:
            self.eng.flip(q)
        if self.reset_error > 0.0 and self.stream.next_uniform() < self.reset_error:
            self.eng.flip(q)

    # -- results --
    @property
    def psi(self):
        return self.eng.psi

    @property
    def words_drawn(self):
        """Philox words this shot consumed (one per measure/reset event, plus the error draws)."""
        return self.stream.event - self.first_event

    def creg_words(self):
        words = [0] * max(1, (len(self.cbits) + 63) // 64)
        for i, b in enumerate(self.cbits):
            words[i // 64] |= b << (i % 64)
        return words


def _val(x):
    return x.v if isinstance(x, Lin) else float(x)


def _wrap64(v):
    """v as a signed 64-bit two's-complement value."""
    v = int(v) & 0xFFFFFFFFFFFFFFFF
    return v - (1 << 64) if v >> 63 else v


# --------------------------------------------------------------------------
# Convenience entry points used by tests, the smoke check and the CPU baseline.
# --------------------------------------------------------------------------
def run_shot(source, theta=None, seed=0, shot=0, forced=None, engine_cls=TensorEngine, first_event=0,
             readout_error=0.0, reset_error=0.0, depolarizing=0.0):
    """Run one shot; returns the finished interpreter (psi, cbits, record, ...)."""
    it = Interpreter(source if isinstance(source, Program) else Program(source), theta, engine_cls)
    return it.run(seed, shot, forced, first_event, readout_error, reset_error, depolarizing)


def run_shots(source, n_shots, theta=None, seed=0, shot_offset=0, forced=None, readout_error=0.0,
              reset_error=0.0, depolarizing=0.0):
    prog = source if isinstance(source, Program) else Program(source)
    out = []
    for s in range(n_shots):
        f = None if forced is None else forced[s]
        it = Interpreter(prog, theta).run(seed, shot_offset + s, f, 0, readout_error, reset_error, depolarizing)
        out.append({"creg": it.creg_words(), "cbits": list(it.cbits), "record": list(it.record),
                    "n_events": it.words_drawn, "record_prob": it.record_prob,
                    "status": it.status, "events": list(it.events)})
    return out


def final_state(source, theta=None, seed=0, shot=0, forced=None):
    return run_shot(source, theta, seed, shot, forced).psi


# --------------------------------------------------------------------------
# Expectation values and gradients (VQE energy, Experiments, hybrid VQE).
# --------------------------------------------------------------------------
def apply_pauli(psi, codes, n):
    """P psi for a Pauli string given as codes[q] in {0:I, 1:X, 2:Y, 3:Z}."""
    eng = TensorEngine(n)
    eng.psi = psi.copy()
    for q, c in enumerate(codes):
        if c:
            eng.apply(G.PAULI["IXYZ"[c]], [q])
    return eng.psi


def apply_hamiltonian(psi, coeffs, codes, n):
    lam = np.zeros_like(psi)
    for c, row in zip(coeffs, codes):
        lam += c * apply_pauli(psi, row, n)
    return lam


def expval(source, theta, coeffs, codes):
    """E = sum_j c_j Re <psi|P_j|psi> for a unitary program."""
    prog = source if isinstance(source, Program) else Program(source)
    if not prog.is_unitary:
        raise OracleError("expval needs a program without measurement or control flow")
    psi = Interpreter(prog, theta).run().psi
    n = prog.n_qubits
    terms = [np.vdot(psi, apply_pauli(psi, row, n)) for row in codes]
    return float(sum(c * t.real for c, t in zip(coeffs, terms)))


def _tape(prog, theta):
    it = Interpreter(prog, theta, with_derivs=True)
    it.tape = []
    it.run()
    return it


def grad_param_shift(source, theta, coeffs, codes):
    """dE/dtheta by the two-term shift rule applied to every gate angle, then the
    chain rule through each angle's (affine or general) dependence on theta."""
    prog = source if isinstance(source, Program) else Program(source)
    theta = np.asarray(theta, dtype=np.float64)
    tape = _tape(prog, theta).tape
    grad = np.zeros(prog.n_params)
    n = prog.n_qubits
    shiftable = {"rx", "ry", "rz", "p", "phase", "u1", "u2", "u3", "u", "U", "cp", "cphase"}
    for g, (name, vals, qs, derivs, chain) in enumerate(tape):
        for j, dj in enumerate(derivs):
            if not dj:
                continue
            if name not in shiftable or any(kind != "inv" for kind, _ in chain):
                raise OracleError(f"no two-term shift rule for gate {name}")
            e = []
            for sgn in (+1.0, -1.0):
                it = Interpreter(prog, theta)
                it.shift = {(g, j): sgn * math.pi / 2.0}
                psi = it.run().psi
                e.append(sum(c * np.vdot(psi, apply_pauli(psi, row, n)).real
                             for c, row in zip(coeffs, codes)))
            dEda = 0.5 * (e[0] - e[1])
            for k, coef in dj.items():
                grad[k] += coef * dEda
    return grad


def grad_adjoint(source, theta, coeffs, codes):
    """Plain adjoint sweep: lambda = H psi; for gates k = N..1: psi <- U_k^dag psi,
    g = 2 Re <lambda| dU_k/da |psi>, lambda <- U_k^dag lambda."""
    prog = source if isinstance(source, Program) else Program(source)
    theta = np.asarray(theta, dtype=np.float64)
    it = _tape(prog, theta)
    n = prog.n_qubits
    psi = it.psi.copy()
    energy = float(np.vdot(psi, apply_hamiltonian(psi, coeffs, codes, n)).real)
    lam_e = TensorEngine(n)
    lam_e.psi = apply_hamiltonian(psi, coeffs, codes, n)
    psi_e = TensorEngine(n)
    psi_e.psi = psi
    grad = np.zeros(prog.n_params)
    for name, vals, qs, derivs, chain in reversed(it.tape):
        m, _ = modify(chain, G.gate_matrix(name, vals)[0], None)
        psi_e.apply(m.conj().T, qs)
        for j, dj in enumerate(derivs):
            if not dj:
                continue
            base = G.gate_matrix(name, vals)[0]
            _, dm = modify(chain, base, G.gate_derivative(name, vals, j))
            tmp = TensorEngine(n)
            tmp.psi = psi_e.psi.copy()
            tmp.apply(dm, qs)
            gj = 2.0 * np.vdot(lam_e.psi, tmp.psi).real
            for k, coef in dj.items():
                grad[k] += coef * gj
        lam_e.apply(m.conj().T, qs)
    return energy, grad
