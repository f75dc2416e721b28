"""OpenQASM 3 subset front end: source text -> syntax tree (product side).

The paper's pipeline parses OpenQASM 3 into a typed AST and resolves a symbol
table separating compile-time constants, runtime ``input`` parameters and
classical registers (Methodology, parsing and semantic analysis). This module
is the project's own small parser for the subset the dynamic-circuit path needs:

  OPENQASM 3[.0];  include "...";  qubit[n] q;  bit[m] c;  qreg/creg;
  input float[64] t;  input array[float[64], N] theta;  const float[64] k = expr;
  gate name(params) a, b { ... }   standard gates, broadcast over registers
  measure q -> c;  c = measure q;  bit[m] c = measure q;  reset q;  barrier ...;
  if (cond) stmt-or-block [else stmt-or-block]   cond: c[i] | c | c[i] OP v | c OP v | !cond
  for [type] i in [a:b] / [a:s:b] { ... }  (inclusive bounds)  break;  continue;

``while`` is rejected: only loops with a static bound can be lowered.
"""
from dataclasses import dataclass, field
from typing import List, Optional


class QasmError(ValueError):
    """Malformed or unsupported OpenQASM 3 (reported as QSV_ERR_PARSE)."""


# ---------------------------------------------------------------------------
# syntax tree
# ---------------------------------------------------------------------------
@dataclass
class Num:
    value: float


@dataclass
class Name:
    ident: str


@dataclass
class Subscript:
    ident: str
    index: object


@dataclass
class Unary:
    op: str
    arg: object


@dataclass
class Binary:
    op: str
    lhs: object
    rhs: object


@dataclass
class Call:
    fn: str
    args: list


@dataclass
class Operand:
    reg: str
    index: Optional[object] = None


@dataclass
class Declare:
    kind: str          # "qubit" | "bit"
    name: str
    size: Optional[int]


@dataclass
class InputDecl:
    name: str
    size: Optional[int]


@dataclass
class ConstDecl:
    name: str
    value: object


@dataclass
class GateDef:
    name: str
    params: List[str]
    qargs: List[str]
    body: list


@dataclass
class GateCall:
    name: str
    args: list
    operands: List[Operand]
    mods: list = None    # [(kind, expr or None)], outermost first: inv, pow, ctrl, negctrl
    sid: Optional[int] = None  # index among the gate statements outside gate definitions, in source order


@dataclass
class Measure:
    qubits: Operand
    target: Optional[Operand]


@dataclass
class Reset:
    qubits: Operand


# Classical integer expressions (conditions included): C precedence, 64-bit
# two's-complement values; `!` takes the whole comparison after it.
@dataclass
class CNum:
    value: int


@dataclass
class CRef:
    operand: Operand           # a register, variable, bit, constant or loop variable


@dataclass
class CUn:
    op: str                    # "!" | "~" | "-"
    arg: object


@dataclass
class CBin:
    op: str                    # || && | ^ & == != < > <= >= << >> + - * / %
    lhs: object
    rhs: object


@dataclass
class Assign:
    """Classical assignment: target <- the low bits of a classical expression."""
    target: Operand
    expr: object


@dataclass
class IfStmt:
    cond: object               # a classical expression, true iff nonzero
    then_body: list
    else_body: list = field(default_factory=list)


@dataclass
class ForStmt:
    var: str
    start: object
    step: object
    stop: object
    body: list


@dataclass
class Break:
    pass


@dataclass
class Continue:
    pass


# ---------------------------------------------------------------------------
# scanner
# ---------------------------------------------------------------------------
_PUNCT3 = ("<<=", ">>=")
_PUNCT2 = ("->", "==", "!=", "<=", ">=", "**", "&&", "||", "<<", ">>", "+=", "-=", "*=", "/=", "%=", "&=", "|=",
           "^=")
_PUNCT1 = set("()[]{};,:=<>!+-*/%@&|^~")


def scan(text):
    """Split source text into (kind, value) tokens: 'n' number, 'w' word, 's' string, 'p' punctuation."""
    out, i, L = [], 0, len(text)
    while i < L:
        ch = text[i]
        if ch.isspace():
            i += 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = L if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            if j < 0:
                raise QasmError("unterminated comment")
            i = j + 2
        elif ch == '"':
            j = text.find('"', i + 1)
            if j < 0:
                raise QasmError("unterminated string")
            out.append(("s", text[i + 1:j]))
            i = j + 1
        elif ch.isdigit() or (ch == "." and i + 1 < L and text[i + 1].isdigit()):
            j = i
            if text.startswith(("0b", "0B", "0x", "0X", "0o", "0O"), i):
                j = i + 2
                while j < L and (text[j].isalnum() or text[j] == "_"):
                    j += 1
                base = {"b": 2, "x": 16, "o": 8}[text[i + 1].lower()]
                out.append(("n", int(text[i + 2:j].replace("_", ""), base)))
                i = j
                continue
            while j < L and (text[j].isdigit() or text[j] == "_"):
                j += 1
            is_float = False
            if j < L and text[j] == ".":
                is_float = True
                j += 1
                while j < L and text[j].isdigit():
                    j += 1
            if j < L and text[j] in "eE" and j + 1 < L and (text[j + 1].isdigit() or text[j + 1] in "+-"):
                is_float = True
                j += 2
                while j < L and text[j].isdigit():
                    j += 1
            lit = text[i:j].replace("_", "")
            out.append(("n", float(lit) if is_float else int(lit)))
            i = j
        elif ch.isalpha() or ch == "_" or ord(ch) > 127:
            j = i + 1
            while j < L and (text[j].isalnum() or text[j] == "_" or ord(text[j]) > 127):
                j += 1
            out.append(("w", text[i:j]))
            i = j
        elif text[i:i + 3] in _PUNCT3:
            out.append(("p", text[i:i + 3]))
            i += 3
        elif text[i:i + 2] in _PUNCT2:
            out.append(("p", text[i:i + 2]))
            i += 2
        elif ch in _PUNCT1:
            out.append(("p", ch))
            i += 1
        else:
            raise QasmError(f"unexpected character {ch!r}")
    out.append(("end", None))
    return out


# ---------------------------------------------------------------------------
# parser
# ---------------------------------------------------------------------------
_CMP_OPS = ("==", "!=", "<", ">", "<=", ">=")
# classical expression operators, loosest first
_CLASSICAL_LEVELS = [("||",), ("&&",), ("|",), ("^",), ("&",), ("==", "!="), ("<", ">", "<=", ">="), ("<<", ">>"),
                     ("+", "-"), ("*", "/", "%")]
_COMPOUND = {"+=": "+", "-=": "-", "*=": "*", "/=": "/", "%=": "%", "&=": "&", "|=": "|", "^=": "^",
             "<<=": "<<", ">>=": ">>"}
_BINARY_PRECEDENCE = [("+", "-"), ("*", "/", "%"), ("**",)]
_FUNCTIONS = ("sin", "cos", "tan", "exp", "ln", "sqrt", "arcsin", "arccos", "arctan")


class Parser:
    def __init__(self, text):
        self.tok = scan(text)
        self.pos = 0
        self.n_calls = 0     # gate statements seen outside gate definitions
        self.in_def = False

    def _peek(self, ahead=0):
        return self.tok[min(self.pos + ahead, len(self.tok) - 1)]

    def _take(self):
        t = self.tok[self.pos]
        self.pos += 1
        return t

    def _is(self, value, ahead=0):
        k, v = self._peek(ahead)
        return k in ("p", "w") and v == value

    def _eat(self, value):
        if self._is(value):
            self.pos += 1
            return True
        return False

    def _need(self, value):
        if not self._eat(value):
            raise QasmError(f"expected {value!r} but found {self._peek()[1]!r}")

    def _word(self):
        k, v = self._take()
        if k != "w":
            raise QasmError(f"expected a name but found {v!r}")
        return v

    def _int_const(self):
        k, v = self._take()
        if k != "n" or not isinstance(v, int):
            raise QasmError("expected an integer literal")
        return v

    # program
    def parse(self):
        stmts = []
        if self._is("OPENQASM"):
            self._take()
            self._take()
            self._need(";")
        while self._peek()[0] != "end":
            stmts.extend(self._statement())
        return stmts

    def _block(self):
        if self._eat("{"):
            body = []
            while not self._eat("}"):
                if self._peek()[0] == "end":
                    raise QasmError("unterminated block")
                body.extend(self._statement())
            return body
        return self._statement()

    def _statement(self):
        k, v = self._peek()
        if k != "w":
            raise QasmError(f"unexpected {v!r} at the start of a statement")
        if v == "include":
            self._take()
            self._take()
            self._need(";")
            return []
        if v in ("qubit", "bit"):
            self._take()
            size = None
            if self._eat("["):
                size = self._int_const()
                self._need("]")
            name = self._word()
            if v == "bit" and self._eat("="):
                self._need("measure")
                src = self._operand()
                self._need(";")
                return [Declare(v, name, size), Measure(src, Operand(name))]
            self._need(";")
            return [Declare(v, name, size)]
        if v in ("uint", "int", "bool"):
            # classical integer variable: uint[n] / int[n] (32 bits without a
            # width), bool (1 bit), optionally initialised
            self._take()
            width = 1 if v == "bool" else 32
            if v != "bool" and self._eat("["):
                width = self._int_const()
                self._need("]")
            if not 1 <= width <= 64:
                raise QasmError("classical variables hold 1..64 bits")
            name = self._word()
            out = [Declare(v, name, width)]
            if self._eat("="):
                out.append(Assign(Operand(name), self._cexpr()))
            self._need(";")
            return out
        if v in ("qreg", "creg"):
            self._take()
            name = self._word()
            size = None
            if self._eat("["):
                size = self._int_const()
                self._need("]")
            self._need(";")
            return [Declare("qubit" if v == "qreg" else "bit", name, size)]
        if v == "input":
            self._take()
            size = self._type()
            name = self._word()
            self._need(";")
            return [InputDecl(name, size)]
        if v == "const":
            self._take()
            self._type()
            name = self._word()
            self._need("=")
            val = self._expr()
            self._need(";")
            return [ConstDecl(name, val)]
        if v == "gate":
            return [self._gate_def()]
        if v == "measure":
            self._take()
            q = self._operand()
            tgt = self._operand() if self._eat("->") else None
            self._need(";")
            return [Measure(q, tgt)]
        if v == "reset":
            self._take()
            q = self._operand()
            self._need(";")
            return [Reset(q)]
        if v == "barrier":
            while not self._eat(";"):
                if self._take()[0] == "end":
                    raise QasmError("unterminated barrier")
            return []
        if v == "if":
            return [self._if()]
        if v == "for":
            return [self._for()]
        if v == "while":
            raise QasmError("while loops have no static bound; use a for loop with break")
        if v == "break":
            self._take()
            self._need(";")
            return [Break()]
        if v == "continue":
            self._take()
            self._need(";")
            return [Continue()]
        # "c[...] = measure q[...];", a classical assignment or a gate call
        nxt = self._peek(1)
        if (nxt[0] == "p" and (nxt[1] == "=" or nxt[1] in _COMPOUND)) or (self._is("[", 1) and self._assignment_ahead()):
            tgt = self._operand()
            k, v = self._take()
            if v in _COMPOUND:
                st = Assign(tgt, CBin(_COMPOUND[v], CRef(tgt), self._cexpr()))
                self._need(";")
                return [st]
            if v != "=":
                raise QasmError(f"expected = after {tgt.reg}")
            if self._eat("measure"):
                q = self._operand()
                self._need(";")
                return [Measure(q, tgt)]
            st = Assign(tgt, self._cexpr())
            self._need(";")
            return [st]
        return [self._gate_call()]

    def _assignment_ahead(self):
        depth, j = 0, self.pos + 1
        while j < len(self.tok):
            k, v = self.tok[j]
            if k == "p" and v == "[":
                depth += 1
            elif k == "p" and v == "]":
                depth -= 1
                if depth == 0:
                    nk, nv = self.tok[j + 1]
                    return nk == "p" and (nv == "=" or nv in _COMPOUND)
            j += 1
        return False

    def _type(self):
        """Parses a type; returns the array length for array types, else None."""
        name = self._word()
        if name == "array":
            self._need("[")
            self._type()
            self._need(",")
            n = self._int_const()
            self._need("]")
            return n
        if self._eat("["):
            self._int_const()
            self._need("]")
        return None

    def _gate_def(self):
        self._need("gate")
        name = self._word()
        params = []
        if self._eat("("):
            while not self._eat(")"):
                params.append(self._word())
                self._eat(",")
        qargs = [self._word()]
        while self._eat(","):
            qargs.append(self._word())
        self._need("{")
        body = []
        self.in_def = True
        while not self._eat("}"):
            body.extend(self._statement())
        self.in_def = False
        return GateDef(name, params, qargs, body)

    def _gate_call(self):
        name = self._word()
        mods = []
        while name in ("inv", "pow", "ctrl", "negctrl") and (self._is("@") or self._is("(")):
            arg = None
            if self._eat("("):
                arg = self._expr()
                self._need(")")
            self._need("@")
            mods.append((name, arg))
            name = self._word()
        args = []
        if self._eat("("):
            if not self._eat(")"):
                args.append(self._expr())
                while self._eat(","):
                    args.append(self._expr())
                self._need(")")
        ops = [self._operand()]
        while self._eat(","):
            ops.append(self._operand())
        self._need(";")
        sid = None
        if not self.in_def:
            sid = self.n_calls
            self.n_calls += 1
        return GateCall(name, args, ops, mods, sid)

    def _operand(self):
        reg = self._word()
        idx = None
        if self._eat("["):
            idx = self._expr()
            self._need("]")
        return Operand(reg, idx)

    def _if(self):
        self._need("if")
        self._need("(")
        cond = self._cexpr()
        self._need(")")
        then_body = self._block()
        else_body = self._block() if self._eat("else") else []
        return IfStmt(cond, then_body, else_body)

    def _cexpr(self, level=0):
        """Classical expression by precedence level (loosest first)."""
        if level == len(_CLASSICAL_LEVELS):
            return self._cunary()
        lhs = self._cexpr(level + 1)
        while self._peek()[0] == "p" and self._peek()[1] in _CLASSICAL_LEVELS[level]:
            op = self._take()[1]
            lhs = CBin(op, lhs, self._cexpr(level + 1))
        return lhs

    def _cunary(self):
        if self._eat("!"):
            return CUn("!", self._cexpr(_CLASSICAL_LEVELS.index(("==", "!="))))
        if self._eat("~"):
            return CUn("~", self._cunary())
        if self._eat("-"):
            return CUn("-", self._cunary())
        if self._eat("+"):
            return self._cunary()
        if self._eat("("):
            e = self._cexpr()
            self._need(")")
            return e
        k, v = self._peek()
        if k == "n":
            self._take()
            if isinstance(v, float):
                raise QasmError(f"classical expressions are integers, got {v}")
            return CNum(v)
        if k == "w" and v in ("true", "false"):
            self._take()
            return CNum(1 if v == "true" else 0)
        return CRef(self._operand())

    def _for(self):
        self._need("for")
        if not self._is("in", 1):
            self._type()
        var = self._word()
        self._need("in")
        self._need("[")
        a = self._expr()
        self._need(":")
        b = self._expr()
        if self._eat(":"):
            step, stop = b, self._expr()
        else:
            step, stop = Num(1), b
        self._need("]")
        return ForStmt(var, a, step, stop, self._block())

    # expressions
    def _expr(self, level=0):
        if level == len(_BINARY_PRECEDENCE):
            return self._unary()
        lhs = self._expr(level + 1)
        ops = _BINARY_PRECEDENCE[level]
        while self._peek()[0] == "p" and self._peek()[1] in ops:
            op = self._take()[1]
            rhs = self._expr(level + 1) if op != "**" else self._expr(level)
            lhs = Binary(op, lhs, rhs)
            if op == "**":
                break
        return lhs

    def _unary(self):
        if self._eat("-"):
            return Unary("-", self._unary())
        if self._eat("+"):
            return self._unary()
        k, v = self._take()
        if k == "n":
            return Num(v)
        if k == "p" and v == "(":
            e = self._expr()
            self._need(")")
            return e
        if k == "w":
            if v in _FUNCTIONS and self._is("("):
                self._take()
                args = [self._expr()]
                while self._eat(","):
                    args.append(self._expr())
                self._need(")")
                return Call(v, args)
            if self._eat("["):
                e = self._expr()
                self._need("]")
                return Subscript(v, e)
            return Name(v)
        raise QasmError(f"unexpected {v!r} in an expression")


def parse(text):
    return Parser(text).parse()
