"""A small OpenQASM 3 subset parser for the oracle (independent of the product's).

TEST INFRASTRUCTURE ONLY: part of the CPU oracle.

The paper's pipeline starts from OpenQASM 3 text parsed into a typed AST and a
symbol table separating compile-time constants, runtime ``input`` parameters and
classical registers (Methodology, parsing and semantic analysis). This module
builds such an AST as plain tuples for the tree-walking interpreter in
``oracle.sim``:

  ('qubit', name, size|None)        ('bit', name, size|None)
  ('var', name, width, signed)      classical integer variable (uint/int/bool)
  ('input', name, size|None)        ('const', name, expr)
  ('gatedef', name, params, qargs, body)
  ('gate', name, [expr], [qref], mods, sid)    ('measure', qref, cref|None)
        sid: index of the gate statement among those outside gate definitions,
        in source order (None inside a definition); names its noise draws
  ('assign', cref, cexpr)           classical assignment (also variable initialisers)
  ('reset', qref)                   ('barrier',)
  ('if', cexpr, then_body, else_body) ('for', var, start, step, stop, body)
  ('break',)                        ('continue',)
  qref/cref = ('ref', name, index_expr|None)
  expr  = ('num', v) | ('id', name) | ('index', name, expr) | ('neg', e)
        | ('bin', op, a, b) | ('call', fn, [e])             (gate angles, constants)
  cexpr = ('cnum', v) | ('cref', ref) | ('cun', op, e) | ('cbin', op, a, b)
          classical integer expressions and conditions, C precedence
          (|| < && < | < ^ < & < == != < relational < shifts < + - < * / % < unary),
          except that `!` applies to the whole comparison after it
          (`!c == 1` is `!(c == 1)`)
"""
import math
import re

_TOKEN = re.compile(r"""
    (?P<ws>\s+|//[^\n]*|/\*.*?\*/)
  | (?P<num>0b[01_]+|0x[0-9a-fA-F_]+|(?:\d+\.\d*|\.\d+|\d+)(?:[eE][+-]?\d+)?)
  | (?P<str>"[^"]*")
  | (?P<id>[A-Za-z_θπτφλ][A-Za-z0-9_θπτφλ]*)
  | (?P<op>->|<<=|>>=|==|!=|<=|>=|&&|\|\||\*\*|<<|>>|\+=|-=|\*=|/=|%=|&=|\|=|\^=|[-+*/%()\[\]{};,:=<>!@&|^~])
""", re.S | re.X)


class QasmSyntaxError(ValueError):
    pass


def tokenize(text):
    toks, pos = [], 0
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m:
            raise QasmSyntaxError(f"unexpected character {text[pos]!r} at offset {pos}")
        pos = m.end()
        kind = m.lastgroup
        if kind == "ws":
            continue
        toks.append((kind, m.group(kind)))
    toks.append(("eof", ""))
    return toks


def _parse_int_literal(s):
    s = s.replace("_", "")
    if s.startswith("0b"):
        return int(s[2:], 2)
    if s.startswith("0x"):
        return int(s[2:], 16)
    return None


class _Parser:
    def __init__(self, text):
        self.toks = tokenize(text)
        self.i = 0
        self.gate_sid = 0   # gate statements seen outside gate definitions
        self.in_def = 0

    # -- token helpers --
    def peek(self, k=0):
        return self.toks[self.i + k]

    def next(self):
        t = self.toks[self.i]
        self.i += 1
        return t

    def accept(self, value):
        if self.peek()[1] == value and self.peek()[0] in ("op", "id"):
            self.i += 1
            return True
        return False

    def expect(self, value):
        t = self.next()
        if t[1] != value:
            raise QasmSyntaxError(f"expected {value!r}, got {t[1]!r}")
        return t

    def ident(self):
        t = self.next()
        if t[0] != "id":
            raise QasmSyntaxError(f"expected identifier, got {t[1]!r}")
        return t[1]

    # -- program --
    def program(self):
        body = []
        if self.peek()[1] == "OPENQASM":
            self.next()
            self.next()  # version number
            self.expect(";")
        while self.peek()[0] != "eof":
            st = self.statement()
            if st is not None:
                body.append(st)
        return body

    def block_or_statement(self):
        if self.accept("{"):
            body = []
            while not self.accept("}"):
                st = self.statement()
                if st is not None:
                    body.append(st)
            return body
        st = self.statement()
        return [] if st is None else [st]

    def statement(self):
        kind, val = self.peek()
        if kind == "id":
            if val == "include":
                self.next()
                self.next()
                self.expect(";")
                return None
            if val in ("qubit", "bit"):
                return self.declaration()
            if val in ("uint", "int", "bool"):
                return self.var_decl()
            if val in ("qreg", "creg"):
                self.next()
                name = self.ident()
                size = None
                if self.accept("["):
                    size = self.const_int()
                    self.expect("]")
                self.expect(";")
                return ("qubit" if val == "qreg" else "bit", name, size)
            if val == "input":
                return self.input_decl()
            if val == "const":
                self.next()
                self.type_spec()
                name = self.ident()
                self.expect("=")
                e = self.expr()
                self.expect(";")
                return ("const", name, e)
            if val == "gate":
                return self.gate_def()
            if val == "measure":
                self.next()
                q = self.ref()
                c = None
                if self.accept("->"):
                    c = self.ref()
                self.expect(";")
                return ("measure", q, c)
            if val == "reset":
                self.next()
                q = self.ref()
                self.expect(";")
                return ("reset", q)
            if val == "barrier":
                while self.next()[1] != ";":
                    pass
                return ("barrier",)
            if val == "if":
                return self.if_stmt()
            if val == "for":
                return self.for_stmt()
            if val == "break":
                self.next()
                self.expect(";")
                return ("break",)
            if val == "continue":
                self.next()
                self.expect(";")
                return ("continue",)
            if val == "while":
                raise QasmSyntaxError("while loops are unbounded and not supported")
            # assignment "c[i] = measure q[j];", classical assignment, or gate call
            if self.peek(1)[1] in ("=", "[") or self.peek(1)[1] in _COMPOUND:
                save = self.i
                target = self.ref()
                if self.accept("="):
                    if self.accept("measure"):
                        q = self.ref()
                        self.expect(";")
                        return ("measure", q, target)
                    rhs = self.cexpr()
                    self.expect(";")
                    return ("assign", target, rhs)
                op = self.peek()[1]
                if op in _COMPOUND:
                    self.next()
                    rhs = self.cexpr()
                    self.expect(";")
                    return ("assign", target, ("cbin", _COMPOUND[op], ("cref", target), rhs))
                self.i = save
            return self.gate_call()
        raise QasmSyntaxError(f"unexpected token {val!r}")

    def type_spec(self):
        name = self.ident()
        if name == "array":
            self.expect("[")
            self.type_spec()
            self.expect(",")
            size = self.const_int()
            self.expect("]")
            return ("array", size)
        width = None
        if self.accept("["):
            width = self.const_int()
            self.expect("]")
        return (name, width)

    def declaration(self):
        kind = self.ident()
        size = None
        if self.accept("["):
            size = self.const_int()
            self.expect("]")
        name = self.ident()
        if kind == "bit" and self.accept("="):
            self.expect("measure")
            q = self.ref()
            self.expect(";")
            return [("bit", name, size), ("measure", q, ("ref", name, None))]
        self.expect(";")
        return (kind, name, size)

    def var_decl(self):
        """uint[n] x; int[n] x; uint x; int x (32 bits); bool b; each with an
        optional initialiser."""
        kind = self.ident()
        width = 1 if kind == "bool" else 32
        if kind != "bool" and self.accept("["):
            width = self.const_int()
            self.expect("]")
        if not 1 <= width <= 64:
            raise QasmSyntaxError("classical variables hold 1..64 bits")
        name = self.ident()
        out = [("var", name, width, kind == "int")]
        if self.accept("="):
            out.append(("assign", ("ref", name, None), self.cexpr()))
        self.expect(";")
        return out

    # -- classical integer expressions and conditions (C precedence) --
    _CPREC = [("||",), ("&&",), ("|",), ("^",), ("&",), ("==", "!="), ("<", ">", "<=", ">="), ("<<", ">>"),
              ("+", "-"), ("*", "/", "%")]

    def cexpr(self, level=0):
        if level == len(self._CPREC):
            return self.cunary()
        lhs = self.cexpr(level + 1)
        while self.peek()[0] == "op" and self.peek()[1] in self._CPREC[level]:
            op = self.next()[1]
            lhs = ("cbin", op, lhs, self.cexpr(level + 1))
        return lhs

    def cunary(self):
        if self.accept("!"):
            # `!` takes the whole comparison after it
            return ("cun", "!", self.cexpr(5))
        if self.accept("~"):
            return ("cun", "~", self.cunary())
        if self.accept("-"):
            return ("cun", "-", self.cunary())
        if self.accept("+"):
            return self.cunary()
        kind, val = self.peek()
        if kind == "num":
            self.next()
            iv = _parse_int_literal(val)
            if iv is None:
                if not re.fullmatch(r"\d+", val):
                    raise QasmSyntaxError(f"classical expressions are integers, got {val}")
                iv = int(val)
            return ("cnum", iv)
        if self.accept("("):
            e = self.cexpr()
            self.expect(")")
            return e
        if kind == "id" and val in ("true", "false"):
            self.next()
            return ("cnum", 1 if val == "true" else 0)
        return ("cref", self.ref())

    def input_decl(self):
        self.expect("input")
        t = self.type_spec()
        name = self.ident()
        self.expect(";")
        size = t[1] if t[0] == "array" else None
        return ("input", name, size)

    def gate_def(self):
        self.expect("gate")
        name = self.ident()
        params = []
        if self.accept("("):
            if not self.accept(")"):
                params.append(self.ident())
                while self.accept(","):
                    params.append(self.ident())
                self.expect(")")
        qargs = [self.ident()]
        while self.accept(","):
            qargs.append(self.ident())
        self.expect("{")
        body = []
        self.in_def += 1
        while not self.accept("}"):
            st = self.statement()
            if st is not None:
                body.append(st)
        self.in_def -= 1
        return ("gatedef", name, params, qargs, body)

    def gate_call(self):
        # gate modifiers, outermost first: inv @, pow(k) @, ctrl @, ctrl(n) @, negctrl @, negctrl(n) @
        mods = []
        name = self.ident()
        while name in ("inv", "pow", "ctrl", "negctrl") and self.peek(0)[1] in ("@", "("):
            arg = None
            if self.accept("("):
                arg = self.expr()
                self.expect(")")
            self.expect("@")
            mods.append((name, arg))
            name = self.ident()
        args = []
        if self.accept("("):
            if not self.accept(")"):
                args.append(self.expr())
                while self.accept(","):
                    args.append(self.expr())
                self.expect(")")
        qs = [self.ref()]
        while self.accept(","):
            qs.append(self.ref())
        self.expect(";")
        sid = None
        if not self.in_def:
            sid = self.gate_sid
            self.gate_sid += 1
        return ("gate", name, args, qs, tuple(mods), sid)

    def ref(self):
        name = self.ident()
        idx = None
        if self.accept("["):
            idx = self.expr()
            self.expect("]")
        return ("ref", name, idx)

    def if_stmt(self):
        self.expect("if")
        self.expect("(")
        cond = self.cexpr()
        self.expect(")")
        then_body = self.block_or_statement()
        else_body = []
        if self.accept("else"):
            else_body = self.block_or_statement()
        return ("if", cond, then_body, else_body)

    def for_stmt(self):
        self.expect("for")
        if self.peek(1)[1] != "in":
            self.type_spec()
        var = self.ident()
        self.expect("in")
        self.expect("[")
        a = self.expr()
        self.expect(":")
        b = self.expr()
        step, stop = ("num", 1), b
        if self.accept(":"):
            step, stop = b, self.expr()
        self.expect("]")
        body = self.block_or_statement()
        return ("for", var, a, step, stop, body)

    def const_int(self):
        e = self.expr()
        if e[0] != "num" or int(e[1]) != e[1]:
            raise QasmSyntaxError("expected an integer constant")
        return int(e[1])

    # -- expressions (precedence climbing) --
    def expr(self):
        return self._binary(0)

    _PREC = {"+": 1, "-": 1, "*": 2, "/": 2, "%": 2, "**": 3}

    def _binary(self, min_prec):
        lhs = self._unary()
        while True:
            op = self.peek()[1]
            if self.peek()[0] != "op" or op not in self._PREC or self._PREC[op] < min_prec:
                return lhs
            self.next()
            nxt = self._PREC[op] + (0 if op == "**" else 1)
            rhs = self._binary(nxt)
            lhs = ("bin", op, lhs, rhs)

    def _unary(self):
        if self.accept("-"):
            return ("neg", self._unary())
        if self.accept("+"):
            return self._unary()
        return self._atom()

    def _atom(self):
        kind, val = self.next()
        if kind == "num":
            iv = _parse_int_literal(val)
            if iv is not None:
                return ("num", iv)
            v = float(val)
            return ("num", int(v) if re.fullmatch(r"\d+", val) else v)
        if kind == "op" and val == "(":
            e = self.expr()
            self.expect(")")
            return e
        if kind == "id":
            if self.peek()[1] == "(" and val in ("sin", "cos", "tan", "exp", "sqrt", "ln", "arccos", "arcsin", "arctan"):
                self.next()
                args = [self.expr()]
                while self.accept(","):
                    args.append(self.expr())
                self.expect(")")
                return ("call", val, args)
            if self.accept("["):
                e = self.expr()
                self.expect("]")
                return ("index", val, e)
            return ("id", val)
        raise QasmSyntaxError(f"unexpected token {val!r} in expression")


_COMPOUND = {"+=": "+", "-=": "-", "*=": "*", "/=": "/", "%=": "%", "&=": "&", "|=": "|", "^=": "^",
             "<<=": "<<", ">>=": ">>"}


def _flatten(body):
    out = []
    for st in body:
        if isinstance(st, list):
            out.extend(st)
        else:
            out.append(st)
    return out


def parse(text):
    """Parse OpenQASM 3 subset text into the oracle's tuple AST (a statement list)."""
    p = _Parser(text)
    return _deep_flatten(p.program())


def _deep_flatten(body):
    res = []
    for st in _flatten(body):
        if st[0] == "if":
            res.append(("if", st[1], _deep_flatten(st[2]), _deep_flatten(st[3])))
        elif st[0] == "for":
            res.append(("for", st[1], st[2], st[3], st[4], _deep_flatten(st[5])))
        elif st[0] == "gatedef":
            res.append(("gatedef", st[1], st[2], st[3], _deep_flatten(st[4])))
        else:
            res.append(st)
    return res


CONSTANTS = {"pi": math.pi, "π": math.pi, "tau": 2 * math.pi, "τ": 2 * math.pi,
             "euler": math.e, "ℇ": math.e}
