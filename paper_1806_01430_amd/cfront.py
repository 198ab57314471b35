"""C front end: loop nests of a restricted C program -> the application IR.

The paper's offloader parses the application's source, finds every for
statement and checks each one for parallelisability (Sec. 4).  This module
does the parsing step for a subset of C, so that an application can be given
as source instead of the JSON IR:

* ``#define NAME <int>`` -- parameters;
* array declarations ``float|double|bf16 NAME[d0][d1]...;`` with an optional
  trailing ``// ofl: output setup=sin mode=MODE`` annotation (the IR's
  buffer metadata; default set-up content is zero);
* statements: ``for (int v = lo; v < hi; v++) stmt``, blocks, assignments
  ``ref (=|+=|-=|*=) expr;`` to array elements, local temporaries
  ``float|double t = expr;``.  Expressions: numbers, parameters,
  array references, locals, ``+ - * /``, parentheses, casts ``(double)x``
  and calls ``f(...)``.

A call statement of its own outside any loop, ``fft_rows(X);``,
``ifft_rows(X);``, ``rfft_rows(X);``, ``irfft_rows(X);``, ``sgemm(A, B, C);`` or one of the level-1 BLAS calls
``saxpy(alpha, X, Y);``, ``scopy(X, Y);``, ``sscal(alpha, X);``, is a
function block (the FFT library calls Sec. 3.2 names beside loop statements
as offloadable parts): one nest with one gene bit, whose GPU and CPU forms
are the library's own.

Every top-level ``for`` is a loop nest: its loops are the for statements it
contains, outermost first; a top-level for from 0 whose body holds only for
statements, two or more of them, is a repeat block (the iterated sweep; the
nests inside it are the candidates).  Accesses come from the array
references, per element in statement order: an element written is "w", or
"rw" when read before its first plain write; an element only read is "r"; a
buffer touched only through ``+=`` at subscripts that use no loop variable of
the nest is a sum reduction ("sum").  A call of anything but ``u01`` (the
counter-based uniform value of an element) and ``bf16`` (the rounding cast)
marks the nest as calling an external routine, which the dependence check
(``ofl_app_load``) rejects, as it rejects loop-carried dependences.

The body of each nest is bound to one of the library's operations by
structural matching against C templates (below): temporaries are substituted
and compound assignments expanded first, then the expression trees must agree
node by node -- the same constants and grouping, operands in the same order
except that one addition or product may have its two operands swapped (which
rounds alike) -- because the library evaluates exactly that expression.  A
nest matching no template (one that leaves its loop with ``break``, for one)
is an error: the library could run it neither on the GPU nor on the CPU.
"""
import hashlib
import json
import os
import re
import subprocess

import numpy as np

# ------------------------------------------------------------------ lexing
_TOKEN = re.compile(r"""
    (?P<ws>\s+|//[^\n]*|/\*.*?\*/)
  | (?P<num>\d+\.\d*(?:[eE][+-]?\d+)?f?|\d*\.\d+(?:[eE][+-]?\d+)?f?|\d+[eE][+-]?\d+f?|\d+f?)
  | (?P<id>\$?[A-Za-z_][A-Za-z_0-9]*)
  | (?P<op>\+\+|\+=|-=|\*=|/=|<=|>=|==|!=|&&|\|\||[-+*/%=<>!()\[\]{};,&@?:])
""", re.X | re.S)

TYPES = {"float": "f32", "double": "f64", "bf16": "bf16", "int": "int"}


class CError(ValueError):
    pass


def _lex(src):
    """Tokens, with the 1-based source line of each, whether it is the first
    token on its line, and its start and end offsets in the text."""
    out, pos, line, last_line = [], 0, 1, 0
    while pos < len(src):
        m = _TOKEN.match(src, pos)
        if not m:
            raise CError("line %d: cannot read %r" % (line, src[pos:pos + 20]))
        if m.lastgroup != "ws":
            out.append((m.group(m.lastgroup), line, line != last_line, m.start(), m.end()))
            last_line = line
        line += src.count("\n", pos, m.end())
        pos = m.end()
    return out


# ------------------------------------------------------------------ parsing
class _Parser:
    def __init__(self, toks):
        self.t = [t[0] for t in toks]
        self.where = [(t[1], t[2]) for t in toks]
        self.span = [(t[3], t[4]) for t in toks]
        self.i = 0
        self.for_at = {}          # id of a parsed for or call statement -> (line, first on its line)
        self.text_at = {}         # id of a parsed for statement -> (start, end) offsets of its text

    def peek(self, k=0):
        return self.t[self.i + k] if self.i + k < len(self.t) else None

    def take(self, want=None):
        tok = self.peek()
        if tok is None or (want is not None and tok != want):
            raise CError("expected %r, found %r" % (want, tok))
        self.i += 1
        return tok

    # expressions: ('num', v, kind) ('var', n) ('ref', n, [subs]) ('bin', op, a, b)
    # ('neg', a) ('call', n, [args]) ('cast', type, a) ('addr', a) ('not', a)
    # ('sel', c, a, b); a number's kind is 'i' (integer literal), 'f' (float
    # literal, suffix f) or 'd' (double literal)
    def cond(self):
        e = self.conj()
        while self.peek() == "||":
            self.take()
            e = ("bin", "||", e, self.conj())
        return e

    def conj(self):
        e = self.rel()
        while self.peek() == "&&":
            self.take()
            e = ("bin", "&&", e, self.rel())
        return e

    def rel(self):
        e = self.expr()
        while self.peek() in ("<", "<=", ">", ">=", "==", "!="):
            op = self.take()
            e = ("bin", op, e, self.expr())
        return e

    def expr(self):
        e = self.term()
        while self.peek() in ("+", "-"):
            op = self.take()
            e = ("bin", op, e, self.term())
        return e

    def term(self):
        e = self.unary()
        while self.peek() in ("*", "/", "%"):
            op = self.take()
            e = ("bin", op, e, self.unary())
        return e

    def unary(self):
        tok = self.peek()
        if tok == "-":
            self.take()
            return ("neg", self.unary())
        if tok == "&":
            self.take()
            return ("addr", self.unary())
        if tok == "!":
            self.take()
            return ("not", self.unary())
        if tok == "(" and self.peek(1) in TYPES and self.peek(2) == ")":
            self.take("(")
            ty = self.take()
            self.take(")")
            return ("cast", TYPES[ty], self.unary())
        return self.primary()

    def primary(self):
        tok = self.take()
        if tok == "(":
            e = self.cond()
            self.take(")")
            return e
        if re.match(r"[\d.]", tok):
            kind = "f" if tok[-1] in "fF" else ("i" if re.fullmatch(r"\d+", tok) else "d")
            return ("num", float(tok.rstrip("fF")), kind)
        if not re.match(r"\$?[A-Za-z_]", tok):
            raise CError("unexpected %r" % tok)
        if self.peek() == "(":
            self.take("(")
            args = []
            if self.peek() != ")":
                args.append(self.expr())
                while self.peek() == ",":
                    self.take(",")
                    args.append(self.expr())
            self.take(")")
            return ("call", tok, args)
        subs = []
        while self.peek() == "[":
            self.take("[")
            subs.append(self.expr())
            self.take("]")
        return ("ref", tok, subs) if subs else ("var", tok)

    # statements: ('for', v, lo, hi, [body]) ('assign', ref, op, e)
    # ('local', type, name, e) ('break',) ('if', cond, [then], [else])
    def stmt(self):
        start = self.span[self.i][0] if self.i < len(self.span) else 0
        out = self._stmt()
        if len(out) == 1 and out[0][0] == "for":
            self.text_at[id(out[0])] = (start, self.span[self.i - 1][1])
        return out

    def _stmt(self):
        tok = self.peek()
        if tok == "if":
            self.take("if")
            self.take("(")
            c = self.cond()
            self.take(")")
            then = self.stmt()
            other = []
            if self.peek() == "else":
                self.take("else")
                other = self.stmt()
            return [("if", c, then, other)]
        if tok == "{":
            self.take("{")
            body = []
            while self.peek() != "}":
                body.extend(self.stmt())
            self.take("}")
            return body
        if tok == "for":
            at = self.where[self.i]
            self.take("for")
            self.take("(")
            if self.peek() == "int":
                self.take()
            v = self.take()
            self.take("=")
            lo = self.expr()
            self.take(";")
            if self.take() != v:
                raise CError("loop condition must test %s" % v)
            cmp = self.take()
            hi = self.expr()
            if cmp == "<=":
                hi = ("bin", "+", hi, ("num", 1.0, "i"))
            elif cmp != "<":
                raise CError("loop condition must be < or <=")
            self.take(";")
            if self.peek() == "++":
                self.take()
                self.take(v)
            else:
                self.take(v)
                if self.take() not in ("++",):
                    raise CError("loops step by one (v++)")
            self.take(")")
            node = ("for", v, lo, hi, self.stmt())
            self.for_at[id(node)] = at
            return [node]
        if tok == "@":
            self.take("@")
            what = self.take()
            val = self.take()
            self.take(";")
            return [("pragma", what, val)]
        if tok == "break":
            self.take()
            self.take(";")
            return [("break",)]
        if tok in TYPES and self.peek(2) == "=":
            ty = TYPES[self.take()]
            name = self.take()
            self.take("=")
            e = self.expr()
            self.take(";")
            return [("local", ty, name, e)]
        at = self.where[self.i]
        lhs = self.primary()
        if lhs[0] == "call" and self.peek() == ";":
            self.take(";")
            node = ("callstmt", lhs[1], lhs[2])
            self.for_at[id(node)] = at
            return [node]
        op = self.take()
        if op not in ("=", "+=", "-=", "*=", "/="):
            raise CError("expected an assignment, found %r" % op)
        e = self.expr()
        self.take(";")
        return [("assign", lhs, op, e)]


def _affine(e):
    """An affine subscript / bound 'name + c', 'c' or 'name - c' -> IR text."""
    if e[0] == "num":
        return str(int(e[1]))
    if e[0] == "var":
        return e[1]
    if e[0] == "bin" and e[1] in "+-" and e[3][0] == "num":
        base = _affine(e[2])
        c = int(e[3][1])
        return "%s%s%d" % (base, e[1], c)
    raise CError("subscript or bound is not 'name + constant': %r" % (e,))


# ------------------------------------------------------------------ templates
# Calls that are part of the language of the nests, not external routines:
# u01(stream, i, j) is the counter-based uniform value of element (i, j) of a
# random stream, bf16(x) the round-to-nearest-even bfloat16 of x.  Any other
# call (lcg01(seed), a sequential generator, for one) is an external routine.
PURE_CALLS = ("u01", "bf16")

# Library routines called as statements of their own, outside any loop, that
# the library implements on the CPU and on the GPU: each call becomes a
# function block (one nest, one gene bit).  fft_rows(X): the forward DFT of
# every row of X[R][2n] (n complex values per row, interleaved);
# ifft_rows(X): the inverse DFT of every row, scaled by 1/n; rfft_rows(X):
# the DFT of every row of X[R][n] (n real values), written packed in place
# ([X0, X(n/2), Re X1, Im X1, ...]); irfft_rows(X): packed spectra back to
# their real rows;
# sgemm(A, B, C): C = A B (FP32 or bf16 operands by their declarations),
# the same nest as the loop form of the product; the level-1 BLAS routines
# on whole float arrays of one shape: saxpy(alpha, X, Y): Y = Y + alpha X,
# scopy(X, Y): Y = X, sscal(alpha, X): X = alpha X, the same nests as the
# loop forms (alpha a number, passed as the routine's float parameter).
FUNCTION_BLOCKS = {"fft_rows": "fft_rows", "ifft_rows": "fft_rows", "rfft_rows": "fft_rows",
                   "irfft_rows": "fft_rows", "sgemm": "gemm",
                   "saxpy": "add_scaled", "scopy": "copy", "sscal": "scale"}

# One C snippet per operation, each the nest's definition in the evaluation
# order the library follows; names beginning with $ are pattern variables
# (buffers, parameters, constants).  Loop variables match any names, renamed
# consistently.  Element-wise results are identical bits to this order; the
# products (gemm) and the FP64 sums (sumsq, the sweep's residual) are the same
# expressions summed in another order, within the library's stated bounds.
TEMPLATES = [
    ("gemm", """for (int i = 0; i < $M; i++) for (int j = 0; j < $N; j++) {
                  $C[i][j] = 0.0f;
                  for (int k = 0; k < $K; k++) $C[i][j] += $A[i][k] * $B[k][j]; }"""),
    ("add_scaled", "for (int i = 0; i < $R; i++) for (int j = 0; j < $S; j++) "
                   "$C[i][j] = $C[i][j] + $alpha * $A[i][j];"),
    ("avg2", "for (int i = 0; i < $R; i++) for (int j = 0; j < $S; j++) $D[i][j] = 0.5f * ($X[i][j] + $Y[i][j]);"),
    ("scale", "for (int i = 0; i < $R; i++) for (int j = 0; j < $S; j++) $D[i][j] = $beta * $D[i][j];"),
    ("transpose", "for (int i = 0; i < $R; i++) for (int j = 0; j < $S; j++) $T[j][i] = $X[i][j];"),
    ("copy", "for (int i = 0; i < $R; i++) for (int j = 0; j < $S; j++) $D[i][j] = $X[i][j];"),
    ("sumsq", """for (int i = 0; i < $R; i++) for (int j = 0; j < $S; j++) {
                   double v = (double)$X[i][j];
                   $s[0] += v * v; }"""),
    ("rec_prefix", "for (int i = 1; i < $N; i++) $v[i] = $v[i - 1] + $S[i][0];"),
    ("rec_decay", "for (int k = 1; k < $K; k++) $w[k] = 0.5f * $w[k - 1] + $p[1][1][k];"),
    ("lcg_fill", "for (int e = 0; e < $N; e++) $L[e] = lcg01($seed);"),
    ("copy_interior", """for (int i = 1; i < $I - 1; i++) for (int j = 1; j < $J - 1; j++)
                           for (int k = 1; k < $K - 1; k++) $p[i][j][k] = $q[i][j][k];"""),
    ("stencil19", """for (int i = 1; i < $I - 1; i++) for (int j = 1; j < $J - 1; j++)
                       for (int k = 1; k < $K - 1; k++) {
        float xm = ($p[i - 1][j - 1][k] + $p[i - 1][j + 1][k]) + ($p[i - 1][j][k - 1] + $p[i - 1][j][k + 1]);
        float x0 = ($p[i][j - 1][k] + $p[i][j + 1][k]) + ($p[i][j][k - 1] + $p[i][j][k + 1]);
        float xp = ($p[i + 1][j - 1][k] + $p[i + 1][j + 1][k]) + ($p[i + 1][j][k - 1] + $p[i + 1][j][k + 1]);
        float y0 = ($p[i][j - 1][k - 1] + $p[i][j - 1][k + 1]) + ($p[i][j + 1][k - 1] + $p[i][j + 1][k + 1]);
        float faces = ($p[i - 1][j][k] + $p[i + 1][j][k]) + x0;
        float edges = (xm + xp) + y0;
        float v = (0.25f * $p[i][j][k] + 0.0625f * faces) + 0.03125f * edges;
        $q[i][j][k] = v;
        double d = (double)v - (double)$p[i][j][k];
        $res[$n] += d * d; }"""),
]


def _parse_stmts(src, where=None, spans=None):
    p = _Parser(_lex(src))
    out = []
    while p.peek() is not None:
        out.extend(p.stmt())
    if where is not None:
        where.update(p.for_at)
    if spans is not None:
        spans.update(p.text_at)
    return out


def _inline(stmts, env=None):
    """Substitute local temporaries into later expressions; drop the locals.
    Compound assignments become plain ones (a += b -> a = a + b)."""
    env = dict(env or {})

    def sub(e):
        if e[0] == "var" and e[1] in env:
            return env[e[1]]
        if e[0] in ("ref",):
            return ("ref", e[1], [sub(x) for x in e[2]])
        if e[0] == "bin":
            return ("bin", e[1], sub(e[2]), sub(e[3]))
        if e[0] in ("neg", "addr", "not"):
            return (e[0], sub(e[1]))
        if e[0] == "cast":
            return ("cast", e[1], sub(e[2]))
        if e[0] == "call":
            return ("call", e[1], [sub(x) for x in e[2]])
        return e

    out = []
    for s in stmts:
        if s[0] == "local":
            env[s[2]] = sub(s[3])
        elif s[0] == "assign" and s[1][0] == "var":
            out.append(s)      # a local assigned again: no template has one
        elif s[0] == "assign":
            lhs, rhs = sub(s[1]), sub(s[3])
            if s[2] != "=":
                rhs = ("bin", s[2][0], lhs, rhs)
            out.append(("assign", lhs, "=", rhs))
        elif s[0] == "for":
            out.append(("for", s[1], sub(s[2]), sub(s[3]), _inline(s[4], env)))
        elif s[0] == "if":
            out.append(("if", sub(s[1]), _inline(s[2], env), _inline(s[3], env)))
        else:
            out.append(s)
    return out


_TPL = [(op, _inline(_parse_stmts(src))[0]) for op, src in TEMPLATES]

# pattern variables of each template that stand for arrays
_BUFFER_OPERANDS = {"gemm": "ABC", "add_scaled": "CA", "avg2": "DXY", "scale": "D", "transpose": "TX",
                    "copy": "DX", "sumsq": "Xs", "rec_prefix": "vS", "rec_decay": "wp", "lcg_fill": "L",
                    "copy_interior": "pq", "stencil19": ["p", "q", "res"]}


def _match(t, s, env):
    """Structural match of template node t against source node s; pattern
    variables and loop-variable renamings are recorded in env."""
    if isinstance(t, list):
        return isinstance(s, list) and len(t) == len(s) and all(_match(a, b, env) for a, b in zip(t, s))
    if not isinstance(t, tuple):
        return t == s
    if not (isinstance(s, tuple) and s and s[0] == t[0] and len(s) == len(t)):
        if t[0] == "var" and t[1].startswith("$") and isinstance(s, tuple):
            pass            # a pattern variable matches any expression
        else:
            return False
    kind = t[0]
    if kind == "num":
        # a float literal of the template matches the same value written as a
        # float or an integer literal (C converts the integer exactly); a
        # double literal makes the expression double arithmetic: no match
        if s[1] != t[1]:
            return False
        return s[2] == t[2] or (t[2] == "f" and s[2] == "i" and abs(s[1]) < 2 ** 24)
    if kind == "var":
        if t[1].startswith("$"):
            if t[1] in env:
                return env[t[1]] == s
            env[t[1]] = s
            return True
        if ("loop", t[1]) in env:
            return s == ("var", env[("loop", t[1])])
        return s == t
    if kind == "ref":
        return _match(("var", t[1]), ("var", s[1]), env) and _match(t[2], s[2], env)
    if kind == "bin" and t[1] in "+*" and s[1] == t[1]:
        # one addition or product may have its operands swapped (a + b and
        # b + a round alike); grouping is kept, (a + b) + c != a + (b + c)
        saved = dict(env)
        if _match(t[2], s[2], env) and _match(t[3], s[3], env):
            return True
        env.clear()
        env.update(saved)
        return _match(t[2], s[3], env) and _match(t[3], s[2], env)
    if kind == "for":
        env[("loop", t[1])] = s[1]
        return _match(t[2], s[2], env) and _match(t[3], s[3], env) and _match(t[4], s[4], env)
    return all(_match(a, b, env) for a, b in zip(t[1:], s[1:]))


class _NoMatch(Exception):
    pass


def _literal(e, what):
    """Value of a float (or integer) literal operand; a double literal, or
    anything but a literal, is not the library's float operation."""
    neg = e[0] == "neg"
    if neg:
        e = e[1]
    if e[0] != "num" or e[2] == "d" or (e[2] == "i" and abs(e[1]) >= 2 ** 24):
        raise _NoMatch(what)
    return -e[1] if neg else e[1]


def _bind(nest, dtypes):
    """(op, args) of a nest by template, or None when no operation of the
    library has its body (the nest then keeps its source text and runs on
    the CPU)."""
    if _has_break(nest):
        return None
    try:
        return _bind_template(nest, dtypes)
    except _NoMatch:
        return None


def _bind_template(nest, dtypes):
    src = _inline([nest])[0]
    for op, tpl in _TPL:
        env = {}
        if not _match(tpl, src, env):
            continue
        v = {k[1:]: e for k, e in env.items() if isinstance(k, str)}
        buf = {k: e[1] for k, e in v.items() if e[0] == "var"}
        for name in _BUFFER_OPERANDS[op]:
            if v[name][0] != "var" or v[name][1] not in dtypes:
                raise _NoMatch(name)
        if op == "gemm":
            kinds = {dtypes.get(buf[x]) for x in "AB"}
            if kinds == {"bf16"}:
                op = "gemm_bf16"
            elif kinds != {"f32"}:
                raise _NoMatch("product operand types")
            return op, {"A": buf["A"], "B": buf["B"], "C": buf["C"]}
        if op == "add_scaled":
            return op, {"C": buf["C"], "A": buf["A"], "alpha": _literal(v["alpha"], "alpha")}
        if op == "avg2":
            return op, {"S": buf["D"], "X": buf["X"], "Y": buf["Y"]}
        if op == "scale":
            return op, {"D": buf["D"], "beta": _literal(v["beta"], "beta")}
        if op == "copy":
            return op, {"dst": buf["D"], "src": buf["X"]}
        if op == "transpose":
            return op, {"src": buf["X"], "dst": buf["T"]}
        if op == "sumsq":
            return op, {"x": buf["X"], "s": buf["s"]}
        if op == "rec_prefix":
            return op, {"v": buf["v"], "S": buf["S"]}
        if op == "rec_decay":
            return op, {"w": buf["w"], "p": buf["p"]}
        if op == "lcg_fill":
            return op, {"L": buf["L"], "seed32": int(_literal(v["seed"], "the generator seed"))}
        if op == "copy_interior":
            return op, {"dst": buf["p"], "src": buf["q"]}
        if op == "stencil19":
            if v["n"][0] != "var":
                raise _NoMatch("the residual slot must be the repeat variable")
            return op, {"p": buf["p"], "q": buf["q"], "res": buf["res"], "slot": v["n"][1]}
    for bind in (_bind_init, _bind_cast):
        got = bind(src)
        if got:
            return got
    return None


def _rows(src):
    """Statements of a two-deep i, j nest and its loop variables, or None."""
    if src[0] != "for" or len(src[4]) != 1 or src[4][0][0] != "for":
        return None
    i, j = src[1], src[4][0][1]
    body = src[4][0][4]
    if not body or any(s[0] != "assign" or s[1][0] != "ref" or s[1][2] != [("var", i), ("var", j)]
                       for s in body):
        return None
    return i, j, body


def _bind_init(src):
    # X[i][j] = u01(stream, i, j); one statement per buffer
    got = _rows(src)
    if not got:
        return None
    i, j, body = got
    outs, streams = [], []
    for s in body:
        e = s[3]
        if not (e[0] == "call" and e[1] == "u01" and len(e[2]) == 3 and e[2][0][0] == "num"
                and e[2][1] == ("var", i) and e[2][2] == ("var", j)):
            return None
        outs.append(s[1][1])
        streams.append(int(e[2][0][1]))
    return "init_uniform", {"out": outs, "streams": streams}


def _bind_cast(src):
    # Xb[i][j] = bf16(X[i][j]); one statement per buffer
    got = _rows(src)
    if not got:
        return None
    i, j, body = got
    dst, srcs = [], []
    for s in body:
        e = s[3]
        if not (e[0] == "call" and e[1] == "bf16" and len(e[2]) == 1 and e[2][0][0] == "ref"
                and e[2][0][2] == [("var", i), ("var", j)]):
            return None
        dst.append(s[1][1])
        srcs.append(e[2][0][1])
    return "cast_bf16", {"dst": dst, "src": srcs}


def _has_break(stmt):
    if stmt[0] == "break":
        return True
    if stmt[0] == "for":
        return any(_has_break(b) for b in stmt[4])
    if stmt[0] == "if":
        return any(_has_break(b) for b in stmt[2] + stmt[3])
    return False


def _loop_vars(stmt):
    out = []
    if stmt[0] == "for":
        out.append(stmt[1])
        for s in stmt[4]:
            for v in _loop_vars(s):
                if v not in out:
                    out.append(v)
    return out


# ------------------------------------------------------------------ nests -> IR
def _loops(stmt):
    out = []

    def walk(s):
        if s[0] != "for":
            return
        if s[1] not in [l[0] for l in out]:
            out.append([s[1], _affine(s[2]), _affine(s[3])])
        for b in s[4]:
            walk(b)
    walk(stmt)
    return out


def _accesses(stmt, loop_vars):
    """IR access list of a nest: [buf, mode, subscript...] and its flags.

    Per array element (buffer + subscripts), in statement order: a read before
    any plain write of the same element is exposed; an element written and
    exposed is "rw", written only "w", read only "r".  A buffer touched only
    by += whose subscripts use none of the nest's loop variables is a sum
    reduction ("sum")."""
    events, flags = [], set()

    def exprs(e):
        if e[0] == "ref":
            events.append(("r", e))
            for x in e[2]:
                exprs(x)
        elif e[0] == "bin":
            exprs(e[2])
            exprs(e[3])
        elif e[0] in ("neg", "addr", "not"):
            exprs(e[1])
        elif e[0] == "cast":
            exprs(e[2])
        elif e[0] == "call":
            if e[1] not in PURE_CALLS:
                flags.add("opaque_call")
            for x in e[2]:
                exprs(x)

    locals_ = set()
    leaves = _has_break(stmt)

    def walk(s, cond):
        # cond: the statement may not run in every iteration (under an if,
        # or in a loop that can be left early), so its writes may leave the
        # old values in place: they count as reads of the element too
        if s[0] == "for":
            for b in s[4]:
                walk(b, cond)
        elif s[0] == "if":
            exprs(s[1])
            for b in s[2] + s[3]:
                walk(b, True)
        elif s[0] == "local":
            locals_.add(s[2])
            exprs(s[3])
        elif s[0] == "assign":
            if s[1][0] == "var":
                if s[1][1] not in locals_:
                    raise CError("assignment to %s: assignments go to array elements or declared locals" % s[1][1])
                exprs(s[3])
                return
            if s[1][0] != "ref":
                raise CError("assignments go to array elements (a local is declared with its type)")
            exprs(s[3])
            for x in s[1][2]:
                exprs(x)
            if s[2] == "=":
                events.append(("cw" if cond else "w", s[1]))
            else:
                events.append(("u+" if s[2] == "+=" and not cond else "u", s[1]))
        elif s[0] == "break":
            flags.add("early_exit")
    walk(stmt, leaves)

    def key(ref):
        return ref[1], tuple(_affine(e) for e in ref[2])

    sums = set()
    for buf in {ref[1] for _, ref in events}:
        mine = [(m, ref) for m, ref in events if ref[1] == buf]
        if all(m == "u+" for m, _ in mine) and not any(
                _names_in(x) & set(loop_vars) for _, ref in mine for x in ref[2]):
            sums.add(buf)
    order, state = [], {}
    for m, ref in events:
        k = key(ref)
        if k not in state:
            order.append(k)
            state[k] = {"w": False, "exposed": False}
        st = state[k]
        if m in ("r", "u", "u+", "cw") and not st["w"]:
            st["exposed"] = True
        if m in ("w", "u", "u+", "cw"):
            st["w"] = True
    writes = [k for k in order if state[k]["w"]]
    reads = [k for k in order if not state[k]["w"]]
    acc = []
    for buf, subs in writes + reads:
        st = state[(buf, subs)]
        if buf in sums:
            mode = "sum"
        elif st["w"]:
            mode = "rw" if st["exposed"] else "w"
        else:
            mode = "r"
        acc.append([buf, mode] + list(subs))
    return acc, sorted(flags)


def _names_in(e):
    out = set()
    if e[0] == "var":
        out.add(e[1])
    elif e[0] == "ref":
        for x in e[2]:
            out |= _names_in(x)
    elif e[0] == "bin":
        out |= _names_in(e[2]) | _names_in(e[3])
    return out


_NEST_NAMES = {
    "init_uniform": lambda a: "init_" + "".join(a["out"]),
    "gemm": lambda a: "gemm_" + a["C"],
    "gemm_bf16": lambda a: "gemm_bf16_" + a["C"],
    "add_scaled": lambda a: "axpy_" + a["C"],
    "avg2": lambda a: "avg_" + a["S"],
    "scale": lambda a: "scale_" + a["D"],
    "copy": lambda a: "copy_" + a["dst"],
    "transpose": lambda a: "transpose_" + a["dst"],
    "sumsq": lambda a: "sumsq_" + a["x"],
    "cast_bf16": lambda a: "cast_bf16",
    "rec_prefix": lambda a: "rec_prefix_" + a["v"],
    "rec_decay": lambda a: "rec_decay_" + a["w"],
    "lcg_fill": lambda a: "lcg_fill_" + a["L"],
    "copy_interior": lambda a: "copy_interior",
    "stencil19": lambda a: "stencil19",
}

def _walk_nodes(x, fn):
    """Call fn on every expression and statement node of a parsed tree."""
    if isinstance(x, list):
        for y in x:
            _walk_nodes(y, fn)
    elif isinstance(x, tuple) and x and isinstance(x[0], str):
        fn(x)
        for y in x[1:]:
            if isinstance(y, (list, tuple)):
                _walk_nodes(y, fn)


def _calls_in(stmt):
    out = set()
    _walk_nodes(stmt, lambda n: out.add(n[1]) if n[0] in ("call", "callstmt") else None)
    return out


def _names_used(stmt):
    out = set()

    def add(n):
        if n[0] in ("var", "ref"):
            out.add(n[1])
    _walk_nodes(stmt, add)
    return out


def _const_int(text, params):
    """Value of a bound written as in the IR ('N-1', '0', 'K')."""
    total, sign, pos = 0, 1, 0
    for m in re.finditer(r"\s*([+-]?)\s*([A-Za-z_]\w*|\d+)", text):
        if m.start() != pos:
            raise CError("bound %r is not a constant" % text)
        pos = m.end()
        sign = -1 if m.group(1) == "-" else 1
        tok = m.group(2)
        if tok.isdigit():
            total += sign * int(tok)
        elif tok in params:
            total += sign * params[tok]
        else:
            return None
    return total if pos == len(text) else None


def _fits(op, args, loops, buffers, params, rvars):
    """Whether a nest bound to `op` is exactly that operation of the library:
    operand types and shapes as the operation takes them and loops over the
    whole index space it covers (the interior of the grid for the sweep and
    the interior copy); otherwise the nest keeps its own source text."""
    info = {}
    for b in buffers:
        dims = [_const_int(d, params) for d in b["dims"]]
        info[b["name"]] = (b["dtype"], dims)
    L = [(_const_int(lo, params), _const_int(hi, params)) for _, lo, hi in loops]
    if any(lo is None or hi is None for lo, hi in L):
        return False

    def dt(n):
        return info[n][0]

    def dims(n):
        return info[n][1]

    def full(n):
        return L == [(0, d) for d in dims(n)]

    def interior(n):
        return L == [(1, d - 1) for d in dims(n)]

    def nbytes(n):
        c = 1
        for d in dims(n):
            c *= d
        return c * {"f32": 4, "f64": 8, "bf16": 2}[dt(n)]

    a = args
    if op == "init_uniform":
        return all(dt(x) == "f32" and full(x) for x in a["out"])
    if op in ("gemm", "gemm_bf16"):
        A, B, C = dims(a["A"]), dims(a["B"]), dims(a["C"])
        return (dt(a["C"]) == "f32" and len(A) == len(B) == len(C) == 2 and A[1] == B[0] and C == [A[0], B[1]]
                and L == [(0, A[0]), (0, B[1]), (0, A[1])])
    if op == "add_scaled":
        return dt(a["C"]) == dt(a["A"]) == "f32" and dims(a["C"]) == dims(a["A"]) and full(a["C"])
    if op == "avg2":
        return (all(dt(a[k]) == "f32" for k in "SXY") and dims(a["S"]) == dims(a["X"]) == dims(a["Y"])
                and full(a["S"]))
    if op == "scale":
        return dt(a["D"]) == "f32" and full(a["D"])
    if op == "copy":
        return dt(a["dst"]) == dt(a["src"]) and dims(a["dst"]) == dims(a["src"]) and full(a["dst"])
    if op == "cast_bf16":
        return all(dt(d) == "bf16" and dt(x) == "f32" and dims(d) == dims(x) and full(d)
                   for d, x in zip(a["dst"], a["src"]))
    if op == "transpose":
        S, T = dims(a["src"]), dims(a["dst"])
        return (dt(a["src"]) == dt(a["dst"]) == "f32" and len(S) == 2 and T == S[::-1] and a["src"] != a["dst"]
                and full(a["src"]))
    if op == "sumsq":
        return dt(a["x"]) == "f32" and dt(a["s"]) == "f64" and full(a["x"])
    if op == "stencil19":
        slot = dict(rvars)
        return (dt(a["p"]) == dt(a["q"]) == "f32" and dt(a["res"]) == "f64" and len(dims(a["p"])) == 3
                and dims(a["p"]) == dims(a["q"]) and a["p"] != a["q"] and interior(a["p"])
                and (dims(a["p"])[0] + 6) * dims(a["p"])[1] * dims(a["p"])[2] * 4 < 2 ** 31 and a["slot"] in slot)
    if op == "copy_interior":
        return (dt(a["dst"]) == dt(a["src"]) == "f32" and len(dims(a["dst"])) == 3
                and dims(a["dst"]) == dims(a["src"]) and interior(a["dst"]) and nbytes(a["dst"]) < 2 ** 31)
    if op == "rec_prefix":
        return dt(a["v"]) == dt(a["S"]) == "f32" and len(dims(a["v"])) == 1 and L == [(1, dims(a["v"])[0])]
    if op == "rec_decay":
        return dt(a["w"]) == dt(a["p"]) == "f32" and len(dims(a["w"])) == 1 and L == [(1, dims(a["w"])[0])]
    if op == "lcg_fill":
        return dt(a["L"]) == "f32" and full(a["L"])
    return True


# The C++ the host object is compiled from: the program's parameters, the
# bf16 storage type and one entry point per host_code nest, whose body is the
# nest's own text.
_HOST_PRELUDE = """// Host forms of loop nests that no operation of the library implements,
// each the nest's own source text (written by the C front end).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <math.h>
#include <stdlib.h>

namespace {
// bf16 storage: bf16(x) rounds a float to the nearest bfloat16 (ties to
// even, NaN kept quiet); reading one gives its exact float value
struct bf16 {
    uint16_t bits;
    bf16() = default;
    bf16(float f) {
        uint32_t u;
        std::memcpy(&u, &f, 4);
        if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) bits = (uint16_t)((u >> 16) | 0x40u);
        else bits = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    }
    operator float() const {
        const uint32_t u = (uint32_t)bits << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return f;
    }
};
static_assert(sizeof(bf16) == 2, "bf16 storage");
}  // namespace
"""

_CTYPE = {"f32": "float", "f64": "double", "bf16": "bf16"}


def host_unit(params, buffers, host_code):
    """Translation unit of an application's host_code nests.  Each entry
    point takes the host copy of every buffer (declaration order) and the
    repeat variables' values (by repeat id)."""
    out = [_HOST_PRELUDE]
    for k, v in params.items():
        out.append("#define %s %d" % (k, v))
    index = {b["name"]: i for i, b in enumerate(buffers)}
    for h in host_code:
        out.append('extern "C" void %s(void *const *ofl_buf, const int64_t *ofl_rep) {' % h["symbol"])
        for name in h["buffers"]:
            b = buffers[index[name]]
            ty, dims = _CTYPE[b["dtype"]], b["dims"]
            if len(dims) == 1:
                out.append("    %s *%s = static_cast<%s *>(ofl_buf[%d]);" % (ty, name, ty, index[name]))
            else:
                inner = "".join("[%s]" % d for d in dims[1:])
                out.append("    %s (*%s)%s = reinterpret_cast<%s (*)%s>(ofl_buf[%d]);"
                           % (ty, name, inner, ty, inner, index[name]))
        for var, rid in h["repeats"]:
            out.append("    const int %s = (int)ofl_rep[%d];" % (var, rid))
        out.append("#line %d" % h["line"])
        out.append(h["text"])
        out.append("}")
    return "\n".join(out) + "\n"


HOST_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_hostobj")
HOST_CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-w"]


def build_host_object(unit):
    """Compile a host translation unit (once per distinct text) into a shared
    object under _hostobj/; returns its path."""
    key = hashlib.sha256(unit.encode()).hexdigest()[:16]
    so = os.path.join(HOST_CACHE, "host_%s.so" % key)
    if os.path.exists(so):
        return so
    os.makedirs(HOST_CACHE, exist_ok=True)
    src = os.path.join(HOST_CACHE, "host_%s.cpp" % key)
    tmp = so + ".tmp%d" % os.getpid()
    with open(src, "w") as f:
        f.write(unit)
    cxx = os.environ.get("OFL_HOST_CXX", "g++")
    r = subprocess.run([cxx] + HOST_CXXFLAGS + [src, "-o", tmp, "-lm"], capture_output=True, text=True)
    if r.returncode != 0:
        raise CError("the host form of a nest does not compile:\n" + r.stderr[-2000:])
    os.replace(tmp, so)
    return so


_DEFINE = re.compile(r"\s*#define\s+([A-Za-z_]\w*)\s+(-?\d+)\s*$")
_ARRAY = re.compile(r"\s*(float|double|bf16)\s+([A-Za-z_]\w*)((?:\s*\[[^\]]+\])+)\s*;\s*(?://\s*ofl:(.*))?$")
_PRAGMA = re.compile(r"\s*#pragma\s+ofl\s+prec\((\w+)\)\s*$")


def parse(src, name="app"):
    """Application IR (a dict, as ofl_app_load_json takes it) of C source.

    ``#pragma ofl prec(bf16x3|fp8x2|f32)`` on the line before a top-level
    product nest sets the arithmetic of its offloaded form; ``#pragma acc``
    lines (as ``offloaded_source`` writes them) are ignored."""
    return _parse(src, name)[0]


def _parse(src, name):
    """(IR, [(line, first on its line)] of each nest's outer for, in program order)."""
    params, buffers, program, at = {}, [], [], []
    body_lines = []
    for line in src.splitlines():
        m = _DEFINE.match(line)
        if m:
            params[m.group(1)] = int(m.group(2))
            body_lines.append("")
            continue
        m = _ARRAY.match(line)
        if m:
            dims = [d.strip() for d in re.findall(r"\[([^\]]+)\]", m.group(3))]
            b = {"name": m.group(2), "dtype": TYPES[m.group(1)], "dims": dims, "setup": "zero",
                 "output": False}
            for opt in (m.group(4) or "").split():
                if opt == "output":
                    b["output"] = True
                elif opt.startswith("setup="):
                    b["setup"] = opt.split("=", 1)[1]
                elif opt.startswith("mode="):
                    b["mode"] = opt.split("=", 1)[1]
                else:
                    raise CError("unknown buffer annotation %r" % opt)
            buffers.append(b)
            body_lines.append("")
            continue
        m = _PRAGMA.match(line)
        if m:
            line = "@prec %s;" % m.group(1)
        elif re.match(r"\s*#pragma\s+acc\b", line):
            line = ""
        elif line.lstrip().startswith("#"):
            raise CError("unsupported directive: %s" % line.strip())
        body_lines.append(line)
    dtypes = {b["name"]: b["dtype"] for b in buffers}
    names_used = {}

    def block_ir(stmt):
        # a call of a library routine the library implements on both sides
        # becomes a function block: one nest, one gene bit
        name, args = stmt[1], stmt[2]
        if name not in FUNCTION_BLOCKS:
            raise CError("call of %s: not a known library routine (only %s)" % (name, ", ".join(FUNCTION_BLOCKS)))
        if name == "sgemm":
            return gemm_block_ir(stmt)
        if name in ("saxpy", "scopy", "sscal"):
            return blas1_block_ir(stmt)
        if len(args) != 1 or args[0][0] != "var" or args[0][1] not in dtypes:
            raise CError("%s takes one declared array" % name)
        x = args[0][1]
        b = next(b for b in buffers if b["name"] == x)
        if b["dtype"] != "f32" or len(b["dims"]) != 2:
            raise CError("%s needs a 2-D float array (rows of interleaved complex values, or of real values "
                         "for rfft_rows / irfft_rows)" % name)
        at.append(where[id(stmt)] + ("call",))
        base = {"fft_rows": "fft_", "ifft_rows": "ifft_", "rfft_rows": "rfft_", "irfft_rows": "irfft_"}[name] + x
        names_used[base] = names_used.get(base, 0) + 1
        fa = {"x": x}
        if name in ("ifft_rows", "irfft_rows"):
            fa["inverse"] = 1
        if name in ("rfft_rows", "irfft_rows"):
            fa["real"] = 1
        return {"nest": base if names_used[base] == 1 else "%s_%d" % (base, names_used[base]),
                "op": FUNCTION_BLOCKS[name], "args": fa,
                "loops": [["r", "0", b["dims"][0]], ["e", "0", b["dims"][1]]], "access": [[x, "rw", "r", "e"]]}

    def blas1_block_ir(stmt):
        name, args = stmt[1], stmt[2]
        nscal = 0 if name == "scopy" else 1
        narr = 1 if name == "sscal" else 2
        if len(args) != nscal + narr:
            raise CError("%s takes %s" % (name, {"saxpy": "alpha, X, Y", "scopy": "X, Y", "sscal": "alpha, X"}[name]))
        alpha = None
        if nscal:
            a = args[0]
            sign = 1.0
            if a[0] == "neg":
                sign, a = -1.0, a[1]
            if a[0] != "num":
                raise CError("%s: alpha must be a number" % name)
            # the routine's float parameter: the literal converted to float
            alpha = float(np.float32(sign * a[1]))
        arrs = args[nscal:]
        if any(a[0] != "var" or a[1] not in dtypes for a in arrs):
            raise CError("%s takes declared arrays" % name)
        bufs = [next(b for b in buffers if b["name"] == a[1]) for a in arrs]
        if any(b["dtype"] != "f32" for b in bufs) or any(b["dims"] != bufs[0]["dims"] for b in bufs):
            raise CError("%s: float arrays of one shape" % name)
        loops = [[v, "0", d] for v, d in zip("ijklmn", bufs[0]["dims"])]
        sub = [l[0] for l in loops]
        if name == "saxpy":
            op, a = "add_scaled", {"C": bufs[1]["name"], "A": bufs[0]["name"], "alpha": alpha}
            acc = [[bufs[1]["name"], "rw"] + sub, [bufs[0]["name"], "r"] + sub]
        elif name == "scopy":
            op, a = "copy", {"dst": bufs[1]["name"], "src": bufs[0]["name"]}
            acc = [[bufs[1]["name"], "w"] + sub, [bufs[0]["name"], "r"] + sub]
        else:
            op, a = "scale", {"D": bufs[0]["name"], "beta": alpha}
            acc = [[bufs[0]["name"], "rw"] + sub]
        at.append(where[id(stmt)] + ("call",))
        base = _NEST_NAMES[op](a)
        names_used[base] = names_used.get(base, 0) + 1
        return {"nest": base if names_used[base] == 1 else "%s_%d" % (base, names_used[base]), "op": op, "args": a,
                "loops": loops, "access": acc}

    def gemm_block_ir(stmt):
        args = stmt[2]
        if len(args) != 3 or any(a[0] != "var" or a[1] not in dtypes for a in args):
            raise CError("sgemm takes three declared arrays: A, B, C")
        A, B, Cm = (next(b for b in buffers if b["name"] == a[1]) for a in args)
        if any(len(b["dims"]) != 2 for b in (A, B, Cm)):
            raise CError("sgemm needs 2-D arrays")
        if A["dims"][1] != B["dims"][0] or Cm["dims"] != [A["dims"][0], B["dims"][1]]:
            raise CError("sgemm: C[M][N] = A[M][K] B[K][N] needs matching extents")
        kinds = {A["dtype"], B["dtype"]}
        if kinds not in ({"f32"}, {"bf16"}) or Cm["dtype"] != "f32":
            raise CError("sgemm: float or bf16 operands and a float result")
        op = "gemm_bf16" if kinds == {"bf16"} else "gemm"
        at.append(where[id(stmt)] + ("call",))
        a = {"A": A["name"], "B": B["name"], "C": Cm["name"]}
        base = _NEST_NAMES[op](a)
        names_used[base] = names_used.get(base, 0) + 1
        return {"nest": base if names_used[base] == 1 else "%s_%d" % (base, names_used[base]), "op": op, "args": a,
                "loops": [["i", "0", A["dims"][0]], ["j", "0", B["dims"][1]], ["k", "0", A["dims"][1]]],
                "access": [[Cm["name"], "w", "i", "j"], [A["name"], "r", "i", "k"], [B["name"], "r", "k", "j"]]}

    def nest_ir(stmt, prec, rvars=()):
        at.append(where[id(stmt)] + ("loop",))
        loops = _loops(stmt)
        acc, flags = _accesses(stmt, [l[0] for l in loops])
        got = _bind(stmt, dtypes)
        if got is not None and not _fits(got[0], got[1], loops, buffers, params, rvars):
            got = None
        if got is None:
            if prec is not None:
                raise CError("prec applies to float products only")
            return host_nest_ir(stmt, loops, acc, flags, rvars)
        op, args = got
        if prec is not None:
            if op != "gemm":
                raise CError("prec applies to float products only")
            args["prec"] = prec
        base = _NEST_NAMES[op](args)
        names_used[base] = names_used.get(base, 0) + 1
        n = {"nest": base if names_used[base] == 1 else "%s_%d" % (base, names_used[base]), "op": op,
             "args": args, "loops": loops, "access": acc}
        if flags:
            n["flags"] = flags
        return n

    def host_nest_ir(stmt, loops, acc, flags, rvars):
        # no operation of the library has this body: the nest keeps its own
        # source text, compiled for the CPU into the application's host
        # object; it never runs on the GPU
        line = where[id(stmt)][0]
        calls = _calls_in(stmt)
        for c in ("u01", "lcg01"):
            if c in calls:
                raise CError("line %d: %s() is available only in the nest forms the library implements" % (line, c))
        name = "host_L%d" % line
        names_used[name] = names_used.get(name, 0) + 1
        if names_used[name] > 1:
            name = "%s_%d" % (name, names_used[name])
        a, b = spans[id(stmt)]
        used = _names_used(stmt)
        host_code.append({"symbol": "ofl_" + name, "text": body_text[a:b], "line": line,
                          "buffers": [bf["name"] for bf in buffers if bf["name"] in used],
                          "repeats": [(v, rid) for v, rid in rvars if v in used]})
        n = {"nest": name, "op": "host_code", "args": {"symbol": "ofl_" + name},
             "loops": loops, "access": acc, "source": body_text[a:b]}
        if flags:
            n["flags"] = flags
        return n

    prec, where, spans, host_code = None, {}, {}, []
    n_repeats = 0
    body_text = "\n".join(body_lines)
    for stmt in _parse_stmts(body_text, where, spans):
        if stmt[0] == "pragma":
            prec = stmt[2]
            continue
        if stmt[0] == "callstmt":
            nest = block_ir(stmt)
            if prec is not None:
                if nest["op"] != "gemm":
                    raise CError("prec applies to float products only")
                nest["args"]["prec"] = prec
            program.append(nest)
            prec = None
            continue
        if stmt[0] != "for":
            raise CError("top-level statements are for loops and library calls")
        inner = stmt[4]
        if len(inner) >= 2 and all(s[0] == "for" for s in inner):
            if _affine(stmt[2]) != "0":
                raise CError("a repeat loop counts from 0")
            rvars = [(stmt[1], n_repeats)]
            n_repeats += 1
            program.append({"repeat": _affine(stmt[3]), "var": stmt[1],
                            "body": [nest_ir(s, None, rvars) for s in inner]})
        else:
            program.append(nest_ir(stmt, prec))
        prec = None
    doc = {"name": name, "params": params, "buffers": buffers, "program": program}
    if host_code:
        doc["host_object"] = build_host_object(host_unit(params, buffers, host_code))
    return doc, at


_REASONS = {1: "a data dependence between iterations", 2: "a call of an external routine",
            3: "a break out of the loop", 4: "no GPU form of its body"}


def offloaded_source(src, verdicts, gene):
    """The program with the offload pattern written in: ``#pragma acc
    kernels`` before each nest whose gene bit is 1 (Sec. 4: the directive
    goes on the loops the gene selects; a 0 bit leaves the loop on the CPU),
    and a comment before each nest the dependence check excluded.

    verdicts: (verdict, reason, gene position) per nest in program order, as
    App.verdicts() gives them; gene: one 0/1 per accepted nest."""
    _, at = _parse(src, "app")
    if len(verdicts) != len(at):
        raise ValueError("%d verdicts for %d nests" % (len(verdicts), len(at)))
    if len(gene) != sum(1 for v in verdicts if v[2] >= 0):
        raise ValueError("gene length does not match the accepted nests")
    lines = src.split("\n")
    insert = {}
    for (verdict, reason, pos), (line, first, kind) in zip(verdicts, at):
        if not first:
            raise CError("line %d: a nest must begin its line to take a directive" % line)
        text = lines[line - 1]
        indent = text[:len(text) - len(text.lstrip())]
        if pos < 0:
            insert[line] = indent + "/* not offloadable: %s */" % _REASONS.get(reason, "rejected")
        elif gene[pos] and kind == "call":
            insert[line] = indent + "/* function block: the GPU implementation replaces this call */"
        elif gene[pos]:
            insert[line] = indent + "#pragma acc kernels"
    out = []
    for n, text in enumerate(lines, 1):
        if n in insert:
            out.append(insert[n])
        out.append(text)
    return "\n".join(out)


def load(path):
    """Application IR of a C source file (named after the file)."""
    with open(path) as f:
        return parse(f.read(), re.sub(r"\.c$", "", path.rsplit("/", 1)[-1]))


def main(argv=None):
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="C loop nests -> application IR (JSON on stdout)")
    ap.add_argument("source")
    ap.add_argument("--name", default=None)
    args = ap.parse_args(argv)
    doc = load(args.source)
    if args.name:
        doc["name"] = args.name
    json.dump(doc, sys.stdout, indent=1)
    print()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
