"""Oracle reader for an application description (test infrastructure only).

An application is what the paper's offloader takes in: a program made of
for-loop nests over arrays (Sec. 4: the source is parsed, every for statement
found and counted).  Here the parsed form is given directly as JSON:

* ``params``   -- named integer sizes (N, I, J, K, S, ...)
* ``buffers``  -- arrays: name, dtype (f32 / f64 / bf16), dims (expressions),
                  set-up content ("zero" or the "sin" mode field), output flag
* ``program``  -- a list of nests and ``repeat`` blocks (a repeat is control
                  flow, never a gene candidate)
* a nest       -- ``op`` (the body kind) with ``args``; ``loops`` as
                  [var, lo, hi) from the outermost level inward; ``access`` as
                  [buf, mode, subscript...] with mode r / w / rw / sum;
                  ``flags`` (opaque_call, early_exit)

Expressions are sums of integers, parameter names and at most one loop or
repeat variable with coefficient +1 (affine subscripts ``var + c``).
"""
import json
import re

_TOK = re.compile(r"\s*([A-Za-z_][A-Za-z_0-9]*|\d+|[+-])")

DTYPE_BYTES = {"f32": 4, "f64": 8, "bf16": 2}


def _tokens(s):
    s = str(s).strip()
    pos, out = 0, []
    while pos < len(s):
        m = _TOK.match(s, pos)
        if not m:
            raise ValueError("bad expression %r" % s)
        out.append(m.group(1))
        pos = m.end()
        while pos < len(s) and s[pos].isspace():
            pos += 1
    return out


def parse_expr(s, params, variables=()):
    """Return (var or None, const) for an affine expression 'var + c'."""
    toks = _tokens(s)
    sign, expect_term = 1, True
    var, const = None, 0
    for t in toks:
        if t in "+-":
            if expect_term:
                sign = -sign if t == "-" else sign
            else:
                sign = -1 if t == "-" else 1
                expect_term = True
            continue
        if not expect_term:
            raise ValueError("missing operator in %r" % s)
        if t.isdigit():
            const += sign * int(t)
        elif t in params:
            const += sign * int(params[t])
        elif t in variables:
            if var is not None or sign != 1:
                raise ValueError("non-affine subscript %r" % s)
            var = t
        else:
            raise ValueError("unknown name %r in %r" % (t, s))
        sign, expect_term = 1, False
    if expect_term:
        raise ValueError("dangling operator in %r" % s)
    return var, const


def eval_const(s, params):
    var, c = parse_expr(s, params)
    if var is not None:
        raise ValueError("expected constant expression: %r" % s)
    return c


class Buffer:
    def __init__(self, d, params):
        self.name = d["name"]
        self.dtype = d.get("dtype", "f32")
        self.dims = [eval_const(x, params) for x in d["dims"]]
        self.setup = d.get("setup", "zero")
        mode = d.get("mode", 1)
        self.mode = eval_const(mode, params) if self.setup == "sin" else 0
        self.output = bool(d.get("output", False))
        n = 1
        for x in self.dims:
            n *= x
        self.count = n
        self.elem_bytes = DTYPE_BYTES[self.dtype]
        self.nbytes = n * self.elem_bytes


class Access:
    """One array reference of a nest: subscripts are (var or None, const)."""

    def __init__(self, buf, mode, subs):
        self.buf, self.mode, self.subs = buf, mode, subs


class Nest:
    def __init__(self, d, params, index, repeat_vars):
        self.index = index
        self.name = d.get("nest", d["op"])
        self.op = d["op"]
        self.args = d.get("args", {})
        self.flags = list(d.get("flags", []))
        self.loops = []
        for var, lo, hi in d["loops"]:
            self.loops.append((var, eval_const(lo, params), eval_const(hi, params)))
        loop_vars = [v for v, _, _ in self.loops]
        allvars = set(loop_vars) | set(repeat_vars)
        self.access = []
        for a in d["access"]:
            buf, mode, subs = a[0], a[1], a[2:]
            if mode not in ("r", "w", "rw", "sum"):
                raise ValueError("bad access mode %r" % mode)
            self.access.append(Access(buf, mode, [parse_expr(s, params, allvars) for s in subs]))
        self.repeat_vars = dict(repeat_vars)   # name -> trip count


class App:
    """Parsed application: buffers, nests in program order, program tree."""

    def __init__(self, doc):
        if isinstance(doc, str):
            doc = json.loads(doc)
        self.doc = doc
        self.name = doc.get("name", "app")
        self.params = {k: int(v) for k, v in doc.get("params", {}).items()}
        self.buffers = [Buffer(b, self.params) for b in doc["buffers"]]
        self.buf_index = {b.name: i for i, b in enumerate(self.buffers)}
        self.nests = []
        self.program = self._walk(doc["program"], {})
        for n in self.nests:
            for a in n.access:
                if a.buf not in self.buf_index:
                    raise ValueError("nest %s: unknown buffer %s" % (n.name, a.buf))

    def _walk(self, items, repeat_vars):
        out = []
        for it in items:
            if "repeat" in it:
                count = eval_const(it["repeat"], self.params)
                rv = dict(repeat_vars)
                rv[it["var"]] = count
                out.append(("repeat", it["var"], count, self._walk(it["body"], rv)))
            else:
                n = Nest(it, self.params, len(self.nests), rv_copy(repeat_vars))
                self.nests.append(n)
                out.append(("nest", n.index))
        return out

    def buffer(self, name):
        return self.buffers[self.buf_index[name]]


def rv_copy(d):
    return dict(d)


def load(path_or_doc, params=None):
    """Load an application; ``params`` overrides entries of its params block."""
    if isinstance(path_or_doc, dict):
        doc = json.loads(json.dumps(path_or_doc))
    elif str(path_or_doc).lstrip().startswith("{"):
        doc = json.loads(path_or_doc)
    else:
        with open(path_or_doc) as f:
            doc = json.load(f)
    if params:
        doc.setdefault("params", {}).update(params)
    return App(doc)
