"""Oracle parallelisability check of each loop nest (test infrastructure only).

Sec. 4 of the paper: every for statement gets the parallel directive on its
own and is compiled; a compile error excludes it.  The error kinds named are an
external routine called in the loop, several levels of one nest specified
twice, leaving the loop early (break), and a data dependence between the loop's
iterations.  The nests that pass number ``a`` and become the gene, one bit
each, 1 = offload, 0 = CPU, in program order.

Reading used here (the paper does not spell the test out):

* the candidate of a nest is its OUTERMOST loop; inner levels are part of the
  same kernel, so the "specified twice" error cannot arise (Sec. 6 speaks of
  detecting the upper-level loop statements);
* ``opaque_call`` -> REJECT(EXTERNAL_CALL); ``early_exit`` -> REJECT(BREAK);
* a buffer touched only through ``sum`` accesses is a sum reduction and makes
  the nest PARALLEL_REDUCTION (if the buffer is also touched otherwise, the sum
  counts as an ordinary read-write);
* otherwise a write W and any access X of the same buffer conflict when two
  iterations with different outer-loop values reach the same element:
  REJECT(DATA_DEP);
* a nest whose body no library operation implements (op ``host_code``: the
  loop kept as source text, compiled for the CPU) cannot be offloaded even
  when its loop is parallel -- the paper's "other" compile errors:
  REJECT(NO_KERNEL), after the reasons above.

The conflict question is answered exactly for subscripts of the form
``var + c`` / ``c``: each subscript equation links two variables by a fixed
offset or pins one to a value, so the solutions are the connected components
of a graph of offsets, each component free to slide over the intersection of
its members' ranges.
"""
PARALLEL, PARALLEL_REDUCTION, REJECT = 0, 1, 2
R_NONE, R_DATA_DEP, R_EXTERNAL_CALL, R_BREAK, R_NO_KERNEL = 0, 1, 2, 3, 4


class _Offsets:
    """Union-find where every node stores value(node) = value(root) + off."""

    def __init__(self):
        self.parent, self.off = {}, {}

    def add(self, x):
        if x not in self.parent:
            self.parent[x], self.off[x] = x, 0

    def find(self, x):
        path = []
        while self.parent[x] != x:
            path.append(x)
            x = self.parent[x]
        root = x
        # compress: recompute offsets along the path from the root side
        total = 0
        for node in reversed(path):
            total += self.off[node]
            self.off[node] = total
            self.parent[node] = root
        return root

    def link(self, a, b, delta):
        """Require value(a) - value(b) == delta; return False if inconsistent."""
        ra, rb = self.find(a), self.find(b)
        oa, ob = self.off[a], self.off[b]
        if ra == rb:
            return oa - ob == delta
        # value(a) = v(ra) + oa ; value(b) = v(rb) + ob ; v(ra) + oa - v(rb) - ob = delta
        # attach ra under rb: v(ra) = v(rb) + (delta + ob - oa)
        self.parent[ra] = rb
        self.off[ra] = delta + ob - oa
        return True


def carried(nest, w, x):
    """Exact test: do iterations it, it' with it[0] != it'[0] exist such that
    access w at it and access x at it' hit the same element?"""
    loops = nest.loops
    for _, lo, hi in loops:
        if lo >= hi:
            return False          # empty iteration space: nothing runs
    rng = {}
    uf = _Offsets()
    ZERO = ("zero",)
    uf.add(ZERO)
    rng[ZERO] = (0, 0)
    for v, lo, hi in loops:
        for side in (0, 1):
            uf.add((side, v))
            rng[(side, v)] = (lo, hi - 1)
    for v, count in nest.repeat_vars.items():
        if count <= 0:
            return False
        uf.add(("rep", v))
        rng[("rep", v)] = (0, count - 1)
    loop_names = {v for v, _, _ in loops}

    def node(side, var):
        if var is None:
            return ZERO
        if var in loop_names:
            return (side, var)
        return ("rep", var)          # repeat variable: shared by both sides

    if len(w.subs) != len(x.subs):
        raise ValueError("rank mismatch on buffer %s" % w.buf)
    for (vw, cw), (vx, cx) in zip(w.subs, x.subs):
        # value(vw) + cw == value(vx) + cx  ->  value(vw) - value(vx) == cx - cw
        if not uf.link(node(0, vw), node(1, vx), cx - cw):
            return False
    # feasible range of every component's root value
    comp = {}
    for n in list(uf.parent):
        r = uf.find(n)
        lo, hi = rng[n]
        o = uf.off[n]
        clo, chi = comp.get(r, (-10**18, 10**18))
        comp[r] = (max(clo, lo - o), min(chi, hi - o))
    for lo, hi in comp.values():
        if lo > hi:
            return False
    outer = loops[0][0]
    a, b = (0, outer), (1, outer)
    ra, rb = uf.find(a), uf.find(b)
    if ra == rb:
        return uf.off[a] != uf.off[b]
    lo_a, hi_a = comp[ra]
    lo_b, hi_b = comp[rb]
    if lo_a == hi_a and lo_b == hi_b:
        return lo_a + uf.off[a] != lo_b + uf.off[b]
    return True


def check_nest(nest):
    """Return (verdict, reason) for one nest."""
    if "opaque_call" in nest.flags:
        return REJECT, R_EXTERNAL_CALL
    if "early_exit" in nest.flags:
        return REJECT, R_BREAK
    by_buf = {}
    for a in nest.access:
        by_buf.setdefault(a.buf, []).append(a)
    reduction = False
    for buf, accs in by_buf.items():
        modes = {a.mode for a in accs}
        if modes == {"sum"}:
            reduction = True
            continue
        writes = [a for a in accs if a.mode in ("w", "rw", "sum")]
        for w in writes:
            for x in accs:
                if carried(nest, w, x):
                    return REJECT, R_DATA_DEP
    if nest.op == "host_code":
        return REJECT, R_NO_KERNEL
    return (PARALLEL_REDUCTION if reduction else PARALLEL), R_NONE


def check_app(app):
    """Verdicts of every nest plus the gene position of each accepted nest
    (-1 when rejected); gene positions follow program order."""
    out, pos = [], 0
    for n in app.nests:
        v, r = check_nest(n)
        if v == REJECT:
            out.append((v, r, -1))
        else:
            out.append((v, r, pos))
            pos += 1
    return out


def gene_length(app):
    return sum(1 for v, _, _ in check_app(app) if v != REJECT)


def brute_force_carried(nest, w, x):
    """Definition written out, for tiny bounds: enumerate every pair of
    iterations (and every repeat-variable value) and compare subscripts."""
    import itertools
    loops = nest.loops
    ranges = [range(lo, hi) for _, lo, hi in loops]
    names = [v for v, _, _ in loops]
    reps = list(nest.repeat_vars.items())
    rep_ranges = [range(c) for _, c in reps]
    iters = list(itertools.product(*ranges))

    def sub(acc, env):
        return tuple((env[v] if v is not None else 0) + c for v, c in acc.subs)

    for repvals in itertools.product(*rep_ranges):
        renv = {reps[t][0]: repvals[t] for t in range(len(reps))}
        for it in iters:
            env1 = dict(renv)
            env1.update(zip(names, it))
            s1 = sub(w, env1)
            for it2 in iters:
                if it2[0] == it[0]:
                    continue
                env2 = dict(renv)
                env2.update(zip(names, it2))
                if s1 == sub(x, env2):
                    return True
    return False
