"""Oracle host<->device transfer plan of one gene (test infrastructure only).

Sec. 3.3: offloading every parallelisable loop is not necessarily fastest
because of CPU-GPU memory transfers and their timing; the search measures each
combination.  This module states which copies a gene implies, buffer by
buffer, so that both byte counts and copy counts are exact integers.

Per nest, a buffer is *read* if any access reads it (r, rw, sum) or if it is
written only in part (a partial write must preserve the rest, so the old
content is needed); it is *written* if any access writes it (w, rw, sum).  A
write is FULL when one plain ``w`` access covers every element: each
subscript is a distinct loop variable plus offset spanning the whole extent.

State per buffer: (host_valid, dev_valid), initially (1, 0).

RESIDENT policy
    GPU nest: H2D each read buffer that is not device-valid; afterwards every
    written buffer is (0, 1).  CPU nest: D2H each read buffer that is not
    host-valid; afterwards every written buffer is (1, 0).  At the end, D2H
    each output that is not host-valid.
PER_REGION policy (the compiler-managed copies around each offloaded region
    that the paper's directive-based toolchain performs, Sec. 2)
    GPU nest: H2D every read buffer, then D2H every written buffer; CPU nests
    copy nothing; the host copy is always current.
SECTIONS policy (RESIDENT with array sections, as a directive's data clause
    may name them): a CPU nest that only reads a buffer stale on the host
    copies out just the bounding box of the elements it reads (per dimension
    the range its subscripts take over the loop and repeat ranges), unless a
    box copied out earlier and still current contains it; a box equal to the
    whole buffer is a whole copy.  Every other copy is RESIDENT's; a write
    anywhere invalidates the host boxes of that buffer.

Flags (both policies): PRESTAGED -- every buffer starts (1, 1), i.e. the
set-up content is already resident on the device; KEEP_OUTPUTS -- no final
D2H (results stay on the device).
"""
RESIDENT, PER_REGION, SECTIONS = 0, 1, 2
FLAG_PRESTAGED, FLAG_KEEP_OUTPUTS = 1, 2


def _full_write(nest, app, acc):
    if acc.mode != "w":
        return False
    buf = app.buffer(acc.buf)
    ranges = {v: (lo, hi) for v, lo, hi in nest.loops}
    seen = set()
    for (v, c), extent in zip(acc.subs, buf.dims):
        if v is None:
            if not (extent == 1 and c == 0):
                return False
            continue
        if v not in ranges or v in seen:
            return False           # repeat variable, or a diagonal use
        seen.add(v)
        lo, hi = ranges[v]
        if lo >= hi or lo + c > 0 or hi + c < extent:
            return False
    return True


def nest_sets(app, nest):
    """(reads, writes) as sorted lists of buffer indices."""
    reads, writes, full = set(), set(), set()
    for a in nest.access:
        b = app.buf_index[a.buf]
        if a.mode in ("r", "rw", "sum"):
            reads.add(b)
        if a.mode in ("w", "rw", "sum"):
            writes.add(b)
        if _full_write(nest, app, a):
            full.add(b)
    for b in writes:
        if b not in full:
            reads.add(b)
    return sorted(reads), sorted(writes)


def read_box(app, nest, b):
    """Bounding box [(lo, hi), ...] of the elements of buffer b that the nest's
    plain reads touch, or None when they touch nothing."""
    ranges = {v: (lo, hi) for v, lo, hi in nest.loops}
    box = None
    for a in nest.access:
        if app.buf_index[a.buf] != b or a.mode != "r":
            continue
        cur = []
        for v, c in a.subs:
            if v is None:
                cur.append((c, c + 1))
            elif v in ranges:
                lo, hi = ranges[v]
                cur.append((lo + c, hi + c))
            else:
                cur.append((c, nest.repeat_vars[v] + c))
        if any(lo >= hi for lo, hi in cur):
            continue
        box = cur if box is None else [(min(p[0], q[0]), max(p[1], q[1])) for p, q in zip(box, cur)]
    return box


def box_bytes(app, b, box):
    n = 1
    for lo, hi in box:
        n *= hi - lo
    return n * app.buffers[b].elem_bytes


def _contains(outer, inner):
    return all(o[0] <= i[0] and i[1] <= o[1] for o, i in zip(outer, inner))


def executions(app):
    """Nest indices in execution order, repeats expanded."""
    out = []

    def walk(items):
        for it in items:
            if it[0] == "nest":
                out.append(it[1])
            else:
                for _ in range(it[2]):
                    walk(it[3])
    walk(app.program)
    return out


def plan(app, placement, policy=RESIDENT, flags=0):
    """placement[nest] = 1 (GPU) / 0 (CPU) for every nest.  Returns the list
    of copies as (direction, buffer index, bytes), direction 'H2D' / 'D2H'."""
    nb = len(app.buffers)
    init = 1 if flags & FLAG_PRESTAGED else 0
    host = [1] * nb
    dev = [init] * nb
    boxes = [[] for _ in range(nb)]
    copies = []
    sets = [nest_sets(app, n) for n in app.nests]
    for ni in executions(app):
        reads, writes = sets[ni]
        if placement[ni]:
            if policy in (RESIDENT, SECTIONS):
                for b in reads:
                    if not dev[b]:
                        copies.append(("H2D", b, app.buffers[b].nbytes))
                        dev[b] = 1
                for b in writes:
                    host[b], dev[b] = 0, 1
                    boxes[b] = []
            else:
                for b in reads:
                    copies.append(("H2D", b, app.buffers[b].nbytes))
                    dev[b] = 1
                for b in writes:
                    copies.append(("D2H", b, app.buffers[b].nbytes))
                    host[b], dev[b] = 1, 1
        else:
            if policy in (RESIDENT, SECTIONS):
                for b in reads:
                    if host[b]:
                        continue
                    if policy == SECTIONS and b not in writes:
                        box = read_box(app, app.nests[ni], b)
                        if box is None:
                            continue
                        whole = all(lo == 0 and hi == d for (lo, hi), d in zip(box, app.buffers[b].dims))
                        if not whole:
                            if not any(_contains(o, box) for o in boxes[b]):
                                copies.append(("D2H", b, box_bytes(app, b, box)))
                                boxes[b].append(box)
                            continue
                    copies.append(("D2H", b, app.buffers[b].nbytes))
                    host[b] = 1
            for b in writes:
                host[b], dev[b] = 1, 0
                boxes[b] = []
    if not flags & FLAG_KEEP_OUTPUTS:
        for b, buf in enumerate(app.buffers):
            if buf.output and not host[b]:
                copies.append(("D2H", b, buf.nbytes))
                host[b] = 1
    return copies


def totals(app, placement, policy=RESIDENT, flags=0):
    """(bytes_h2d, bytes_d2h, n_copies)."""
    cs = plan(app, placement, policy, flags)
    h2d = sum(c[2] for c in cs if c[0] == "H2D")
    d2h = sum(c[2] for c in cs if c[0] == "D2H")
    return h2d, d2h, len(cs)


def placement_of_gene(app, verdicts, gene):
    """Expand a gene (one bit per accepted nest) to a per-nest placement;
    rejected nests always stay on the CPU."""
    out = []
    for v, r, pos in verdicts:
        out.append(int(gene[pos]) if pos >= 0 else 0)
    return out
