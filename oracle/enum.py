"""Oracle exhaustive enumeration of every gene of a small application
(test infrastructure only).

The prior work the paper cites (Sec. 2) tries every for statement on and off
and measures each combination.  For an application with a small gene length
this brute force is the ground truth the GA is checked against: every gene's
transfer plan under both policies and, since offloading never changes the
values computed, one serial run whose outputs all genes must reproduce.
"""
from . import depcheck, xfer


def genes(a):
    """All 2^a genes; gene index idx has bit i at position i."""
    return [tuple((idx >> i) & 1 for i in range(a)) for idx in range(1 << a)]


def enumerate_plans(app, flags=0):
    """[(gene, (h2d, d2h, copies) RESIDENT, (...) PER_REGION)] for all genes."""
    verdicts = depcheck.check_app(app)
    a = sum(1 for v in verdicts if v[0] != depcheck.REJECT)
    out = []
    for g in genes(a):
        pl = xfer.placement_of_gene(app, verdicts, g)
        out.append((g, xfer.totals(app, pl, xfer.RESIDENT, flags),
                    xfer.totals(app, pl, xfer.PER_REGION, flags)))
    return out
