"""Oracle for the GA-driven GPU-offload method -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously-correct CPU statement of what the
offload path computes.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product library never does,
and it shares no code with the product (no common kernels, helpers, tables or
pre/post-processing).  The only thing both sides read is the application
description (JSON) and the seeded generators in ``workloads``, which hold none
of the method's arithmetic.

Modules
-------
nests.c / cnests.py
    serial C loops for every nest kind (FP32 in a fixed order, plus FP64 twins)
ir.py
    reads an application description: buffers, loop nests, affine accesses
depcheck.py
    the parallelisability verdict per nest (Sec. 4: a nest that cannot take
    the parallel directive is excluded and gets no gene bit)
xfer.py
    host<->device transfer plan of one gene (Sec. 3.3: transfers decide
    whether a combination of offloaded loops is fast)
run.py
    serial execution of the whole application (the all-CPU gene)
ga.py
    the Simple GA of Sec. 3.3 / Sec. 4 with the Sec. 5.1.2 settings
enum.py
    exhaustive enumeration of every gene of a small application
"""
