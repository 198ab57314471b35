"""Writes large_grid_513x513x1025_S50.txt: the oracle's serial run of the
large application's grid nests at full size (calls only oracle/).

The grid nests of the large application are independent of its matrix
nests: the sine field (mode 1) on 513 x 513 x 1025, then 50 repetitions of
the 19-point sweep (q from p, FP64 residual of the repetition) followed by the
interior copy (p from q), then the decay recurrence w[k] = 0.5 w[k-1] +
p[1][1][k] from w = 0.  The serial oracle takes about a minute and a half
on one core, too long for a test, so its results are stored:

* the SHA-256 of the final p's bytes (little-endian FP32, i-j-k order) and of
  w's bytes: a GPU run whose field is bit-identical to the oracle's has the
  same digests;
* the 50 residuals (FP64, shortest round-trip repr);
* 4096 probes of the final p at indices drawn from a seeded generator
  (numpy PCG64, seed 2024), each with the FP32 bit pattern, so that a
  mismatch can be located.

    python tests/golden/make_large_grid.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cnests as C  # noqa: E402

I, J, K, SWEEPS, MODE = 513, 513, 1025, 50, 1
N_PROBES, PROBE_SEED = 4096, 2024
NAME = "large_grid_%dx%dx%d_S%d.txt" % (I, J, K, SWEEPS)


def probe_indices():
    rng = np.random.default_rng(PROBE_SEED)
    return np.stack([rng.integers(0, n, N_PROBES) for n in (I, J, K)], axis=1)


def main():
    p = C.sin_field(I, J, K, MODE)
    q = np.zeros_like(p)
    res = np.zeros(SWEEPS, np.float64)
    for n in range(SWEEPS):
        cell = res[n:n + 1]
        C.stencil19(p, q, cell)
        C.copy_interior(p, q)
        print("sweep", n + 1, repr(float(res[n])), flush=True)
    w = np.zeros(K, np.float32)
    C.rec_decay(w, p)
    idx = probe_indices()
    bits = p.view(np.uint32)[idx[:, 0], idx[:, 1], idx[:, 2]]
    with open(os.path.join(HERE, NAME), "w") as f:
        f.write("# Oracle serial run of the large application's grid nests (written by make_large_grid.py):\n")
        f.write("# sine field m=%d on %d x %d x %d, %d x (19-point sweep + FP64 residual, interior copy),\n"
                % (MODE, I, J, K, SWEEPS))
        f.write("# then w[k] = 0.5 w[k-1] + p[1][1][k].  Lines: p_sha256 / w_sha256 of the final bytes,\n")
        f.write("# res n r_n (n = 1..%d), probe i j k fp32-bits of the final p (PCG64 seed %d).\n"
                % (SWEEPS, PROBE_SEED))
        f.write("p_sha256 %s\n" % hashlib.sha256(p.tobytes()).hexdigest())
        f.write("w_sha256 %s\n" % hashlib.sha256(w.tobytes()).hexdigest())
        for n in range(SWEEPS):
            f.write("res %d %r\n" % (n + 1, float(res[n])))
        for (i, j, k), b in zip(idx, bits):
            f.write("probe %d %d %d %08x\n" % (i, j, k, int(b)))


if __name__ == "__main__":
    main()
