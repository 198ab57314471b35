"""Oracle serial run of a whole application (test infrastructure only).

Every nest runs on the CPU, one core, in program order with repeats expanded:
this is the all-zero gene of the paper, whose time is the CPU-only baseline of
Sec. 5.2, and whose values every other gene must reproduce (offloading a loop
must not change what the program computes).

``run_app(app, seed)`` returns {buffer name: numpy array} in the application's
own precision (FP32 evaluated in the fixed order of the C nests).
``run_app(app, seed, twin=True)`` evaluates the same program with FP32
arrays widened to FP64 where a double twin exists (GEMM, stencil, element-wise
ops), as the accuracy reference for GPU results whose rounding order differs.
"""
import numpy as np

from . import cnests as C
from .dft import dft_rows, idft_rows, irdft_packed_rows, rdft_packed_rows
from .ir import load  # noqa: F401  (re-exported for callers)

_NP = {"f32": np.float32, "f64": np.float64, "bf16": np.uint16}


def setup_buffers(app, twin=False):
    bufs = {}
    for b in app.buffers:
        dt = _NP[b.dtype]
        if twin and b.dtype == "f32":
            dt = np.float64
        if b.setup == "sin":
            I, J, K = b.dims
            f32, f64 = C.sin_field(I, J, K, b.mode, want64=True)
            arr = f64 if (twin and dt == np.float64) else f32
            bufs[b.name] = np.ascontiguousarray(arr.astype(dt, copy=False))
        else:
            bufs[b.name] = np.zeros(b.dims, dt)
    return bufs


def _bf16_to_f64(x16):
    return (x16.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def run_nest(app, nest, bufs, seed, repeat_env, twin=False, offloaded=False):
    op, a = nest.op, nest.args
    if op == "init_uniform":
        for name, stream in zip(a["out"], a["streams"]):
            x = bufs[name]
            v = C.init_uniform(x.size, seed, stream).reshape(x.shape)
            x[...] = v
    elif op == "gemm" and offloaded and a.get("prec", "f32") != "f32":
        # the offloaded form of a GEMM nest marked with a split precision: the
        # split product's own definition, summed in FP64; the FP32 run holds
        # that value rounded to FP32.  On the CPU the nest is plain FP32.
        A, B, Cm = bufs[a["A"]], bufs[a["B"]], bufs[a["C"]]
        Cm[...] = C.gemm_split_f64(np.asarray(A, np.float32), np.asarray(B, np.float32), a["prec"])
    elif op == "gemm":
        A, B, Cm = bufs[a["A"]], bufs[a["B"]], bufs[a["C"]]
        if twin:
            Cm[...] = np.matmul(A.astype(np.float64), B.astype(np.float64)) if A.dtype == np.float64 \
                else C.gemm_f64(A, B)
        else:
            Cm[...] = C.gemm_f32(A, B)
    elif op == "gemm_bf16":
        A, B, Cm = bufs[a["A"]], bufs[a["B"]], bufs[a["C"]]
        if twin:
            Cm[...] = C.gemm_bf16_f64(A, B)
        else:
            Cm[...] = C.gemm_bf16(A, B)
    elif op == "add_scaled":
        Cm, A = bufs[a["C"]], bufs[a["A"]]
        if twin:
            Cm += float(a["alpha"]) * A
        else:
            C.add_scaled(Cm, A, float(a["alpha"]))
    elif op == "avg2":
        S, X, Y = bufs[a["S"]], bufs[a["X"]], bufs[a["Y"]]
        if twin:
            S[...] = 0.5 * (X + Y)
        else:
            C.avg2(S, X, Y)
    elif op == "scale":
        D = bufs[a["D"]]
        if twin:
            D *= float(a["beta"])
        else:
            C.scale(D, float(a["beta"]))
    elif op == "copy":
        bufs[a["dst"]][...] = bufs[a["src"]]
    elif op == "cast_bf16":
        for d, s in zip(a["dst"], a["src"]):
            src = bufs[s]
            bufs[d][...] = C.cast_bf16(src.astype(np.float32) if twin else src)
    elif op == "transpose":
        X = bufs[a["src"]]
        bufs[a["dst"]][...] = X.T if twin else C.transpose(X)
    elif op == "sumsq":
        x, s = bufs[a["x"]], bufs[a["s"]]
        if twin:
            s[0] += float(np.sum(x.astype(np.float64) ** 2))
        else:
            C.sumsq(x, s)
    elif op == "stencil19":
        p, q, res = bufs[a["p"]], bufs[a["q"]], bufs[a["res"]]
        slot = repeat_env[a["slot"]]
        cell = res[slot:slot + 1]
        if twin:
            C.stencil19_f64(p, q, cell)
        else:
            C.stencil19(p, q, cell)
        res[slot] = cell[0]
    elif op == "copy_interior":
        C.copy_interior(bufs[a["dst"]], bufs[a["src"]])
    elif op == "rec_prefix":
        v, S = bufs[a["v"]], bufs[a["S"]]
        if twin:
            for i in range(1, v.shape[0]):
                v[i] = v[i - 1] + S[i, 0]
        else:
            C.rec_prefix(v, S)
    elif op == "rec_decay":
        w, p = bufs[a["w"]], bufs[a["p"]]
        if twin:
            row = p[1, 1, :]
            for k in range(1, w.shape[0]):
                w[k] = 0.5 * w[k - 1] + row[k]
        else:
            C.rec_decay(w, p)
    elif op == "fft_rows":
        # the FFT call: the exact transform (forward, inverse scaled by 1/n,
        # or of real rows, packed), rounded to the buffer's precision
        X = bufs[a["x"]]
        if a.get("real"):
            X[...] = (irdft_packed_rows(X) if a.get("inverse") else rdft_packed_rows(X)).astype(X.dtype)
        else:
            X[...] = (idft_rows(X) if a.get("inverse") else dft_rows(X)).astype(X.dtype)
    elif op == "lcg_fill":
        L = bufs[a["L"]]
        if twin:
            tmp = np.empty(L.shape, np.float32)
            C.lcg_fill(tmp, int(a["seed32"]))
            L[...] = tmp
        else:
            C.lcg_fill(L, int(a["seed32"]))
    else:
        raise ValueError("unknown op %r" % op)


def run_app(app, seed, twin=False, bufs=None, offloaded=()):
    """Serial run of the whole program; returns the final buffers.

    ``offloaded`` names the nests (by index) that the gene places on the GPU;
    it matters only for GEMM nests marked with a split precision, whose GPU
    form computes a different (documented) value than the FP32 loop."""
    if bufs is None:
        bufs = setup_buffers(app, twin)
    offloaded = set(offloaded)

    def walk(items, env):
        for it in items:
            if it[0] == "nest":
                run_nest(app, app.nests[it[1]], bufs, seed, env, twin, it[1] in offloaded)
            else:
                _, var, count, body = it
                for n in range(count):
                    e2 = dict(env)
                    e2[var] = n
                    walk(body, e2)
    walk(app.program, {})
    return bufs
