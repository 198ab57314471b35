"""Builders of application descriptions (tiny / medium / precision / large and
single-nest test applications); ``python -m workloads.appgen`` rewrites the
JSON files under paper_1806_01430_amd/apps/.

Each application is a program of for-loop nests over arrays, the input the
offloader works on (Sec. 4 of the paper: the source is parsed and every for
statement found).  The JSON holds the parsed form: loops with bounds, affine
array accesses, the body kind (``op``) with its arguments, and ``repeat``
blocks for the iterated sweep.

Shapes: matrices are row-major N x N; grids are p[i][j][k] with k contiguous.
"""
import json
import os

HERE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1806_01430_amd", "apps")

ALL2 = [["i", "0", "N"], ["j", "0", "N"]]


def init_nest(outs, streams):
    return {"nest": "init_" + "".join(outs), "op": "init_uniform",
            "args": {"out": outs, "streams": streams},
            "loops": ALL2, "access": [[b, "w", "i", "j"] for b in outs]}


def gemm_nest(A, B, C, op="gemm", prec=None):
    args = {"A": A, "B": B, "C": C}
    if prec:
        args["prec"] = prec
    return {"nest": op + "_" + C, "op": op, "args": args,
            "loops": [["i", "0", "N"], ["j", "0", "N"], ["k", "0", "N"]],
            "access": [[C, "w", "i", "j"], [A, "r", "i", "k"], [B, "r", "k", "j"]]}


def add_scaled_nest(C, A, alpha):
    return {"nest": "axpy_" + C, "op": "add_scaled", "args": {"C": C, "A": A, "alpha": alpha},
            "loops": ALL2, "access": [[C, "rw", "i", "j"], [A, "r", "i", "j"]]}


def transpose_nest(src, dst):
    return {"nest": "transpose_" + dst, "op": "transpose", "args": {"src": src, "dst": dst},
            "loops": ALL2, "access": [[dst, "w", "j", "i"], [src, "r", "i", "j"]]}


def avg2_nest(S, X, Y):
    return {"nest": "avg_" + S, "op": "avg2", "args": {"S": S, "X": X, "Y": Y},
            "loops": ALL2, "access": [[S, "w", "i", "j"], [X, "r", "i", "j"], [Y, "r", "i", "j"]]}


def rec_prefix_nest(v, S):
    return {"nest": "rec_prefix_" + v, "op": "rec_prefix", "args": {"v": v, "S": S},
            "loops": [["i", "1", "N"]],
            "access": [[v, "w", "i"], [v, "r", "i-1"], [S, "r", "i", "0"]]}


def sumsq_nest(x, s):
    return {"nest": "sumsq_" + x, "op": "sumsq", "args": {"x": x, "s": s},
            "loops": ALL2, "access": [[s, "sum", "0"], [x, "r", "i", "j"]]}


STENCIL_OFFSETS = [(0, 0, 0),
                   (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1),
                   (-1, -1, 0), (-1, 1, 0), (1, -1, 0), (1, 1, 0),
                   (-1, 0, -1), (-1, 0, 1), (1, 0, -1), (1, 0, 1),
                   (0, -1, -1), (0, -1, 1), (0, 1, -1), (0, 1, 1)]


def _sub(v, d):
    return v if d == 0 else ("%s%+d" % (v, d))


def stencil_nest(p, q, res, slot):
    acc = [[q, "w", "i", "j", "k"]]
    for di, dj, dk in STENCIL_OFFSETS:
        acc.append([p, "r", _sub("i", di), _sub("j", dj), _sub("k", dk)])
    acc.append([res, "sum", slot])
    return {"nest": "stencil19", "op": "stencil19",
            "args": {"p": p, "q": q, "res": res, "slot": slot},
            "loops": [["i", "1", "I-1"], ["j", "1", "J-1"], ["k", "1", "K-1"]],
            "access": acc}


def copy_interior_nest(dst, src):
    return {"nest": "copy_interior", "op": "copy_interior", "args": {"dst": dst, "src": src},
            "loops": [["i", "1", "I-1"], ["j", "1", "J-1"], ["k", "1", "K-1"]],
            "access": [[dst, "w", "i", "j", "k"], [src, "r", "i", "j", "k"]]}


def rec_decay_nest(w, p):
    return {"nest": "rec_decay_" + w, "op": "rec_decay", "args": {"w": w, "p": p},
            "loops": [["k", "1", "K"]],
            "access": [[w, "w", "k"], [w, "r", "k-1"], [p, "r", "1", "1", "k"]]}


def copy_nest(dst, src):
    return {"nest": "copy_" + dst, "op": "copy", "args": {"dst": dst, "src": src},
            "loops": ALL2, "access": [[dst, "w", "i", "j"], [src, "r", "i", "j"]]}


def scale_nest(D, beta):
    return {"nest": "scale_" + D, "op": "scale", "args": {"D": D, "beta": beta},
            "loops": ALL2, "access": [[D, "rw", "i", "j"]]}


def cast_nest(dsts, srcs):
    acc = []
    for d, s in zip(dsts, srcs):
        acc += [[d, "w", "i", "j"], [s, "r", "i", "j"]]
    return {"nest": "cast_bf16", "op": "cast_bf16", "args": {"dst": dsts, "src": srcs},
            "loops": ALL2, "access": acc}


def lcg_nest(L, seed32):
    return {"nest": "lcg_fill_" + L, "op": "lcg_fill", "args": {"L": L, "seed32": seed32},
            "loops": [["e", "0", "N"]], "access": [[L, "w", "e"]], "flags": ["opaque_call"]}


def fft_nest(x, rows="R", width="M", inverse=False, real=False):
    """The FFT library call on x[rows][width] (width = 2n floats per row: n
    complex values, interleaved) as a function block: one gene bit; its
    iteration space is the rows and the floats of a row, all read and written
    in place.  inverse: the inverse transform scaled by 1/n; real: rows of
    `width` real values, replaced by their packed spectrum (with inverse:
    packed spectra replaced by their real rows)."""
    args = {"x": x}
    if inverse:
        args["inverse"] = 1
    if real:
        args["real"] = 1
    prefix = {(False, False): "fft_", (True, False): "ifft_", (False, True): "rfft_", (True, True): "irfft_"}
    return {"nest": prefix[(bool(inverse), bool(real))] + x, "op": "fft_rows", "args": args,
            "loops": [["r", "0", rows], ["e", "0", width]], "access": [[x, "rw", "r", "e"]]}


def mat(name, output=False, dtype="f32"):
    return {"name": name, "dtype": dtype, "dims": ["N", "N"], "setup": "zero", "output": output}


def grid(name, setup="zero", output=False):
    d = {"name": name, "dtype": "f32", "dims": ["I", "J", "K"], "setup": setup, "output": output}
    if setup == "sin":
        d["mode"] = "MODE"
    return d


def sweep_block():
    return {"repeat": "SWEEPS", "var": "n",
            "body": [stencil_nest("p", "q", "res", "n"), copy_interior_nest("p", "q")]}


def tiny():
    return {
        "name": "tiny",
        "params": {"N": 64, "I": 33, "J": 33, "K": 65, "SWEEPS": 10, "MODE": 1},
        "buffers": [mat("A"), mat("B"), mat("C", True), mat("T", True),
                    grid("p", "sin", True), grid("q"),
                    {"name": "res", "dtype": "f64", "dims": ["SWEEPS"], "setup": "zero", "output": True}],
        "program": [init_nest(["A", "B"], [0, 1]), gemm_nest("A", "B", "C"),
                    add_scaled_nest("C", "A", 0.5), sweep_block(), transpose_nest("C", "T")],
    }


def _medium_buffers():
    return [mat("A"), mat("B"), mat("C", True), mat("T", True), mat("S", True),
            {"name": "v", "dtype": "f32", "dims": ["N"], "setup": "zero", "output": True},
            {"name": "s", "dtype": "f64", "dims": ["1"], "setup": "zero", "output": True},
            grid("p", "sin", True), grid("q"),
            {"name": "res", "dtype": "f64", "dims": ["SWEEPS"], "setup": "zero", "output": True},
            {"name": "w", "dtype": "f32", "dims": ["K"], "setup": "zero", "output": True},
            mat("D", True)]


def _medium_program():
    return [init_nest(["A", "B"], [0, 1]), gemm_nest("A", "B", "C"),
            add_scaled_nest("C", "A", 0.5), transpose_nest("C", "T"),
            avg2_nest("S", "C", "T"), rec_prefix_nest("v", "S"), sumsq_nest("S", "s"),
            sweep_block(), rec_decay_nest("w", "p"), copy_nest("D", "C"), scale_nest("D", 2.0)]


def medium():
    return {"name": "medium",
            "params": {"N": 1024, "I": 129, "J": 129, "K": 257, "SWEEPS": 100, "MODE": 1},
            "buffers": _medium_buffers(), "program": _medium_program()}


def precision():
    return {"name": "precision",
            "params": {"N": 4096, "I": 257, "J": 257, "K": 513, "SWEEPS": 200, "MODE": 1},
            "buffers": [mat("A"), mat("B"), mat("C", True), grid("p", "sin", True), grid("q"),
                        {"name": "res", "dtype": "f64", "dims": ["SWEEPS"], "setup": "zero",
                         "output": True}],
            "program": [init_nest(["A", "B"], [0, 1]), gemm_nest("A", "B", "C", prec="f32"),
                        sweep_block()]}


def large():
    bufs = _medium_buffers() + [mat("Y"), mat("Cb", False, "bf16"), mat("Yb", False, "bf16"),
                                mat("Z", True),
                                {"name": "L", "dtype": "f32", "dims": ["N"], "setup": "zero",
                                 "output": True}]
    prog = _medium_program() + [init_nest(["Y"], [2]), cast_nest(["Cb", "Yb"], ["C", "Y"]),
                                gemm_nest("Cb", "Yb", "Z", op="gemm_bf16"),
                                lcg_nest("L", 12345)]
    return {"name": "large",
            "params": {"N": 8192, "I": 513, "J": 513, "K": 1025, "SWEEPS": 50, "MODE": 1},
            "buffers": bufs, "program": prog}


def batch():
    """One instance of the batching configuration: product, then the iterated
    sweep on the instance's own grid (sizes set per instance)."""
    return {"name": "batch",
            "params": {"N": 64, "I": 17, "J": 17, "K": 33, "SWEEPS": 10, "MODE": 1},
            "buffers": [mat("A"), mat("B"), mat("C", True), grid("p", "sin", True), grid("q"),
                        {"name": "res", "dtype": "f64", "dims": ["SWEEPS"], "setup": "zero",
                         "output": True}],
            "program": [init_nest(["A", "B"], [0, 1]), gemm_nest("A", "B", "C"), sweep_block()]}


def spectral():
    """Spectra of R rows of n = M/2 complex samples: random samples, the FFT
    call, the total energy (Parseval: n times the samples' energy), the
    spectra scaled by 1/n."""
    rows = [["i", "0", "R"], ["j", "0", "M"]]

    def on(n):
        n["loops"] = rows
        return n
    return {"name": "spectral",
            "params": {"R": 4096, "M": 2048},
            "buffers": [{"name": "X", "dtype": "f32", "dims": ["R", "M"], "setup": "zero", "output": True},
                        {"name": "s", "dtype": "f64", "dims": ["1"], "setup": "zero", "output": True}],
            "program": [on(init_nest(["X"], [0])), fft_nest("X"), on(sumsq_nest("X", "s")),
                        on(scale_nest("X", 1.0 / 1024))]}


APPS = {"tiny": tiny, "medium": medium, "precision": precision, "large": large, "batch": batch,
        "spectral": spectral}


# ---------------------------------------------------------------- test apps
def gemm_app(M, N, K, op="gemm", prec=None):
    """One GEMM nest C[M][N] = A[M][K] B[K][N] with caller-supplied A, B."""
    dt = "bf16" if op == "gemm_bf16" else "f32"
    nest = gemm_nest("A", "B", "C", op=op, prec=prec)
    nest["loops"] = [["i", "0", "M"], ["j", "0", "NN"], ["k", "0", "KK"]]
    return {"name": "gemm", "params": {"M": M, "NN": N, "KK": K},
            "buffers": [{"name": "A", "dtype": dt, "dims": ["M", "KK"]},
                        {"name": "B", "dtype": dt, "dims": ["KK", "NN"]},
                        {"name": "C", "dtype": "f32", "dims": ["M", "NN"], "output": True}],
            "program": [nest]}


def stencil_app(I, J, K, sweeps, mode=1):
    """The iterated sweep alone on an I x J x K grid (sine set-up unless the
    caller supplies p)."""
    return {"name": "stencil", "params": {"I": I, "J": J, "K": K, "SWEEPS": sweeps, "MODE": mode},
            "buffers": [grid("p", "sin", True), grid("q", "zero", True),
                        {"name": "res", "dtype": "f64", "dims": ["SWEEPS"], "output": True}],
            "program": [sweep_block()]}


def fft_app(R, n, inverse=False, real=False):
    """The FFT call alone (forward or inverse) on R rows of n complex values,
    or (real) on R rows of n real values (caller-supplied)."""
    return {"name": "fft", "params": {"R": R, "M": n if real else 2 * n},
            "buffers": [{"name": "X", "dtype": "f32", "dims": ["R", "M"], "output": True}],
            "program": [fft_nest("X", inverse=inverse, real=real)]}


def rfft_roundtrip_app(R, n):
    """The real FFT call, then its inverse, on rows of n real values."""
    return {"name": "rfft_roundtrip", "params": {"R": R, "M": n},
            "buffers": [{"name": "X", "dtype": "f32", "dims": ["R", "M"], "output": True}],
            "program": [fft_nest("X", real=True), fft_nest("X", inverse=True, real=True)]}


def fft_roundtrip_app(R, n):
    """The forward FFT call, then the inverse one, on the same rows: two
    function blocks, two gene bits."""
    return {"name": "fft_roundtrip", "params": {"R": R, "M": 2 * n},
            "buffers": [{"name": "X", "dtype": "f32", "dims": ["R", "M"], "output": True}],
            "program": [fft_nest("X"), fft_nest("X", inverse=True)]}


def ewise_app(R, Cc):
    """Element-wise nests, transpose, cast and reduction on R x Cc matrices."""
    def m(name, dims=("R", "CC"), dtype="f32"):
        return {"name": name, "dtype": dtype, "dims": list(dims), "output": True}
    L2 = [["i", "0", "R"], ["j", "0", "CC"]]

    def on(n):
        n = json.loads(json.dumps(n))
        n["loops"] = L2
        return n
    tr = transpose_nest("C", "T")
    tr["loops"] = L2
    return {"name": "ewise", "params": {"R": R, "CC": Cc},
            "buffers": [m("A"), m("C"), m("T", ("CC", "R")), m("S"), m("D"), m("Cb", dtype="bf16"),
                        {"name": "s", "dtype": "f64", "dims": ["1"], "output": True}],
            "program": [on(init_nest(["A", "C"], [0, 1])), on(add_scaled_nest("C", "A", 0.5)), tr,
                        on(avg2_nest("S", "C", "A")), on(copy_nest("D", "S")), on(scale_nest("D", 2.0)),
                        on(cast_nest(["Cb"], ["D"])), on(sumsq_nest("S", "s"))]}


def main():
    for name, fn in APPS.items():
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(fn(), f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
