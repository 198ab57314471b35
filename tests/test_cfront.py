"""The C front end (parsing loop nests of a C subset into the application
description, Sec. 4): each application's C source yields its hand-built
description, the library and the oracle give the parsed nests the same
verdicts, and the access modes, bindings and errors follow the source."""
import json
import os

import pytest

import paper_1806_01430_amd as ofl
from paper_1806_01430_amd import cfront
from oracle import depcheck as D
from oracle import ir

APPS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1806_01430_amd", "apps")


def _norm(n):
    n = dict(n)
    if "access" in n:
        n["access"] = sorted(tuple(a) for a in n["access"])
    if "body" in n:
        n["body"] = [_norm(x) for x in n["body"]]
    return n


@pytest.mark.parametrize("name", ["tiny", "medium", "precision", "large", "batch", "spectral"])
def test_c_source_parses_to_the_description(name):
    got = cfront.load(os.path.join(APPS, name + ".c"))
    with open(os.path.join(APPS, name + ".json")) as f:
        want = json.load(f)
    assert got["name"] == want["name"]
    assert got["params"] == want["params"]
    assert got["buffers"] == want["buffers"]
    assert [_norm(n) for n in got["program"]] == [_norm(n) for n in want["program"]]


@pytest.mark.parametrize("name", ["medium", "large"])
def test_library_and_oracle_verdicts_of_parsed_source(name):
    app = ofl.App(os.path.join(APPS, name + ".c"))
    o = ir.load(cfront.load(os.path.join(APPS, name + ".c")))
    v = [tuple(x) for x in D.check_app(o)]
    assert app.verdicts() == v
    by_name = {app.nest_name(i): v[i] for i in range(app.n_nests)}
    # the two recurrences carry a dependence, the generator is an external call
    assert by_name["rec_prefix_v"][:2] == (D.REJECT, D.R_DATA_DEP)
    assert by_name["rec_decay_w"][:2] == (D.REJECT, D.R_DATA_DEP)
    assert by_name["sumsq_S"][:2] == (D.PARALLEL_REDUCTION, D.R_NONE)
    assert by_name["stencil19"][:2] == (D.PARALLEL_REDUCTION, D.R_NONE)
    if name == "large":
        assert by_name["lcg_fill_L"][:2] == (D.REJECT, D.R_EXTERNAL_CALL)


DECLS = """#define R 5
#define CC 7
float X[R][CC];
float Y[R][CC];
float Z[CC][R];
double t[1];
"""


def _one(body):
    doc = cfront.parse(DECLS + body, "t")
    assert len(doc["program"]) == 1
    return doc["program"][0]


def test_renamed_loops_and_buffers_bind():
    n = _one("for (int r = 0; r < R; r++) for (int c = 0; c < CC; c++) Z[c][r] = X[r][c];")
    assert (n["op"], n["args"]) == ("transpose", {"src": "X", "dst": "Z"})
    assert n["loops"] == [["r", "0", "R"], ["c", "0", "CC"]]
    assert sorted(map(tuple, n["access"])) == [("X", "r", "r", "c"), ("Z", "w", "c", "r")]
    n = _one("for (int a = 0; a < R; a++) for (int b = 0; b < CC; b++) Y[a][b] = 0.5f * (Y[a][b] + X[a][b]);")
    assert (n["op"], n["args"]) == ("avg2", {"S": "Y", "X": "Y", "Y": "X"})
    # Y read at the element it writes, before the write: read-write
    assert sorted(map(tuple, n["access"])) == [("X", "r", "a", "b"), ("Y", "rw", "a", "b")]


def test_compound_assignment_and_commuted_operands():
    for body in ("X[i][j] += 0.25f * Y[i][j];", "X[i][j] = X[i][j] + Y[i][j] * 0.25f;",
                 "X[i][j] = 0.25f * Y[i][j] + X[i][j];"):
        n = _one("for (int i = 0; i < R; i++) for (int j = 0; j < CC; j++) " + body)
        assert (n["op"], n["args"]) == ("add_scaled", {"C": "X", "A": "Y", "alpha": 0.25}), body
        assert sorted(map(tuple, n["access"])) == [("X", "rw", "i", "j"), ("Y", "r", "i", "j")]
    n = _one("for (int i = 0; i < R; i++) for (int j = 0; j < CC; j++) X[i][j] *= -3.0f;")
    assert (n["op"], n["args"]) == ("scale", {"D": "X", "beta": -3.0})


def test_sum_reduction_through_temporary():
    n = _one("""for (int i = 0; i < R; i++) for (int j = 0; j < CC; j++) {
                    double u = (double)X[i][j];
                    t[0] += u * u; }""")
    assert (n["op"], n["args"]) == ("sumsq", {"x": "X", "s": "t"})
    assert sorted(map(tuple, n["access"])) == [("X", "r", "i", "j"), ("t", "sum", "0")]


@pytest.mark.parametrize("body", [
    # grouping differs from the operation's: another rounding
    "X[i][j] = 0.5f * X[i][j] + 0.5f * Y[i][j];",
    # another constant
    "Y[i][j] = 0.25f * (X[i][j] + Y[i][j]);",
    # element-wise with a shifted operand: no operation reads a neighbour
    "Y[i][j] = X[i][j];\n X[i][j] = Y[i][j];",
])
def test_unmatched_bodies_keep_their_source(body):
    # no operation of the library has these bodies: the nest keeps its text,
    # compiled for the CPU, and gets no gene bit (Sec. 4: a loop whose
    # directive does not compile stays on the CPU)
    n = _one("for (int i = 0; i < R; i++) for (int j = 0; j < CC; j++) { " + body + " }")
    assert n["op"] == "host_code" and body.split(";")[0].strip() in n["source"]
    _check_host_only(DECLS + "for (int i = 0; i < R; i++) for (int j = 0; j < CC; j++) { " + body + " }",
                     D.R_NO_KERNEL)


def _check_host_only(src, reason):
    doc = cfront.parse(src, "t")
    app = ofl.App(doc)
    want = [tuple(x) for x in D.check_app(ir.load(doc))]
    assert app.verdicts() == want
    assert want[-1] == (D.REJECT, reason, -1)


@pytest.mark.parametrize("body,reason", [
    # over part of the array: the library's add would cover all of it
    ("for (int i = 0; i < 2; i++) for (int j = 0; j < CC; j++) X[i][j] = X[i][j] + 0.5f * Y[i][j];",
     "no_kernel"),
    # a double literal makes the update double arithmetic
    ("for (int i = 0; i < R; i++) for (int j = 0; j < CC; j++) X[i][j] = X[i][j] + 0.1 * Y[i][j];",
     "no_kernel"),
    # a product over part of the inner dimension
    ("for (int i = 0; i < R; i++) for (int j = 0; j < R; j++) { Z[i][j] = 0.0f;"
     " for (int k = 0; k < 3; k++) Z[i][j] += Y[i][k] * X[k][j]; }", "bounds"),
    # a math routine, a branch, an early exit
    ("for (int i = 0; i < R; i++) for (int j = 0; j < CC; j++) Y[i][j] = sqrtf(X[i][j]);", "call"),
    ("for (int i = 0; i < R; i++) for (int j = 0; j < CC; j++) { float u = X[i][j];"
     " if (u < 0.5f) u = 0.5f - u; Y[i][j] = u; }", "no_kernel"),
    ("for (int i = 0; i < R; i++) { if (X[i][0] > 0.5f) break; Y[i][0] = X[i][0]; }", "break"),
])
def test_nests_the_library_does_not_implement_stay_on_the_cpu(body, reason):
    n = _one(body)
    assert n["op"] == "host_code"
    want = {"no_kernel": D.R_NO_KERNEL, "call": D.R_EXTERNAL_CALL, "break": D.R_BREAK}.get(reason)
    if reason == "bounds":
        # Z is 7 x 5 here, not the 5 x 5 the loops cover: no product binds
        want = D.R_NO_KERNEL
    _check_host_only(DECLS + body, want)
    if reason == "break":
        # a write in a loop that can be left early may not happen: read-write
        assert ["Y", "rw", "i", "0"] in n["access"]


def test_residual_slot_must_be_the_repeat_variable():
    src = """#define I 5
#define J 6
#define K 7
float p[I][J][K];
float q[I][J][K];
double res[3];
for (int n = 0; n < 3; n++) {
    for (int i = 1; i < I - 1; i++) for (int j = 1; j < J - 1; j++) for (int k = 1; k < K - 1; k++) {
        float xm = (p[i - 1][j - 1][k] + p[i - 1][j + 1][k]) + (p[i - 1][j][k - 1] + p[i - 1][j][k + 1]);
        float x0 = (p[i][j - 1][k] + p[i][j + 1][k]) + (p[i][j][k - 1] + p[i][j][k + 1]);
        float xp = (p[i + 1][j - 1][k] + p[i + 1][j + 1][k]) + (p[i + 1][j][k - 1] + p[i + 1][j][k + 1]);
        float y0 = (p[i][j - 1][k - 1] + p[i][j - 1][k + 1]) + (p[i][j + 1][k - 1] + p[i][j + 1][k + 1]);
        float faces = (p[i - 1][j][k] + p[i + 1][j][k]) + x0;
        float edges = (xm + xp) + y0;
        float r = (0.25f * p[i][j][k] + 0.0625f * faces) + 0.03125f * edges;
        q[i][j][k] = r;
        double d = (double)r - (double)p[i][j][k];
        res[SLOT] += d * d; }
    for (int i = 1; i < I - 1; i++) for (int j = 1; j < J - 1; j++) for (int k = 1; k < K - 1; k++)
        p[i][j][k] = q[i][j][k];
}
"""
    doc = cfront.parse(src.replace("SLOT", "n"), "t")
    assert doc["program"][0]["body"][0]["op"] == "stencil19"
    doc = cfront.parse(src.replace("SLOT", "0"), "t")
    assert doc["program"][0]["body"][0]["op"] == "host_code"
    app = ofl.App(doc)
    assert app.verdicts() == [tuple(x) for x in D.check_app(ir.load(doc))]


def test_source_errors():
    loop = "for (int i = 0; i < R; i++) for (int j = 0; j < CC; j++) "
    with pytest.raises(cfront.CError, match="u01"):
        _one(loop + "{ Y[i][j] = u01(0, i, j) * X[i][j]; }")
    with pytest.raises(cfront.CError, match="name \\+ constant"):
        _one(loop + "Y[i][j] = X[2 * i][j];")
    with pytest.raises(cfront.CError, match="step by one"):
        _one("for (int i = 0; i < R; i += 2) Y[i][0] = X[i][0];")
    with pytest.raises(cfront.CError, match="unsupported directive"):
        cfront.parse("#include <math.h>\n" + DECLS, "t")
    with pytest.raises(cfront.CError, match="prec"):
        cfront.parse(DECLS + "#pragma ofl prec(bf16x3)\n" + loop + "Y[i][j] = X[i][j];", "t")
    with pytest.raises(cfront.CError, match="annotation"):
        cfront.parse("float P[3]; // ofl: outptu\n", "t")


def test_repeat_block_and_prec_pragma():
    src = """#define N 16
#define STEPS 3
float A[N][N];
float B[N][N];
float C[N][N];
#pragma ofl prec(bf16x3)
for (int i = 0; i < N; i++) for (int j = 0; j < N; j++) {
    C[i][j] = 0;
    for (int k = 0; k < N; k++) C[i][j] += A[i][k] * B[k][j]; }
for (int s = 0; s < STEPS; s++) {
    for (int i = 0; i < N; i++) for (int j = 0; j < N; j++) A[i][j] = C[i][j];
    for (int i = 0; i < N; i++) for (int j = 0; j < N; j++) C[i][j] = 2.0f * C[i][j];
}
"""
    doc = cfront.parse(src, "r")
    g, rep = doc["program"]
    assert (g["op"], g["args"]) == ("gemm", {"A": "A", "B": "B", "C": "C", "prec": "bf16x3"})
    assert sorted(map(tuple, g["access"])) == [("A", "r", "i", "k"), ("B", "r", "k", "j"), ("C", "w", "i", "j")]
    assert rep["repeat"] == "STEPS" and rep["var"] == "s"
    assert [n["nest"] for n in rep["body"]] == ["copy_A", "scale_C"]
    app = ofl.App(doc)
    assert app.verdicts() == [tuple(x) for x in D.check_app(ir.load(doc))]
    assert app.gene_len == 3


def test_command_line_prints_the_description(capsys):
    assert cfront.main([os.path.join(APPS, "tiny.c")]) == 0
    doc = json.loads(capsys.readouterr().out)
    with open(os.path.join(APPS, "tiny.json")) as f:
        want = json.load(f)
    assert [_norm(n) for n in doc["program"]] == [_norm(n) for n in want["program"]]


def test_offloaded_source_marks_the_gene():
    path = os.path.join(APPS, "medium.c")
    with open(path) as f:
        src = f.read()
    app = ofl.App(path)
    v = app.verdicts()
    for gene in ([1] * app.gene_len, [0] * app.gene_len, [(i * 7) % 3 % 2 for i in range(app.gene_len)]):
        text = cfront.offloaded_source(src, v, gene)
        lines = text.split("\n")
        assert len(lines) == len(src.split("\n")) + sum(gene) + sum(1 for x in v if x[2] < 0)
        # the directive sits right before the outer for of each offloaded nest
        fors = [i for i, t in enumerate(lines) if t.strip() == "#pragma acc kernels"]
        assert len(fors) == sum(gene)
        assert all(lines[i + 1].lstrip().startswith("for (") for i in fors)
        assert text.count("not offloadable: a data dependence") == 2
        # the written program parses to the same description
        assert cfront.parse(text, "medium") == cfront.parse(src, "medium")
    # nests marked in program order: the product is the first accepted nest after init
    text = cfront.offloaded_source(src, v, [0, 1] + [0] * (app.gene_len - 2))
    i = text.index("#pragma acc kernels")
    assert text[i:].split("\n")[3].strip() == "C[i][j] = 0.0f;"
    with pytest.raises(ValueError):
        cfront.offloaded_source(src, v, [1] * (app.gene_len + 1))
    with pytest.raises(cfront.CError, match="begin its line"):
        cfront.offloaded_source(DECLS + "{ } for (int i = 0; i < R; i++) for (int j = 0; j < CC; j++) Y[i][j] = X[i][j];",
                                [(0, 0, 0)], [1])


def test_library_call_is_a_function_block():
    path = os.path.join(APPS, "spectral.c")
    doc = cfront.load(path)
    fft = doc["program"][1]
    assert (fft["nest"], fft["op"], fft["args"]) == ("fft_X", "fft_rows", {"x": "X"})
    app = ofl.App(path)
    v = app.verdicts()
    assert v == [tuple(x) for x in D.check_app(ir.load(doc))]
    assert v[1] == (D.PARALLEL, D.R_NONE, 1)          # the call holds gene bit 1
    with open(path) as f:
        src = f.read()
    text = cfront.offloaded_source(src, v, [1, 1, 0, 1])
    lines = text.split("\n")
    i = lines.index("/* function block: the GPU implementation replaces this call */")
    assert lines[i + 1] == "fft_rows(X);"
    assert text.count("#pragma acc kernels") == 2
    assert cfront.parse(text, "spectral") == doc
    with pytest.raises(cfront.CError, match="not a known library routine"):
        cfront.parse(DECLS + "qsort(X);", "t")
    with pytest.raises(cfront.CError, match="2-D float"):
        cfront.parse(DECLS + "fft_rows(t);", "t")


def test_inverse_fft_call_is_a_function_block():
    # ifft_rows(X): the same op with the inverse flag, one more gene bit; a
    # forward call then an inverse one parse to the round-trip application
    from workloads import appgen
    src = ("#define R 37\n#define M 512\nfloat X[R][M]; // ofl: output\n"
           "fft_rows(X);\nifft_rows(X);\n")
    doc = cfront.parse(src, "fft_roundtrip")
    want = appgen.fft_roundtrip_app(37, 256)
    assert [(n["nest"], n["op"], n["args"]) for n in doc["program"]] == \
        [(n["nest"], n["op"], n["args"]) for n in want["program"]]
    app = ofl.App(json.dumps(doc))
    assert app.gene_len == 2
    assert app.verdicts() == [tuple(x) for x in D.check_app(ir.load(doc))]
    # rfft_rows(X): rows of real values, the same op with the real flag
    real = cfront.parse("#define R 5\n#define M 64\nfloat X[R][M]; // ofl: output\n"
                        "rfft_rows(X);\nirfft_rows(X);\n", "r")
    assert [(n["nest"], n["op"], n["args"]) for n in real["program"]] == \
        [(n["nest"], n["op"], n["args"]) for n in appgen.rfft_roundtrip_app(5, 64)["program"]]


BLAS1_SRC = open(os.path.join(APPS, "blas1.c")).read()


def test_level1_blas_calls_are_the_loop_nests():
    # saxpy / scopy / sscal on whole arrays become the nests of their loop
    # forms (alpha as the routine's float parameter: a double literal is
    # converted to float); one gene bit each
    import numpy as np
    doc = cfront.parse(BLAS1_SRC, "blas1")
    prog = doc["program"]
    assert [(n["op"], n["args"]) for n in prog[1:]] == [
        ("add_scaled", {"C": "Y", "A": "X", "alpha": float(np.float32(0.1))}),
        ("copy", {"dst": "Z", "src": "Y"}),
        ("scale", {"D": "Z", "beta": -2.5}),
        ("add_scaled", {"C": "Z", "A": "X", "alpha": 0.5})]
    assert prog[1]["loops"] == prog[4]["loops"] and prog[1]["access"][1] == prog[4]["access"][1]
    app = ofl.App(json.dumps(doc))
    assert app.gene_len == 5
    assert app.verdicts() == [tuple(x) for x in D.check_app(ir.load(doc))]
    for bad, msg in (("saxpy(X, Y);", "takes"), ("saxpy(a, X, Y);", "alpha must be a number"),
                     ("scopy(X, W);", "one shape"), ("sscal(2.0f, t);", "declared arrays")):
        with pytest.raises(cfront.CError, match=msg):
            cfront.parse(BLAS1_SRC.replace("sscal(-2.5f, Z);", bad).replace(
                "float Z[N][M];", "float Z[N][M];\nfloat W[N][N];"), "t")


def test_matrix_product_call_is_the_product_nest():
    # sgemm(A, B, C) as a function block gives the same nest as the loop form
    loop = cfront.load(os.path.join(APPS, "tiny.c"))
    with open(os.path.join(APPS, "tiny.c")) as f:
        src = f.read()
    i = src.index("/* C = A B */")
    j = src.index("for (int i = 0; i < N; i++)\n    for (int j = 0; j < N; j++)\n        C[i][j] = C[i][j]")
    call = cfront.parse(src[:i] + "#pragma ofl prec(bf16x3)\nsgemm(A, B, C);\n\n" + src[j:], "tiny")
    want = json.loads(json.dumps(loop))
    want["program"][1]["args"]["prec"] = "bf16x3"
    assert [_norm(n) for n in call["program"]] == [_norm(n) for n in want["program"]]
    with pytest.raises(cfront.CError, match="matching extents"):
        cfront.parse(DECLS + "sgemm(X, Y, Z);", "t")


def _rename_nest(nest, loop_map, buf_map):
    """A description nest with its loop variables and buffers renamed."""
    import re as _re

    def sub(text):
        return _re.sub(r"[A-Za-z_]\w*", lambda m: loop_map.get(m.group(0), m.group(0)), text)
    out = json.loads(json.dumps(nest))
    out["loops"] = [[loop_map[v], lo, hi] for v, lo, hi in out["loops"]]
    out["access"] = [[buf_map[a[0]], a[1]] + [sub(x) for x in a[2:]] for a in out["access"]]
    out["args"] = {k: (buf_map.get(v, v) if isinstance(v, str) else v) for k, v in out["args"].items()}
    return out


def test_random_renamings_and_commutations_bind():
    # each element-wise operation written with random loop and array names
    # and randomly swapped operands of single additions and products parses
    # to the generator's nest for the same operation, renamed
    import random
    from workloads import appgen
    rng = random.Random(11)
    names = ["P", "Q", "U", "V", "W"]
    for trial in range(60):
        i, j = rng.sample(["i", "j", "r", "c", "ii", "jj"], 2)
        X, Y, Z = rng.sample(names, 3)

        def sw(a, b, op):
            return "%s %s %s" % ((a, op, b) if rng.random() < 0.5 else (b, op, a))
        xi, yi, zi = "%s[%s][%s]" % (X, i, j), "%s[%s][%s]" % (Y, i, j), "%s[%s][%s]" % (Z, i, j)
        kind = trial % 5
        if kind == 0:
            body, want = "%s = %s;" % (zi, sw(zi, sw("0.5f", xi, "*"), "+")), appgen.add_scaled_nest("C", "A", 0.5)
            bm = {"C": Z, "A": X}
        elif kind == 1:
            body, want = "%s = %s;" % (zi, sw("0.5f", "(%s)" % sw(xi, yi, "+"), "*")), appgen.avg2_nest("S", "C", "T")
            bm = {"S": Z, "C": X, "T": Y}
            if body.count(yi) and body.index(yi) < body.index(xi):
                bm = {"S": Z, "C": Y, "T": X}
        elif kind == 2:
            body, want = "%s = %s;" % (zi, sw("2.0f", zi, "*")), appgen.scale_nest("D", 2.0)
            bm = {"D": Z}
        elif kind == 3:
            body, want = "%s = %s;" % (zi, xi), appgen.copy_nest("D", "C")
            bm = {"D": Z, "C": X}
        else:
            body = "%s[%s][%s] = %s;" % (Z, j, i, xi)
            want, bm = appgen.transpose_nest("C", "T"), {"C": X, "T": Z}
        decl = "#define N 6\n" + "".join("float %s[N][N];\n" % b for b in names)
        src = decl + "for (int %s = 0; %s < N; %s++) for (int %s = 0; %s < N; %s++) %s" % (i, i, i, j, j, j, body)
        got = cfront.parse(src, "t")["program"][0]
        exp = _rename_nest(want, {"i": i, "j": j}, bm)
        assert (got["op"], got["args"], got["loops"]) == (exp["op"], exp["args"], exp["loops"]), (src, got)
        assert sorted(map(tuple, got["access"])) == sorted(map(tuple, exp["access"])), src
