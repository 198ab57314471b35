// Application IR: parsing and validation.
#include "ir.hpp"

#include <cctype>
#include <set>

#include "../../include/ofl.h"

namespace ofl {

static const char *kOpNames[OP_COUNT] = {
    "none",       "init_uniform", "gemm",       "gemm_bf16",     "add_scaled", "avg2",
    "scale",      "copy",         "cast_bf16",  "transpose",     "sumsq",      "stencil19",
    "copy_interior", "rec_prefix", "rec_decay", "lcg_fill", "fft_rows", "host_code"};

const char *op_name(Op op) { return (op >= 0 && op < OP_COUNT) ? kOpNames[op] : "?"; }

bool op_has_device_kernel(Op op) {
    switch (op) {
    case OP_INIT_UNIFORM: case OP_GEMM: case OP_GEMM_BF16: case OP_ADD_SCALED: case OP_AVG2:
    case OP_SCALE: case OP_COPY: case OP_CAST_BF16: case OP_TRANSPOSE: case OP_SUMSQ:
    case OP_STENCIL19: case OP_COPY_INTERIOR: case OP_FFT_ROWS:
        return true;
    default:
        return false;
    }
}

namespace {

struct Ctx {
    AppIR &app;
    std::string &err;
    int status = OFL_OK;
    bool fail(int code, const std::string &m) {
        if (status == OFL_OK) {
            status = code;
            err = m;
        }
        return false;
    }
};

// Affine expression: optional single variable with coefficient +1 plus an
// integer built from literals and parameters joined by + and -.
struct Affine {
    std::string var;   // empty = constant
    int64_t c = 0;
};

bool parse_affine(Ctx &cx, const std::string &s, const std::set<std::string> &vars, Affine &out) {
    size_t i = 0, n = s.size();
    int sign = 1;
    bool expect_term = true;
    out = Affine();
    while (i < n) {
        char ch = s[i];
        if (std::isspace((unsigned char)ch)) { ++i; continue; }
        if (ch == '+' || ch == '-') {
            if (expect_term) sign = (ch == '-') ? -sign : sign;
            else { sign = (ch == '-') ? -1 : 1; expect_term = true; }
            ++i;
            continue;
        }
        if (!expect_term) return cx.fail(OFL_E_PARSE, "missing operator in '" + s + "'");
        if (std::isdigit((unsigned char)ch)) {
            int64_t v = 0;
            while (i < n && std::isdigit((unsigned char)s[i])) v = v * 10 + (s[i++] - '0');
            out.c += sign * v;
        } else if (std::isalpha((unsigned char)ch) || ch == '_') {
            size_t j = i;
            while (j < n && (std::isalnum((unsigned char)s[j]) || s[j] == '_')) ++j;
            std::string name = s.substr(i, j - i);
            i = j;
            auto it = cx.app.params.find(name);
            if (it != cx.app.params.end()) {
                out.c += sign * it->second;
            } else if (vars.count(name)) {
                if (!out.var.empty() || sign != 1)
                    return cx.fail(OFL_E_PARSE, "non-affine subscript '" + s + "'");
                out.var = name;
            } else {
                return cx.fail(OFL_E_PARSE, "unknown name '" + name + "' in '" + s + "'");
            }
        } else {
            return cx.fail(OFL_E_PARSE, "bad character in expression '" + s + "'");
        }
        sign = 1;
        expect_term = false;
    }
    if (expect_term) return cx.fail(OFL_E_PARSE, "incomplete expression '" + s + "'");
    return true;
}

bool json_expr_string(const Json &j, std::string &out) {
    if (j.kind == Json::Str) { out = j.str; return true; }
    if (j.kind == Json::Num && j.is_int) { out = std::to_string(j.inum); return true; }
    return false;
}

bool const_expr(Ctx &cx, const Json &j, int64_t &v) {
    std::string s;
    if (!json_expr_string(j, s)) return cx.fail(OFL_E_PARSE, "expected an integer expression");
    Affine a;
    if (!parse_affine(cx, s, {}, a)) return false;
    v = a.c;
    return true;
}

int find_buf(const AppIR &app, const std::string &name) {
    for (size_t i = 0; i < app.bufs.size(); ++i)
        if (app.bufs[i].name == name) return (int)i;
    return -1;
}

bool arg_buf(Ctx &cx, const Nest &n, const Json *args, const char *key, int &out) {
    const Json *j = args ? args->get(key) : nullptr;
    if (!j || j->kind != Json::Str) return cx.fail(OFL_E_IR, "nest " + n.name + ": missing buffer argument '" + key + "'");
    out = find_buf(cx.app, j->str);
    if (out < 0) return cx.fail(OFL_E_IR, "nest " + n.name + ": unknown buffer '" + j->str + "'");
    return true;
}

bool arg_buf_list(Ctx &cx, const Nest &n, const Json *args, const char *key, std::vector<int> &out) {
    const Json *j = args ? args->get(key) : nullptr;
    if (!j || j->kind != Json::Arr || j->arr.empty())
        return cx.fail(OFL_E_IR, "nest " + n.name + ": missing buffer list '" + key + "'");
    for (const auto &e : j->arr) {
        if (e.kind != Json::Str) return cx.fail(OFL_E_IR, "nest " + n.name + ": bad buffer list");
        int b = find_buf(cx.app, e.str);
        if (b < 0) return cx.fail(OFL_E_IR, "nest " + n.name + ": unknown buffer '" + e.str + "'");
        out.push_back(b);
    }
    return true;
}

bool arg_num(Ctx &cx, const Nest &n, const Json *args, const char *key, double &out) {
    const Json *j = args ? args->get(key) : nullptr;
    if (!j || j->kind != Json::Num) return cx.fail(OFL_E_IR, "nest " + n.name + ": missing number '" + key + "'");
    out = j->num;
    return true;
}

bool need(Ctx &cx, const Nest &n, bool cond, const std::string &what) {
    if (!cond) return cx.fail(OFL_E_IR, "nest " + n.name + " (" + op_name(n.op) + "): " + what);
    return true;
}

// Resolve and check the op-specific operands of a nest.
bool resolve_op(Ctx &cx, Nest &n, const Json *args, const std::vector<int64_t> &rep_counts) {
    AppIR &app = cx.app;
    auto B = [&](int i) -> const Buffer & { return app.bufs[n.b[i]]; };
    auto is = [&](int i, DType t) { return B(i).dtype == t; };
    int x;
    switch (n.op) {
    case OP_NONE:
        return true;
    case OP_INIT_UNIFORM: {
        if (!arg_buf_list(cx, n, args, "out", n.b)) return false;
        const Json *st = args->get("streams");
        if (!st || st->kind != Json::Arr || st->arr.size() != n.b.size())
            return need(cx, n, false, "streams must list one id per output");
        for (const auto &e : st->arr) {
            if (e.kind != Json::Num || !e.is_int || e.inum < 0 || e.inum > 0xFFFFFFFFll)
                return need(cx, n, false, "bad stream id");
            n.streams.push_back((uint32_t)e.inum);
        }
        for (size_t i = 0; i < n.b.size(); ++i)
            if (!need(cx, n, is((int)i, DT_F32), "outputs must be f32")) return false;
        return true;
    }
    case OP_GEMM:
    case OP_GEMM_BF16: {
        if (!arg_buf(cx, n, args, "A", x)) return false;
        n.b.push_back(x);
        if (!arg_buf(cx, n, args, "B", x)) return false;
        n.b.push_back(x);
        if (!arg_buf(cx, n, args, "C", x)) return false;
        n.b.push_back(x);
        DType in = n.op == OP_GEMM ? DT_F32 : DT_BF16;
        if (!need(cx, n, is(0, in) && is(1, in) && is(2, DT_F32), "dtype mismatch")) return false;
        if (!need(cx, n, B(0).dims.size() == 2 && B(1).dims.size() == 2 && B(2).dims.size() == 2,
                  "operands must be 2-D")) return false;
        if (!need(cx, n, B(0).dims[1] == B(1).dims[0] && B(2).dims[0] == B(0).dims[0] &&
                          B(2).dims[1] == B(1).dims[1], "shape mismatch")) return false;
        if (!need(cx, n, B(0).dims[0] < (1ll << 31) && B(1).dims[1] < (1ll << 31) && B(0).dims[1] < (1ll << 31),
                  "extent too large")) return false;
        const Json *pr = args->get("prec");
        if (pr && n.op == OP_GEMM) {
            if (pr->kind != Json::Str) return need(cx, n, false, "prec must be a string");
            if (pr->str == "f32") n.prec = PREC_F32;
            else if (pr->str == "bf16x3") n.prec = PREC_BF16X3;
            else if (pr->str == "fp8x2") n.prec = PREC_FP8X2;
            else return need(cx, n, false, "unknown prec '" + pr->str + "'");
        }
        return true;
    }
    case OP_ADD_SCALED:
        if (!arg_buf(cx, n, args, "C", x)) return false;
        n.b.push_back(x);
        if (!arg_buf(cx, n, args, "A", x)) return false;
        n.b.push_back(x);
        if (!arg_num(cx, n, args, "alpha", n.alpha)) return false;
        return need(cx, n, is(0, DT_F32) && is(1, DT_F32) && B(0).count == B(1).count, "operand mismatch");
    case OP_AVG2:
        for (const char *k : {"S", "X", "Y"}) {
            if (!arg_buf(cx, n, args, k, x)) return false;
            n.b.push_back(x);
        }
        return need(cx, n, is(0, DT_F32) && is(1, DT_F32) && is(2, DT_F32) && B(0).count == B(1).count &&
                               B(0).count == B(2).count, "operand mismatch");
    case OP_SCALE:
        if (!arg_buf(cx, n, args, "D", x)) return false;
        n.b.push_back(x);
        if (!arg_num(cx, n, args, "beta", n.alpha)) return false;
        return need(cx, n, is(0, DT_F32), "operand must be f32");
    case OP_COPY:
        if (!arg_buf(cx, n, args, "dst", x)) return false;
        n.b.push_back(x);
        if (!arg_buf(cx, n, args, "src", x)) return false;
        n.b.push_back(x);
        return need(cx, n, B(0).dtype == B(1).dtype && B(0).count == B(1).count, "operand mismatch");
    case OP_CAST_BF16: {
        std::vector<int> d, s;
        if (!arg_buf_list(cx, n, args, "dst", d) || !arg_buf_list(cx, n, args, "src", s)) return false;
        if (!need(cx, n, d.size() == s.size(), "dst/src lists differ in length")) return false;
        for (size_t i = 0; i < d.size(); ++i) {
            n.b.push_back(d[i]);
            n.b.push_back(s[i]);
            const Buffer &bd = app.bufs[d[i]], &bs = app.bufs[s[i]];
            if (!need(cx, n, bd.dtype == DT_BF16 && bs.dtype == DT_F32 && bd.count == bs.count, "operand mismatch"))
                return false;
        }
        return true;
    }
    case OP_TRANSPOSE:
        if (!arg_buf(cx, n, args, "src", x)) return false;
        n.b.push_back(x);
        if (!arg_buf(cx, n, args, "dst", x)) return false;
        n.b.push_back(x);
        return need(cx, n, is(0, DT_F32) && is(1, DT_F32) && B(0).dims.size() == 2 && B(1).dims.size() == 2 &&
                               B(0).dims[0] == B(1).dims[1] && B(0).dims[1] == B(1).dims[0] && n.b[0] != n.b[1],
                    "needs distinct R x C -> C x R f32 operands");
    case OP_SUMSQ:
        if (!arg_buf(cx, n, args, "x", x)) return false;
        n.b.push_back(x);
        if (!arg_buf(cx, n, args, "s", x)) return false;
        n.b.push_back(x);
        return need(cx, n, is(0, DT_F32) && is(1, DT_F64) && B(1).count >= 1, "operand mismatch");
    case OP_STENCIL19: {
        for (const char *k : {"p", "q", "res"}) {
            if (!arg_buf(cx, n, args, k, x)) return false;
            n.b.push_back(x);
        }
        if (!need(cx, n, is(0, DT_F32) && is(1, DT_F32) && is(2, DT_F64) && B(0).dims.size() == 3 &&
                              B(0).dims == B(1).dims && n.b[0] != n.b[1], "needs distinct f32 grids and an f64 residual"))
            return false;
        // the sweep forms 32-bit byte offsets up to five planes past the grid
        if (!need(cx, n, B(0).dims[0] >= 1 && B(0).dims[1] >= 1 && B(0).dims[2] >= 1 &&
                              (B(0).dims[0] + 6) * B(0).dims[1] * B(0).dims[2] * 4 < (1ll << 31),
                  "grid extents (the grid plus six planes must hold under 2 GiB: the sweep addresses it with "
                  "32-bit byte offsets)")) return false;
        const Json *sl = args->get("slot");
        if (!sl || sl->kind != Json::Str) return need(cx, n, false, "missing residual slot");
        for (size_t r = 0; r < n.repeats.size(); ++r)
            if (app.repeat_names[n.repeats[r].first] == sl->str) n.slot_repeat = n.repeats[r].first;
        if (!need(cx, n, n.slot_repeat >= 0, "slot must name an enclosing repeat variable")) return false;
        return need(cx, n, rep_counts[n.slot_repeat] <= B(2).count, "residual buffer shorter than the repeat");
    }
    case OP_COPY_INTERIOR:
        if (!arg_buf(cx, n, args, "dst", x)) return false;
        n.b.push_back(x);
        if (!arg_buf(cx, n, args, "src", x)) return false;
        n.b.push_back(x);
        if (!need(cx, n, is(0, DT_F32) && is(1, DT_F32) && B(0).dims.size() == 3 && B(0).dims == B(1).dims,
                  "needs equal f32 grids")) return false;
        return need(cx, n, B(0).nbytes < (1ull << 31),
                    "a grid must hold under 2 GiB (the copy addresses it with 32-bit byte offsets)");
    case OP_REC_PREFIX:
        if (!arg_buf(cx, n, args, "v", x)) return false;
        n.b.push_back(x);
        if (!arg_buf(cx, n, args, "S", x)) return false;
        n.b.push_back(x);
        return need(cx, n, is(0, DT_F32) && is(1, DT_F32) && B(0).dims.size() == 1 && B(1).dims.size() == 2 &&
                               B(1).dims[0] == B(0).dims[0], "needs v[N] and S[N][*] f32");
    case OP_REC_DECAY:
        if (!arg_buf(cx, n, args, "w", x)) return false;
        n.b.push_back(x);
        if (!arg_buf(cx, n, args, "p", x)) return false;
        n.b.push_back(x);
        return need(cx, n, is(0, DT_F32) && is(1, DT_F32) && B(0).dims.size() == 1 && B(1).dims.size() == 3 &&
                               B(1).dims[2] == B(0).dims[0] && B(1).dims[0] >= 2 && B(1).dims[1] >= 2,
                    "needs w[K] and p[I][J][K] f32");
    case OP_FFT_ROWS: {
        // x[R][2n]: R rows of n complex values, real and imaginary parts
        // interleaved; n a power of two up to kFftMaxPoints
        if (!arg_buf(cx, n, args, "x", x)) return false;
        n.b.push_back(x);
        if (!need(cx, n, is(0, DT_F32) && B(0).dims.size() == 2, "needs a 2-D f32 buffer")) return false;
        // optional flags "inverse" (the inverse transform) and "real" (rows
        // of real values), each true / false or 0 / 1
        for (const char *key : {"inverse", "real"}) {
            if (const Json *f = args->get(key)) {
                const bool ok = (f->kind == Json::Bool) ||
                                (f->kind == Json::Num && f->is_int && (f->inum == 0 || f->inum == 1));
                if (!need(cx, n, ok, std::string(key) + " must be true / false or 0 / 1")) return false;
                (key[0] == 'i' ? n.inverse : n.real) = f->kind == Json::Bool ? f->b : f->inum == 1;
            }
        }
        if (n.real) {
            // x[R][n]: R rows of n real values, n a power of two from 2 to
            // kFftMaxPoints, replaced by their packed spectrum (inverse: a
            // packed spectrum replaced by its real row)
            const int64_t nr = B(0).dims[1];
            return need(cx, n, nr >= 2 && nr <= kFftMaxPoints && (nr & (nr - 1)) == 0 && B(0).dims[0] < (1ll << 31),
                        "real rows must hold n values, n a power of two from 2 to " +
                            std::to_string(kFftMaxPoints));
        }
        const int64_t pts = B(0).dims[1] / 2;
        return need(cx, n, B(0).dims[1] % 2 == 0 && pts >= 1 && pts <= kFftMaxPoints && (pts & (pts - 1)) == 0 &&
                               B(0).dims[0] < (1ll << 31),
                    "row length must be 2 n floats, n a power of two up to " + std::to_string(kFftMaxPoints));
    }
    case OP_HOST_CODE: {
        // a nest no library operation matches, compiled from its own source
        // text into the application's host object; it runs on the CPU only
        const Json *sy = args->get("symbol");
        if (!sy || sy->kind != Json::Str || sy->str.empty()) return need(cx, n, false, "missing symbol");
        n.symbol = sy->str;
        return true;
    }
    case OP_LCG_FILL: {
        if (!arg_buf(cx, n, args, "L", x)) return false;
        n.b.push_back(x);
        double s = 0;
        if (!arg_num(cx, n, args, "seed32", s)) return false;
        n.seed32 = (uint32_t)(int64_t)s;
        return need(cx, n, is(0, DT_F32), "operand must be f32");
    }
    default:
        return cx.fail(OFL_E_IR, "unknown op");
    }
}

// The loops of a nest must run over exactly the index space its operation
// covers: the library's kernel and host code of an op process that whole
// space, so a nest over part of it (a partial update, a smaller product) is
// a different program and must not bind to the op.
bool check_span(Ctx &cx, const Nest &n) {
    const AppIR &app = cx.app;
    auto full = [&](const std::vector<int64_t> &dims) {
        if (n.loops.size() != dims.size()) return false;
        for (size_t l = 0; l < dims.size(); ++l)
            if (n.loops[l].lo != 0 || n.loops[l].hi != dims[l]) return false;
        return true;
    };
    auto interior = [&](const std::vector<int64_t> &dims) {
        if (n.loops.size() != dims.size()) return false;
        for (size_t l = 0; l < dims.size(); ++l)
            if (n.loops[l].lo != 1 || n.loops[l].hi != dims[l] - 1) return false;
        return true;
    };
    auto D = [&](int i) -> const std::vector<int64_t> & { return app.bufs[n.b[i]].dims; };
    bool ok = true;
    switch (n.op) {
    case OP_INIT_UNIFORM:
        for (size_t i = 0; i < n.b.size(); ++i) ok = ok && full(D((int)i));
        break;
    case OP_GEMM:
    case OP_GEMM_BF16:
        ok = n.loops.size() == 3 && n.loops[0].lo == 0 && n.loops[0].hi == D(0)[0] && n.loops[1].lo == 0 &&
             n.loops[1].hi == D(1)[1] && n.loops[2].lo == 0 && n.loops[2].hi == D(0)[1];
        break;
    case OP_ADD_SCALED: case OP_AVG2: case OP_SCALE: case OP_COPY: case OP_CAST_BF16: case OP_TRANSPOSE:
    case OP_SUMSQ: case OP_LCG_FILL: case OP_FFT_ROWS:
        ok = full(D(0));
        break;
    case OP_STENCIL19:
    case OP_COPY_INTERIOR:
        ok = interior(D(0));
        break;
    case OP_REC_PREFIX:
    case OP_REC_DECAY: {
        const int64_t len = D(0)[0];
        ok = n.loops.size() == 1 && n.loops[0].lo == 1 && n.loops[0].hi == len;
        break;
    }
    default:
        break;
    }
    return ok ? true : need(cx, n, false, "its loops do not span the index space of the operation");
}

bool parse_nest(Ctx &cx, const Json &j, const std::vector<std::pair<int, int64_t>> &repeats,
                const std::vector<int64_t> &rep_counts, ProgItem &item) {
    AppIR &app = cx.app;
    Nest n;
    const Json *op = j.get("op");
    if (!op || op->kind != Json::Str) return cx.fail(OFL_E_PARSE, "nest without op");
    n.op = OP_COUNT;
    for (int k = 0; k < OP_COUNT; ++k)
        if (op->str == kOpNames[k]) n.op = (Op)k;
    if (n.op == OP_COUNT) return cx.fail(OFL_E_IR, "unknown op '" + op->str + "'");
    const Json *nm = j.get("nest");
    n.name = (nm && nm->kind == Json::Str) ? nm->str : op->str;
    n.repeats = repeats;
    const Json *loops = j.get("loops");
    if (!loops || loops->kind != Json::Arr || loops->arr.empty())
        return cx.fail(OFL_E_PARSE, "nest " + n.name + ": needs at least one loop");
    std::set<std::string> vars;
    for (const auto &L : loops->arr) {
        if (L.kind != Json::Arr || L.arr.size() != 3 || L.arr[0].kind != Json::Str)
            return cx.fail(OFL_E_PARSE, "nest " + n.name + ": loop must be [var, lo, hi]");
        Loop lp;
        lp.var = L.arr[0].str;
        if (vars.count(lp.var) || app.params.count(lp.var))
            return cx.fail(OFL_E_PARSE, "nest " + n.name + ": loop variable '" + lp.var + "' reused");
        if (!const_expr(cx, L.arr[1], lp.lo) || !const_expr(cx, L.arr[2], lp.hi)) return false;
        vars.insert(lp.var);
        n.loops.push_back(lp);
    }
    std::set<std::string> allvars = vars;
    for (auto &r : repeats) allvars.insert(app.repeat_names[r.first]);
    const Json *acc = j.get("access");
    if (!acc || acc->kind != Json::Arr) return cx.fail(OFL_E_PARSE, "nest " + n.name + ": missing access list");
    for (const auto &A : acc->arr) {
        if (A.kind != Json::Arr || A.arr.size() < 3 || A.arr[0].kind != Json::Str || A.arr[1].kind != Json::Str)
            return cx.fail(OFL_E_PARSE, "nest " + n.name + ": access must be [buf, mode, subscripts...]");
        Access a;
        a.buf = find_buf(app, A.arr[0].str);
        if (a.buf < 0) return cx.fail(OFL_E_IR, "nest " + n.name + ": unknown buffer '" + A.arr[0].str + "'");
        const std::string &m = A.arr[1].str;
        if (m == "r") a.mode = M_R;
        else if (m == "w") a.mode = M_W;
        else if (m == "rw") a.mode = M_RW;
        else if (m == "sum") a.mode = M_SUM;
        else return cx.fail(OFL_E_PARSE, "nest " + n.name + ": bad access mode '" + m + "'");
        const Buffer &buf = app.bufs[a.buf];
        if (A.arr.size() - 2 != buf.dims.size())
            return cx.fail(OFL_E_IR, "nest " + n.name + ": rank mismatch on '" + buf.name + "'");
        for (size_t d = 2; d < A.arr.size(); ++d) {
            std::string s;
            if (!json_expr_string(A.arr[d], s)) return cx.fail(OFL_E_PARSE, "nest " + n.name + ": bad subscript");
            Affine af;
            if (!parse_affine(cx, s, allvars, af)) return false;
            Sub sub;
            sub.c = af.c;
            if (af.var.empty()) {
                sub.kind = S_CONST;
            } else if (vars.count(af.var)) {
                sub.kind = S_LOOP;
                for (size_t l = 0; l < n.loops.size(); ++l)
                    if (n.loops[l].var == af.var) sub.idx = (int)l;
            } else {
                sub.kind = S_REPEAT;
                for (auto &r : repeats)
                    if (app.repeat_names[r.first] == af.var) sub.idx = r.first;
            }
            a.subs.push_back(sub);
        }
        n.access.push_back(a);
    }
    const Json *fl = j.get("flags");
    if (fl) {
        if (fl->kind != Json::Arr) return cx.fail(OFL_E_PARSE, "nest " + n.name + ": flags must be a list");
        for (const auto &f : fl->arr) {
            if (f.kind != Json::Str) return cx.fail(OFL_E_PARSE, "bad flag");
            if (f.str == "opaque_call") n.opaque_call = true;
            else if (f.str == "early_exit") n.early_exit = true;
            else return cx.fail(OFL_E_PARSE, "nest " + n.name + ": unknown flag '" + f.str + "'");
        }
    }
    // every access must stay inside its buffer for every iteration
    bool empty_space = false;
    for (const auto &lp : n.loops)
        if (lp.lo >= lp.hi) empty_space = true;
    if (!empty_space) {
        for (const auto &a : n.access) {
            const Buffer &buf = app.bufs[a.buf];
            for (size_t d = 0; d < a.subs.size(); ++d) {
                const Sub &s = a.subs[d];
                int64_t lo = s.c, hi = s.c;
                if (s.kind == S_LOOP) {
                    lo += n.loops[s.idx].lo;
                    hi += n.loops[s.idx].hi - 1;
                } else if (s.kind == S_REPEAT) {
                    if (rep_counts[s.idx] <= 0) continue;
                    hi += rep_counts[s.idx] - 1;
                }
                if (lo < 0 || hi >= buf.dims[d])
                    return cx.fail(OFL_E_IR, "nest " + n.name + ": access to '" + buf.name + "' out of bounds");
            }
        }
    }
    const Json *args = j.get("args");
    if (n.op != OP_NONE && (!args || args->kind != Json::Obj))
        return cx.fail(OFL_E_IR, "nest " + n.name + ": missing args");
    if (!resolve_op(cx, n, args, rep_counts)) return false;
    if (!check_span(cx, n)) return false;
    // each operand of the body must be declared among the accesses
    for (int b : n.b) {
        bool found = false;
        for (const auto &a : n.access) found |= (a.buf == b);
        if (!found)
            return cx.fail(OFL_E_IR, "nest " + n.name + ": operand '" + app.bufs[b].name + "' has no declared access");
    }
    item.is_repeat = false;
    item.nest = (int)app.nests.size();
    app.nests.push_back(std::move(n));
    return true;
}

bool parse_program(Ctx &cx, const Json &arr, std::vector<std::pair<int, int64_t>> repeats,
                   std::vector<int64_t> &rep_counts, std::vector<ProgItem> &out) {
    if (arr.kind != Json::Arr) return cx.fail(OFL_E_PARSE, "program must be a list");
    for (const auto &it : arr.arr) {
        if (it.kind != Json::Obj) return cx.fail(OFL_E_PARSE, "program item must be an object");
        ProgItem pi;
        if (it.get("repeat")) {
            int64_t cnt = 0;
            if (!const_expr(cx, *it.get("repeat"), cnt)) return false;
            const Json *v = it.get("var");
            const Json *body = it.get("body");
            if (!v || v->kind != Json::Str || !body) return cx.fail(OFL_E_PARSE, "repeat needs var and body");
            if (cnt < 0) return cx.fail(OFL_E_IR, "negative repeat count");
            if (cx.app.params.count(v->str)) return cx.fail(OFL_E_PARSE, "repeat variable shadows a parameter");
            for (auto &r : repeats)
                if (cx.app.repeat_names[r.first] == v->str)
                    return cx.fail(OFL_E_PARSE, "repeat variable reused");
            pi.is_repeat = true;
            pi.rep_id = (int)cx.app.repeat_names.size();
            pi.count = cnt;
            cx.app.repeat_names.push_back(v->str);
            rep_counts.push_back(cnt);
            auto inner = repeats;
            inner.emplace_back(pi.rep_id, cnt);
            if (!parse_program(cx, *body, inner, rep_counts, pi.body)) return false;
        } else {
            if (!parse_nest(cx, it, repeats, rep_counts, pi)) return false;
        }
        out.push_back(std::move(pi));
    }
    return true;
}

}  // namespace

int parse_app(const std::string &text, AppIR &app, std::string &err,
              const std::map<std::string, int64_t> *overrides) {
    Json doc;
    JsonParser jp(text);
    if (!jp.parse(doc, err)) return OFL_E_PARSE;
    if (doc.kind != Json::Obj) {
        err = "application must be a JSON object";
        return OFL_E_PARSE;
    }
    Ctx cx{app, err};
    const Json *nm = doc.get("name");
    app.name = (nm && nm->kind == Json::Str) ? nm->str : "app";
    const Json *params = doc.get("params");
    if (params) {
        if (params->kind != Json::Obj) return (cx.fail(OFL_E_PARSE, "params must be an object"), cx.status);
        for (const auto &kv : params->obj) {
            if (kv.second.kind != Json::Num || !kv.second.is_int) {
                cx.fail(OFL_E_PARSE, "param '" + kv.first + "' must be an integer");
                return cx.status;
            }
            app.params[kv.first] = kv.second.inum;
        }
    }
    if (overrides) {
        for (const auto &kv : *overrides) {
            auto it = app.params.find(kv.first);
            if (it == app.params.end()) {
                cx.fail(OFL_E_ARG, "unknown parameter '" + kv.first + "'");
                return cx.status;
            }
            it->second = kv.second;
        }
    }
    const Json *bufs = doc.get("buffers");
    if (!bufs || bufs->kind != Json::Arr) {
        cx.fail(OFL_E_PARSE, "missing buffers");
        return cx.status;
    }
    for (const auto &bj : bufs->arr) {
        Buffer b;
        const Json *n = bj.get("name");
        if (!n || n->kind != Json::Str || n->str.empty()) { cx.fail(OFL_E_PARSE, "buffer without name"); return cx.status; }
        b.name = n->str;
        if (find_buf(app, b.name) >= 0) { cx.fail(OFL_E_IR, "duplicate buffer '" + b.name + "'"); return cx.status; }
        const Json *dt = bj.get("dtype");
        std::string dts = (dt && dt->kind == Json::Str) ? dt->str : "f32";
        int esz;
        if (dts == "f32") { b.dtype = DT_F32; esz = 4; }
        else if (dts == "f64") { b.dtype = DT_F64; esz = 8; }
        else if (dts == "bf16") { b.dtype = DT_BF16; esz = 2; }
        else { cx.fail(OFL_E_IR, "buffer '" + b.name + "': unknown dtype"); return cx.status; }
        const Json *dims = bj.get("dims");
        if (!dims || dims->kind != Json::Arr || dims->arr.empty()) { cx.fail(OFL_E_PARSE, "buffer '" + b.name + "': dims"); return cx.status; }
        b.count = 1;
        for (const auto &d : dims->arr) {
            int64_t v;
            if (!const_expr(cx, d, v)) return cx.status;
            if (v < 1 || v > (1ll << 34)) { cx.fail(OFL_E_IR, "buffer '" + b.name + "': bad extent"); return cx.status; }
            b.dims.push_back(v);
            b.count *= v;
            if (b.count > (1ll << 36)) { cx.fail(OFL_E_IR, "buffer '" + b.name + "': too large"); return cx.status; }
        }
        b.nbytes = (uint64_t)b.count * (uint64_t)esz;
        const Json *su = bj.get("setup");
        std::string sus = (su && su->kind == Json::Str) ? su->str : "zero";
        if (sus == "sin") {
            b.setup_sin = true;
            if (b.dims.size() != 3 || b.dtype != DT_F32 || b.dims[0] < 2 || b.dims[1] < 2 || b.dims[2] < 2) {
                cx.fail(OFL_E_IR, "buffer '" + b.name + "': sin set-up needs an f32 3-D grid with extents >= 2");
                return cx.status;
            }
            const Json *m = bj.get("mode");
            int64_t mv = 1;
            if (m && !const_expr(cx, *m, mv)) return cx.status;
            b.sin_mode = (int32_t)mv;
        } else if (sus != "zero") {
            cx.fail(OFL_E_IR, "buffer '" + b.name + "': unknown set-up '" + sus + "'");
            return cx.status;
        }
        const Json *o = bj.get("output");
        b.output = o && o->kind == Json::Bool && o->b;
        app.bufs.push_back(b);
    }
    const Json *ho = doc.get("host_object");
    if (ho) {
        if (ho->kind != Json::Str || ho->str.empty()) { cx.fail(OFL_E_PARSE, "host_object must be a path"); return cx.status; }
        app.host_object = ho->str;
    }
    const Json *prog = doc.get("program");
    if (!prog) { cx.fail(OFL_E_PARSE, "missing program"); return cx.status; }
    std::vector<int64_t> rep_counts;
    if (!parse_program(cx, *prog, {}, rep_counts, app.program)) return cx.status;
    if (app.nests.empty()) { cx.fail(OFL_E_IR, "program has no nests"); return cx.status; }
    for (const auto &n : app.nests)
        if (n.op == OP_HOST_CODE && app.host_object.empty()) {
            cx.fail(OFL_E_IR, "nest " + n.name + " is host code but the application names no host_object");
            return cx.status;
        }
    analyse(app);
    for (const auto &n : app.nests)
        if (n.verdict != V_REJECT && n.op != OP_NONE && !op_has_device_kernel(n.op)) {
            cx.fail(OFL_E_IR, "nest " + n.name + " is parallel but op '" + std::string(op_name(n.op)) +
                                  "' has no device kernel");
            return cx.status;
        }
    return OFL_OK;
}

}  // namespace ofl
