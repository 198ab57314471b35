// Application IR: buffers, loop nests with affine accesses, repeat blocks.
//
// This is the parsed form of the program the offloader works on: Sec. 4 of
// the paper parses the C/C++ source, finds and counts the for statements and
// tries each one with the parallel directive.  A nest here carries its loop
// bounds (outermost first), its array references with subscripts of the form
// `var + c` or `c`, flags for an external call or an early exit, and the body
// kind (`op`) that selects the GPU kernel and the serial host code.
#pragma once

#include "fft_limits.hpp"

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "json.hpp"

namespace ofl {

enum DType { DT_F32 = 0, DT_F64 = 1, DT_BF16 = 2 };
enum Mode { M_R = 0, M_W = 1, M_RW = 2, M_SUM = 3 };
enum SubKind { S_CONST = 0, S_LOOP = 1, S_REPEAT = 2 };
enum Verdict { V_PARALLEL = 0, V_PARALLEL_REDUCTION = 1, V_REJECT = 2 };
enum Reason { RS_NONE = 0, RS_DATA_DEP = 1, RS_EXTERNAL_CALL = 2, RS_BREAK = 3, RS_NO_KERNEL = 4 };

enum Op {
    OP_NONE = 0,        // analysis-only nest (no body)
    OP_INIT_UNIFORM,
    OP_GEMM,
    OP_GEMM_BF16,
    OP_ADD_SCALED,
    OP_AVG2,
    OP_SCALE,
    OP_COPY,
    OP_CAST_BF16,
    OP_TRANSPOSE,
    OP_SUMSQ,
    OP_STENCIL19,
    OP_COPY_INTERIOR,
    OP_REC_PREFIX,
    OP_REC_DECAY,
    OP_LCG_FILL,
    OP_FFT_ROWS,        // function block: complex DFT of each row (forward, or inverse / n)
    OP_HOST_CODE,       // a nest compiled from its own source text, CPU only
    OP_COUNT
};

const char *op_name(Op op);
bool op_has_device_kernel(Op op);

enum GemmPrec { PREC_F32 = 0, PREC_BF16X3 = 1, PREC_FP8X2 = 2 };

struct Buffer {
    std::string name;
    DType dtype = DT_F32;
    std::vector<int64_t> dims;
    int64_t count = 0;
    uint64_t nbytes = 0;
    bool setup_sin = false;   // otherwise zero
    int32_t sin_mode = 1;
    bool output = false;
};

struct Sub {
    SubKind kind = S_CONST;
    int idx = -1;             // loop index or repeat id
    int64_t c = 0;
};

struct Access {
    int buf = -1;
    Mode mode = M_R;
    std::vector<Sub> subs;
};

struct Loop {
    std::string var;
    int64_t lo = 0, hi = 0;   // [lo, hi)
};

struct Nest {
    std::string name;
    Op op = OP_NONE;
    std::vector<Loop> loops;
    std::vector<Access> access;
    bool opaque_call = false, early_exit = false;
    std::vector<std::pair<int, int64_t>> repeats;   // enclosing repeat ids and trip counts

    // resolved op arguments
    std::vector<int> b;          // buffer operands, op-specific order
    std::vector<uint32_t> streams;
    double alpha = 0.0;          // add_scaled alpha / scale beta
    uint32_t seed32 = 0;         // lcg_fill
    bool inverse = false;        // fft_rows: the inverse transform (scaled by 1/n)
    bool real = false;           // fft_rows: rows of n real values, packed spectrum
    int slot_repeat = -1;        // stencil residual slot: repeat id
    GemmPrec prec = PREC_F32;
    std::string symbol;          // host_code: entry point in the application's host object
    void (*host_fn)(void *const *bufs, const int64_t *repeat_env) = nullptr;

    // analysis results
    Verdict verdict = V_PARALLEL;
    Reason reason = RS_NONE;
    int gene_pos = -1;
    std::vector<int> reads, writes;   // buffer-level sets for transfer planning
};

struct ProgItem {
    bool is_repeat = false;
    int nest = -1;
    int rep_id = -1;
    int64_t count = 0;
    std::vector<ProgItem> body;
};

struct AppIR {
    std::string name;
    std::map<std::string, int64_t> params;
    std::vector<Buffer> bufs;
    std::vector<Nest> nests;
    std::vector<ProgItem> program;
    std::vector<std::string> repeat_names;
    int gene_len = 0;
    std::string host_object;     // shared object holding the host_code nests (empty: none)
};

// Parse + validate; returns an OFL_* status and fills `err` on failure.
// `overrides` replaces the values of parameters the description declares.
int parse_app(const std::string &text, AppIR &app, std::string &err,
              const std::map<std::string, int64_t> *overrides = nullptr);

// Parallelisability verdict of every nest and gene positions.
void analyse(AppIR &app);

// Exact carried-dependence test between write `w` and access `x` of a nest.
bool carried_dependence(const Nest &n, const Access &w, const Access &x);

}  // namespace ofl
