// C ABI, application object and pattern executor.
#include "../../include/ofl.h"

#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <fstream>
#include <limits>
#include <map>
#include <memory>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "ga.hpp"
#include "host_nests.hpp"
#include "ir.hpp"
#include "kernels.hpp"
#include "launch.hpp"
#include "plan.hpp"
#include "status.hpp"

using namespace ofl;

namespace {
thread_local std::string g_last_error;
}  // namespace

int ofl::fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int ofl::hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return OFL_E_HIP;
}

namespace {

using clk = std::chrono::steady_clock;

}  // namespace

struct ofl_app;

namespace {

bool timed_nest(const ofl_app *app, const Nest &n, int32_t *exec_count);

// Host work recorded into a graph: one serial nest, or the restore of set-up
// content into host copies.  They live as long as the graph that calls them.
// Time limit of a captured run's host nests: the run graph's first node
// stamps the start, every host nest of the run checks start + limit_s as an
// eager run checks its deadline, and a nest that runs out sets `cut`.
// limit_s <= 0: no limit.  Written by host callbacks, read by the thread that
// submitted the graphs after it synchronised the stream.
struct GraphClock {
    std::chrono::steady_clock::time_point start;
    double limit_s = 0.0;
    std::atomic<bool> cut{false};
};
struct HostTask {
    ofl_app *app = nullptr;
    int nest = -1;
    std::vector<int64_t> env;
    GraphClock *clock = nullptr;
};
struct HostRestore {
    ofl_app *app = nullptr;
    std::vector<int> bufs;    // set-up content the run consumes on the host
    std::vector<int> marks;   // host copies the run writes
};

// Captured graphs of one (placement, policy, flags, device buffers).
struct GraphEntry {
    hipGraphExec_t reset = nullptr, run = nullptr;
    Plan plan;
    std::vector<char> host_written;
    std::vector<std::unique_ptr<HostTask>> tasks;
    std::unique_ptr<HostRestore> restore;
    std::unique_ptr<GraphClock> clock;
    int32_t launches = 0, host_nests = 0;
    // with kernel timing: an event record node before and after every GPU
    // nest (nest index, start event, stop event)
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> timed;
    ~GraphEntry() {
        if (reset) (void)hipGraphExecDestroy(reset);
        if (run) (void)hipGraphExecDestroy(run);
        for (auto &t : timed) {
            (void)hipEventDestroy(t.second.first);
            (void)hipEventDestroy(t.second.second);
        }
    }
};

}  // namespace

struct ofl_app {
    AppIR ir;
    uint64_t seed = 0;

    // pinned host copies of every buffer and the set-up content of sine fields
    std::vector<void *> host;
    std::vector<char> host_dirty;            // differs from the set-up content
    std::vector<std::vector<unsigned char>> setup;   // non-zero set-up content (empty = zeros)

    // device side owned by the library
    int device = -1;
    std::vector<void *> dev_setup;           // device copies of sine set-up content
    double *d_partials = nullptr;
    int64_t partial_cap = 0;
    void *d_gemm_ws = nullptr;               // operand workspace of split-precision GEMM nests
    int64_t gemm_ws_bytes = 0;
    float *d_twiddles = nullptr;             // FFT twiddle tables (fft_twiddle_packed), if any FFT call

    // state after the last completed run
    bool ran = false;
    std::vector<char> host_valid, dev_valid, host_written;
    std::vector<void *> last_dev;
    hipStream_t last_stream = nullptr;

    // per-kernel timing
    bool timing = false;
    uint64_t timing_ops = 0;                 // bit per Op of the timed kinds; 0: every kind
    int32_t timing_stride = 1, timing_phase = 0;   // time executions i of a kind with i % stride == phase
    std::vector<hipEvent_t> events;
    std::map<std::string, std::pair<int64_t, double>> kstats;

    // event pairs of batched population evaluation
    std::vector<hipEvent_t> chain_events;

    // concurrent runs (OFL_RUN_CONCURRENT): component of every buffer and
    // nest (nests that share no buffer, nor the product workspace, are in
    // different components), and per component beyond the first a stream and
    // reduction scratch of its own
    bool comps_done = false;
    int n_comps = 1;
    std::vector<int> buf_comp, nest_comp;
    std::vector<hipStream_t> side_streams;
    std::vector<double *> side_partials;

    // captured graphs and the stream they are captured on
    std::map<std::vector<uint64_t>, std::unique_ptr<GraphEntry>> graphs;
    hipStream_t capture_stream = nullptr;

    void *host_lib = nullptr;                // dlopen handle of the host object, if any

    // output check: probe positions per output buffer and the all-zero
    // gene's values there (valid until the inputs change)
    bool ref_valid = false, ref_bufs_done = false;
    std::vector<int> ref_bufs;
    std::vector<std::vector<int64_t>> ref_pos;
    std::vector<std::vector<double>> ref_val;
    int64_t *d_probe_idx = nullptr;
    double *d_probe_val = nullptr;

    ~ofl_app() {
        graphs.clear();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        for (void *p : host)
            if (p) (void)hipHostFree(p);
        for (void *p : dev_setup)
            if (p) (void)hipFree(p);
        if (d_partials) (void)hipFree(d_partials);
        if (d_gemm_ws) (void)hipFree(d_gemm_ws);
        if (d_twiddles) (void)hipFree(d_twiddles);
        for (auto e : events) (void)hipEventDestroy(e);
        for (auto e : chain_events) (void)hipEventDestroy(e);
        for (auto st : side_streams)
            if (st) (void)hipStreamDestroy(st);
        for (double *p : side_partials)
            if (p) (void)hipFree(p);
        if (host_lib) dlclose(host_lib);
        if (d_probe_idx) (void)hipFree(d_probe_idx);
        if (d_probe_val) (void)hipFree(d_probe_val);
    }
};

namespace {

int check_gene(const ofl_app *app, const uint8_t *gene, int32_t gene_len, std::vector<uint8_t> &placement) {
    if (!gene && gene_len > 0) return fail(OFL_E_ARG, "null gene");
    if (gene_len != app->ir.gene_len)
        return fail(OFL_E_GENE_LEN, "gene length " + std::to_string(gene_len) + " != " + std::to_string(app->ir.gene_len));
    for (int i = 0; i < gene_len; ++i)
        if (gene[i] > 1) return fail(OFL_E_GENE_BIT, "gene byte " + std::to_string(i) + " is not 0/1");
    placement.assign(app->ir.nests.size(), 0);
    for (size_t n = 0; n < app->ir.nests.size(); ++n) {
        const Nest &ns = app->ir.nests[n];
        if (ns.gene_pos >= 0) placement[n] = gene[ns.gene_pos];
    }
    return OFL_OK;
}

int ensure_host(ofl_app *app) {
    if (!app->host.empty()) return OFL_OK;
    const size_t nb = app->ir.bufs.size();
    if (app->setup.size() != nb) app->setup.resize(nb);
    std::vector<void *> host(nb, nullptr);
    for (size_t b = 0; b < nb; ++b) {
        const Buffer &buf = app->ir.bufs[b];
        hipError_t e = hipHostMalloc(&host[b], buf.nbytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            for (void *p : host)
                if (p) (void)hipHostFree(p);
            return e == hipErrorOutOfMemory ? fail(OFL_E_NOMEM, "pinned host allocation failed")
                                            : hip_fail(e, "hipHostMalloc");
        }
        if (buf.setup_sin && app->setup[b].empty()) {
            app->setup[b].resize(buf.nbytes);
            fill_setup_sin(buf, reinterpret_cast<float *>(app->setup[b].data()));
        }
        if (!app->setup[b].empty()) std::memcpy(host[b], app->setup[b].data(), buf.nbytes);
        else std::memset(host[b], 0, buf.nbytes);
    }
    app->host = host;
    app->host_dirty.assign(nb, 0);
    app->dev_setup.assign(nb, nullptr);
    return OFL_OK;
}

void restore_host(ofl_app *app, int b) {
    const Buffer &buf = app->ir.bufs[b];
    if (!app->setup[b].empty()) std::memcpy(app->host[b], app->setup[b].data(), buf.nbytes);
    else std::memset(app->host[b], 0, buf.nbytes);
    app->host_dirty[b] = 0;
}

// Kernel variant of a GEMM nest (as numbered by the k:: GEMM launchers).
int gemm_variant(const Nest &n) {
    if (n.op == OP_GEMM_BF16) return 3;
    return n.prec == PREC_BF16X3 ? 1 : (n.prec == PREC_FP8X2 ? 2 : 0);
}

int ensure_device(ofl_app *app) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (app->device >= 0 && app->device != dev)
        return fail(OFL_E_STATE, "application already bound to another device");
    app->device = dev;
    if (app->d_partials) return OFL_OK;
    int64_t cap = 1;
    for (const auto &n : app->ir.nests) {
        if (n.op == OP_SUMSQ) cap = std::max(cap, k::sumsq_partials(app->ir.bufs[n.b[0]].count));
        if (n.op == OP_STENCIL19) {
            const auto &d = app->ir.bufs[n.b[0]].dims;
            cap = std::max(cap, k::stencil_partials(d[0], d[1], d[2]));
        }
    }
    void *mem = nullptr;
    const size_t bytes = (size_t)cap * sizeof(double) + 256;
    e = hipMalloc(&mem, bytes);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(OFL_E_NOMEM, "device scratch") : hip_fail(e, "hipMalloc");
    e = hipMemset(mem, 0, bytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return hip_fail(e, "scratch init");
    }
    int64_t ws = 0;
    for (const auto &n : app->ir.nests) {
        if ((n.op != OP_GEMM && n.op != OP_GEMM_BF16) || gemm_variant(n) == 0) continue;
        const auto &a = app->ir.bufs[n.b[0]].dims, &bb = app->ir.bufs[n.b[1]].dims;
        ws = std::max(ws, k::gemm_workspace_bytes(a[0], bb[1], a[1], gemm_variant(n)));
    }
    if (ws > 0) {
        void *w = nullptr;
        e = hipMalloc(&w, (size_t)ws);
        if (e != hipSuccess) {
            (void)hipFree(mem);
            return e == hipErrorOutOfMemory ? fail(OFL_E_NOMEM, "GEMM workspace") : hip_fail(e, "hipMalloc");
        }
        app->d_gemm_ws = w;
        app->gemm_ws_bytes = ws;
    }
    bool fft = false;
    for (const auto &n : app->ir.nests) fft = fft || n.op == OP_FFT_ROWS;
    if (fft) {
        std::vector<float> tw(2 * (kFftMaxPoints - 1));
        fft_twiddle_packed(tw.data());
        void *t = nullptr;
        e = hipMalloc(&t, tw.size() * sizeof(float));
        if (e == hipSuccess) e = hipMemcpy(t, tw.data(), tw.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (t) (void)hipFree(t);
            (void)hipFree(mem);
            return e == hipErrorOutOfMemory ? fail(OFL_E_NOMEM, "FFT twiddles") : hip_fail(e, "twiddle table");
        }
        app->d_twiddles = static_cast<float *>(t);
    }
    app->d_partials = static_cast<double *>(mem);
    app->partial_cap = cap;
    return OFL_OK;
}

int ensure_dev_setup(ofl_app *app, int b) {
    if (app->dev_setup[b]) return OFL_OK;
    const Buffer &buf = app->ir.bufs[b];
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, buf.nbytes);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(OFL_E_NOMEM, "device set-up copy") : hip_fail(e, "hipMalloc");
    e = hipMemcpy(p, app->setup[b].data(), buf.nbytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p);
        return hip_fail(e, "set-up upload");
    }
    app->dev_setup[b] = p;
    return OFL_OK;
}

int check_bufs(const ofl_app *app, void *const *dev_bufs, int32_t n_bufs) {
    if (n_bufs != (int32_t)app->ir.bufs.size())
        return fail(OFL_E_BUF, "n_bufs " + std::to_string(n_bufs) + " != " + std::to_string(app->ir.bufs.size()));
    if (!dev_bufs) return fail(OFL_E_BUF, "null buffer table");
    for (int32_t b = 0; b < n_bufs; ++b) {
        if (!dev_bufs[b]) return fail(OFL_E_BUF, "null device pointer for buffer '" + app->ir.bufs[b].name + "'");
        if (reinterpret_cast<uintptr_t>(dev_bufs[b]) % 16)
            return fail(OFL_E_BUF, "device buffer '" + app->ir.bufs[b].name + "' not 16-byte aligned");
    }
    return OFL_OK;
}

// `fin`: the residual finish owed by the last sweep launched on `s`; a sweep
// sets it, an interior copy runs it as its extra block.  The callers run it
// by itself (k::residual_finish) before any other step.
hipError_t launch_nest(ofl_app *app, const Nest &n, void *const *dev, const int64_t *env, hipStream_t s,
                       k::ResidualFinish &fin, const k::ReduceScratch &rs) {
    const AppIR &ir = app->ir;
    auto F = [&](int i) { return static_cast<float *>(dev[n.b[i]]); };
    auto cnt = [&](int i) { return ir.bufs[n.b[i]].count; };
    hipError_t e = hipSuccess;
    switch (n.op) {
    case OP_INIT_UNIFORM:
        for (size_t t = 0; t < n.b.size() && e == hipSuccess; ++t)
            e = k::init_uniform(static_cast<float *>(dev[n.b[t]]), ir.bufs[n.b[t]].count,
                                uniform_stream_key(app->seed, n.streams[t]), s);
        return e;
    case OP_GEMM: {
        const auto &a = ir.bufs[n.b[0]].dims, &bb = ir.bufs[n.b[1]].dims;
        if (n.prec == PREC_F32) return k::gemm_f32(F(0), F(1), F(2), a[0], bb[1], a[1], s);
        return k::gemm_split(F(0), F(1), F(2), a[0], bb[1], a[1], gemm_variant(n), app->d_gemm_ws,
                             app->gemm_ws_bytes, s);
    }
    case OP_GEMM_BF16: {
        const auto &a = ir.bufs[n.b[0]].dims, &bb = ir.bufs[n.b[1]].dims;
        return k::gemm_bf16(static_cast<const uint16_t *>(dev[n.b[0]]), static_cast<const uint16_t *>(dev[n.b[1]]),
                            F(2), a[0], bb[1], a[1], app->d_gemm_ws, app->gemm_ws_bytes, s);
    }
    case OP_ADD_SCALED: return k::add_scaled(F(0), F(1), (float)n.alpha, cnt(0), s);
    case OP_AVG2: return k::avg2(F(0), F(1), F(2), cnt(0), s);
    case OP_SCALE: return k::scale(F(0), (float)n.alpha, cnt(0), s);
    case OP_COPY: return k::copy_bytes(dev[n.b[0]], dev[n.b[1]], ir.bufs[n.b[0]].nbytes, s);
    case OP_CAST_BF16:
        for (size_t t = 0; t + 1 < n.b.size() && e == hipSuccess; t += 2)
            e = k::cast_bf16(static_cast<uint16_t *>(dev[n.b[t]]), static_cast<const float *>(dev[n.b[t + 1]]),
                             ir.bufs[n.b[t]].count, s);
        return e;
    case OP_TRANSPOSE: {
        const auto &d = ir.bufs[n.b[0]].dims;
        return k::transpose(F(0), F(1), d[0], d[1], s);
    }
    case OP_SUMSQ: return k::sumsq(F(0), cnt(0), static_cast<double *>(dev[n.b[1]]), rs, s);
    case OP_STENCIL19: {
        const auto &d = ir.bufs[n.b[0]].dims;
        double *slot = static_cast<double *>(dev[n.b[2]]) + env[n.slot_repeat];
        return k::stencil19_sweep(F(0), F(1), d[0], d[1], d[2], slot, rs, s, fin);
    }
    case OP_COPY_INTERIOR: {
        const auto &d = ir.bufs[n.b[0]].dims;
        return k::copy_interior(F(0), F(1), d[0], d[1], d[2], s, &fin);
    }
    case OP_FFT_ROWS: {
        const auto &d = ir.bufs[n.b[0]].dims;
        if (n.real) return k::rfft_rows(F(0), d[0], d[1], app->d_twiddles, n.inverse, s);
        return k::fft_rows(F(0), d[0], d[1] / 2, app->d_twiddles, n.inverse, s);
    }
    default:
        return hipErrorInvalidValue;
    }
}

int32_t kernel_launch_count(const AppIR &ir, const Nest &n) {
    if (n.op == OP_INIT_UNIFORM) return (int32_t)n.b.size();
    if (n.op == OP_CAST_BF16) return (int32_t)(n.b.size() / 2);
    if (n.op == OP_SUMSQ) return 2;   // block partials + ordered finish
    if (n.op == OP_FFT_ROWS && n.real)  // the half-length complex transform (none for 2 values) + the (un)packing
        return ir.bufs[n.b[0]].dims[1] > 2 ? 2 : 1;
    if (n.op == OP_GEMM || n.op == OP_GEMM_BF16) {
        const auto &a = ir.bufs[n.b[0]].dims, &bb = ir.bufs[n.b[1]].dims;
        return k::gemm_launches(a[0], bb[1], a[1], gemm_variant(n));
    }
    return 1;   // a sweep's residual finish is counted where it is launched
}

// Whether `step` takes the residual finish still owed by the last sweep: an
// interior copy on the GPU runs it as an extra block of its launch; before
// any other step (and at the end of the run) it runs by itself.
bool takes_finish(const Step &step, const AppIR &ir) {
    return step.kind == ST_GPU && ir.nests[step.idx].op == OP_COPY_INTERIOR;
}

struct RunResult {
    int code = OFL_OK;
    ofl_run_stats st{};
};

// Components of the application: buffers joined by every nest that touches
// them (and every product nest that uses the shared operand workspace), so
// that nests of different components share no data and may run at once.
void ensure_components(ofl_app *app) {
    if (app->comps_done) return;
    const AppIR &ir = app->ir;
    const size_t nb = ir.bufs.size();
    std::vector<int> parent(nb + 1);   // + 1: the product workspace
    for (size_t i = 0; i <= nb; ++i) parent[i] = (int)i;
    auto find = [&](int x) {
        while (parent[x] != x) x = parent[x] = parent[parent[x]];
        return x;
    };
    auto unite = [&](int x, int y) { parent[find(x)] = find(y); };
    for (const Nest &n : ir.nests) {
        std::vector<int> bs = n.b;
        bs.insert(bs.end(), n.reads.begin(), n.reads.end());
        bs.insert(bs.end(), n.writes.begin(), n.writes.end());
        if ((n.op == OP_GEMM || n.op == OP_GEMM_BF16) && gemm_variant(n) != 0) bs.push_back((int)nb);
        for (size_t i = 1; i < bs.size(); ++i) unite(bs[0], bs[i]);
    }
    // number the components of buffers some nest touches, in program order
    std::map<int, int> id;
    app->nest_comp.assign(ir.nests.size(), 0);
    for (size_t k = 0; k < ir.nests.size(); ++k) {
        const Nest &n = ir.nests[k];
        const int b0 = !n.b.empty() ? n.b[0] : !n.writes.empty() ? n.writes[0] : !n.reads.empty() ? n.reads[0] : -1;
        if (b0 < 0) continue;
        const int root = find(b0);
        if (!id.count(root)) id[root] = (int)id.size();
        app->nest_comp[k] = id[root];
    }
    app->buf_comp.assign(nb, 0);
    for (size_t b = 0; b < nb; ++b) {
        const auto it = id.find(find((int)b));
        app->buf_comp[b] = it == id.end() ? 0 : it->second;
    }
    app->n_comps = std::max<int>(1, (int)id.size());
    app->comps_done = true;
}

int step_comp(const ofl_app *app, const Step &step) {
    return (step.kind == ST_H2D || step.kind == ST_D2H) ? app->buf_comp[step.idx] : app->nest_comp[step.idx];
}

// A stream (default priority) and reduction scratch for every component
// beyond the first.
int ensure_side_streams(ofl_app *app) {
    while ((int)app->side_streams.size() < app->n_comps - 1) {
        hipStream_t st = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
        app->side_streams.push_back(st);
        void *mem = nullptr;
        e = hipMalloc(&mem, (size_t)app->partial_cap * sizeof(double) + 256);
        if (e != hipSuccess) {
            app->side_partials.push_back(nullptr);
            return e == hipErrorOutOfMemory ? fail(OFL_E_NOMEM, "device scratch") : hip_fail(e, "hipMalloc");
        }
        app->side_partials.push_back(static_cast<double *>(mem));
    }
    for (double *p : app->side_partials)
        if (!p) return fail(OFL_E_NOMEM, "device scratch");
    return OFL_OK;
}

// What one component's part of a run did.
struct StepsOut {
    int code = OFL_OK;
    std::string msg;
    bool timed_out = false;
    uint64_t h2d = 0, d2h = 0;
    int32_t copies = 0, launches = 0, host_nests = 0;
    std::vector<char> host_written;
    std::vector<std::pair<int, int>> timed;   // (nest, event index)
};

hipError_t copy_box_d2h(const Buffer &buf, void *host, const void *dev, const Box &bx, hipStream_t s);

// The timed part of an eager run for the steps `idx` (indices into
// plan.steps, in program order) on `stream`: copies and kernels issued
// asynchronously, the stream synchronised before each host nest, the
// deadline checked before each step and inside host nests.  step_ev[i] is
// the event pair of step i (-1: not timed).
void run_steps(ofl_app *app, const Plan &plan, const std::vector<int> &idx, const std::vector<int> &step_ev,
               void *const *dev, hipStream_t stream, const k::ReduceScratch &rs, const Deadline &dl, StepsOut &out) {
    const AppIR &ir = app->ir;
    bool pending = false;
    hipError_t e = hipSuccess;
    k::ResidualFinish fin;
    auto failed = [&](int code) {
        out.code = code;
        out.msg = ofl_last_error();
    };
    for (int i : idx) {
        const Step &step = plan.steps[i];
        if (dl.expired()) {
            out.timed_out = true;
            break;
        }
        if (fin.n > 0 && !takes_finish(step, ir)) {
            e = k::residual_finish(fin, stream);
            if (e != hipSuccess) {
                failed(hip_fail(e, "launch of a residual finish"));
                break;
            }
            out.launches++;
        }
        switch (step.kind) {
        case ST_H2D:
            e = hipMemcpyAsync(dev[step.idx], app->host[step.idx], ir.bufs[step.idx].nbytes, hipMemcpyHostToDevice,
                               stream);
            if (e != hipSuccess) {
                failed(hip_fail(e, "H2D copy"));
                break;
            }
            out.h2d += ir.bufs[step.idx].nbytes;
            out.copies++;
            pending = true;
            break;
        case ST_D2H:
            e = step.box < 0 ? hipMemcpyAsync(app->host[step.idx], dev[step.idx], ir.bufs[step.idx].nbytes,
                                              hipMemcpyDeviceToHost, stream)
                             : copy_box_d2h(ir.bufs[step.idx], app->host[step.idx], dev[step.idx],
                                            plan.boxes[step.box], stream);
            if (e != hipSuccess) {
                failed(hip_fail(e, "D2H copy"));
                break;
            }
            out.d2h += step.box < 0 ? ir.bufs[step.idx].nbytes : box_bytes(ir.bufs[step.idx], plan.boxes[step.box]);
            out.copies++;
            out.host_written[step.idx] = 1;
            pending = true;
            break;
        case ST_GPU: {
            const Nest &n = ir.nests[step.idx];
            const int ev = step_ev[i];
            // a single-launch nest gets its events in the dispatch packet itself
            // (kernel-only interval); a multi-launch nest is bracketed by events
            const bool single = kernel_launch_count(ir, n) == 1;
            if (ev >= 0 && single) k::arm_launch_events(app->events[ev], app->events[ev + 1]);
            if (ev >= 0 && !single) (void)hipEventRecord(app->events[ev], stream);
            e = launch_nest(app, n, dev, plan.env.data() + step.env, stream, fin, rs);
            k::arm_launch_events(nullptr, nullptr);
            if (e != hipSuccess) {
                failed(hip_fail(e, (std::string("launch of nest ") + n.name).c_str()));
                break;
            }
            if (ev >= 0) {
                if (!single) (void)hipEventRecord(app->events[ev + 1], stream);
                out.timed.emplace_back(step.idx, ev);
            }
            out.launches += kernel_launch_count(ir, n);
            pending = true;
            break;
        }
        case ST_CPU: {
            if (pending) {
                e = hipStreamSynchronize(stream);
                if (e != hipSuccess) {
                    failed(hip_fail(e, "hipStreamSynchronize"));
                    break;
                }
                pending = false;
            }
            const Nest &n = ir.nests[step.idx];
            if (!run_host_nest(ir, n, app->host, plan.env.data() + step.env, app->seed, dl)) out.timed_out = true;
            for (int b : n.writes) out.host_written[b] = 1;
            out.host_nests++;
            break;
        }
        }
        if (out.code != OFL_OK || out.timed_out) break;
    }
    if (out.code == OFL_OK && !out.timed_out && fin.n > 0) {
        e = k::residual_finish(fin, stream);
        if (e != hipSuccess) failed(hip_fail(e, "launch of a residual finish"));
        else out.launches++;
    }
}

// Copy box `bx` of buffer b from the device to the same place in its host
// copy: the trailing dimensions the box covers whole and the first partial
// one form contiguous runs; the next dimension out becomes the rows of one
// 2-D copy, and any further dimensions are looped over.
hipError_t copy_box_d2h(const Buffer &buf, void *host, const void *dev, const Box &bx, hipStream_t s) {
    const int r = (int)buf.dims.size();
    const size_t elem = buf.nbytes / (size_t)std::max<int64_t>(1, buf.count);
    std::vector<size_t> stride(r, 1);   // elements per step of each dimension
    for (int d = r - 2; d >= 0; --d) stride[d] = stride[d + 1] * (size_t)buf.dims[d + 1];
    int t = r - 1;                      // innermost dimension not covered whole
    while (t > 0 && bx.lo[t] == 0 && bx.hi[t] == buf.dims[t]) --t;
    const size_t width = (size_t)(bx.hi[t] - bx.lo[t]) * stride[t] * elem;
    const int rd = t - 1;               // dimension of the rows (-1: none)
    const size_t rows = rd >= 0 ? (size_t)(bx.hi[rd] - bx.lo[rd]) : 1;
    const size_t pitch = rd >= 0 ? stride[rd] * elem : width;
    // loop over the dimensions outside the rows
    std::vector<int64_t> idx(r, 0);
    for (int d = 0; d < r; ++d) idx[d] = bx.lo[d];
    while (true) {
        size_t off = 0;
        for (int d = 0; d < r; ++d) off += (size_t)idx[d] * stride[d];
        off *= elem;
        hipError_t e = hipMemcpy2DAsync(static_cast<char *>(host) + off, pitch,
                                        static_cast<const char *>(dev) + off, pitch, width, rows,
                                        hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        int d = rd - 1;
        while (d >= 0 && ++idx[d] == bx.hi[d]) {
            idx[d] = bx.lo[d];
            --d;
        }
        if (d < 0) break;
    }
    return hipSuccess;
}

RunResult run_once(ofl_app *app, const std::vector<uint8_t> &placement, void *const *dev, hipStream_t stream,
                   int policy, int flags, double deadline_s) {
    RunResult rr;
    ofl_run_stats &st = rr.st;
    std::memset(&st, 0, sizeof(st));
    const AppIR &ir = app->ir;
    const size_t nb = ir.bufs.size();
    int rc = ensure_host(app);
    if (rc == OFL_OK) rc = ensure_device(app);
    if (rc != OFL_OK) {
        rr.code = rc;
        st.status = OFL_ST_FAILED;
        return rr;
    }
    Plan plan;
    build_plan(ir, placement, policy, flags, plan);
    app->ran = false;
    ensure_components(app);

    // ---- untimed reset: restore only set-up content that this run consumes
    for (size_t b = 0; b < nb; ++b)
        if (plan.host_init_used[b] && app->host_dirty[b]) restore_host(app, (int)b);
    if (flags & OFL_RUN_PRESTAGED) {
        for (size_t b = 0; b < nb; ++b) {
            if (!plan.dev_init_used[b]) continue;
            hipError_t e;
            if (!app->setup[b].empty()) {
                if ((rc = ensure_dev_setup(app, (int)b)) != OFL_OK) {
                    rr.code = rc;
                    st.status = OFL_ST_FAILED;
                    return rr;
                }
                e = k::copy_bytes(dev[b], app->dev_setup[b], ir.bufs[b].nbytes, stream);
            } else {
                e = k::fill_zero(dev[b], ir.bufs[b].nbytes, stream);
            }
            if (e != hipSuccess) {
                rr.code = hip_fail(e, "device set-up restore");
                st.status = OFL_ST_FAILED;
                return rr;
            }
        }
    }
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        rr.code = hip_fail(e, "hipStreamSynchronize");
        st.status = OFL_ST_FAILED;
        return rr;
    }

    // per-kernel timing events: two per GPU nest step
    if (app->timing) {
        const size_t need = 2 * (size_t)plan.launches;
        while (app->events.size() < need) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess) break;
            app->events.push_back(ev);
        }
    }

    // which GPU steps carry timing events (program order, as a sequential
    // run samples them) and their event pairs
    std::vector<int> step_ev(plan.steps.size(), -1);
    {
        size_t ev_next = 0;
        int32_t exec_count[OP_COUNT] = {};
        for (size_t i = 0; i < plan.steps.size(); ++i) {
            const Step &step = plan.steps[i];
            if (step.kind != ST_GPU) continue;
            if (timed_nest(app, ir.nests[step.idx], exec_count) && ev_next + 2 <= app->events.size()) {
                step_ev[i] = (int)ev_next;
                ev_next += 2;
            }
        }
    }
    // the steps of each component, in program order
    const bool concurrent = (flags & OFL_RUN_CONCURRENT) && app->n_comps > 1;
    if (concurrent && (rc = ensure_side_streams(app)) != OFL_OK) {
        rr.code = rc;
        st.status = OFL_ST_FAILED;
        return rr;
    }
    const int nc = concurrent ? app->n_comps : 1;
    std::vector<std::vector<int>> comp_steps(nc);
    for (size_t i = 0; i < plan.steps.size(); ++i)
        comp_steps[concurrent ? step_comp(app, plan.steps[i]) : 0].push_back((int)i);

    Deadline dl;
    const auto t0 = clk::now();
    if (deadline_s > 0) {
        dl.active = true;
        dl.until = t0 + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(deadline_s));
    }
    std::vector<StepsOut> outs(nc);
    for (auto &o : outs) o.host_written.assign(nb, 0);
    auto exec = [&](int c) {
        const hipStream_t cs = c == 0 ? stream : app->side_streams[c - 1];
        const k::ReduceScratch rs{c == 0 ? app->d_partials : app->side_partials[c - 1], app->partial_cap};
        run_steps(app, plan, comp_steps[c], step_ev, dev, cs, rs, dl, outs[c]);
    };
    if (nc == 1) {
        exec(0);
    } else {
        // every component from a host thread of its own (a host nest blocks
        // only its own component), on its own stream
        std::vector<std::thread> th;
        for (int c = 1; c < nc; ++c)
            if (!comp_steps[c].empty()) th.emplace_back(exec, c);
        exec(0);
        for (auto &t : th) t.join();
    }
    e = hipSuccess;
    for (int c = 0; c < nc; ++c) {
        const hipError_t ec = hipStreamSynchronize(c == 0 ? stream : app->side_streams[c - 1]);
        if (e == hipSuccess) e = ec;
    }
    const auto t1 = clk::now();
    st.t_total_s = std::chrono::duration<double>(t1 - t0).count();
    std::vector<char> host_written(nb, 0);
    bool timed_out = false;
    std::vector<std::pair<int, int>> timed;   // (nest, event index)
    for (const StepsOut &o : outs) {
        if (rr.code == OFL_OK && o.code != OFL_OK) rr.code = fail(o.code, o.msg);
        timed_out = timed_out || o.timed_out;
        st.bytes_h2d += o.h2d;
        st.bytes_d2h += o.d2h;
        st.n_copies += o.copies;
        st.n_launches += o.launches;
        st.n_host_nests += o.host_nests;
        for (size_t b = 0; b < nb; ++b) host_written[b] = host_written[b] || o.host_written[b];
        timed.insert(timed.end(), o.timed.begin(), o.timed.end());
    }
    for (size_t b = 0; b < nb; ++b)
        if (host_written[b]) app->host_dirty[b] = 1;
    if (rr.code == OFL_OK && e != hipSuccess) rr.code = hip_fail(e, "hipStreamSynchronize");
    if (rr.code != OFL_OK) {
        st.status = OFL_ST_FAILED;
        return rr;
    }
    if (timed_out || dl.expired()) {
        st.status = OFL_ST_TIMEOUT;
        rr.code = fail(OFL_E_TIMEOUT, "run exceeded its deadline");
        return rr;
    }
    for (const auto &te : timed) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, app->events[te.second], app->events[te.second + 1]) == hipSuccess) {
            auto &ks = app->kstats[op_name(ir.nests[te.first].op)];
            ks.first += 1;
            ks.second += ms;
        }
    }
    st.status = OFL_ST_OK;
    app->ran = true;
    app->host_valid = plan.host_valid;
    app->dev_valid = plan.dev_valid;
    app->host_written = host_written;
    app->last_dev.assign(dev, dev + nb);
    app->last_stream = stream;
    return rr;
}

// ------------------------------------------------------------ graph runs
void host_task_cb(void *p) {
    const HostTask *t = static_cast<const HostTask *>(p);
    // a gene already cut is a TIMEOUT whatever its later runs do: skip the
    // host work of its remaining runs (their results are not used)
    if (t->clock && t->clock->limit_s > 0.0 && t->clock->cut) return;
    Deadline dl;
    if (t->clock && t->clock->limit_s > 0.0) {
        dl.active = true;
        dl.until = t->clock->start + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                         std::chrono::duration<double>(t->clock->limit_s));
    }
    if (!run_host_nest(t->app->ir, t->app->ir.nests[t->nest], t->app->host, t->env.data(), t->app->seed, dl) &&
        t->clock)
        t->clock->cut = true;
}

void clock_start_cb(void *p) { static_cast<GraphClock *>(p)->start = std::chrono::steady_clock::now(); }

// Reset node of a run graph: restore the consumed host copies that differ
// from their set-up content (as an eager run does), then mark the ones the
// run after it writes -- the run follows this node on the stream, and the
// flags are read by the submitting thread only after it synchronised.
void host_restore_cb(void *p) {
    const HostRestore *r = static_cast<const HostRestore *>(p);
    for (int b : r->bufs) {
        if (!r->app->host_dirty[b]) continue;
        const Buffer &buf = r->app->ir.bufs[b];
        if (!r->app->setup[b].empty()) std::memcpy(r->app->host[b], r->app->setup[b].data(), buf.nbytes);
        else std::memset(r->app->host[b], 0, buf.nbytes);
        r->app->host_dirty[b] = 0;
    }
    for (int b : r->marks) r->app->host_dirty[b] = 1;
}

// Whether this execution of nest n is timed; exec_count[op] counts the
// executions of each kind in the run (or the captured graph) so far.
bool timed_nest(const ofl_app *app, const Nest &n, int32_t *exec_count) {
    const int32_t i = exec_count[n.op]++;
    if (!app->timing || !(app->timing_ops == 0 || ((app->timing_ops >> n.op) & 1u))) return false;
    return i % app->timing_stride == app->timing_phase;
}

// Append an event record node to the graph being captured on `cs` after the
// work captured so far, and make later captured work depend on it (a plain
// event record inside a capture only orders work and leaves no node).
hipError_t capture_event_node(hipStream_t cs, hipEvent_t ev) {
    hipStreamCaptureStatus status;
    unsigned long long id = 0;
    hipGraph_t g = nullptr;
    const hipGraphNode_t *deps = nullptr;
    size_t nd = 0;
    hipError_t e = hipStreamGetCaptureInfo_v2(cs, &status, &id, &g, &deps, &nd);
    if (e != hipSuccess) return e;
    if (status != hipStreamCaptureStatusActive || !g) return hipErrorInvalidValue;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddEventRecordNode(&node, g, deps, nd, ev);
    if (e != hipSuccess) return e;
    return hipStreamUpdateCaptureDependencies(cs, &node, 1, hipStreamSetCaptureDependencies);
}

int capture_begin(ofl_app *app) {
    if (!app->capture_stream) {
        hipError_t e = hipStreamCreateWithFlags(&app->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    }
    hipError_t e = hipStreamBeginCapture(app->capture_stream, hipStreamCaptureModeThreadLocal);
    return e == hipSuccess ? OFL_OK : hip_fail(e, "hipStreamBeginCapture");
}

int capture_end(ofl_app *app, hipGraphExec_t *exec, int status) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(app->capture_stream, &g);
    if (status != OFL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return status;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e == hipSuccess ? OFL_OK : hip_fail(e, "hipGraphInstantiate");
}

// Capture the reset graph (set-up content consumed by the run, restored on
// host and -- with PRESTAGED -- on device) and the run graph (the plan's
// copies and launches; CPU nests as host nodes).  No memset nodes: device
// zeroing uses the fill kernel.
int build_graphs(ofl_app *app, const std::vector<uint8_t> &placement, void *const *dev, int policy, int flags,
                 GraphEntry &ge) {
    const AppIR &ir = app->ir;
    const size_t nb = ir.bufs.size();
    build_plan(ir, placement, policy, flags, ge.plan);
    const Plan &plan = ge.plan;
    ge.host_written.assign(nb, 0);
    for (const Step &st : plan.steps) {
        if (st.kind == ST_D2H) ge.host_written[st.idx] = 1;
        if (st.kind == ST_CPU)
            for (int b : ir.nests[st.idx].writes) ge.host_written[b] = 1;
    }
    if (flags & OFL_RUN_PRESTAGED)
        for (size_t b = 0; b < nb; ++b)
            if (plan.dev_init_used[b] && !app->setup[b].empty()) {
                int rc = ensure_dev_setup(app, (int)b);
                if (rc != OFL_OK) return rc;
            }
    ge.restore.reset(new HostRestore());
    ge.restore->app = app;
    for (size_t b = 0; b < nb; ++b) {
        if (plan.host_init_used[b]) ge.restore->bufs.push_back((int)b);
        if (ge.host_written[b]) ge.restore->marks.push_back((int)b);
    }

    hipStream_t cs;
    int rc = capture_begin(app);
    if (rc != OFL_OK) return rc;
    cs = app->capture_stream;
    hipError_t e = hipLaunchHostFunc(cs, host_restore_cb, ge.restore.get());
    if (e == hipSuccess && (flags & OFL_RUN_PRESTAGED))
        for (size_t b = 0; b < nb && e == hipSuccess; ++b) {
            if (!plan.dev_init_used[b]) continue;
            e = !app->setup[b].empty() ? k::copy_bytes(dev[b], app->dev_setup[b], ir.bufs[b].nbytes, cs)
                                       : k::fill_zero(dev[b], ir.bufs[b].nbytes, cs);
        }
    rc = capture_end(app, &ge.reset, e == hipSuccess ? OFL_OK : hip_fail(e, "capture of the reset graph"));
    if (rc != OFL_OK) return rc;

    if ((rc = capture_begin(app)) != OFL_OK) return rc;
    e = hipSuccess;
    // a run with host nests starts with a host node that stamps its start
    // (the limit of a batched measurement applies to its host nests)
    ge.clock.reset(new GraphClock());
    const bool has_host = std::any_of(plan.steps.begin(), plan.steps.end(),
                                      [](const Step &st) { return st.kind == ST_CPU; });
    if (has_host) e = hipLaunchHostFunc(cs, clock_start_cb, ge.clock.get());
    k::ResidualFinish fin;
    int32_t exec_count[OP_COUNT] = {};
    for (const Step &st : plan.steps) {
        const Buffer *buf = (st.kind == ST_H2D || st.kind == ST_D2H) ? &ir.bufs[st.idx] : nullptr;
        if (fin.n > 0 && !takes_finish(st, ir)) {
            e = k::residual_finish(fin, cs);
            if (e != hipSuccess) break;
            ge.launches++;
        }
        switch (st.kind) {
        case ST_H2D: e = hipMemcpyAsync(dev[st.idx], app->host[st.idx], buf->nbytes, hipMemcpyHostToDevice, cs); break;
        case ST_D2H:
            e = st.box < 0 ? hipMemcpyAsync(app->host[st.idx], dev[st.idx], buf->nbytes, hipMemcpyDeviceToHost, cs)
                           : copy_box_d2h(*buf, app->host[st.idx], dev[st.idx], plan.boxes[st.box], cs);
            break;
        case ST_GPU: {
            hipEvent_t ev0 = nullptr, ev1 = nullptr;
            const bool tm = timed_nest(app, ir.nests[st.idx], exec_count);
            if (tm) {
                e = hipEventCreate(&ev0);
                if (e == hipSuccess) e = hipEventCreate(&ev1);
                if (e == hipSuccess) ge.timed.push_back({st.idx, {ev0, ev1}});
                else {
                    if (ev0) (void)hipEventDestroy(ev0);
                    break;
                }
                e = capture_event_node(cs, ev0);
            }
            if (e == hipSuccess)
                e = launch_nest(app, ir.nests[st.idx], dev, plan.env.data() + st.env, cs, fin,
                                k::ReduceScratch{app->d_partials, app->partial_cap});
            if (e == hipSuccess && tm) e = capture_event_node(cs, ev1);
            ge.launches += kernel_launch_count(ir, ir.nests[st.idx]);
            break;
        }
        case ST_CPU: {
            std::unique_ptr<HostTask> t(new HostTask());
            t->app = app;
            t->nest = st.idx;
            t->env.assign(plan.env.begin() + st.env, plan.env.begin() + st.env + ir.repeat_names.size());
            t->clock = ge.clock.get();
            e = hipLaunchHostFunc(cs, host_task_cb, t.get());
            ge.tasks.push_back(std::move(t));
            ge.host_nests++;
            break;
        }
        }
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess && fin.n > 0) {
        e = k::residual_finish(fin, cs);
        if (e == hipSuccess) ge.launches++;
    }
    return capture_end(app, &ge.run, e == hipSuccess ? OFL_OK : hip_fail(e, "capture of the run graph"));
}

int get_graph(ofl_app *app, const std::vector<uint8_t> &placement, void *const *dev, int policy, int flags,
              GraphEntry **out) {
    const size_t nb = app->ir.bufs.size();
    const int gflags = flags & ~(OFL_RUN_GRAPH | OFL_RUN_BATCHED | OFL_RUN_CONCURRENT);
    std::vector<uint64_t> key(placement.begin(), placement.end());
    key.push_back((uint64_t)policy);
    key.push_back((uint64_t)gflags);
    key.push_back(app->timing ? 1u : 0u);
    key.push_back(app->timing ? app->timing_ops : 0u);
    key.push_back(app->timing ? ((uint64_t)app->timing_stride << 32 | (uint32_t)app->timing_phase) : 0u);
    for (size_t b = 0; b < nb; ++b) key.push_back(reinterpret_cast<uint64_t>(dev[b]));
    auto it = app->graphs.find(key);
    if (it == app->graphs.end()) {
        std::unique_ptr<GraphEntry> ge(new GraphEntry());
        int rc = build_graphs(app, placement, dev, policy, gflags, *ge);
        if (rc != OFL_OK) return rc;
        it = app->graphs.emplace(key, std::move(ge)).first;
    }
    *out = it->second.get();
    return OFL_OK;
}

// Host-side state after a run of `ge` (its reset restored the host copies it
// lists, its run wrote the ones it marks).
void note_graph_run(ofl_app *app, const GraphEntry &ge, void *const *dev, hipStream_t stream) {
    const size_t nb = app->ir.bufs.size();
    for (int b : ge.restore->bufs) app->host_dirty[b] = 0;
    for (size_t b = 0; b < nb; ++b)
        if (ge.host_written[b]) app->host_dirty[b] = 1;
    app->ran = true;
    app->host_valid = ge.plan.host_valid;
    app->dev_valid = ge.plan.dev_valid;
    app->host_written = ge.host_written;
    app->last_dev.assign(dev, dev + nb);
    app->last_stream = stream;
}

RunResult run_graph(ofl_app *app, const std::vector<uint8_t> &placement, void *const *dev, hipStream_t stream,
                    int policy, int flags) {
    RunResult rr;
    ofl_run_stats &st = rr.st;
    std::memset(&st, 0, sizeof(st));
    st.status = OFL_ST_FAILED;
    const size_t nb = app->ir.bufs.size();
    int rc = ensure_host(app);
    if (rc == OFL_OK) rc = ensure_device(app);
    GraphEntry *gep = nullptr;
    if (rc == OFL_OK) rc = get_graph(app, placement, dev, policy, flags, &gep);
    if (rc != OFL_OK) {
        rr.code = rc;
        return rr;
    }
    GraphEntry &ge = *gep;
    app->ran = false;
    hipError_t e = hipGraphLaunch(ge.reset, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        rr.code = hip_fail(e, "reset graph");
        return rr;
    }
    for (int b : ge.restore->bufs) app->host_dirty[b] = 0;
    const auto t0 = clk::now();
    e = hipGraphLaunch(ge.run, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    const auto t1 = clk::now();
    for (size_t b = 0; b < nb; ++b)
        if (ge.host_written[b]) app->host_dirty[b] = 1;
    if (e != hipSuccess) {
        rr.code = hip_fail(e, "run graph");
        return rr;
    }
    st.t_total_s = std::chrono::duration<double>(t1 - t0).count();
    for (const auto &te : ge.timed) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, te.second.first, te.second.second) == hipSuccess) {
            auto &ks = app->kstats[op_name(app->ir.nests[te.first].op)];
            ks.first += 1;
            ks.second += ms;
        }
    }
    st.bytes_h2d = ge.plan.h2d;
    st.bytes_d2h = ge.plan.d2h;
    st.n_copies = ge.plan.copies;
    st.n_launches = ge.launches;
    st.n_host_nests = ge.host_nests;
    st.status = OFL_ST_OK;
    app->ran = true;
    app->host_valid = ge.plan.host_valid;
    app->dev_valid = ge.plan.dev_valid;
    app->host_written = ge.host_written;
    app->last_dev.assign(dev, dev + nb);
    app->last_stream = stream;
    return rr;
}

// One run, eager or as graphs.
RunResult run_any(ofl_app *app, const std::vector<uint8_t> &placement, void *const *dev, hipStream_t stream,
                  int policy, int flags, double deadline_s) {
    if (flags & OFL_RUN_GRAPH) return run_graph(app, placement, dev, stream, policy, flags);
    return run_once(app, placement, dev, stream, policy, flags, deadline_s);
}

// ------------------------------------------------------------ output check
// The outputs of a pattern against those of the all-zero gene (the program
// as written, every nest on the CPU): at up to kProbes fixed positions per
// output buffer, read from the host copy or, when the device holds the
// newest values, gathered there by one small kernel.
constexpr int kProbes = 4096;

void probe_positions(ofl_app *app) {
    if (!app->ref_pos.empty() || app->ref_bufs_done) return;
    const AppIR &ir = app->ir;
    for (size_t b = 0; b < ir.bufs.size(); ++b) {
        if (!ir.bufs[b].output) continue;
        const int64_t cnt = ir.bufs[b].count;
        std::vector<int64_t> pos;
        if (cnt <= kProbes) {
            for (int64_t e = 0; e < cnt; ++e) pos.push_back(e);
        } else {
            // a fixed pseudo-random sample (the SplitMix64 mix of buffer and
            // probe number), sorted
            for (int i = 0; i < kProbes; ++i) {
                uint64_t z = ((uint64_t)b << 32) + (uint64_t)i + 1;
                z *= 0x9E3779B97F4A7C15ull;
                z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
                z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
                z ^= z >> 31;
                pos.push_back((int64_t)(z % (uint64_t)cnt));
            }
            std::sort(pos.begin(), pos.end());
        }
        app->ref_bufs.push_back((int)b);
        app->ref_pos.push_back(pos);
    }
    app->ref_bufs_done = true;
}

double host_value(const Buffer &buf, const void *p, int64_t e) {
    if (buf.dtype == DT_F64) return static_cast<const double *>(p)[e];
    if (buf.dtype == DT_BF16) {
        const uint32_t u = (uint32_t) static_cast<const uint16_t *>(p)[e] << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return f;
    }
    return static_cast<const float *>(p)[e];
}

// Probe values of every output buffer after the last completed run.
int read_probes(ofl_app *app, std::vector<std::vector<double>> &vals) {
    probe_positions(app);
    vals.assign(app->ref_bufs.size(), {});
    for (size_t k = 0; k < app->ref_bufs.size(); ++k) {
        const int b = app->ref_bufs[k];
        const Buffer &buf = app->ir.bufs[b];
        const std::vector<int64_t> &pos = app->ref_pos[k];
        vals[k].resize(pos.size());
        if (app->host_valid[b]) {
            if (!app->host_written[b] && app->host_dirty[b]) restore_host(app, b);
            for (size_t i = 0; i < pos.size(); ++i) vals[k][i] = host_value(buf, app->host[b], pos[i]);
            continue;
        }
        hipError_t e = hipSuccess;
        if (!app->d_probe_idx) {
            e = hipMalloc(&app->d_probe_idx, kProbes * sizeof(int64_t));
            if (e == hipSuccess) e = hipMalloc(&app->d_probe_val, kProbes * sizeof(double));
            if (e != hipSuccess) return hip_fail(e, "probe buffers");
        }
        const hipStream_t s = app->last_stream;
        const int dt = buf.dtype == DT_F64 ? 1 : (buf.dtype == DT_BF16 ? 2 : 0);
        e = hipMemcpyAsync(app->d_probe_idx, pos.data(), pos.size() * sizeof(int64_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = k::gather_probes(app->last_dev[b], dt, app->d_probe_idx, (int)pos.size(), app->d_probe_val, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(vals[k].data(), app->d_probe_val, pos.size() * sizeof(double), hipMemcpyDeviceToHost,
                               s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "output probes");
    }
    return OFL_OK;
}

// The reference probes: one run of the all-zero gene, untimed, no deadline;
// kept until the inputs change.
int ensure_reference(ofl_app *app, void *const *dev, hipStream_t s, int policy) {
    if (app->ref_valid) return OFL_OK;
    const std::vector<uint8_t> zero(app->ir.nests.size(), 0);
    RunResult rr = run_once(app, zero, dev, s, policy, 0, 0.0);
    if (rr.code != OFL_OK) return rr.code;
    const int rc = read_probes(app, app->ref_val);
    if (rc != OFL_OK) return rc;
    app->ref_valid = true;
    return OFL_OK;
}

// Whether the last run's outputs agree with the reference within rtol of
// each buffer's largest reference probe (NaN only where the reference has
// NaN).
int outputs_agree(ofl_app *app, double rtol, bool *agree) {
    std::vector<std::vector<double>> got;
    const int rc = read_probes(app, got);
    if (rc != OFL_OK) return rc;
    *agree = true;
    for (size_t k = 0; k < got.size() && *agree; ++k) {
        const std::vector<double> &ref = app->ref_val[k];
        double scale = 0.0;
        for (double r : ref)
            if (std::isfinite(r)) scale = std::max(scale, std::fabs(r));
        for (size_t i = 0; i < ref.size(); ++i) {
            const double x = got[k][i], r = ref[i];
            if (std::isnan(r) || std::isnan(x)) {
                if (!(std::isnan(r) && std::isnan(x))) *agree = false;
            } else if (std::isinf(r) || std::isinf(x)) {
                if (x != r) *agree = false;
            } else if (std::fabs(x - r) > rtol * scale) {
                *agree = false;
            }
            if (!*agree) {
                (void)fail(OFL_E_MISMATCH, "output '" + app->ir.bufs[app->ref_bufs[k]].name + "' differs from the all-CPU run at "
                               "element " + std::to_string(app->ref_pos[k][i]));
                break;
            }
        }
    }
    return OFL_OK;
}

double median_of(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    const size_t n = v.size();
    return (n % 2) ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

// warmup + reps runs of one gene; median time
Measurement measure(ofl_app *app, const std::vector<uint8_t> &placement, void *const *dev, hipStream_t s,
                    int reps, int warmup, int policy, int flags, double deadline_s, int *hard_error,
                    double verify_rtol = 0.0) {
    Measurement m;
    std::vector<double> ts;
    if (verify_rtol > 0) {
        const int rc = ensure_reference(app, dev, s, policy);
        if (rc != OFL_OK) {
            *hard_error = rc;
            return Measurement{0.0, OFL_ST_FAILED};
        }
    }
    for (int r = 0; r < warmup + reps; ++r) {
        RunResult rr = run_any(app, placement, dev, s, policy, flags, deadline_s);
        if (r == 0 && verify_rtol > 0 && rr.code == OFL_OK) {
            bool agree = false;
            const int rc = outputs_agree(app, verify_rtol, &agree);
            if (rc != OFL_OK) {
                *hard_error = rc;
                return Measurement{0.0, OFL_ST_FAILED};
            }
            if (!agree) return Measurement{0.0, OFL_ST_MISMATCH};
        }
        if (rr.code == OFL_E_TIMEOUT) {
            m.status = OFL_ST_TIMEOUT;
            m.t = rr.st.t_total_s;
            return m;
        }
        if (rr.code != OFL_OK) {
            m.status = OFL_ST_FAILED;
            m.t = rr.st.t_total_s;
            if (rr.code == OFL_E_HIP || rr.code == OFL_E_NOMEM || rr.code == OFL_E_STATE) *hard_error = rr.code;
            return m;
        }
        if (r >= warmup) ts.push_back(rr.st.t_total_s);
    }
    m.status = OFL_ST_OK;
    m.t = median_of(ts);
    return m;
}

// All genes together, one submission per round of runs (the warm-up
// rounds, then the timed ones): each gene's reset graph and run graph back
// to back on the stream, an event pair around every run graph, one
// synchronisation per round; per gene the median of its timed intervals.
// limit > 0: a run over it (or a host nest cut at it) makes the gene
// OFL_ST_TIMEOUT at the limit and drops it from the later rounds.
int measure_batched_all(ofl_app *app, const std::vector<std::vector<uint8_t>> &placements, void *const *dev,
                        hipStream_t s, int reps, int warmup, int policy, int flags, double limit,
                        std::vector<Measurement> &out) {
    const size_t n = placements.size();
    out.assign(n, Measurement{0.0, OFL_ST_FAILED});
    if (n == 0) return OFL_OK;
    int rc = ensure_host(app);
    if (rc == OFL_OK) rc = ensure_device(app);
    if (rc != OFL_OK) return rc;
    std::vector<GraphEntry *> ge(n);
    for (size_t g = 0; g < n; ++g)
        if ((rc = get_graph(app, placements[g], dev, policy, flags, &ge[g])) != OFL_OK) return rc;
    while (app->chain_events.size() < 2 * n) {
        hipEvent_t e = nullptr;
        hipError_t he = hipEventCreate(&e);
        if (he != hipSuccess) return hip_fail(he, "hipEventCreate");
        app->chain_events.push_back(e);
    }
    app->ran = false;
    // the limit also cuts host nests short (counted from each run's start)
    for (size_t g = 0; g < n; ++g) {
        ge[g]->clock->limit_s = limit > 0 ? limit : 0.0;
        ge[g]->clock->cut = false;
    }
    std::vector<char> dead(n, 0), ran(n, 0), eager_warm(n, 0);
    // A cut inside a captured run stops its host nests, but every later copy
    // and kernel of the run still executes.  A host nest inside a repeated
    // block (an iterated sweep left on the CPU) interleaves host work with
    // copies in every repetition, so after a cut such a run still moves the
    // buffers across PCIe once per repetition.  With a limit, these genes
    // take their warm-up runs eagerly, where the limit ends the whole run, and
    // join the submitted rounds only if they stay within it.
    if (limit > 0 && warmup > 0) {
        const size_t nn = app->ir.nests.size();
        for (size_t g = 0; g < n; ++g) {
            std::vector<int> cpu_runs(nn, 0);
            for (const Step &st : ge[g]->plan.steps)
                if (st.kind == ST_CPU && ++cpu_runs[st.idx] > 1) eager_warm[g] = 1;
        }
        for (size_t g = 0; g < n; ++g) {
            if (!eager_warm[g]) continue;
            for (int r = 0; r < warmup && !dead[g]; ++r) {
                RunResult rr = run_once(app, placements[g], dev, s, policy, flags & ~(OFL_RUN_GRAPH | OFL_RUN_BATCHED),
                                        limit);
                if (rr.code == OFL_E_TIMEOUT || (rr.code == OFL_OK && rr.st.t_total_s > limit)) dead[g] = 1;
                else if (rr.code != OFL_OK) return rr.code;
            }
        }
    }
    // one submission per round (the warm-up runs, then each timed run): the
    // reset and run graphs of every gene still measured, back to back, an
    // event pair around each run graph.  A gene whose run went over the
    // limit, or whose host nests were cut, is a TIMEOUT and leaves the later
    // rounds (as an eager measurement stops at its first run over the limit)
    std::vector<std::vector<double>> ts(n);
    std::vector<size_t> last_round;
    hipError_t e = hipSuccess;
    for (int r = 0; r < warmup + reps && e == hipSuccess; ++r) {
        std::vector<size_t> round;
        for (size_t g = 0; g < n; ++g)
            if (!dead[g] && !(r < warmup && eager_warm[g])) round.push_back(g);
        if (round.empty()) {
            if (r < warmup) continue;   // every gene left took its warm-up eagerly
            break;
        }
        for (size_t k = 0; k < round.size() && e == hipSuccess; ++k) {
            const size_t g = round[k];
            e = hipGraphLaunch(ge[g]->reset, s);
            if (e == hipSuccess) e = hipEventRecord(app->chain_events[2 * k], s);
            if (e == hipSuccess) e = hipGraphLaunch(ge[g]->run, s);
            if (e == hipSuccess) e = hipEventRecord(app->chain_events[2 * k + 1], s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) break;
        for (size_t k = 0; k < round.size(); ++k) {
            const size_t g = round[k];
            ran[g] = 1;
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, app->chain_events[2 * k], app->chain_events[2 * k + 1]);
            if (e != hipSuccess) break;
            const double t = 1e-3 * ms;
            if (r >= warmup) ts[g].push_back(t);
            if (limit > 0 && (t > limit || ge[g]->clock->cut)) dead[g] = 1;
        }
        last_round = round;
    }
    for (size_t g = 0; g < n; ++g) ge[g]->clock->limit_s = 0.0;   // later graph runs are not limited
    if (e != hipSuccess) return hip_fail(e, "batched evaluation");
    for (size_t g = 0; g < n; ++g) {
        if (dead[g]) {
            out[g] = Measurement{limit, OFL_ST_TIMEOUT};
            continue;
        }
        out[g] = Measurement{median_of(ts[g]), OFL_ST_OK};
    }
    // host / device state: every gene that ran, those of the last round last
    // and in order, so the state is that of the last run
    for (size_t g = 0; g < n; ++g)
        if (ran[g] && std::find(last_round.begin(), last_round.end(), g) == last_round.end())
            note_graph_run(app, *ge[g], dev, s);
    for (size_t g : last_round) note_graph_run(app, *ge[g], dev, s);
    return OFL_OK;
}

// Runs of this length (seconds) or longer gain nothing from a batched GA
// generation: at the large application (130 ms to 0.5 s per run) the search
// took 195 s batched against 177 s gene by gene in one session, the difference
// being the capture and instantiation of every gene's graphs.  A batched GA
// measures its generations gene by gene until the best run so far is shorter
// than this; OFL_BATCH_EAGER_S overrides it (0: always gene by gene).
double batch_eager_threshold() {
    if (const char *e = std::getenv("OFL_BATCH_EAGER_S")) {
        char *end = nullptr;
        const double v = std::strtod(e, &end);
        if (end != e && v >= 0) return v;
    }
    return 0.02;
}

// Batched measurement with the optional output check: each gene runs once
// eagerly first (with the limit) and is checked; genes that fail the check
// or time out there are left out of the submission.
int measure_batched(ofl_app *app, const std::vector<std::vector<uint8_t>> &placements, void *const *dev,
                    hipStream_t s, int reps, int warmup, int policy, int flags, double limit,
                    std::vector<Measurement> &out, double verify_rtol = 0.0) {
    if (!(verify_rtol > 0)) return measure_batched_all(app, placements, dev, s, reps, warmup, policy, flags, limit, out);
    const size_t n = placements.size();
    out.assign(n, Measurement{0.0, OFL_ST_FAILED});
    int rc = ensure_reference(app, dev, s, policy);
    if (rc != OFL_OK) return rc;
    std::vector<size_t> keep;
    std::vector<std::vector<uint8_t>> kept;
    const int eager = flags & ~(OFL_RUN_GRAPH | OFL_RUN_BATCHED);
    for (size_t g = 0; g < n; ++g) {
        RunResult rr = run_once(app, placements[g], dev, s, policy, eager, limit > 0 ? limit : 0.0);
        if (rr.code == OFL_E_TIMEOUT) {
            out[g] = Measurement{limit > 0 ? limit : rr.st.t_total_s, OFL_ST_TIMEOUT};
            continue;
        }
        if (rr.code != OFL_OK) {
            if (rr.code == OFL_E_HIP || rr.code == OFL_E_NOMEM || rr.code == OFL_E_STATE) return rr.code;
            continue;
        }
        bool agree = false;
        if ((rc = outputs_agree(app, verify_rtol, &agree)) != OFL_OK) return rc;
        if (!agree) {
            out[g] = Measurement{0.0, OFL_ST_MISMATCH};
            continue;
        }
        keep.push_back(g);
        kept.push_back(placements[g]);
    }
    std::vector<Measurement> got;
    rc = measure_batched_all(app, kept, dev, s, reps, warmup, policy, flags, limit, got);
    if (rc != OFL_OK) return rc;
    for (size_t i = 0; i < keep.size(); ++i) out[keep[i]] = got[i];
    return OFL_OK;
}

void copy_name(const std::string &s, char *out, int32_t cap) {
    if (!out || cap <= 0) return;
    const size_t n = std::min((size_t)cap - 1, s.size());
    std::memcpy(out, s.data(), n);
    out[n] = 0;
}

void fill_ga_result(const GaTrace &tr, int a, int M, ofl_ga_result *res) {
    if (res->best_gene && !tr.best_gene.empty()) std::memcpy(res->best_gene, tr.best_gene.data(), a);
    for (size_t g = 0; g < tr.pops.size(); ++g)
        for (int m = 0; m < M; ++m) {
            const size_t o = g * M + m;
            if (res->pop_trace) std::memcpy(res->pop_trace + o * a, tr.pops[g][m].data(), a);
            if (res->time_trace) res->time_trace[o] = tr.meas[g][m].t;
            if (res->status_trace) res->status_trace[o] = tr.meas[g][m].status;
        }
    res->best_time = tr.best_t;
    res->best_fitness = tr.best_f;
    res->t_all0 = tr.t_all0;
    res->n_measured = tr.n_measured;
    res->n_generations = (int32_t)tr.pops.size();
    res->search_wall_s = tr.wall_s;
    res->time_to_best_s = tr.time_to_best_s;
}

int check_ga_params(const ofl_ga_params *p, int a) {
    if (!p) return fail(OFL_E_ARG, "null GA parameters");
    if (p->M < 1 || p->T < 1 || a < 1) return fail(OFL_E_ARG, "need M >= 1, T >= 1 and a non-empty gene");
    if (!(p->Pc >= 0 && p->Pc <= 1 && p->Pm >= 0 && p->Pm <= 1 && p->p > 0))
        return fail(OFL_E_ARG, "rates must lie in [0,1] and the exponent be > 0");
    return OFL_OK;
}

GaConfig ga_config(const ofl_ga_params *p) {
    GaConfig c;
    c.M = p->M;
    c.T = p->T;
    c.Pc = p->Pc;
    c.Pm = p->Pm;
    c.p = p->p;
    c.seed = p->seed;
    c.deadline_factor = p->deadline_factor;
    c.timeout_s = p->timeout_s;
    return c;
}

// Identity of a search for its log: every parameter the trajectory depends
// on (not T: a longer search continues a shorter one) and what is searched.
std::string search_identity(const ofl_ga_params *p, int a, const std::string &what) {
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "a=%d;M=%d;Pc=%.17g;Pm=%.17g;p=%.17g;seed=%llu;deadline_factor=%.17g;timeout=%.17g;"
                  "reps=%d;warmup=%d;policy=%d;flags=%d;",
                  a, p->M, p->Pc, p->Pm, p->p, (unsigned long long)p->seed, p->deadline_factor, p->timeout_s,
                  p->reps, p->warmup, p->policy, p->flags & ~OFL_RUN_PROGRESS);
    return std::string(buf) + what;
}

// run_ga with the measurement log of params->cache_path (if set): logged
// measurements are replayed in order, fresh ones appended.  A log that
// disagrees with this search (another gene where its next measurement is,
// another random state at a generation's end) stops the measuring and
// returns OFL_E_STATE.
int run_logged_ga(int a, const ofl_ga_params *params, const std::string &what, const Evaluator &ev,
                  const BatchEvaluator &bev, bool print, GaTrace &tr, const BatchGate *gate = nullptr) {
    GaLog log;
    if (params->cache_path && params->cache_path[0]) {
        std::string err;
        const int rc = log.open(params->cache_path, search_identity(params, a, what), err);
        if (rc != OFL_OK) return fail(rc, err);
    }
    bool bad = false;
    Evaluator lev = [&](const std::vector<uint8_t> &g, double limit) -> Measurement {
        if (bad) return Measurement{0.0, OFL_ST_FAILED};
        Measurement m;
        const int r = log.take(g, m);
        if (r == 1) return m;
        if (r < 0) {
            bad = true;
            return Measurement{0.0, OFL_ST_FAILED};
        }
        m = ev(g, limit);
        log.add(g, m);
        return m;
    };
    BatchEvaluator lbev = [&](const std::vector<std::vector<uint8_t>> &gs, double limit) {
        std::vector<Measurement> out(gs.size(), Measurement{0.0, OFL_ST_FAILED});
        if (bad) return out;
        size_t i = 0;
        for (; i < gs.size(); ++i) {
            const int r = log.take(gs[i], out[i]);
            if (r == 0) break;
            if (r < 0) {
                bad = true;
                return out;
            }
        }
        if (i < gs.size()) {
            const std::vector<std::vector<uint8_t>> rest(gs.begin() + i, gs.end());
            const std::vector<Measurement> got = bev(rest, limit);
            for (size_t k = 0; k < rest.size(); ++k) {
                out[i + k] = k < got.size() ? got[k] : Measurement{0.0, OFL_ST_FAILED};
                log.add(rest[k], out[i + k]);
            }
        }
        return out;
    };
    GaProgress prog = [&](int gen, const GaTrace &t, double wall) {
        if (!log.generation(gen, t.rng_state)) bad = true;
        if (print) {
            std::fprintf(stderr, "ga generation %d/%d: best %.6f s, %d genes measured (%d from the log), %.1f s\n",
                         gen, params->T, t.best_t, t.n_measured, log.replayed(), wall);
            std::fflush(stderr);
        }
    };
    run_ga(a, ga_config(params), lev, tr, (params->flags & OFL_RUN_BATCHED) ? &lbev : nullptr, &prog, gate);
    if (bad) return fail(OFL_E_STATE, std::string("GA log ") + params->cache_path +
                                          " disagrees with this search (another gene or random state)");
    return OFL_OK;
}

int load_common(const std::string &text, uint64_t seed, ofl_app **out) {
    if (!out) return fail(OFL_E_ARG, "null output pointer");
    *out = nullptr;
    ofl_app *app = new (std::nothrow) ofl_app();
    if (!app) return fail(OFL_E_NOMEM, "out of memory");
    std::string err;
    int rc = parse_app(text, app->ir, err);
    if (rc != OFL_OK) {
        delete app;
        return fail(rc, err);
    }
    if (!app->ir.host_object.empty()) {
        // the host object holds one entry point per host_code nest
        app->host_lib = dlopen(app->ir.host_object.c_str(), RTLD_NOW | RTLD_LOCAL);
        if (!app->host_lib) {
            const char *why = dlerror();
            delete app;
            return fail(OFL_E_IO, std::string("cannot load host object: ") + (why ? why : "?"));
        }
        for (auto &n : app->ir.nests) {
            if (n.op != OP_HOST_CODE) continue;
            void *sym = dlsym(app->host_lib, n.symbol.c_str());
            if (!sym) {
                const std::string name = n.name, symbol = n.symbol;
                delete app;
                return fail(OFL_E_IR, "nest " + name + ": host object has no entry point " + symbol);
            }
            n.host_fn = reinterpret_cast<void (*)(void *const *, const int64_t *)>(sym);
        }
    }
    app->seed = seed;
    *out = app;
    return OFL_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int ofl_app_load_json(const char *json_text, uint64_t seed, ofl_app **out) {
    if (!json_text) return fail(OFL_E_ARG, "null JSON text");
    return load_common(json_text, seed, out);
}

int ofl_app_load(const char *path, uint64_t seed, ofl_app **out) {
    if (!path) return fail(OFL_E_ARG, "null path");
    std::ifstream f(path);
    if (!f) return fail(OFL_E_IO, std::string("cannot open ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    return load_common(ss.str(), seed, out);
}

void ofl_app_free(ofl_app *app) { delete app; }

int ofl_app_info(const ofl_app *app, int32_t *n_nests, int32_t *gene_len, int32_t *n_bufs) {
    if (!app) return fail(OFL_E_ARG, "null app");
    if (n_nests) *n_nests = (int32_t)app->ir.nests.size();
    if (gene_len) *gene_len = app->ir.gene_len;
    if (n_bufs) *n_bufs = (int32_t)app->ir.bufs.size();
    return OFL_OK;
}

int ofl_nest_info(const ofl_app *app, int32_t nest, int32_t *verdict, int32_t *reason, int32_t *gene_pos) {
    if (!app) return fail(OFL_E_ARG, "null app");
    if (nest < 0 || nest >= (int32_t)app->ir.nests.size()) return fail(OFL_E_RANGE, "nest index out of range");
    const Nest &n = app->ir.nests[nest];
    if (verdict) *verdict = n.verdict;
    if (reason) *reason = n.reason;
    if (gene_pos) *gene_pos = n.gene_pos;
    return OFL_OK;
}

int ofl_nest_name(const ofl_app *app, int32_t nest, char *out, int32_t cap) {
    if (!app || !out || cap <= 0) return fail(OFL_E_ARG, "bad arguments");
    if (nest < 0 || nest >= (int32_t)app->ir.nests.size()) return fail(OFL_E_RANGE, "nest index out of range");
    copy_name(app->ir.nests[nest].name, out, cap);
    return OFL_OK;
}

int ofl_buf_info(const ofl_app *app, int32_t buf, uint64_t *bytes, int32_t *dtype, int32_t *is_output) {
    if (!app) return fail(OFL_E_ARG, "null app");
    if (buf < 0 || buf >= (int32_t)app->ir.bufs.size()) return fail(OFL_E_RANGE, "buffer index out of range");
    const Buffer &b = app->ir.bufs[buf];
    if (bytes) *bytes = b.nbytes;
    if (dtype) *dtype = b.dtype;
    if (is_output) *is_output = b.output ? 1 : 0;
    return OFL_OK;
}

int ofl_buf_name(const ofl_app *app, int32_t buf, char *out, int32_t cap) {
    if (!app || !out || cap <= 0) return fail(OFL_E_ARG, "bad arguments");
    if (buf < 0 || buf >= (int32_t)app->ir.bufs.size()) return fail(OFL_E_RANGE, "buffer index out of range");
    copy_name(app->ir.bufs[buf].name, out, cap);
    return OFL_OK;
}

int ofl_buf_dims(const ofl_app *app, int32_t buf, int64_t *dims, int32_t cap, int32_t *ndim) {
    if (!app || !ndim || (cap > 0 && !dims)) return fail(OFL_E_ARG, "null argument");
    if (buf < 0 || buf >= (int32_t)app->ir.bufs.size()) return fail(OFL_E_RANGE, "buffer index out of range");
    const auto &d = app->ir.bufs[buf].dims;
    *ndim = (int32_t)d.size();
    for (int32_t i = 0; i < cap && i < (int32_t)d.size(); ++i) dims[i] = d[i];
    return OFL_OK;
}

int ofl_set_input(ofl_app *app, int32_t buf, const void *src, uint64_t bytes) {
    if (!app || !src) return fail(OFL_E_ARG, "null argument");
    if (buf < 0 || buf >= (int32_t)app->ir.bufs.size()) return fail(OFL_E_RANGE, "buffer index out of range");
    const Buffer &b = app->ir.bufs[buf];
    if (bytes != b.nbytes) return fail(OFL_E_ARG, "input size differs from the buffer size");
    if (app->setup.size() != app->ir.bufs.size()) app->setup.resize(app->ir.bufs.size());
    try {
        app->setup[buf].assign(static_cast<const unsigned char *>(src), static_cast<const unsigned char *>(src) + bytes);
    } catch (const std::bad_alloc &) {
        return fail(OFL_E_NOMEM, "out of memory");
    }
    if (!app->host.empty()) app->host_dirty[buf] = 1;   // host copy must be refreshed
    app->graphs.clear();   // captured reset graphs refer to the old device copy
    app->ref_valid = false;   // the reference outputs belong to the old inputs
    if (!app->dev_setup.empty() && app->dev_setup[buf]) {
        (void)hipFree(app->dev_setup[buf]);
        app->dev_setup[buf] = nullptr;
    }
    return OFL_OK;
}

int ofl_mask_to_gene(const ofl_app *app, const uint8_t *mask, int32_t n_nests, uint8_t *gene_out) {
    if (!app || !mask || (!gene_out && app->ir.gene_len > 0)) return fail(OFL_E_ARG, "null argument");
    if (n_nests != (int32_t)app->ir.nests.size()) return fail(OFL_E_ARG, "mask length differs from the nest count");
    for (int32_t n = 0; n < n_nests; ++n) {
        if (mask[n] > 1) return fail(OFL_E_GENE_BIT, "mask byte is not 0/1");
        const Nest &ns = app->ir.nests[n];
        if (ns.gene_pos < 0) {
            if (mask[n]) return fail(OFL_E_NOT_PARALLEL, "nest " + ns.name + " was rejected and cannot run on the GPU");
        } else {
            gene_out[ns.gene_pos] = mask[n];
        }
    }
    return OFL_OK;
}

int ofl_plan_transfers(const ofl_app *app, const uint8_t *gene, int32_t gene_len, int32_t policy, int32_t flags,
                       uint64_t *bytes_h2d, uint64_t *bytes_d2h, int32_t *n_copies) {
    if (!app) return fail(OFL_E_ARG, "null app");
    if (policy < OFL_POLICY_RESIDENT || policy > OFL_POLICY_SECTIONS) return fail(OFL_E_ARG, "bad policy");
    if (flags & ~(OFL_RUN_PRESTAGED | OFL_RUN_KEEP_OUTPUTS | OFL_RUN_GRAPH | OFL_RUN_CONCURRENT))
        return fail(OFL_E_ARG, "bad flags");
    std::vector<uint8_t> placement;
    int rc = check_gene(app, gene, gene_len, placement);
    if (rc != OFL_OK) return rc;
    Plan plan;
    build_plan(app->ir, placement, policy, flags, plan);
    if (bytes_h2d) *bytes_h2d = plan.h2d;
    if (bytes_d2h) *bytes_d2h = plan.d2h;
    if (n_copies) *n_copies = plan.copies;
    return OFL_OK;
}

int ofl_run_pattern(ofl_app *app, const uint8_t *gene, int32_t gene_len, void *const *dev_bufs, int32_t n_bufs,
                    void *stream, const ofl_run_opts *opts, ofl_run_stats *stats) {
    if (!app) return fail(OFL_E_ARG, "null app");
    for (const auto &n : app->ir.nests)
        if (n.op == OP_NONE) return fail(OFL_E_IR, "application has analysis-only nests and cannot run");
    std::vector<uint8_t> placement;
    int rc = check_gene(app, gene, gene_len, placement);
    if (rc != OFL_OK) return rc;
    if ((rc = check_bufs(app, dev_bufs, n_bufs)) != OFL_OK) return rc;
    const int policy = opts ? opts->policy : OFL_POLICY_RESIDENT;
    const int flags = opts ? opts->flags : 0;
    const double deadline = opts ? opts->deadline_s : 0.0;
    if (policy < OFL_POLICY_RESIDENT || policy > OFL_POLICY_SECTIONS) return fail(OFL_E_ARG, "bad policy");
    if (flags & ~(OFL_RUN_PRESTAGED | OFL_RUN_KEEP_OUTPUTS | OFL_RUN_GRAPH | OFL_RUN_CONCURRENT))
        return fail(OFL_E_ARG, "bad flags");
    const double rtol = opts ? opts->verify_rtol : 0.0;
    if (rtol > 0 && (rc = ensure_reference(app, dev_bufs, static_cast<hipStream_t>(stream), policy)) != OFL_OK)
        return rc;
    RunResult rr = run_any(app, placement, dev_bufs, static_cast<hipStream_t>(stream), policy, flags, deadline);
    if (rr.code == OFL_OK && rtol > 0) {
        bool agree = false;
        if ((rc = outputs_agree(app, rtol, &agree)) != OFL_OK) return rc;
        if (!agree) {
            rr.st.status = OFL_ST_MISMATCH;
            rr.code = OFL_E_MISMATCH;   // the message names the buffer and element
        }
    }
    if (stats) *stats = rr.st;
    return rr.code;
}

int ofl_eval_population(ofl_app *app, const uint8_t *genes, int32_t pop, int32_t gene_len, void *const *dev_bufs,
                        int32_t n_bufs, void *stream, const ofl_eval_opts *opts, double *time_out,
                        int32_t *status_out) {
    if (!app || !genes || !time_out || !status_out || !opts || pop < 0) return fail(OFL_E_ARG, "null argument");
    if (opts->reps < 1 || opts->warmup < 0) return fail(OFL_E_ARG, "need reps >= 1 and warmup >= 0");
    int rc = check_bufs(app, dev_bufs, n_bufs);
    if (rc != OFL_OK) return rc;
    if (opts->flags & ~(OFL_RUN_PRESTAGED | OFL_RUN_KEEP_OUTPUTS | OFL_RUN_GRAPH | OFL_RUN_BATCHED | OFL_RUN_CONCURRENT))
        return fail(OFL_E_ARG, "bad flags");
    std::map<std::vector<uint8_t>, Measurement> seen;
    std::vector<uint8_t> placement;
    for (int32_t m = 0; m < pop; ++m) {
        rc = check_gene(app, genes + (size_t)m * gene_len, gene_len, placement);
        if (rc != OFL_OK) return rc;
    }
    if (opts->flags & OFL_RUN_BATCHED) {
        std::vector<std::vector<uint8_t>> uniq, places;
        for (int32_t m = 0; m < pop; ++m) {
            std::vector<uint8_t> g(genes + (size_t)m * gene_len, genes + (size_t)(m + 1) * gene_len);
            if (std::find(uniq.begin(), uniq.end(), g) != uniq.end()) continue;
            check_gene(app, g.data(), gene_len, placement);
            uniq.push_back(g);
            places.push_back(placement);
        }
        std::vector<Measurement> got;
        rc = measure_batched(app, places, dev_bufs, static_cast<hipStream_t>(stream), opts->reps, opts->warmup,
                             opts->policy, opts->flags, opts->deadline_s, got, opts->verify_rtol);
        if (rc != OFL_OK) return rc;
        for (int32_t m = 0; m < pop; ++m) {
            std::vector<uint8_t> g(genes + (size_t)m * gene_len, genes + (size_t)(m + 1) * gene_len);
            const size_t k = std::find(uniq.begin(), uniq.end(), g) - uniq.begin();
            time_out[m] = got[k].t;
            status_out[m] = got[k].status;
        }
        return OFL_OK;
    }
    for (int32_t m = 0; m < pop; ++m) {
        std::vector<uint8_t> g(genes + (size_t)m * gene_len, genes + (size_t)(m + 1) * gene_len);
        auto it = seen.find(g);
        Measurement meas;
        if (it != seen.end()) {
            meas = it->second;
        } else {
            check_gene(app, g.data(), gene_len, placement);
            int hard = OFL_OK;
            meas = measure(app, placement, dev_bufs, static_cast<hipStream_t>(stream), opts->reps, opts->warmup,
                           opts->policy, opts->flags, opts->deadline_s, &hard, opts->verify_rtol);
            if (hard != OFL_OK) return hard;
            seen[g] = meas;
        }
        time_out[m] = meas.t;
        status_out[m] = meas.status;
    }
    return OFL_OK;
}

int ofl_ga_run(ofl_app *app, const ofl_ga_params *params, void *const *dev_bufs, int32_t n_bufs, void *stream,
               ofl_ga_result *result) {
    if (!app || !result) return fail(OFL_E_ARG, "null argument");
    int rc = check_ga_params(params, app->ir.gene_len);
    if (rc != OFL_OK) return rc;
    if ((rc = check_bufs(app, dev_bufs, n_bufs)) != OFL_OK) return rc;
    if (params->reps < 1 || params->warmup < 0) return fail(OFL_E_ARG, "need reps >= 1 and warmup >= 0");
    int hard = OFL_OK;
    const int a = app->ir.gene_len;
    // the gene-by-gene evaluator; in a batched search (the generations that
    // do not go to a submission, and the all-CPU reference gene) it runs
    // eagerly, so that no gene's graphs are captured for a handful of runs
    const int eager = (params->flags & OFL_RUN_BATCHED) ? params->flags & ~(OFL_RUN_GRAPH | OFL_RUN_BATCHED)
                                                         : params->flags;
    Evaluator ev = [&](const std::vector<uint8_t> &g, double limit) -> Measurement {
        if (hard != OFL_OK) return Measurement{0.0, OFL_ST_FAILED};
        std::vector<uint8_t> placement;
        check_gene(app, g.data(), a, placement);
        return measure(app, placement, dev_bufs, static_cast<hipStream_t>(stream), params->reps, params->warmup,
                       params->policy, eager, limit > 0 ? limit : 0.0, &hard, params->verify_rtol);
    };
    BatchEvaluator bev = [&](const std::vector<std::vector<uint8_t>> &gs, double limit) {
        std::vector<Measurement> out(gs.size(), Measurement{0.0, OFL_ST_FAILED});
        if (hard != OFL_OK) return out;
        std::vector<std::vector<uint8_t>> places(gs.size());
        for (size_t i = 0; i < gs.size(); ++i) check_gene(app, gs[i].data(), a, places[i]);
        const int rc2 = measure_batched(app, places, dev_bufs, static_cast<hipStream_t>(stream), params->reps,
                                        params->warmup, params->policy, params->flags, limit, out,
                                        params->verify_rtol);
        if (rc2 != OFL_OK) hard = rc2;
        return out;
    };
    // A generation's fresh genes go to one submission once the best run
    // measured so far is shorter than batch_eager_threshold(); until then
    // (the first generation included) the search measures them gene by gene,
    // exactly as without OFL_RUN_BATCHED: for long runs, capturing each
    // gene's graphs costs more than the launch overhead a submission saves
    const double eager_from = batch_eager_threshold();
    const BatchGate gate = [eager_from](const GaTrace &t) { return t.best_f > 0.0 && t.best_t < eager_from; };
    GaTrace tr;
    std::string what = "app=" + app->ir.name + ":" + std::to_string(app->ir.nests.size());
    for (const auto &n : app->ir.nests) what += ":" + n.name;
    rc = run_logged_ga(a, params, what, ev, bev, (params->flags & OFL_RUN_PROGRESS) != 0, tr, &gate);
    if (hard != OFL_OK) return hard;
    if (rc != OFL_OK) return rc;
    fill_ga_result(tr, a, params->M, result);
    return OFL_OK;
}

int ofl_ga_run_table(int32_t gene_len, const ofl_ga_params *params, const double *t_table,
                     const int32_t *status_table, ofl_ga_result *result) {
    if (!t_table || !result) return fail(OFL_E_ARG, "null argument");
    if (gene_len < 1 || gene_len > 24) return fail(OFL_E_ARG, "gene_len must be in [1, 24]");
    int rc = check_ga_params(params, gene_len);
    if (rc != OFL_OK) return rc;
    Evaluator ev = [&](const std::vector<uint8_t> &g, double limit) -> Measurement {
        uint64_t idx = 0;
        for (int i = 0; i < gene_len; ++i) idx |= (uint64_t)g[i] << i;
        Measurement m{t_table[idx], status_table ? status_table[idx] : OFL_ST_OK};
        if (m.status == OFL_ST_OK && limit > 0 && m.t > limit) {
            m.t = limit;
            m.status = OFL_ST_TIMEOUT;
        }
        return m;
    };
    BatchEvaluator bev = [&](const std::vector<std::vector<uint8_t>> &gs, double limit) {
        std::vector<Measurement> out;
        for (const auto &g : gs) out.push_back(ev(g, limit));
        return out;
    };
    // what is searched: the table (FNV-1a over its bytes)
    uint64_t h = 1469598103934665603ull;
    auto mixin = [&](const void *p, size_t n) {
        for (size_t i = 0; i < n; ++i) h = (h ^ static_cast<const unsigned char *>(p)[i]) * 1099511628211ull;
    };
    mixin(t_table, sizeof(double) << gene_len);
    if (status_table) mixin(status_table, sizeof(int32_t) << gene_len);
    char what[64];
    std::snprintf(what, sizeof what, "table=%016llx", (unsigned long long)h);
    GaTrace tr;
    rc = run_logged_ga(gene_len, params, what, ev, bev, false, tr);
    if (rc != OFL_OK) return rc;
    fill_ga_result(tr, gene_len, params->M, result);
    return OFL_OK;
}

int ofl_read_buffer(ofl_app *app, int32_t buf, void *host_dst, uint64_t bytes) {
    if (!app || !host_dst) return fail(OFL_E_ARG, "null argument");
    if (buf < 0 || buf >= (int32_t)app->ir.bufs.size()) return fail(OFL_E_RANGE, "buffer index out of range");
    if (!app->ran) return fail(OFL_E_STATE, "no completed run");
    const Buffer &b = app->ir.bufs[buf];
    if (bytes < b.nbytes) return fail(OFL_E_ARG, "destination too small");
    if (app->host_valid[buf]) {
        // a host copy this run never touched still holds stale content from an
        // earlier run when its restore was skipped: its true value is the set-up
        if (!app->host_written[buf] && app->host_dirty[buf]) restore_host(app, buf);
        std::memcpy(host_dst, app->host[buf], b.nbytes);
        return OFL_OK;
    }
    hipError_t e = hipMemcpyAsync(host_dst, app->last_dev[buf], b.nbytes, hipMemcpyDeviceToHost, app->last_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(app->last_stream);
    return e == hipSuccess ? OFL_OK : hip_fail(e, "read_buffer");
}

int ofl_set_kernel_timing(ofl_app *app, int32_t enable) {
    if (!app) return fail(OFL_E_ARG, "null app");
    app->timing = enable != 0;
    if (app->timing) app->kstats.clear();
    return OFL_OK;
}

int ofl_set_kernel_timing_sample(ofl_app *app, int32_t stride, int32_t phase) {
    if (!app) return fail(OFL_E_ARG, "null app");
    if (stride < 1 || phase < 0 || phase >= stride) return fail(OFL_E_ARG, "need stride >= 1 and 0 <= phase < stride");
    app->timing_stride = stride;
    app->timing_phase = phase;
    return OFL_OK;
}

static_assert(OP_COUNT <= 64, "timed kinds are a 64-bit mask");

int ofl_set_kernel_timing_op(ofl_app *app, const char *op) {
    if (!app) return fail(OFL_E_ARG, "null app");
    uint64_t ops = 0;
    const std::string list = op ? op : "";
    // every comma-separated piece must name a kind (an empty piece does not)
    for (size_t at = 0; !list.empty() && at <= list.size();) {
        size_t end = list.find(',', at);
        if (end == std::string::npos) end = list.size();
        const std::string name = list.substr(at, end - at);
        int found = OP_NONE;
        for (int o = OP_NONE + 1; o < OP_COUNT; ++o)
            if (name == op_name((Op)o)) found = o;
        if (found == OP_NONE) return fail(OFL_E_ARG, "unknown nest kind '" + name + "'");
        ops |= 1ull << found;
        at = end + 1;
    }
    app->timing_ops = ops;
    return OFL_OK;
}

int ofl_kernel_stats(const ofl_app *app, const char *op, int64_t *executions, double *total_ms) {
    if (!app || !op) return fail(OFL_E_ARG, "null argument");
    auto it = app->kstats.find(op);
    if (executions) *executions = it == app->kstats.end() ? 0 : it->second.first;
    if (total_ms) *total_ms = it == app->kstats.end() ? 0.0 : it->second.second;
    return OFL_OK;
}

const char *ofl_status_str(int32_t code) {
    switch (code) {
    case OFL_OK: return "ok";
    case OFL_E_ARG: return "invalid argument";
    case OFL_E_IO: return "I/O error";
    case OFL_E_PARSE: return "parse error";
    case OFL_E_IR: return "invalid application";
    case OFL_E_GENE_LEN: return "gene length mismatch";
    case OFL_E_GENE_BIT: return "gene byte not 0/1";
    case OFL_E_NOT_PARALLEL: return "nest not parallelisable";
    case OFL_E_BUF: return "bad device buffer";
    case OFL_E_HIP: return "HIP runtime error";
    case OFL_E_TIMEOUT: return "deadline exceeded";
    case OFL_E_MISMATCH: return "output mismatch";
    case OFL_E_STATE: return "invalid state";
    case OFL_E_NOMEM: return "out of memory";
    case OFL_E_RANGE: return "index out of range";
    case OFL_E_UNSUPPORTED: return "not supported in a batch";
    default: return "unknown status";
    }
}

const char *ofl_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
