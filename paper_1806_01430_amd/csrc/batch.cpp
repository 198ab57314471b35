// Instance batches: many instances of one program with uneven sizes, every
// nest on the GPU, each nest run for all instances by one grouped launch.
//
// The paper evaluates one application at a time; the batching configuration
// widens the GPU side of the method to many small instances, where launching
// each instance's kernels separately leaves the device idle between tiny
// launches.  Here every nest execution of the common program becomes one
// persistent launch over a work table that lists the nest's work units in all
// instances (biggest instances first, so the tail of the launch is made of
// small units), the sweeps are captured with everything else in one HIP
// graph, and the tile shapes and grid sizes come from a tuner that times the
// candidates on the batch itself.
#include "../../include/ofl.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "batch_jobs.hpp"
#include "host_nests.hpp"
#include "ir.hpp"
#include "kernels.hpp"
#include "status.hpp"

using namespace ofl;

namespace {

using clk = std::chrono::steady_clock;

struct BatchGraph {
    hipGraphExec_t exec = nullptr;
    int launches = 0;
    ~BatchGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};

// Device work table of one nest (offset into the table allocation).
struct NestTable {
    size_t off = 0;          // byte offset of the job array
    int njobs = 0;
    int64_t nunits = 0;      // units / tiles / items
    unsigned blocks = 0;     // persistent grid
};

constexpr int kMaxBlocksPerCu = 8;

}  // namespace

struct ofl_batch {
    std::vector<AppIR> inst;
    std::vector<uint64_t> seed;
    int n_bufs = 0;
    ofl_batch_config cfg{};
    int device = -1;

    // tables built for (bufs, cfg); graphs are keyed by the same
    std::vector<const void *> tab_bufs;
    ofl_batch_config tab_cfg{};
    bool tab_valid = false;
    std::vector<NestTable> tabs;      // per nest
    void *d_tables = nullptr;
    size_t tables_cap = 0;
    double *d_partials = nullptr;     // per sweep item (grouped) / per block (per-instance launches)
    int64_t partial_cap = 0;
    void *d_scratch = nullptr;        // the reduction partials
    std::unique_ptr<BatchGraph> graph;
    hipStream_t capture_stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};

    ~ofl_batch() {
        graph.reset();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        if (d_tables) (void)hipFree(d_tables);
        if (d_scratch) (void)hipFree(d_scratch);
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

bool same_structure(const AppIR &a, const AppIR &b, std::string &why) {
    if (a.bufs.size() != b.bufs.size() || a.nests.size() != b.nests.size()) {
        why = "buffer or nest count";
        return false;
    }
    for (size_t i = 0; i < a.bufs.size(); ++i)
        if (a.bufs[i].name != b.bufs[i].name || a.bufs[i].dtype != b.bufs[i].dtype ||
            a.bufs[i].dims.size() != b.bufs[i].dims.size() || a.bufs[i].setup_sin != b.bufs[i].setup_sin) {
            why = "buffer '" + a.bufs[i].name + "'";
            return false;
        }
    for (size_t i = 0; i < a.nests.size(); ++i)
        if (a.nests[i].op != b.nests[i].op || a.nests[i].b != b.nests[i].b || a.nests[i].prec != b.nests[i].prec) {
            why = "nest '" + a.nests[i].name + "'";
            return false;
        }
    // same program tree, same trip counts
    std::vector<std::pair<const std::vector<ProgItem> *, const std::vector<ProgItem> *>> st{{&a.program, &b.program}};
    while (!st.empty()) {
        auto [x, y] = st.back();
        st.pop_back();
        if (x->size() != y->size()) {
            why = "program shape";
            return false;
        }
        for (size_t i = 0; i < x->size(); ++i) {
            const ProgItem &p = (*x)[i], &q = (*y)[i];
            if (p.is_repeat != q.is_repeat || p.nest != q.nest || p.count != q.count) {
                why = "program shape or repeat count";
                return false;
            }
            if (p.is_repeat) st.push_back({&p.body, &q.body});
        }
    }
    return true;
}

int check_nest_supported(const AppIR &ir, const Nest &n) {
    switch (n.op) {
    case OP_INIT_UNIFORM:
    case OP_STENCIL19:
    case OP_COPY_INTERIOR:
        break;
    case OP_GEMM:
        if (n.prec != PREC_F32) return fail(OFL_E_UNSUPPORTED, "nest '" + n.name + "': split-precision product");
        break;
    default:
        return fail(OFL_E_UNSUPPORTED, "nest '" + n.name + "' (" + op_name(n.op) + ") has no grouped kernel");
    }
    if (n.op == OP_STENCIL19 || n.op == OP_COPY_INTERIOR) {
        const auto &d = ir.bufs[n.b[0]].dims;
        if ((d[0] + 6) * d[1] * d[2] * 4 >= ((int64_t)1 << 31))
            return fail(OFL_E_UNSUPPORTED, "nest '" + n.name + "': grid too large for a batch");
    }
    if (n.op == OP_GEMM) {
        const auto &a = ir.bufs[n.b[0]].dims, &bb = ir.bufs[n.b[1]].dims;
        if (a[0] > (1 << 24) || bb[1] > (1 << 24) || a[1] > (1 << 24))
            return fail(OFL_E_UNSUPPORTED, "nest '" + n.name + "': product too large for a batch");
    }
    return OFL_OK;
}

int check_ptrs(const ofl_batch *b, void *const *bufs, int32_t n_ptrs) {
    const int64_t want = (int64_t)b->inst.size() * b->n_bufs;
    if (!bufs || n_ptrs != want)
        return fail(OFL_E_BUF, "expected " + std::to_string(want) + " device pointers, got " + std::to_string(n_ptrs));
    for (int64_t i = 0; i < want; ++i) {
        if (!bufs[i]) return fail(OFL_E_BUF, "null device pointer at " + std::to_string(i));
        if (reinterpret_cast<uintptr_t>(bufs[i]) % 16) return fail(OFL_E_BUF, "device pointer not 16-byte aligned");
    }
    return OFL_OK;
}

int bind_device(ofl_batch *b) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (b->device >= 0 && b->device != dev) return fail(OFL_E_STATE, "batch already bound to another device");
    b->device = dev;
    for (auto &ev : b->ev)
        if (!ev) {
            e = hipEventCreate(&ev);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        }
    return OFL_OK;
}

// Planes per sweep item for a grid: the configured count, else the
// single-grid rule (12 planes below 192 interior planes).
int planes_for(const ofl_batch *b, int64_t I) {
    if (b->cfg.stencil_planes > 0) return b->cfg.stencil_planes;
    return I - 2 >= 192 ? 48 : 12;
}

// Instances in decreasing order of a size measure (ties: instance order).
std::vector<int> order_by(const ofl_batch *b, const std::vector<int64_t> &size) {
    std::vector<int> o(b->inst.size());
    std::iota(o.begin(), o.end(), 0);
    std::stable_sort(o.begin(), o.end(), [&](int x, int y) { return size[x] > size[y]; });
    return o;
}

unsigned grid_of(int64_t units_per_block_round, int64_t units, int64_t cap_blocks) {
    int64_t blocks = (units + units_per_block_round - 1) / units_per_block_round;
    if (blocks > cap_blocks) blocks = cap_blocks;
    if (blocks < 1) blocks = 1;
    return (unsigned)blocks;
}

// Build every nest's work table for (bufs, cfg) and upload it; grows the
// scratch for the sweep partials.  Synchronous (no launch of this batch is in
// flight when it runs: every run ends with a stream synchronisation).
int build_tables(ofl_batch *b, void *const *bufs) {
    const AppIR &ir0 = b->inst[0];
    const int nb = b->n_bufs;
    const int cu = k::cu_count();
    auto P = [&](int inst, int buf) { return bufs[(size_t)inst * nb + buf]; };
    std::vector<unsigned char> host;
    auto put = [&](const void *src, size_t bytes) {
        size_t off = (host.size() + 63) / 64 * 64;
        host.resize(off + bytes);
        std::memcpy(host.data() + off, src, bytes);
        return off;
    };
    b->tabs.assign(ir0.nests.size(), NestTable{});
    int64_t max_items = 1, max_block_partials = 1;
    for (size_t ni = 0; ni < ir0.nests.size(); ++ni) {
        const Nest &n0 = ir0.nests[ni];
        NestTable &t = b->tabs[ni];
        if (n0.op == OP_INIT_UNIFORM) {
            std::vector<k::InitJob> jobs;
            int64_t u = 0;
            for (size_t i = 0; i < b->inst.size(); ++i) {
                const Nest &n = b->inst[i].nests[ni];
                for (size_t s = 0; s < n.b.size(); ++s) {
                    const int64_t cnt = b->inst[i].bufs[n.b[s]].count;
                    if (cnt <= 0) continue;
                    jobs.push_back({static_cast<float *>(P((int)i, n.b[s])), cnt,
                                    uniform_stream_key(b->seed[i], n.streams[s]), u});
                    u += (cnt + k::kInitUnit - 1) / k::kInitUnit;
                }
            }
            t.njobs = (int)jobs.size();
            t.nunits = u;
            t.blocks = grid_of(1, u, (int64_t)cu * 8);
            if (!jobs.empty()) t.off = put(jobs.data(), jobs.size() * sizeof(jobs[0]));
        } else if (n0.op == OP_GEMM) {
            int bm = 64, bk = 32;
            k::gemm_cfg_shape(b->cfg.gemm_cfg, &bm, &bk);
            std::vector<int64_t> work(b->inst.size());
            for (size_t i = 0; i < b->inst.size(); ++i) {
                const Nest &n = b->inst[i].nests[ni];
                const auto &a = b->inst[i].bufs[n.b[0]].dims;
                work[i] = a[1];   // per-tile cost grows with K
            }
            std::vector<k::GemmJob> jobs;
            int tiles = 0;
            for (int i : order_by(b, work)) {
                const Nest &n = b->inst[i].nests[ni];
                const auto &a = b->inst[i].bufs[n.b[0]].dims, &bb = b->inst[i].bufs[n.b[1]].dims;
                const int M = (int)a[0], K = (int)a[1], N = (int)bb[1];
                if (M <= 0 || N <= 0) continue;
                const int tn = (N + bm - 1) / bm, tm = (M + bm - 1) / bm;
                jobs.push_back({static_cast<const float *>(P(i, n.b[0])), static_cast<const float *>(P(i, n.b[1])),
                                static_cast<float *>(P(i, n.b[2])), M, N, K, tn, tiles,
                                (K % 4 == 0 && N % 4 == 0) ? 1 : 0});
                tiles += tm * tn;
            }
            t.njobs = (int)jobs.size();
            t.nunits = tiles;
            const int occ = std::min(k::grouped_gemm_occupancy(b->cfg.gemm_cfg), b->cfg.gemm_blocks_per_cu);
            t.blocks = grid_of(1, tiles, (int64_t)cu * std::max(1, occ));
            if (!jobs.empty()) t.off = put(jobs.data(), jobs.size() * sizeof(jobs[0]));
        } else if (n0.op == OP_STENCIL19) {
            const int JR = b->cfg.stencil_rows;
            std::vector<k::Geo> geo(b->inst.size());
            std::vector<int64_t> work(b->inst.size());
            for (size_t i = 0; i < b->inst.size(); ++i) {
                const auto &d = b->inst[i].bufs[b->inst[i].nests[ni].b[0]].dims;
                geo[i] = k::make_geo(d[0], d[1], d[2], JR, planes_for(b, d[0]));
                work[i] = d[0] * d[1] * d[2];
                max_block_partials = std::max(max_block_partials, k::stencil_partials(d[0], d[1], d[2]));
            }
            std::vector<k::StencilJob> jobs;
            int items = 0;
            for (int i : order_by(b, work)) {
                const Nest &n = b->inst[i].nests[ni];
                if (geo[i].items <= 0) continue;
                jobs.push_back({static_cast<const float *>(P(i, n.b[0])), static_cast<float *>(P(i, n.b[1])),
                                static_cast<double *>(P(i, n.b[2])), geo[i], items});
                items += geo[i].items;
            }
            t.njobs = (int)jobs.size();
            t.nunits = items;
            max_items = std::max<int64_t>(max_items, items);
            const int occ = std::min(k::grouped_stencil_occupancy(JR), b->cfg.stencil_blocks_per_cu);
            t.blocks = grid_of(4, items, (int64_t)cu * std::max(1, occ));
            if (!jobs.empty()) t.off = put(jobs.data(), jobs.size() * sizeof(jobs[0]));
        } else if (n0.op == OP_COPY_INTERIOR) {
            std::vector<int64_t> work(b->inst.size());
            for (size_t i = 0; i < b->inst.size(); ++i) {
                const auto &d = b->inst[i].bufs[b->inst[i].nests[ni].b[0]].dims;
                work[i] = d[0] * d[1] * d[2];
            }
            std::vector<k::CopyJob> jobs;
            int units = 0;
            for (int i : order_by(b, work)) {
                const Nest &n = b->inst[i].nests[ni];
                const auto &d = b->inst[i].bufs[n.b[0]].dims;
                const int rows = (int)((d[0] - 2) * (d[1] - 2));
                if (rows <= 0 || d[2] < 3) continue;
                jobs.push_back({static_cast<float *>(P(i, n.b[0])), static_cast<const float *>(P(i, n.b[1])),
                                (int)d[0], (int)d[1], (int)d[2], rows, units});
                units += (rows + k::kRows - 1) / k::kRows;
            }
            t.njobs = (int)jobs.size();
            t.nunits = units;
            t.blocks = grid_of(4, units, (int64_t)cu * k::grouped_copy_occupancy());
            if (!jobs.empty()) t.off = put(jobs.data(), jobs.size() * sizeof(jobs[0]));
        }
    }
    hipError_t e = hipSuccess;
    if (host.size() > b->tables_cap) {
        if (b->d_tables) (void)hipFree(b->d_tables);
        b->d_tables = nullptr;
        b->tables_cap = 0;
        e = hipMalloc(&b->d_tables, host.size());
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(OFL_E_NOMEM, "batch tables") : hip_fail(e, "hipMalloc");
        b->tables_cap = host.size();
    }
    if (!host.empty()) {
        e = hipMemcpy(b->d_tables, host.data(), host.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "batch tables upload");
    }
    const int64_t need = std::max(max_items, max_block_partials);
    if (need > b->partial_cap) {
        if (b->d_scratch) (void)hipFree(b->d_scratch);
        b->d_scratch = nullptr;
        b->partial_cap = 0;
        const size_t bytes = (size_t)need * sizeof(double) + 256;
        e = hipMalloc(&b->d_scratch, bytes);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(OFL_E_NOMEM, "batch scratch") : hip_fail(e, "hipMalloc");
        e = hipMemset(b->d_scratch, 0, bytes);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "batch scratch init");
        b->d_partials = static_cast<double *>(b->d_scratch);
        b->partial_cap = need;
    }
    b->tab_bufs.assign(bufs, bufs + (size_t)b->inst.size() * nb);
    b->tab_cfg = b->cfg;
    b->tab_valid = true;
    b->graph.reset();
    return OFL_OK;
}

bool same_cfg(const ofl_batch_config &x, const ofl_batch_config &y) { return std::memcmp(&x, &y, sizeof(x)) == 0; }

int ensure_tables(ofl_batch *b, void *const *bufs) {
    const size_t n = b->inst.size() * (size_t)b->n_bufs;
    if (b->tab_valid && same_cfg(b->tab_cfg, b->cfg) && std::equal(b->tab_bufs.begin(), b->tab_bufs.end(), bufs) &&
        b->tab_bufs.size() == n)
        return OFL_OK;
    return build_tables(b, bufs);
}

template <typename Job>
const Job *table(const ofl_batch *b, int nest) {
    return reinterpret_cast<const Job *>(static_cast<const char *>(b->d_tables) + b->tabs[nest].off);
}

// One grouped execution of nest `ni` (residual slot from the repeat env).
hipError_t launch_grouped(ofl_batch *b, int ni, const std::vector<int64_t> &env, hipStream_t s, int *launches) {
    const Nest &n = b->inst[0].nests[ni];
    const NestTable &t = b->tabs[ni];
    switch (n.op) {
    case OP_INIT_UNIFORM:
        ++*launches;
        return k::init_grouped(table<k::InitJob>(b, ni), t.njobs, t.nunits, t.blocks, s);
    case OP_GEMM:
        ++*launches;
        return k::gemm_grouped(b->cfg.gemm_cfg, table<k::GemmJob>(b, ni), t.njobs, (int)t.nunits, t.blocks, s);
    case OP_STENCIL19: {
        *launches += 2;
        hipError_t e = k::stencil_grouped(b->cfg.stencil_rows, table<k::StencilJob>(b, ni), t.njobs, (int)t.nunits,
                                          b->d_partials, t.blocks, s);
        if (e != hipSuccess) return e;
        return k::stencil_finish(table<k::StencilJob>(b, ni), t.njobs, (int)t.nunits, b->d_partials,
                                 env[n.slot_repeat], s);
    }
    case OP_COPY_INTERIOR:
        ++*launches;
        return k::copy_grouped(table<k::CopyJob>(b, ni), t.njobs, (int)t.nunits, t.blocks, s);
    default:
        return hipErrorInvalidValue;
    }
}

// The single-instance launchers for instance `i` (the comparison path).
hipError_t launch_single(ofl_batch *b, int i, int ni, const std::vector<int64_t> &env, void *const *bufs,
                         hipStream_t s, int *launches) {
    const AppIR &ir = b->inst[i];
    const Nest &n = ir.nests[ni];
    auto F = [&](int t) { return static_cast<float *>(bufs[(size_t)i * b->n_bufs + n.b[t]]); };
    hipError_t e = hipSuccess;
    switch (n.op) {
    case OP_INIT_UNIFORM:
        for (size_t t = 0; t < n.b.size() && e == hipSuccess; ++t, ++*launches)
            e = k::init_uniform(F((int)t), ir.bufs[n.b[t]].count, uniform_stream_key(b->seed[i], n.streams[t]), s);
        return e;
    case OP_GEMM: {
        const auto &a = ir.bufs[n.b[0]].dims, &bb = ir.bufs[n.b[1]].dims;
        ++*launches;
        return k::gemm_f32(F(0), F(1), F(2), a[0], bb[1], a[1], s);
    }
    case OP_STENCIL19: {
        const auto &d = ir.bufs[n.b[0]].dims;
        k::ReduceScratch rs{b->d_partials, b->partial_cap};
        *launches += 2;   // sweep + residual finish
        return k::stencil19(F(0), F(1), d[0], d[1], d[2],
                            reinterpret_cast<double *>(F(2)) + env[n.slot_repeat], rs, s);
    }
    case OP_COPY_INTERIOR: {
        const auto &d = ir.bufs[n.b[0]].dims;
        ++*launches;
        return k::copy_interior(F(0), F(1), d[0], d[1], d[2], s);
    }
    default:
        return hipErrorInvalidValue;
    }
}

// Walk the common program; `fn(nest, env)` launches one nest execution.
template <typename Fn>
hipError_t walk(const std::vector<ProgItem> &items, std::vector<int64_t> &env, Fn &&fn) {
    for (const ProgItem &it : items) {
        if (!it.is_repeat) {
            hipError_t e = fn(it.nest, env);
            if (e != hipSuccess) return e;
            continue;
        }
        for (int64_t r = 0; r < it.count; ++r) {
            env[it.rep_id] = r;
            hipError_t e = walk(it.body, env, fn);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t enqueue_grouped(ofl_batch *b, hipStream_t s, int *launches) {
    std::vector<int64_t> env(b->inst[0].repeat_names.size(), 0);
    return walk(b->inst[0].program, env,
                [&](int ni, const std::vector<int64_t> &e) { return launch_grouped(b, ni, e, s, launches); });
}

int ensure_graph(ofl_batch *b) {
    if (b->graph) return OFL_OK;
    if (!b->capture_stream) {
        hipError_t e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    }
    auto g = std::make_unique<BatchGraph>();
    hipError_t e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    int launches = 0;
    hipError_t le = enqueue_grouped(b, b->capture_stream, &launches);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->capture_stream, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le != hipSuccess ? le : e, "batch graph capture");
    }
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    g->launches = launches;
    b->graph = std::move(g);
    return OFL_OK;
}

bool cfg_ok(const ofl_batch_config &c) {
    auto bpc_ok = [](int v) { return v >= 1 && v <= kMaxBlocksPerCu; };
    return c.gemm_cfg >= 0 && c.gemm_cfg < k::kGemmCfgs && bpc_ok(c.gemm_blocks_per_cu) &&
           (c.stencil_rows == 2 || c.stencil_rows == 4 || c.stencil_rows == 8) && c.stencil_planes >= 0 &&
           c.stencil_planes <= 4096 && bpc_ok(c.stencil_blocks_per_cu);
}

// Median of `reps` event-timed executions of `fn` on stream s (after one warm-up).
template <typename Fn>
int time_median(ofl_batch *b, hipStream_t s, int reps, Fn &&fn, double *ms) {
    std::vector<double> t;
    for (int r = -1; r < reps; ++r) {
        hipError_t e = hipEventRecord(b->ev[0], s);
        if (e == hipSuccess) e = fn();
        if (e == hipSuccess) e = hipEventRecord(b->ev[1], s);
        if (e == hipSuccess) e = hipEventSynchronize(b->ev[1]);
        float x = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&x, b->ev[0], b->ev[1]);
        if (e != hipSuccess) return hip_fail(e, "tuning launch");
        if (r >= 0) t.push_back(x);
    }
    std::sort(t.begin(), t.end());
    *ms = t.empty() ? 0.0 : t[t.size() / 2];
    return OFL_OK;
}

}  // namespace

extern "C" {

int ofl_batch_create(const char *app_json, int32_t n_inst, const char *const *param_names, int32_t n_params,
                     const int64_t *param_values, const uint64_t *seeds, ofl_batch **out) {
    if (!out) return fail(OFL_E_ARG, "null out");
    *out = nullptr;
    if (!app_json || n_inst < 1 || n_params < 0 || (n_params > 0 && (!param_names || !param_values)) || !seeds)
        return fail(OFL_E_ARG, "bad batch arguments");
    std::unique_ptr<ofl_batch> b(new (std::nothrow) ofl_batch());
    if (!b) return fail(OFL_E_NOMEM, "batch");
    const std::string text(app_json);
    b->inst.resize(n_inst);
    b->seed.assign(seeds, seeds + n_inst);
    for (int32_t i = 0; i < n_inst; ++i) {
        std::map<std::string, int64_t> ov;
        for (int32_t p = 0; p < n_params; ++p) {
            if (!param_names[p]) return fail(OFL_E_ARG, "null parameter name");
            ov[param_names[p]] = param_values[(size_t)i * n_params + p];
        }
        std::string err;
        const int rc = parse_app(text, b->inst[i], err, &ov);
        if (rc != OFL_OK) return fail(rc, "instance " + std::to_string(i) + ": " + err);
        analyse(b->inst[i]);
        std::string why;
        if (i > 0 && !same_structure(b->inst[0], b->inst[i], why))
            return fail(OFL_E_UNSUPPORTED, "instance " + std::to_string(i) + " differs in " + why);
    }
    for (const Nest &n : b->inst[0].nests)
        if (n.verdict == V_REJECT) return fail(OFL_E_NOT_PARALLEL, "nest '" + n.name + "' is not parallelisable");
    for (const Nest &n : b->inst[0].nests)
        for (const AppIR &ir : b->inst) {
            const int rc = check_nest_supported(ir, ir.nests[&n - &b->inst[0].nests[0]]);
            if (rc != OFL_OK) return rc;
        }
    b->n_bufs = (int)b->inst[0].bufs.size();
    b->cfg = ofl_batch_config{1, 2, 4, 0, 8};
    *out = b.release();
    return OFL_OK;
}

void ofl_batch_free(ofl_batch *batch) { delete batch; }

int ofl_batch_info(const ofl_batch *b, int32_t *n_inst, int32_t *n_bufs, int32_t *n_nests) {
    if (!b) return fail(OFL_E_ARG, "null batch");
    if (n_inst) *n_inst = (int32_t)b->inst.size();
    if (n_bufs) *n_bufs = b->n_bufs;
    if (n_nests) *n_nests = (int32_t)b->inst[0].nests.size();
    return OFL_OK;
}

int ofl_batch_buf_info(const ofl_batch *b, int32_t inst, int32_t buf, uint64_t *bytes, int32_t *dtype,
                       int32_t *rank) {
    if (!b) return fail(OFL_E_ARG, "null batch");
    if (inst < 0 || inst >= (int32_t)b->inst.size() || buf < 0 || buf >= b->n_bufs)
        return fail(OFL_E_RANGE, "instance or buffer index");
    const Buffer &bf = b->inst[inst].bufs[buf];
    if (bytes) *bytes = bf.nbytes;
    if (dtype) *dtype = (int32_t)bf.dtype;
    if (rank) *rank = (int32_t)bf.dims.size();
    return OFL_OK;
}

int ofl_batch_buf_dims(const ofl_batch *b, int32_t inst, int32_t buf, int64_t *dims, int32_t cap) {
    if (!b || (cap > 0 && !dims)) return fail(OFL_E_ARG, "null argument");
    if (inst < 0 || inst >= (int32_t)b->inst.size() || buf < 0 || buf >= b->n_bufs)
        return fail(OFL_E_RANGE, "instance or buffer index");
    const auto &d = b->inst[inst].bufs[buf].dims;
    for (int32_t i = 0; i < cap && i < (int32_t)d.size(); ++i) dims[i] = d[i];
    return OFL_OK;
}

int ofl_batch_buf_name(const ofl_batch *b, int32_t buf, char *name, int32_t cap) {
    if (!b || !name || cap < 1) return fail(OFL_E_ARG, "null argument");
    if (buf < 0 || buf >= b->n_bufs) return fail(OFL_E_RANGE, "buffer index");
    const std::string &s = b->inst[0].bufs[buf].name;
    const size_t n = std::min(s.size(), (size_t)cap - 1);
    std::memcpy(name, s.data(), n);
    name[n] = 0;
    return OFL_OK;
}

int ofl_batch_setup(ofl_batch *b, void *const *bufs, int32_t n_ptrs, void *stream) {
    if (!b) return fail(OFL_E_ARG, "null batch");
    int rc = check_ptrs(b, bufs, n_ptrs);
    if (rc == OFL_OK) rc = bind_device(b);
    if (rc != OFL_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<float> tmp;
    for (size_t i = 0; i < b->inst.size(); ++i)
        for (int j = 0; j < b->n_bufs; ++j) {
            const Buffer &buf = b->inst[i].bufs[j];
            void *d = bufs[i * b->n_bufs + j];
            hipError_t e;
            if (buf.setup_sin) {
                tmp.resize((size_t)buf.count);
                fill_setup_sin(buf, tmp.data());
                e = hipMemcpyAsync(d, tmp.data(), buf.nbytes, hipMemcpyHostToDevice, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
            } else {
                e = k::fill_zero(d, buf.nbytes, s);
            }
            if (e != hipSuccess) return hip_fail(e, "batch set-up");
        }
    hipError_t e = hipStreamSynchronize(s);
    return e == hipSuccess ? OFL_OK : hip_fail(e, "batch set-up");
}

int ofl_batch_run(ofl_batch *b, void *const *bufs, int32_t n_ptrs, void *stream, int32_t mode,
                  ofl_batch_stats *stats) {
    if (!b) return fail(OFL_E_ARG, "null batch");
    if (mode < OFL_BATCH_LOOP || mode > OFL_BATCH_GROUPED_GRAPH) return fail(OFL_E_ARG, "bad batch mode");
    ofl_batch_stats st{};
    st.status = OFL_ST_FAILED;
    int rc = check_ptrs(b, bufs, n_ptrs);
    if (rc == OFL_OK) rc = bind_device(b);
    if (rc == OFL_OK) rc = ensure_tables(b, bufs);
    if (rc == OFL_OK && mode == OFL_BATCH_GROUPED_GRAPH) rc = ensure_graph(b);
    if (rc != OFL_OK) {
        if (stats) *stats = st;
        return rc;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int launches = 0, subs = 0;
    const auto t0 = clk::now();
    hipError_t e = hipSuccess;
    if (mode == OFL_BATCH_GROUPED_GRAPH) {
        e = hipGraphLaunch(b->graph->exec, s);
        launches = b->graph->launches;
        subs = 1;
    } else if (mode == OFL_BATCH_GROUPED) {
        e = enqueue_grouped(b, s, &launches);
        subs = launches;
    } else {
        std::vector<int64_t> env(b->inst[0].repeat_names.size(), 0);
        for (size_t i = 0; i < b->inst.size() && e == hipSuccess; ++i)
            e = walk(b->inst[i].program, env, [&](int ni, const std::vector<int64_t> &en) {
                return launch_single(b, (int)i, ni, en, bufs, s, &launches);
            });
        subs = launches;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    st.t_total_s = std::chrono::duration<double>(clk::now() - t0).count();
    st.n_launches = launches;
    st.n_submissions = subs;
    st.status = e == hipSuccess ? OFL_ST_OK : OFL_ST_FAILED;
    if (stats) *stats = st;
    return e == hipSuccess ? OFL_OK : hip_fail(e, "batch run");
}

int ofl_batch_get_config(const ofl_batch *b, ofl_batch_config *cfg) {
    if (!b || !cfg) return fail(OFL_E_ARG, "null argument");
    *cfg = b->cfg;
    return OFL_OK;
}

int ofl_batch_set_config(ofl_batch *b, const ofl_batch_config *cfg) {
    if (!b || !cfg) return fail(OFL_E_ARG, "null argument");
    if (!cfg_ok(*cfg)) return fail(OFL_E_ARG, "batch configuration out of range");
    b->cfg = *cfg;
    return OFL_OK;
}

int ofl_batch_tune(ofl_batch *b, void *const *bufs, int32_t n_ptrs, void *stream, int32_t reps,
                   ofl_tune_entry *entries, int32_t cap, int32_t *n_entries) {
    if (!b) return fail(OFL_E_ARG, "null batch");
    if (reps < 1 || cap < 0 || (cap > 0 && !entries)) return fail(OFL_E_ARG, "bad tuning arguments");
    int rc = check_ptrs(b, bufs, n_ptrs);
    if (rc == OFL_OK) rc = bind_device(b);
    if (rc != OFL_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const AppIR &ir0 = b->inst[0];
    int gemm_nest = -1, stencil_nest = -1;
    for (size_t i = 0; i < ir0.nests.size(); ++i) {
        if (ir0.nests[i].op == OP_GEMM && gemm_nest < 0) gemm_nest = (int)i;
        if (ir0.nests[i].op == OP_STENCIL19 && stencil_nest < 0) stencil_nest = (int)i;
    }
    std::vector<ofl_tune_entry> all;
    const ofl_batch_config start = b->cfg;
    ofl_batch_config best = start;
    const int bpcs[4] = {1, 2, 4, 8};
    if (gemm_nest >= 0) {
        double best_ms = 1e300;
        for (int c = 0; c < k::kGemmCfgs; ++c)
            for (int bpc : bpcs) {
                if (bpc > k::grouped_gemm_occupancy(c)) continue;
                b->cfg = best;
                b->cfg.gemm_cfg = c;
                b->cfg.gemm_blocks_per_cu = bpc;
                rc = ensure_tables(b, bufs);
                double ms = 0;
                std::vector<int64_t> env(ir0.repeat_names.size(), 0);
                if (rc == OFL_OK)
                    rc = time_median(b, s, reps, [&] {
                        int l = 0;
                        return launch_grouped(b, gemm_nest, env, s, &l);
                    }, &ms);
                if (rc != OFL_OK) {
                    b->cfg = start;
                    return rc;
                }
                all.push_back({0, b->cfg, ms});
                if (ms < best_ms) {
                    best_ms = ms;
                    best.gemm_cfg = c;
                    best.gemm_blocks_per_cu = bpc;
                }
            }
    }
    if (stencil_nest >= 0) {
        double best_ms = 1e300;
        const int rows[3] = {2, 4, 8}, planes[3] = {8, 16, 32};
        for (int jr : rows)
            for (int ic : planes)
                for (int bpc : bpcs) {
                    if (bpc > k::grouped_stencil_occupancy(jr)) continue;
                    b->cfg = best;
                    b->cfg.stencil_rows = jr;
                    b->cfg.stencil_planes = ic;
                    b->cfg.stencil_blocks_per_cu = bpc;
                    rc = ensure_tables(b, bufs);
                    double ms = 0;
                    std::vector<int64_t> env(ir0.repeat_names.size(), 0);
                    if (rc == OFL_OK)
                        rc = time_median(b, s, reps, [&] {
                            int l = 0;
                            return launch_grouped(b, stencil_nest, env, s, &l);
                        }, &ms);
                    if (rc != OFL_OK) {
                        b->cfg = start;
                        return rc;
                    }
                    all.push_back({1, b->cfg, ms});
                    if (ms < best_ms) {
                        best_ms = ms;
                        best.stencil_rows = jr;
                        best.stencil_planes = ic;
                        best.stencil_blocks_per_cu = bpc;
                    }
                }
    }
    b->cfg = best;
    for (int32_t i = 0; i < cap && i < (int32_t)all.size(); ++i) entries[i] = all[i];
    if (n_entries) *n_entries = (int32_t)all.size();
    return OFL_OK;
}

}  // extern "C"
