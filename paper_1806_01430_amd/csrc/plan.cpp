// Transfer planner.
//
// Each buffer has a host copy and a device copy, each either current or
// stale; at the start the host copy holds the set-up content and the device
// copy is stale (with OFL_RUN_PRESTAGED both hold it).
//
// RESIDENT: a GPU nest first copies in what it reads that is stale on the
// device, a CPU nest first copies out what it reads that is stale on the host;
// after a nest, what it wrote is current only where it ran.  At the end the
// outputs that are stale on the host are copied out (unless KEEP_OUTPUTS).
//
// PER_REGION: the implicit copies a directive compiler places around each
// offloaded region (Sec. 2 of the paper): a GPU nest copies in everything it
// reads and copies out everything it writes; CPU nests copy nothing.
#include "plan.hpp"

#include "../../include/ofl.h"

namespace ofl {

namespace {

struct Planner {
    const AppIR &app;
    const std::vector<uint8_t> &placement;
    int policy, flags;
    Plan &P;
    std::vector<char> host, dev;
    std::vector<char> host_pristine, dev_pristine;   // still holding set-up content
    std::vector<int64_t> env;

    void copy_in(int b) {
        P.steps.push_back({ST_H2D, b, -1});
        P.h2d += app.bufs[b].nbytes;
        P.copies++;
        if (host_pristine[b]) P.host_init_used[b] = 1;
        dev[b] = 1;
        dev_pristine[b] = 0;
    }
    void copy_out(int b) {
        P.steps.push_back({ST_D2H, b, -1});
        P.d2h += app.bufs[b].nbytes;
        P.copies++;
        if (dev_pristine[b]) P.dev_init_used[b] = 1;
        host[b] = 1;
        host_pristine[b] = 0;
    }
    void exec(int ni) {
        const Nest &n = app.nests[ni];
        bool gpu = placement[ni] != 0;
        if (gpu) {
            for (int b : n.reads) {
                if (policy == OFL_POLICY_PER_REGION || !dev[b]) copy_in(b);
                else if (dev_pristine[b]) P.dev_init_used[b] = 1;
            }
        } else if (policy == OFL_POLICY_RESIDENT) {
            for (int b : n.reads) {
                if (!host[b]) copy_out(b);
                else if (host_pristine[b]) P.host_init_used[b] = 1;
            }
        } else {
            for (int b : n.reads)
                if (host_pristine[b]) P.host_init_used[b] = 1;
        }
        int env_off = (int)P.env.size();
        P.env.insert(P.env.end(), env.begin(), env.end());
        P.steps.push_back({gpu ? ST_GPU : ST_CPU, ni, env_off});
        if (gpu) P.launches++;
        else P.host_nests++;
        for (int b : n.writes) {
            if (gpu) {
                host[b] = 0;
                dev[b] = 1;
                dev_pristine[b] = 0;
            } else {
                host[b] = 1;
                dev[b] = 0;
                host_pristine[b] = 0;
            }
        }
        if (gpu && policy == OFL_POLICY_PER_REGION)
            for (int b : n.writes) copy_out(b);
    }
    void walk(const std::vector<ProgItem> &items) {
        for (const auto &it : items) {
            if (!it.is_repeat) {
                exec(it.nest);
                continue;
            }
            for (int64_t r = 0; r < it.count; ++r) {
                env[it.rep_id] = r;
                walk(it.body);
            }
        }
    }
};

}  // namespace

void build_plan(const AppIR &app, const std::vector<uint8_t> &placement, int policy, int flags, Plan &out) {
    out = Plan();
    size_t nb = app.bufs.size();
    out.host_init_used.assign(nb, 0);
    out.dev_init_used.assign(nb, 0);
    Planner pl{app, placement, policy, flags, out};
    bool pre = (flags & OFL_RUN_PRESTAGED) != 0;
    pl.host.assign(nb, 1);
    pl.dev.assign(nb, pre ? 1 : 0);
    pl.host_pristine.assign(nb, 1);
    pl.dev_pristine.assign(nb, pre ? 1 : 0);
    pl.env.assign(app.repeat_names.size(), 0);
    pl.walk(app.program);
    if (!(flags & OFL_RUN_KEEP_OUTPUTS))
        for (size_t b = 0; b < nb; ++b)
            if (app.bufs[b].output && !pl.host[b]) pl.copy_out((int)b);
    out.host_valid = pl.host;
    out.dev_valid = pl.dev;
}

}  // namespace ofl
