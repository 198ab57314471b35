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
//
// SECTIONS: RESIDENT, except that a CPU nest which only reads a buffer that
// is stale on the host copies out just the bounding box of the elements its
// reads touch (per dimension the range its subscripts take over the loop and
// repeat ranges), unless an earlier box of that buffer, still current,
// contains it; a box covering the whole buffer is a whole copy.  Any write to
// the buffer drops its boxes.
#include "plan.hpp"

#include <algorithm>

#include "../../include/ofl.h"

namespace ofl {

namespace {

// Bounding box of the elements of buffer b read by plain reads of nest n;
// false when they touch nothing.
bool read_box(const Nest &n, int b, int rank, Box &box) {
    bool any = false;
    for (const Access &a : n.access) {
        if (a.buf != b || a.mode != M_R) continue;
        Box cur;
        bool empty = false;
        for (const Sub &s : a.subs) {
            int64_t lo = s.c, hi = s.c + 1;
            if (s.kind == S_LOOP) {
                lo = n.loops[s.idx].lo + s.c;
                hi = n.loops[s.idx].hi + s.c;
            } else if (s.kind == S_REPEAT) {
                int64_t count = 0;
                for (const auto &r : n.repeats)
                    if (r.first == s.idx) count = r.second;
                hi = count + s.c;
            }
            if (lo >= hi) empty = true;
            cur.lo.push_back(lo);
            cur.hi.push_back(hi);
        }
        if (empty || (int)cur.lo.size() != rank) continue;
        if (!any) {
            box = cur;
            any = true;
        } else {
            for (int d = 0; d < rank; ++d) {
                box.lo[d] = std::min(box.lo[d], cur.lo[d]);
                box.hi[d] = std::max(box.hi[d], cur.hi[d]);
            }
        }
    }
    return any;
}

bool contains(const Box &outer, const Box &inner) {
    for (size_t d = 0; d < outer.lo.size(); ++d)
        if (outer.lo[d] > inner.lo[d] || inner.hi[d] > outer.hi[d]) return false;
    return true;
}

struct Planner {
    const AppIR &app;
    const std::vector<uint8_t> &placement;
    int policy, flags;
    Plan &P;
    std::vector<char> host, dev;
    std::vector<char> host_pristine, dev_pristine;   // still holding set-up content
    std::vector<std::vector<int>> host_boxes;        // SECTIONS: current boxes (indices into P.boxes)
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
    // SECTIONS: copy out only box `bx` of buffer b (the host copy stays stale
    // outside the current boxes)
    void copy_out_box(int b, const Box &bx) {
        const uint64_t n = box_bytes(app.bufs[b], bx);
        Step st{ST_D2H, b, -1};
        st.box = (int)P.boxes.size();
        P.boxes.push_back(bx);
        P.steps.push_back(st);
        P.d2h += n;
        P.copies++;
        if (dev_pristine[b]) P.dev_init_used[b] = 1;
        host_pristine[b] = 0;
        host_boxes[b].push_back(st.box);
    }
    bool writes_buf(const Nest &n, int b) const {
        for (int w : n.writes)
            if (w == b) return true;
        return false;
    }
    void exec(int ni) {
        const Nest &n = app.nests[ni];
        bool gpu = placement[ni] != 0;
        if (gpu) {
            for (int b : n.reads) {
                if (policy == OFL_POLICY_PER_REGION || !dev[b]) copy_in(b);
                else if (dev_pristine[b]) P.dev_init_used[b] = 1;
            }
        } else if (policy == OFL_POLICY_RESIDENT || policy == OFL_POLICY_SECTIONS) {
            for (int b : n.reads) {
                if (host[b]) {
                    if (host_pristine[b]) P.host_init_used[b] = 1;
                    continue;
                }
                if (policy == OFL_POLICY_SECTIONS && !writes_buf(n, b)) {
                    Box bx;
                    const Buffer &buf = app.bufs[b];
                    if (!read_box(n, b, (int)buf.dims.size(), bx)) continue;
                    bool whole = true;
                    for (size_t d = 0; d < buf.dims.size(); ++d)
                        if (bx.lo[d] != 0 || bx.hi[d] != buf.dims[d]) whole = false;
                    if (!whole) {
                        bool covered = false;
                        for (int k : host_boxes[b]) covered = covered || contains(P.boxes[k], bx);
                        if (!covered) copy_out_box(b, bx);
                        continue;
                    }
                }
                copy_out(b);
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
            host_boxes[b].clear();
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

uint64_t box_bytes(const Buffer &buf, const Box &bx) {
    uint64_t n = buf.nbytes / (uint64_t)std::max<int64_t>(1, buf.count);
    for (size_t d = 0; d < bx.lo.size(); ++d) n *= (uint64_t)(bx.hi[d] - bx.lo[d]);
    return n;
}

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
    pl.host_boxes.assign(nb, {});
    pl.env.assign(app.repeat_names.size(), 0);
    pl.walk(app.program);
    if (!(flags & OFL_RUN_KEEP_OUTPUTS))
        for (size_t b = 0; b < nb; ++b)
            if (app.bufs[b].output && !pl.host[b]) pl.copy_out((int)b);
    out.host_valid = pl.host;
    out.dev_valid = pl.dev;
}

}  // namespace ofl
