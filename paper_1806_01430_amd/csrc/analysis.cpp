// Parallelisability check of every loop nest (the analogue of the paper's
// trial compile with the parallel directive on one loop at a time, Sec. 4)
// and the buffer-level read / write sets used by the transfer planner.
//
// Verdict rules: an external call rejects (EXTERNAL_CALL), an early exit
// rejects (BREAK); a buffer touched only by `sum` accesses is a reduction
// (PARALLEL_REDUCTION); otherwise a write and any access of the same buffer
// that reach one element from two iterations with different outer-loop values
// reject (DATA_DEP).  The candidate is always the outermost loop of the nest,
// so inner levels never get a directive of their own.
#include <algorithm>
#include <climits>
#include <vector>

#include "ir.hpp"

namespace ofl {

namespace {

// Nodes: 0 = the constant zero; 1..L = loop vars of the first iteration;
// L+1..2L = loop vars of the second iteration; then the repeat variables
// (shared by both, since both iterations belong to one execution of the nest).
struct Graph {
    struct Edge { int to; int64_t d; };   // value(to) = value(from) + d
    std::vector<std::vector<Edge>> adj;
    void add(int a, int b, int64_t delta) {   // value(a) - value(b) = delta
        adj[b].push_back({a, delta});
        adj[a].push_back({b, -delta});
    }
};

}  // namespace

bool carried_dependence(const Nest &n, const Access &w, const Access &x) {
    const int L = (int)n.loops.size();
    for (const auto &lp : n.loops)
        if (lp.lo >= lp.hi) return false;
    for (const auto &r : n.repeats)
        if (r.second <= 0) return false;
    // map repeat ids to node numbers
    std::vector<int> rep_ids;
    for (const auto &r : n.repeats) rep_ids.push_back(r.first);
    const int nodes = 1 + 2 * L + (int)rep_ids.size();
    std::vector<int64_t> lo(nodes), hi(nodes);
    lo[0] = hi[0] = 0;
    for (int l = 0; l < L; ++l) {
        lo[1 + l] = lo[1 + L + l] = n.loops[l].lo;
        hi[1 + l] = hi[1 + L + l] = n.loops[l].hi - 1;
    }
    for (size_t r = 0; r < rep_ids.size(); ++r) {
        lo[1 + 2 * L + r] = 0;
        hi[1 + 2 * L + r] = n.repeats[r].second - 1;
    }
    auto node_of = [&](const Sub &s, int side) -> int {
        if (s.kind == S_CONST) return 0;
        if (s.kind == S_LOOP) return 1 + side * L + s.idx;
        for (size_t r = 0; r < rep_ids.size(); ++r)
            if (rep_ids[r] == s.idx) return 1 + 2 * L + (int)r;
        return 0;
    };
    Graph g;
    g.adj.resize(nodes);
    for (size_t d = 0; d < w.subs.size(); ++d) {
        // value(nw) + cw == value(nx) + cx
        int nw = node_of(w.subs[d], 0), nx = node_of(x.subs[d], 1);
        g.add(nw, nx, x.subs[d].c - w.subs[d].c);
    }
    // potentials by breadth-first search; a contradiction means no solution
    std::vector<int> comp(nodes, -1);
    std::vector<int64_t> pot(nodes, 0);
    std::vector<int64_t> clo, chi;   // feasible range of each component's anchor
    for (int s = 0; s < nodes; ++s) {
        if (comp[s] >= 0) continue;
        int c = (int)clo.size();
        clo.push_back(LLONG_MIN / 4);
        chi.push_back(LLONG_MAX / 4);
        std::vector<int> queue{s};
        comp[s] = c;
        pot[s] = 0;
        for (size_t qi = 0; qi < queue.size(); ++qi) {
            int u = queue[qi];
            for (const auto &e : g.adj[u]) {
                int64_t want = pot[u] + e.d;
                if (comp[e.to] < 0) {
                    comp[e.to] = c;
                    pot[e.to] = want;
                    queue.push_back(e.to);
                } else if (pot[e.to] != want) {
                    return false;
                }
            }
        }
        for (int u : queue) {
            clo[c] = std::max(clo[c], lo[u] - pot[u]);
            chi[c] = std::min(chi[c], hi[u] - pot[u]);
        }
        if (clo[c] > chi[c]) return false;
    }
    // outer loop variable of each iteration: must be able to differ
    int a = 1, b = 1 + L;
    if (comp[a] == comp[b]) return pot[a] != pot[b];
    bool fixed_a = clo[comp[a]] == chi[comp[a]];
    bool fixed_b = clo[comp[b]] == chi[comp[b]];
    if (fixed_a && fixed_b) return clo[comp[a]] + pot[a] != clo[comp[b]] + pot[b];
    return true;
}

static bool covers_buffer(const Nest &n, const Access &a, const Buffer &buf) {
    if (a.mode != M_W) return false;
    std::vector<char> used(n.loops.size(), 0);
    for (size_t d = 0; d < a.subs.size(); ++d) {
        const Sub &s = a.subs[d];
        if (s.kind == S_CONST) {
            if (!(buf.dims[d] == 1 && s.c == 0)) return false;
            continue;
        }
        if (s.kind != S_LOOP || used[s.idx]) return false;
        used[s.idx] = 1;
        const Loop &lp = n.loops[s.idx];
        if (lp.lo >= lp.hi || lp.lo + s.c > 0 || lp.hi + s.c < buf.dims[d]) return false;
    }
    return true;
}

void analyse(AppIR &app) {
    int pos = 0;
    for (auto &n : app.nests) {
        // buffer-level sets
        std::vector<char> rd(app.bufs.size(), 0), wr(app.bufs.size(), 0), full(app.bufs.size(), 0);
        for (const auto &a : n.access) {
            if (a.mode != M_W) rd[a.buf] = 1;
            if (a.mode != M_R) wr[a.buf] = 1;
            if (covers_buffer(n, a, app.bufs[a.buf])) full[a.buf] = 1;
        }
        n.reads.clear();
        n.writes.clear();
        for (size_t b = 0; b < app.bufs.size(); ++b) {
            if (wr[b] && !full[b]) rd[b] = 1;
            if (rd[b]) n.reads.push_back((int)b);
            if (wr[b]) n.writes.push_back((int)b);
        }
        // verdict
        n.reason = RS_NONE;
        if (n.opaque_call) {
            n.verdict = V_REJECT;
            n.reason = RS_EXTERNAL_CALL;
        } else if (n.early_exit) {
            n.verdict = V_REJECT;
            n.reason = RS_BREAK;
        } else {
            bool reduction = false, dep = false;
            for (size_t b = 0; b < app.bufs.size() && !dep; ++b) {
                bool any = false, only_sum = true;
                for (const auto &a : n.access)
                    if (a.buf == (int)b) {
                        any = true;
                        only_sum &= (a.mode == M_SUM);
                    }
                if (!any) continue;
                if (only_sum) {
                    reduction = true;
                    continue;
                }
                for (const auto &w : n.access) {
                    if (w.buf != (int)b || w.mode == M_R) continue;
                    for (const auto &x : n.access) {
                        if (x.buf != (int)b) continue;
                        if (carried_dependence(n, w, x)) {
                            dep = true;
                            break;
                        }
                    }
                    if (dep) break;
                }
            }
            if (dep) {
                n.verdict = V_REJECT;
                n.reason = RS_DATA_DEP;
            } else {
                n.verdict = reduction ? V_PARALLEL_REDUCTION : V_PARALLEL;
            }
        }
        // a nest that only has a host form (compiled from its own source)
        // stays on the CPU even when its loop could run in parallel
        if (n.verdict != V_REJECT && n.op == OP_HOST_CODE) {
            n.verdict = V_REJECT;
            n.reason = RS_NO_KERNEL;
        }
        n.gene_pos = (n.verdict == V_REJECT) ? -1 : pos++;
    }
    app.gene_len = pos;
}

}  // namespace ofl
