// Transfer planning: the ordered list of copies, kernel launches and host
// nest executions one gene implies (repeats expanded).
#pragma once

#include <cstdint>
#include <vector>

#include "ir.hpp"

namespace ofl {

enum StepKind { ST_H2D = 0, ST_D2H = 1, ST_GPU = 2, ST_CPU = 3 };

struct Step {
    StepKind kind;
    int idx;            // buffer (copies) or nest (executions)
    int env;            // offset into Plan::env (values of the repeat variables)
    int box = -1;       // copies: index into Plan::boxes, -1 = the whole buffer
};

// A box of a buffer: per dimension the index range [lo, hi).
struct Box {
    std::vector<int64_t> lo, hi;
};

struct Plan {
    std::vector<Step> steps;
    std::vector<int64_t> env;        // repeat-variable values, one block per nest step
    std::vector<Box> boxes;          // sections copied by SECTIONS-policy steps
    uint64_t h2d = 0, d2h = 0;
    int32_t copies = 0, launches = 0, host_nests = 0;
    // Whether the set-up content of a buffer's host / device copy is consumed
    // before that copy is overwritten (only then must it be restored).
    std::vector<char> host_init_used, dev_init_used;
    // State of every buffer after the run.
    std::vector<char> host_valid, dev_valid;
};

// Bytes of buffer `buf` inside box `bx`.
uint64_t box_bytes(const Buffer &buf, const Box &bx);

// placement[nest] = 1 for GPU.  policy: OFL_POLICY_*; flags: OFL_RUN_*.
void build_plan(const AppIR &app, const std::vector<uint8_t> &placement, int policy, int flags, Plan &out);

}  // namespace ofl
