// Layout of the SWEEP path in device memory, computed on the host.
#pragma once

#include <stdint.h>

#include <vector>

#include "sto_internal.hpp"

namespace sto {

// Device layout of a sweep of `count` reservoirs of n[r] nodes and n_in
// input channels: each reservoir's row pitch (rows per lane group and pitch
// from the measured table, STO_SWEEP_ROWS / STO_SWEEP_PITCH /
// STO_SWEEP_TABLE for measurements) and its offsets into the concatenated
// arrays, every reservoir's W and state starting on a 256-byte boundary; the
// wave tasks in reservoir order; and the element counts of the concatenated
// W, state (per array of m, ms[], acc) and w_in arrays.
struct SweepLayout {
    std::vector<SweepRes> res;
    std::vector<SweepTask> tasks;
    int64_t w_elems = 0, s_elems = 0, win_elems = 0, nodes = 0;
};

SweepLayout sweep_layout(int elem_bytes, int count, const int64_t* n, int n_in);

}  // namespace sto
