// Launch shapes of the streaming kernels by element type and size, chosen
// by measurement.  Written by paper_2312_01121_amd/autotune.py; entries are
// scanned in order and the first with n <= n_max applies.
#pragma once

namespace sto {

struct StreamTuneEntry {
    int elem_bytes;
    int n_max;
    int rows;
    int unroll;
};

// Sweep at N = 10,000 on MI355X (rows x unroll over the compiled variants).
constexpr StreamTuneEntry kStreamTune[] = {
    {4, 1 << 30, 2, 2},
    {8, 1 << 30, 2, 4},
};

}  // namespace sto
