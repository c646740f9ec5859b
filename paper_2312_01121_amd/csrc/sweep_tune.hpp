// Rows per lane group and row pitch of the sweep kernel by element type and
// reservoir size, chosen by measurement.  Written by
// paper_2312_01121_amd/autotune.py --sweep, which times candidate tables on
// the 256-reservoir FP32 sweep workload (N log-uniform in [32, 2048]) and
// keeps the fastest; FP64 sweeps keep 8 rows and a 64-element pitch.
// Entries are scanned in order and the first with n <= n_max applies.
#pragma once

namespace sto {

struct SweepTuneEntry {
    int elem_bytes;
    int n_max;
    int rows;    // rows of W per lane group (2, 4 or 8)
    int pitch;   // row pitch of W and the state, in elements (a multiple of 16 bytes)
};

constexpr SweepTuneEntry kSweepTune[] = {
    {4, 1073741824, 8, 32},
    {8, 1073741824, 8, 64},
};

// Measured (candidate table n_max:rows:pitch,...): us per RK4 step of the sweep
// {"1073741824:4:64": 364.68, "1073741824:8:16": 348.13, "1073741824:8:32": 338.91, "1073741824:8:64": 341.44, "1792:8:32,1073741824:4:32": 341.28, "192:8:16,1073741824:8:32": 338.91, "192:8:16,1073741824:8:64": 341.65, "48:8:16,1073741824:8:64": 341.53}

}  // namespace sto
