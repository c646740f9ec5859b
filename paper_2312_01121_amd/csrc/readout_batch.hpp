// Many ridge readouts fitted together (readout_fit_batch_device).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace sto {

// Fit `count` readouts.  Item i's fitted rows are records rec[i] + r *
// stride[i] (elements), r < rows, each n[i] x 3 AoS (FP32 if rec_f32,
// else FP64); y[i] (device) holds the rows' targets; w_dev[i]
// receives the item's F + 1 weights and nmse_host[i] its NMSE.  Returns 0,
// or as readout_solve: 1 not positive definite, 2 device error, 3
// non-finite input; *bad_item is then the first item concerned (-1 for a
// device error).
int readout_solve_batch(int count, const void* const* rec, const int64_t* stride, int rec_f32, int rows,
                        const int64_t* n, int features, const double* const* y, double lam, double* const* w_dev,
                        double* nmse_host, hipStream_t stream, const char** err, int* bad_item);

}  // namespace sto
