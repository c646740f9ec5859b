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

// Bytes of device workspace one batched fit of these items needs.
size_t readout_workspace_bytes(int count, const int64_t* n, int rows, int features);

// The allocation-free fit of one record set (readout_fit_device_noalloc):
// the same kernels as readout_solve_batch, with their workspace in the
// library's static scratch array of kReadoutScratchBytes on the current
// device.  Returns as readout_solve_batch, or 4 when the workspace would
// exceed the scratch.  Concurrent calls on one device share the scratch
// and race.
constexpr size_t kReadoutScratchBytes = size_t(96) << 20;
int readout_solve_scratch(const void* rec, int rec_f32, int rows, int64_t n, int features, const double* y,
                          double lam, double* w_dev, double* nmse_host, hipStream_t stream, const char** err);
// Device address of the scratch array on the current device (resolved with
// hipGetSymbolAddress on the first call per device).
hipError_t readout_scratch_address(void** ptr);

}  // namespace sto
