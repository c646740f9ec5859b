// Internal (C++) interface between the C-ABI runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sto_device.hpp"

namespace sto {

// Device buffers of one reservoir, in the handle's arithmetic type T.
//   W      n rows x ld columns, row-major; columns n..ld-1 are zero
//   w_in   n x n_in, row-major
//   m      current state, SoA: m[c*ld + k] for component c of node k
//          (streams > 1: m[(s*3 + c)*ld + k] for stream s)
//   ms[2]  RK4 stage inputs (ping-pong), same layout as m; entries k >= n
//          stay zero, so the padded columns of W meet zeros
//   acc    RK4 accumulator k1 + 2k2 + 2k3, same layout
template <typename T>
struct DevState {
    const T* W;
    const T* w_in;
    T* m;
    T* ms[2];
    T* acc;
    T* xchg;         // resident/multi paths: 3 rotating stage-input buffers
    int* bad;        // first sample index whose state is not finite (INT_MAX: none)
    int* sync;       // grid-barrier words (cooperative kernels)
    int n, n_in;
    int64_t ld;
};

// SWEEP path: per-reservoir offsets into the concatenated device arrays.
struct SweepRes {
    int n;             // nodes
    int pad;
    int64_t ld;        // row pitch of W and of the state arrays (n rounded up to 64)
    int64_t woff;      // element offset of W (n x ld)
    int64_t soff;      // element offset of m, ms[], acc (3 x ld each)
    int64_t winoff;    // element offset of w_in (n x n_in)
    int64_t noff;      // nodes of the reservoirs before this one
};

// One wave task of the sweep: consecutive rows of one reservoir.  It
// carries the offsets its coupling pass needs, so the loads of W can start
// after this one table read.
struct SweepTask {
    int64_t woff;      // element offset of the reservoir's W
    int64_t soff;      // element offset of its m, ms[], acc
    int ld;            // row pitch
    int n;             // nodes of the reservoir
    int res;           // reservoir index (constants, w_in, records)
    int row;           // first row of the task
    int rpg;           // rows per lane group (2, 4 or 8)
    int pad;
};

template <typename T>
struct SweepDev {
    const T* W;
    const T* w_in;
    T* m;
    T* ms[2];
    T* acc;
    T* states;         // records [reservoir][sample][node][3], or nullptr
    int* bad;
    const SweepRes* res;
    const Coef<T>* coef;
    const SweepTask* task;   // every wave task
    int tasks;
    int n_in;
    int64_t rec_samples;   // samples of the current run (record layout)
    int* sample;           // device: index of the input sample being stepped
};

struct RunSpec {
    const double* u;     // device, samples x n_in
    void* states;        // device, samples x n x 3 (T), or nullptr
    int samples;
    int substeps;
    int cur;             // which ms buffer holds the current state
    int renorm;
    int xyz;
    hipStream_t stream;
    // persistent paths: device-clock stamps of the exchange phases of the
    // first trace_stages stages, 4 per stage and workgroup (nullptr: none)
    unsigned long long* trace = nullptr;
    int trace_stages = 0;
    int trace_groups = 0;    // workgroups the trace buffer holds
};

// Launch-shape choices, fixed defaults overridable through the environment
// for measurements (STO_STREAM_ALTERNATE, STO_STREAM_NT: 0 or 1;
// STO_STREAM_ROWS, STO_STREAM_UNROLL: a compiled variant).
struct Tune {
    int stream_alternate;    // reverse the row order of the stream kernel on odd stages
    int stream_nontemporal;  // W loads: 1 non-temporal, 0 cached, -1 by the size of W
    int stream_rows;         // rows per wave of the stream kernel (0: default)
    int stream_unroll;       // column-loop unroll of the stream kernel (0: default)
};
const Tune& tune();
// Process-wide override of the stream kernel shape (0, 0: table).
bool set_stream_variant(int rows, int unroll);
// Rows per wave and unroll of the stream kernels for element size and n.
void stream_shape(int elem_bytes, int n, int* rows, int* unroll);

// Path launchers; each returns the HIP status of its launches.
template <typename T> hipError_t run_stream(const DevState<T>& d, const Coef<T>& k, const RunSpec& r);
template <typename T> hipError_t run_small(const DevState<T>& d, const Coef<T>& k, const RunSpec& r);
template <typename T> hipError_t run_resident(const DevState<T>& d, const Coef<T>& k, const RunSpec& r);

// MULTI path (S streams, FP32 MFMA): whether n x streams fits and runs.
bool multi_fits(int n, int streams, int xyz, int* grid_x, int* grid_y);
hipError_t run_multi(const DevState<float>& d, const Coef<float>& k, const RunSpec& r, int streams);

// SWEEP path launcher (one launch per RK4 stage over every reservoir).
// With a capture stream, the launches of `graph_samples` samples are
// captured once into a HIP graph that is replayed on r.stream (the caller
// destroys *graph and *exec after the stream has finished); without, every
// launch is issued directly.
template <typename T>
hipError_t run_sweep(const SweepDev<T>& d, const RunSpec& r, hipStream_t capture, int graph_samples,
                     hipGraph_t* graph, hipGraphExec_t* exec);

// Largest n the single-workgroup kernel holds (W in LDS).
int small_max_n(int elem_bytes, int xyz);
// Measured path for a single-stream reservoir of n nodes (sto_path value:
// 1 small, 2 resident, 3 stream; 0 if no table entry) and, for the resident
// path, its measured waves per workgroup and rows per workgroup (0: ceil(n /
// CUs)).
int tuned_path(int elem_bytes, int xyz, int n, int* waves, int* rpb, int* split = nullptr);
// Whether the resident kernel can hold n on this device (W split across
// co-resident workgroups' LDS); fills the chosen grid size.
bool resident_fits(int n, int elem_bytes, int xyz, int* grid_out);
// The resident kernel's launch shape for n (grid, rows per workgroup,
// threads per workgroup); false if it does not fit.
bool resident_shape(int n, int elem_bytes, int xyz, int* grid_out, int* rpb_out, int* block_out,
                    int* split_out = nullptr);

// Offset (in ints) of the abort flag in DevState::sync; non-zero after a
// resident run means a grid barrier timed out.
constexpr int kSyncAbortWord = 32;

// Attainable HBM read bandwidth of a plain streaming kernel (GB/s).
hipError_t read_bandwidth(int64_t bytes, int reps, double* gbs);

// Readout (FP64): see readout.hip.
// rec_dev: rows x n x 3 records of type rec_f32 ? float : double; y_dev:
// rows targets; w_dev: cols weights.  Returns 0 on success, 1 if the
// normal-equation matrix is not positive definite, 2 on a HIP error
// (message in *err), 3 if a record or target is not finite.
int readout_solve(const void* rec_dev, int rec_f32, int rows, int n, int features, const double* y_dev,
                  double lam, double* w_dev, double* nmse_host, hipStream_t stream, const char** err);

}  // namespace sto
