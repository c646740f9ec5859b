// Internal interface of the adjoint (reverse-mode gradient) of the RK4
// trajectory: the host runtime fills an AdjArgs and calls adjoint_run.
#pragma once

#include "sto_internal.hpp"

namespace sto {

template <typename T>
struct AdjArgs {
    // reservoir (device, the handle's buffers; read only)
    const T* W;          // n x ld, row-major, zero padding
    const T* Wt;         // n x ld, the transpose of W, zero padding
    const T* w_in;       // n x n_in
    int n, n_in;
    int streams;         // S input streams sharing W (S > 1: FP32 only)
    int64_t ld;
    Coef<T> k;
    int substeps, renorm, xyz;
    // run
    const double* u;     // device, (steps / substeps) x S x n_in
    int64_t steps;
    const T* m_start;    // device, S x n x 3 AoS
    const T* g_rec;      // device, (steps / substeps) x S x n x 3 AoS: dL/d(record); or nullptr
    const T* g_fin;      // device, S x n x 3 AoS: dL/d(final state); or nullptr
    const T* records;    // device, (steps / substeps) x S x n x 3 AoS: the run's records, which then serve as
                         // the segments' checkpoints (seg_steps a multiple of substeps); or nullptr
    // outputs (device; each may be nullptr)
    T* g_W;              // n x n, row-major, no padding
    T* g_win;            // n x n_in
    T* g_m0;             // S x n x 3 AoS
    double* g_scal;      // 4: a_cp, a_in, h_s, h_appl
    int64_t seg_steps;   // RK4 steps per recomputed segment (>= 1)
    int* bad;            // device flag: first non-finite sample (INT_MAX: none)
    hipStream_t stream;
    int* kernels;        // host, or nullptr: receives the ADJ_* kernel families the call ran
};

// Kernel families an adjoint call ran (bit mask; reservoir_adjoint_kernels).
enum : int {
    ADJ_FWD_STAGE = 1,        // forward passes with one launch per RK4 stage
    ADJ_FWD_PERSISTENT = 2,   // forward passes in one persistent launch per segment
    ADJ_REV_STAGE = 4,        // reversed stages with one launch per stage
    ADJ_REV_PERSISTENT = 8,   // reversed stages in one persistent launch per segment
};

// Bytes of the per-step stage trace (the workspace per step of a segment).
int64_t adjoint_trace_bytes_per_step(int64_t ld, int elem_bytes, int xyz, int streams);

template <typename T>
hipError_t transpose_matrix(const T* W, T* Wt, int n, int64_t ld, hipStream_t st);

// Runs the forward from m_start with checkpoints, then reverses it segment
// by segment.  Allocates and frees its own workspace.
template <typename T>
hipError_t adjoint_run(const AdjArgs<T>& a);

// One plain run of the BATCH path (S streams, one launch per RK4 stage,
// coupling of all streams as one FP32 MFMA product; sto_batch.hip).
struct BatchRun {
    const float* W;      // n x ld
    const float* Wt;     // n x ld, transpose of W
    const float* w_in;   // n x n_in
    float* m;            // [S][3][ld]
    float* ms[2];        // [S][3][ld]; the state is in ms[cur] between steps
    float* acc;          // [S][3][ld]
    int* bad;
    const double* u;     // samples x S x n_in
    float* states;       // samples x S x n x 3, or nullptr
    Coef<float> k;
    int n, n_in, streams, substeps, renorm, xyz, samples, cur;
    int64_t ld;
    hipStream_t stream;
};
hipError_t run_batch(const BatchRun& b);

// Gradient of the ridge objective at its optimum with respect to the records
// (readout.hip).  rec_dev: T x n x 3 records (FP32 if rec_f32); w_dev: the
// fitted weights; grad_dev: T x n x 3 of the same type; loss_host may be null.
hipError_t readout_grad(const void* rec_dev, int rec_f32, int T, int washout, int n, int features,
                        const double* y_dev, const double* w_dev, double lambda, void* grad_dev, double* loss_host,
                        hipStream_t stream);

}  // namespace sto
