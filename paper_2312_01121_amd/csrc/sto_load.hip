// Loading a handle's arrays from caller device buffers of doubles: the
// coupling matrix W of Eq. (coup) and the input weights of Eq. (in) into the
// handle's element type and row pitch (zero padding), the state from the
// array-of-structures layout of the entry points into the structure-of-arrays
// layout of the kernels.  One coalesced pass over each array: a workgroup
// per row (per 256 nodes for the state).  Non-finite values, and states off
// the unit sphere where the caller asks for that check, set bits of a flag
// word that the host reads after the stream has finished.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "sto_load.hpp"

namespace sto {

namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_load_rows(const double* __restrict__ src, int64_t rows, int64_t cols,
                                                   T* __restrict__ dst, int64_t ld, int* flags) {
    bool bad = false;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const double* s = src + row * cols;
        T* d = dst + row * ld;
        for (int64_t c = threadIdx.x; c < ld; c += 256) {
            double v = 0.0;
            if (c < cols) {
                v = s[c];
                bad |= !isfinite(v);
            }
            d[c] = (T)v;
        }
    }
    if (bad) atomicOr(flags, kLoadNonFinite);
}

// Thread per (stream, node) of the padded state: node k < n reads its three
// components, k in [n, ld) writes the zero padding.
template <typename T>
__global__ void __launch_bounds__(256) k_load_state(const double* __restrict__ m_aos, int64_t n, int64_t streams,
                                                    int64_t ld, T* __restrict__ m, T* __restrict__ ms,
                                                    int check_norm, int* flags) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= streams * ld) return;
    const int64_t st = i / ld, k = i - st * ld;
    double v[3] = {0.0, 0.0, 0.0};
    if (k < n) {
        const double* p = m_aos + (st * n + k) * 3;
        v[0] = p[0];
        v[1] = p[1];
        v[2] = p[2];
        int f = 0;
        if (!isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2])) f |= kLoadNonFinite;
        else if (check_norm && fabs(sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - 1.0) > 1e-12) f |= kLoadOffSphere;
        if (f) atomicOr(flags, f);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t o = (st * 3 + c) * ld + k;
        m[o] = (T)v[c];
        if (ms) ms[o] = (T)v[c];
    }
}

}  // namespace

template <typename T>
hipError_t load_matrix(const double* src, int64_t rows, int64_t cols, T* dst, int64_t ld, int* flags,
                       hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>(rows, 16384);
    hipLaunchKernelGGL(k_load_rows<T>, dim3(grid), dim3(256), 0, st, src, rows, cols, dst, ld, flags);
    return hipGetLastError();
}

template <typename T>
hipError_t load_state(const double* m_aos, int64_t n, int64_t streams, int64_t ld, T* m, T* ms, int check_norm,
                      int* flags, hipStream_t st) {
    const int64_t total = streams * ld;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_load_state<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, m_aos, n, streams,
                       ld, m, ms, check_norm, flags);
    return hipGetLastError();
}

template hipError_t load_matrix<double>(const double*, int64_t, int64_t, double*, int64_t, int*, hipStream_t);
template hipError_t load_matrix<float>(const double*, int64_t, int64_t, float*, int64_t, int*, hipStream_t);
template hipError_t load_state<double>(const double*, int64_t, int64_t, int64_t, double*, double*, int, int*,
                                       hipStream_t);
template hipError_t load_state<float>(const double*, int64_t, int64_t, int64_t, float*, float*, int, int*,
                                      hipStream_t);

}  // namespace sto
