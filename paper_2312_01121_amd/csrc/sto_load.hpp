// Loading a handle's W, w_in and state from device buffers of doubles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sto {

// Bits of the flag word the load kernels set (atomic OR; the caller clears it).
constexpr int kLoadNonFinite = 1;   // a value is NaN or infinite
constexpr int kLoadOffSphere = 2;   // | |m_k| - 1 | > 1e-12 (state loads that check it)

// dst (rows x ld, element type T) <- src (rows x cols doubles, row-major),
// zeros in columns [cols, ld).
template <typename T>
hipError_t load_matrix(const double* src, int64_t rows, int64_t cols, T* dst, int64_t ld, int* flags,
                       hipStream_t st);

// m (and ms unless NULL), [stream][xyz][ld] <- m_aos [stream][node][xyz] of
// n nodes, zeros in nodes [n, ld).
template <typename T>
hipError_t load_state(const double* m_aos, int64_t n, int64_t streams, int64_t ld, T* m, T* ms, int check_norm,
                      int* flags, hipStream_t st);

}  // namespace sto
