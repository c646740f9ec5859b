// The resident (cooperative, W in LDS) kernels as the adjoint uses them: the
// recompute of a segment with its stage trace, and the reversed stages of a
// segment, each in one cooperative launch (sto_resident.hip).
#pragma once

#include "sto_adjoint_dev.hpp"
#include "sto_internal.hpp"

namespace sto {

// Where the traced forward writes the adjoint's stage trace (AdjDev layout
// with one stream): stage inputs xt [step][stage][3][ld], raw coupling sums
// wx [step][stage][C][ld], norms before the projection pn [step][ld].
template <typename T>
struct ResTrace {
    T* xt;
    T* wx;
    T* pn;
};

// Whether one stream of n nodes runs on the persistent adjoint kernels (both
// the traced forward and the reverse have a co-resident shape); the reverse
// keeps the per-node parameter partials of up to 4 input channels in registers.
bool resident_adjoint_fits(int n, int elem_bytes, int xyz, int n_in);

// Recompute of `samples` whole input samples from the state in d.m / d.ms[0]
// (u: the segment's first sample), writing the trace; the final state is left
// in d.m and d.ms[0].  sample0: global index of the segment's first sample
// (for the non-finite report).
template <typename T>
hipError_t run_resident_traced(const DevState<T>& d, const Coef<T>& k, const RunSpec& r, const ResTrace<T>& tr,
                               int sample0);

// The 4 kn reversed stages of one segment (AdjDev with S = 1), from (kn - 1, 3)
// down to (0, 0); d.st at (kn - 1, 3) holds the first stage's coupling
// adjoint (k_adj_prep).  xbuf: 3 x C x ld exchange buffers; sync: 256 bytes,
// abort word at kSyncAbortWord.
template <typename T>
hipError_t run_resident_reverse(const AdjDev<T>& d, const Coef<T>& k, int kn, int xyz, T* xbuf, int* sync,
                                hipStream_t st);

}  // namespace sto
