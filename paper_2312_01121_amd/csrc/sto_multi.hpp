// The persistent multi-stream kernel as the forward of the multi-stream
// adjoint: one segment of whole input samples, optionally writing the stage
// trace that the reversed stages read.
#pragma once

#include "sto_adjoint_dev.hpp"
#include "sto_internal.hpp"

namespace sto {

// Stage trace of a segment, laid out as the adjoint's kernels expect.
struct MultiTrace {
    float* xt;   // [step][stage][stream][3][ld] stage inputs, or nullptr: no trace
    float* wx;   // [step][stage][stream][C][ld] coupling sums before a_cp
    float* pn;   // [step][stream][ld] norm before the projection (renormalised runs)
};

// Whether the traced kernel can run n x streams (all tiles co-resident).
bool multi_segment_fits(int n, int streams, int xyz);

// r.samples whole samples from the state in d.m (left there at the end);
// sample0 is the global index of the first sample (reported on a non-finite
// state).  The caller checks multi_segment_fits first when tr.xt is set.
hipError_t run_multi_segment(const DevState<float>& d, const Coef<float>& k, const RunSpec& r, int streams,
                             int sample0, const MultiTrace& tr);

// Whether k_multi_rev runs n nodes x S streams with n_in input channels.
bool multi_reverse_fits(int n, int streams, int xyz, int n_in);

// All reversed stages of one segment of kn steps, from (kn - 1, 3) down to
// (0, 0), in one cooperative launch (xchg: 3 C S ld floats, sync: 256
// bytes); the bbar of (kn - 1, 3) must be in d.st.  Requires
// multi_reverse_fits.
hipError_t run_multi_reverse(const AdjDev<float>& d, const Coef<float>& k, int kn, int xyz, float* xchg, int* sync,
                             hipStream_t stream);

}  // namespace sto
