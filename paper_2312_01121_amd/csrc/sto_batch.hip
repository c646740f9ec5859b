// S input streams driving S copies of one reservoir, one launch per RK4
// stage (the BATCH path, and the forward and reversed stages of the
// multi-stream adjoint).  Per stage the coupling of all streams is one
// matrix product, C = a_cp W X with X the N x (S C) block of stage inputs
// (paper, Eq. (coup); Sec. 3.3 writes the single-stream case as W^cp x),
// evaluated on the matrix cores in FP32 (v_mfma_f32_16x16x4f32, FP32
// accumulation); the reversed stage forms W^T Bbar the same way.  Each
// element of the product feeds the pointwise epilogue of its (node, stream)
// pair: the right-hand side of Eq. (gov) and the RK4 bookkeeping (Sec. 3.2),
// or their adjoint.
//
// Tiling.  Workgroup (bi, bj) owns nodes 16 bi .. 16 bi + 15 and streams
// 16 bj .. 16 bj + 15.  Its four waves split the contraction over the nodes
// j into quarters; per MFMA step lane l supplies A[l%16][l/16] = M[j][i]
// (M = W^T for W X, M = W for W^T Bbar; rows of M are contiguous in i, so 16
// lanes read 64 consecutive bytes) and B[l/16][l%16] = X[s][c][j].  The four
// partial tiles meet in LDS and are summed in a fixed order; thread t then
// owns the pair (node 16 bi + t/16, stream 16 bj + t%16).  W (1 MB at
// N = 512) stays in the L2 and MALL between launches.
//
// Unlike the persistent multi-stream kernel (k_multi, x coupling only), this
// path handles both couplings and any N, at one launch per stage.

#include <algorithm>

#include "sto_adjoint.hpp"
#include "sto_adjoint_dev.hpp"

namespace sto {

namespace {

typedef float bf4 __attribute__((ext_vector_type(4)));

constexpr int kT = 16;   // tile edge (nodes and streams)

// Partial products of the tile over one quarter of the contraction, summed
// across the four waves in LDS.  M: n x ld (rows j, contiguous in i); X:
// stream s, component c at X + s * xs + c * xc (contiguous in j).  On return
// out[c] holds the (node i0 + t/16, stream s0 + t%16) element for thread t.
template <int C>
__device__ __forceinline__ void tile_product(const float* __restrict__ M, int64_t ld, int n, int i0,
                                             const float* __restrict__ X, int64_t xs, int64_t xc, int S, int s0,
                                             float* cs, float* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kr = lane >> 4, c16 = lane & 15;
    const int steps = (n + 3) / 4;             // MFMA steps of 4 nodes over the contraction
    const int per = (steps + 3) / 4;           // steps of one wave
    const int t0 = wave * per, t1 = min(steps, t0 + per);
    const int i = i0 + c16;                    // i < ld: i0 + 15 < n rounded up to 16 <= ld
    const int s = min(s0 + c16, S - 1);        // clamped; masked below
    const bool vs = s0 + c16 < S;
    bf4 acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = bf4{0.f, 0.f, 0.f, 0.f};
    for (int t = t0; t < t1; ++t) {
        const int j = 4 * t + kr;
        const bool vj = j < n;
        const int jc = vj ? j : n - 1;
        const unsigned ma = vj ? 0xffffffffu : 0u, mb = (vj && vs) ? 0xffffffffu : 0u;
        const float a = __uint_as_float(__float_as_uint(M[(int64_t)jc * ld + i]) & ma);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float b = __uint_as_float(__float_as_uint(X[(int64_t)s * xs + c * xc + jc]) & mb);
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
        }
    }
    // D of lane l: rows (nodes) 4 (l/16) + r, column (stream) l%16
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) cs[((wave * C + c) * kT + 4 * kr + r) * kT + c16] = acc[c][r];
    __syncthreads();
    const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
#pragma unroll
    for (int c = 0; c < C; ++c)
        out[c] = ((cs[((0 * C + c) * kT + ti) * kT + tj] + cs[((1 * C + c) * kT + ti) * kT + tj]) +
                  cs[((2 * C + c) * kT + ti) * kT + tj]) +
                 cs[((3 * C + c) * kT + ti) * kT + tj];
}

// Forward stage of all streams (records for plain runs, trace for the adjoint).
template <bool XYZ>
__global__ void __launch_bounds__(256) k_bfwd(AdjDev<float> d, Coef<float> k, int kk, int stage, int cur, int trace) {
    constexpr int C = XYZ ? 3 : 1;
    __shared__ float cs[4 * C * kT * kT];
    const int i0 = blockIdx.x * kT, s0 = blockIdx.y * kT;
    float out[3] = {0.f, 0.f, 0.f};
    tile_product<C>(d.Wt, d.ld, d.n, i0, d.ms[cur], 3 * d.ld, d.ld, d.S, s0, cs, out);
    const int i = i0 + (threadIdx.x >> 4), s = s0 + (threadIdx.x & 15);
    if (i < d.n && s < d.S) fwd_epilogue<float, XYZ>(d, k, i, s, kk, stage, cur, trace, out[0], out[1], out[2]);
}

// Reversed stage of all streams: W^T Bbar, then the adjoint epilogue.
template <bool XYZ>
__global__ void __launch_bounds__(256) k_brev(AdjDev<float> d, Coef<float> k, int kk, int stage) {
    constexpr int C = XYZ ? 3 : 1;
    __shared__ float cs[4 * C * kT * kT];
    const int i0 = blockIdx.x * kT, s0 = blockIdx.y * kT;
    const float* bbar = d.st + adj_slot<C>(kk, stage, d.S, d.ld);
    float out[3] = {0.f, 0.f, 0.f};
    tile_product<C>(d.W, d.ld, d.n, i0, bbar, C * d.ld, d.ld, d.S, s0, cs, out);
    const int i = i0 + (threadIdx.x >> 4), s = s0 + (threadIdx.x & 15);
    if (i < d.n && s < d.S) rev_epilogue<float, XYZ>(d, k, i, s, kk, stage, out[0], out[1], out[2]);
}

}  // namespace

void launch_batch_fwd(const AdjDev<float>& d, const Coef<float>& k, int kk, int stage, int cur, int trace, int xyz,
                      hipStream_t st) {
    const dim3 grid((d.n + kT - 1) / kT, (d.S + kT - 1) / kT), block(256);
    if (xyz)
        hipLaunchKernelGGL(k_bfwd<true>, grid, block, 0, st, d, k, kk, stage, cur, trace);
    else
        hipLaunchKernelGGL(k_bfwd<false>, grid, block, 0, st, d, k, kk, stage, cur, trace);
}

void launch_batch_rev(const AdjDev<float>& d, const Coef<float>& k, int kk, int stage, int xyz, hipStream_t st) {
    const dim3 grid((d.n + kT - 1) / kT, (d.S + kT - 1) / kT), block(256);
    if (xyz)
        hipLaunchKernelGGL(k_brev<true>, grid, block, 0, st, d, k, kk, stage);
    else
        hipLaunchKernelGGL(k_brev<false>, grid, block, 0, st, d, k, kk, stage);
}

hipError_t run_batch(const BatchRun& b) {
    AdjDev<float> d{};
    d.W = b.W;
    d.Wt = b.Wt;
    d.w_in = b.w_in;
    d.m = b.m;
    d.ms[0] = b.ms[0];
    d.ms[1] = b.ms[1];
    d.acc = b.acc;
    d.bad = b.bad;
    d.u = b.u;
    d.rec = b.states;
    d.n = b.n;
    d.n_in = b.n_in;
    d.substeps = b.substeps;
    d.renorm = b.renorm;
    d.S = b.streams;
    d.ld = b.ld;
    d.steps = (int64_t)b.samples * b.substeps;
    // the state is in ms[cur] between steps; a step's four stages alternate
    // ms[cur] -> ms[cur^1] -> ms[cur] -> ms[cur^1] -> ms[cur]
    for (int64_t j = 0; j < d.steps; ++j) {
        d.j0 = j;
        for (int stage = 0; stage < 4; ++stage)
            launch_batch_fwd(d, b.k, 0, stage, b.cur ^ (stage & 1), 0, b.xyz, b.stream);
    }
    return hipGetLastError();
}

}  // namespace sto
