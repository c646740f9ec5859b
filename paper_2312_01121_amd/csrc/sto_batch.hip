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
// Tiling.  The columns of X are (stream, component) pairs.  Workgroup
// (bi, bj) owns nodes 16 bi .. 16 bi + 15 against 16 columns: 16 streams of
// one component, or 5 streams of three components with the 16th column
// empty.  The contraction over the nodes j runs in blocks of 256 staged
// through LDS with coalesced loads (M = W^T for W X, M = W for W^T Bbar:
// rows of M are contiguous in i; X's rows are contiguous in j); per MFMA step
// lane l supplies A[l%16][l/16] = M[j][i] and B[l/16][l%16] = X[column][j]
// from LDS, and the eight waves take alternate steps.  Their partial tiles
// meet in LDS and are summed in a fixed order; one thread per (node, stream)
// pair then takes its C columns.  W (1 MB at N = 512) stays in the L2 and
// MALL between launches.
//
// Unlike the persistent multi-stream kernel (k_multi, N <= 1024), this path
// handles any N, at one launch per stage.

#include <algorithm>

#include "sto_adjoint.hpp"
#include "sto_adjoint_dev.hpp"

namespace sto {

namespace {

typedef float bf4 __attribute__((ext_vector_type(4)));

constexpr int kT = 16;   // tile edge (nodes and columns)

// Streams per workgroup: the 16 columns hold SPW streams of C components.
template <int C> constexpr int batch_spw() { return C == 3 ? 5 : 16; }

// Partial products of the tile, the contraction over the nodes j taken in
// blocks of kJB staged through LDS, and summed across the waves.  M: n x ld
// (rows j, contiguous in i); X: stream s, component c at X + s * xs + c * xc
// (contiguous in j).  Per block the workgroup loads the M rows of its 16
// nodes and the X rows of its 16 columns with coalesced 16-byte loads (X's
// rows are padded by 4 floats so that the 16 column lanes of an MFMA operand
// read fall in distinct banks); each wave then runs one eighth of the
// block's MFMA steps.  On return, out[c] holds the coupling sum of component
// c for the pair (node i0 + t/16, stream s0 + (t%16)/C) on the threads t <
// 256 whose t%16 is the pair's first column.
constexpr int kWaves = 8;
constexpr int kJB = 512;          // contraction rows per LDS block
constexpr int kXP = kJB + 4;      // padded row of the X block

struct TileLds {
    float a[kJB][kT];             // M[j][i0 .. i0 + 15]
    float x[kT][kXP];             // X[column][j], column = stream * C + component
    float cs[kWaves * kT * kT];
};

template <int C>
__device__ __forceinline__ void tile_product(const float* __restrict__ M, int64_t ld, int n, int i0,
                                             const float* __restrict__ X, int64_t xs, int64_t xc, int S, int s0,
                                             TileLds& sh, float* out) {
    constexpr int SPW = batch_spw<C>();
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kr = lane >> 4, c16 = lane & 15;
    bf4 acc = bf4{0.f, 0.f, 0.f, 0.f};
    for (int jb = 0; jb < n; jb += kJB) {
        const int tb = (min(kJB, n - jb) + 3) / 4;   // MFMA steps of this block (4 rows each)
        // A block: 4 tb rows x 16 floats, one float4 per thread and pass
        for (int e = tid; e < tb * kT; e += 64 * kWaves) {
            const int r = e >> 2, q = e & 3;
            const int j = jb + r;
            bf4 v = bf4{0.f, 0.f, 0.f, 0.f};
            if (j < n) v = *reinterpret_cast<const bf4*>(M + (int64_t)j * ld + i0 + 4 * q);
            *reinterpret_cast<bf4*>(&sh.a[r][4 * q]) = v;
        }
        // X block: 16 column rows of 4 tb floats; the empty column, streams
        // beyond S and nodes beyond n read as zero (X's rows are ld >= n long
        // and 16-byte aligned)
        for (int e = tid; e < kT * tb; e += 64 * kWaves) {
            const int col = e / tb, q = e - col * tb;
            const int sl = col / C, c = col - sl * C;
            const int j = jb + 4 * q;
            bf4 v = bf4{0.f, 0.f, 0.f, 0.f};
            if (sl < SPW && s0 + sl < S && j < n)
                v = *reinterpret_cast<const bf4*>(X + (int64_t)(s0 + sl) * xs + c * xc + j);
            *reinterpret_cast<bf4*>(&sh.x[col][4 * q]) = v;
        }
        __syncthreads();
        // MFMA steps of 4 rows: wave w takes steps w, w + 8, ...
        for (int t = wave; t < tb; t += kWaves) {
            const int jl = 4 * t + kr;
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(sh.a[jl][c16], sh.x[c16][jl], acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // D of lane l: rows (nodes) 4 (l/16) + r, column l%16
#pragma unroll
    for (int r = 0; r < 4; ++r) sh.cs[(wave * kT + 4 * kr + r) * kT + c16] = acc[r];
    __syncthreads();
    if (tid < kT * kT) {
        const int ti = tid >> 4, tj = tid & 15;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int col = min(tj + c, kT - 1);   // stays in the tile for threads that own no pair
            float v = sh.cs[(0 * kT + ti) * kT + col];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) v += sh.cs[(w * kT + ti) * kT + col];
            out[c] = v;
        }
    }
}

// The (node, stream) pair of thread t of a tile: t < 256 and t%16 the
// first of the stream's C columns.
template <int C>
struct TilePair {
    int i, s;
    bool own;
    __device__ TilePair(int n, int S) {
        constexpr int SPW = batch_spw<C>();
        const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
        i = blockIdx.x * kT + ti;
        s = blockIdx.y * SPW + tj / C;
        own = threadIdx.x < kT * kT && tj % C == 0 && tj / C < SPW && i < n && s < S;
    }
};

// Forward stage of all streams (records for plain runs, trace for the adjoint).
template <bool XYZ>
__global__ void __launch_bounds__(512) k_bfwd(AdjDev<float> d, Coef<float> k, int kk, int stage, int cur, int trace) {
    constexpr int C = XYZ ? 3 : 1;
    __shared__ TileLds sh;
    const TilePair<C> p(d.n, d.S);
    // the epilogue's inputs do not depend on the product: load them first
    FwdIn<float> in{};
    if (p.own) in = fwd_load<float>(d, k, p.i, p.s, kk, stage, cur);
    float out[3] = {0.f, 0.f, 0.f};
    tile_product<C>(d.Wt, d.ld, d.n, blockIdx.x * kT, d.ms[cur], 3 * d.ld, d.ld, d.S, blockIdx.y * batch_spw<C>(), sh,
                    out);
    if (p.own) fwd_finish<float, XYZ>(d, k, p.i, p.s, kk, stage, cur, trace, in, out[0], out[1], out[2]);
}

// Reversed stage of all streams: W^T Bbar, then the adjoint epilogue.
template <bool XYZ>
__global__ void __launch_bounds__(512) k_brev(AdjDev<float> d, Coef<float> k, int kk, int stage) {
    constexpr int C = XYZ ? 3 : 1;
    __shared__ TileLds sh;
    const TilePair<C> p(d.n, d.S);
    // the epilogue's inputs do not depend on the product: load them first
    RevIn<float> in{};
    if (p.own) in = rev_load<float, XYZ>(d, p.i, p.s, kk, stage);
    const float* bbar = d.st + adj_slot<C>(kk, stage, d.S, d.ld);
    float out[3] = {0.f, 0.f, 0.f};
    tile_product<C>(d.W, d.ld, d.n, blockIdx.x * kT, bbar, C * d.ld, d.ld, d.S, blockIdx.y * batch_spw<C>(), sh, out);
    GlobalSink sink;
    if (p.own) rev_finish<float, XYZ>(d, k, p.i, p.s, kk, stage, in, out[0], out[1], out[2], sink);
}

}  // namespace

static dim3 batch_grid(const AdjDev<float>& d, int xyz) {
    const int spw = xyz ? batch_spw<3>() : batch_spw<1>();
    return dim3((d.n + kT - 1) / kT, (d.S + spw - 1) / spw);
}

void launch_batch_fwd(const AdjDev<float>& d, const Coef<float>& k, int kk, int stage, int cur, int trace, int xyz,
                      hipStream_t st) {
    const dim3 grid = batch_grid(d, xyz), block(64 * kWaves);
    if (xyz)
        hipLaunchKernelGGL(k_bfwd<true>, grid, block, 0, st, d, k, kk, stage, cur, trace);
    else
        hipLaunchKernelGGL(k_bfwd<false>, grid, block, 0, st, d, k, kk, stage, cur, trace);
}

void launch_batch_rev(const AdjDev<float>& d, const Coef<float>& k, int kk, int stage, int xyz, hipStream_t st) {
    const dim3 grid = batch_grid(d, xyz), block(64 * kWaves);
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
