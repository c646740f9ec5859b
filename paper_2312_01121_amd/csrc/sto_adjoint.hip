// Adjoint (reverse-mode gradient) of the RK4 trajectory of N coupled
// spin-torque oscillators: exact derivatives of the discrete map of
// Eq. (gov) with the coupling of Eq. (coup) and the input of Eq. (in),
// classic RK4 (paper, Sec. 3.1 and 3.2), for a loss given through its
// gradient on the records.
//
// Reverse of one step from m (stage inputs x1..x4, k_i = F(x_i)), given
// a = dL/dm' after the optional projection has been reversed:
//   kbar4 = (dt/6) a,                 xbar4 = dF(x4)^T kbar4
//   kbar3 = (dt/3) a + dt   xbar4,    xbar3 = dF(x3)^T kbar3
//   kbar2 = (dt/3) a + dt/2 xbar3,    xbar2 = dF(x2)^T kbar2
//   kbar1 = (dt/6) a + dt/2 xbar2,    xbar1 = dF(x1)^T kbar1
//   dL/dm = a + xbar1 + xbar2 + xbar3 + xbar4
// with dF(x)^T v = (pointwise part at x) + a_cp W^T bbar along the coupled
// components, bbar being the adjoint of the effective field b.
//
// Schedule.  Pass 1 runs the forward from m_start and stores a checkpoint
// of the state at the start of every segment of seg_steps steps; the last
// segment is traced directly.  Then, from the last segment to the first:
// recompute the segment from its checkpoint while tracing every stage
// (stage input, raw coupling sums, the norm before projection), then
// reverse its steps, one launch per reversed stage.  A reversed stage
// streams the rows of W^T against the stage's bbar (the same HBM-bound
// shape as the forward stage kernel) and its epilogue applies the pointwise
// adjoint of the next stage to be reversed, so every reversed stage is one
// pass over W^T.  The per-stage bbar vectors of the segment are kept, and
// dL/dW = a_cp sum_stages outer(bbar, x) is one matrix product per segment
// (k_gw_mfma on the matrix cores in FP32, k_gw in FP64).  The scalar derivatives are accumulated per node in FP64 and
// summed in a fixed order at the end.
//
// FP64 stage sums of the forward use the same double-double accumulation as
// every other kernel, so the recomputed trajectory equals the plain run; the
// adjoint's own sums use plain fma in the arithmetic type.

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <vector>

#include "sto_adjoint.hpp"
#include "sto_adjoint_dev.hpp"
#include "sto_multi.hpp"
#include "sto_resident.hpp"

namespace sto {

namespace {

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv4 __attribute__((ext_vector_type(4)));
template <typename T> struct AVec;
template <> struct AVec<double> { using type = dv2; static constexpr int n = 2; };
template <> struct AVec<float> { using type = fv4; static constexpr int n = 4; };


// Sum over the 64 lanes of a wave (every lane ends with the total).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    return lane_sum<T>(v);
}

// ---------------------------------------------------------------------------
// Forward stage with trace (the stage kernel's shape: R rows of W per wave,
// 16-byte non-temporal loads, fused epilogue).
// ---------------------------------------------------------------------------
template <typename T, bool XYZ, int R, int U>
__global__ void __launch_bounds__(256) k_fwd_trace(AdjDev<T> d, Coef<T> k, int kk, int stage, int cur, int trace) {
    using A = Acc<T>;
    using AT = typename A::type;
    using V = typename AVec<T>::type;
    constexpr int VN = AVec<T>::n;
    const int lane = threadIdx.x & 63;
    const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * R;
    const int n = d.n;
    if (row0 >= n) return;   // wave-uniform
    const int64_t ld = d.ld;
    const T* __restrict__ xin = d.ms[cur];
    const T* wrow[R];
#pragma unroll
    for (int r = 0; r < R; ++r) wrow[r] = d.W + (int64_t)min(row0 + r, n - 1) * ld;
    AT ax[R], ay[R], az[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ax[r] = ay[r] = az[r] = A::zero();
#pragma unroll U
    for (int64_t c = (int64_t)lane * VN; c < ld; c += 64 * VN) {
        const V xv = *reinterpret_cast<const V*>(xin + c);
        V yv, zv;
        if (XYZ) {
            yv = *reinterpret_cast<const V*>(xin + ld + c);
            zv = *reinterpret_cast<const V*>(xin + 2 * ld + c);
        }
        V wv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) wv[r] = __builtin_nontemporal_load(reinterpret_cast<const V*>(wrow[r] + c));
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int e = 0; e < VN; ++e) {
                A::fma(ax[r], wv[r][e], xv[e]);
                if (XYZ) {
                    A::fma(ay[r], wv[r][e], yv[e]);
                    A::fma(az[r], wv[r][e], zv[e]);
                }
            }
    }
    T dx = T(0), dy = T(0), dz = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const AT sx = group_reduce<T>(ax[r], 64);
        AT sy = sx, sz = sx;
        if (XYZ) {
            sy = group_reduce<T>(ay[r], 64);
            sz = group_reduce<T>(az[r], 64);
        }
        if (lane == r) {
            dx = A::round(sx);
            if (XYZ) {
                dy = A::round(sy);
                dz = A::round(sz);
            }
        }
    }
    const int row = row0 + lane;
    if (lane >= R || row >= n) return;
    fwd_epilogue<T, XYZ>(d, k, row, 0, kk, stage, cur, trace, dx, dy, dz);
}

// ---------------------------------------------------------------------------
// Reverse of stage `stage` of local step kk: t = W^T bbar over the stage's
// coupling adjoint (all nodes), then per node xbar = loc + a_cp t along the
// coupled components, dL/dm += xbar, and the pointwise adjoint of the next
// stage to reverse (or, after the first stage, the start of the previous step).
// ---------------------------------------------------------------------------
template <typename T, bool XYZ, int R, int U>
__global__ void __launch_bounds__(256) k_adj_stage(AdjDev<T> d, Coef<T> k, int kk, int stage) {
    using V = typename AVec<T>::type;
    constexpr int VN = AVec<T>::n;
    constexpr int C = XYZ ? 3 : 1;
    const int lane = threadIdx.x & 63;
    const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * R;
    const int n = d.n;
    if (row0 >= n) return;   // wave-uniform
    const int64_t ld = d.ld;
    const T* __restrict__ s = d.st + adj_slot<C>(kk, stage, 1, ld);
    const T* wrow[R];
#pragma unroll
    for (int r = 0; r < R; ++r) wrow[r] = d.Wt + (int64_t)min(row0 + r, n - 1) * ld;
    T tx[R], ty[R], tz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) tx[r] = ty[r] = tz[r] = T(0);
#pragma unroll U
    for (int64_t c = (int64_t)lane * VN; c < ld; c += 64 * VN) {
        const V sx = *reinterpret_cast<const V*>(s + c);
        V sy, sz;
        if (XYZ) {
            sy = *reinterpret_cast<const V*>(s + ld + c);
            sz = *reinterpret_cast<const V*>(s + 2 * ld + c);
        }
        V wv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) wv[r] = __builtin_nontemporal_load(reinterpret_cast<const V*>(wrow[r] + c));
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int e = 0; e < VN; ++e) {
                tx[r] = __builtin_fma(wv[r][e], sx[e], tx[r]);
                if (XYZ) {
                    ty[r] = __builtin_fma(wv[r][e], sy[e], ty[r]);
                    tz[r] = __builtin_fma(wv[r][e], sz[e], tz[r]);
                }
            }
    }
    T dx = T(0), dy = T(0), dz = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const T sx = wave_sum<T>(tx[r]);
        T sy = sx, sz = sx;
        if (XYZ) {
            sy = wave_sum<T>(ty[r]);
            sz = wave_sum<T>(tz[r]);
        }
        if (lane == r) {
            dx = sx;
            if (XYZ) {
                dy = sy;
                dz = sz;
            }
        }
    }
    const int i = row0 + lane;
    if (lane >= R || i >= n) return;
    rev_epilogue<T, XYZ>(d, k, i, 0, kk, stage, dx, dy, dz);
}

// Start reversing the last step (local kk) of a segment: the carry is the
// dL/dm left in mbar by the later segment (zero for the last one), and the
// state after the step is the forward state m after the recompute.
template <typename T, bool XYZ>
__global__ void __launch_bounds__(256) k_adj_prep(AdjDev<T> d, Coef<T> k, int kk) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= d.n) return;
    const int64_t ld = d.ld;
    const int64_t sb = (int64_t)s * 3 * ld;
    const T pn = d.renorm ? d.pn[((int64_t)kk * d.S + s) * ld + i] : T(1);
    GlobalSink sink;
    prep_step<T, XYZ>(d, k, i, s, kk, d.m + sb, pn, d.mbar[sb + i], d.mbar[sb + ld + i], d.mbar[sb + 2 * ld + i],
                      sink);
}

// ---------------------------------------------------------------------------
// dL/dW over one segment: G (+)= alpha * sum_l S[l][i] X[l][j], a product of
// two L x n panels (rows strided by sld / xld).  64 x 64 output tile per
// workgroup, 4 x 4 per thread, panels staged through LDS 16 rows at a time.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_gw(const T* __restrict__ S, int64_t sld, const T* __restrict__ X,
                                            int64_t xld, int L, int n, T alpha, T* __restrict__ G, int accumulate) {
    __shared__ T As[16][64];
    __shared__ T Bs[16][64];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    T acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = T(0);
    for (int l0 = 0; l0 < L; l0 += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q;
            const int lr = e >> 6, cc = e & 63;
            const int l = l0 + lr;
            As[lr][cc] = l < L ? S[(int64_t)l * sld + i0 + cc] : T(0);
            Bs[lr][cc] = l < L ? X[(int64_t)l * xld + j0 + cc] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int lr = 0; lr < 16; ++lr) {
            T a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[lr][4 * ty + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[lr][4 * tx + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = __builtin_fma(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + 4 * ty + r;
        if (i >= n) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = j0 + 4 * tx + c;
            if (j >= n) continue;
            T* g = G + (int64_t)i * n + j;
            *g = accumulate ? *g + alpha * acc[r][c] : alpha * acc[r][c];
        }
    }
}

// FP32 dL/dW on the matrix cores: G (+)= alpha * S^T X as above, with
// v_mfma_f32_16x16x4f32 (FP32 accumulation).  A wave owns a 64 x 64 block of
// G as 4 x 4 tiles of 16 x 16, a workgroup of four waves 128 x 128.  Per MFMA
// step of four panel rows, lane l supplies A[l%16][l/16] = S[l0 + l/16][i]
// and B[l/16][l%16] = X[l0 + l/16][j], so both panels are read along their
// contiguous dimension (16 lanes cover 64 consecutive bytes); the result tile
// holds D[4 (l/16) + r][l%16] in lane l.  Columns at or beyond ld (the panel
// pitch) read as zero; the kernel has no barrier, so waves outside G leave early.
typedef float mf4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_gw_mfma(const float* __restrict__ S, int64_t sld, const float* __restrict__ X,
                                                 int64_t xld, int L, int n, int64_t ld, float alpha,
                                                 float* __restrict__ G, int accumulate, int lchunk,
                                                 float* __restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // slice z of the contraction (rows [lb, le)); with part, its partial
    // tile goes to part[z] and k_gw_reduce sums the slices
    const int lb = blockIdx.z * lchunk, le = min(L, lb + lchunk);
    const int i0 = blockIdx.y * 128 + (wave >> 1) * 64;
    const int j0 = blockIdx.x * 128 + (wave & 1) * 64;
    if (i0 >= n || j0 >= n) return;   // wave-uniform
    const int kr = lane >> 4, c16 = lane & 15;
    bool va[4], vb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        va[q] = i0 + 16 * q + c16 < ld;
        vb[q] = j0 + 16 * q + c16 < ld;
    }
    const float* sp = S + i0 + c16;
    const float* xp = X + j0 + c16;
    mf4 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mf4{0.f, 0.f, 0.f, 0.f};
    // operands of step l0 + 4 are loaded while the MFMAs of step l0 run
    float a[4], b[4];
    // Loads are unconditional from clamped addresses (row L - 1, column
    // offset 0: i0 + c16 < n <= ld), out-of-range operands are zeroed after.
    auto load = [&](int l0, float* ra, float* rb) {
        const int l = l0 + kr;
        const bool vl = l < le;
        const int64_t lc = vl ? l : le - 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float x = sp[lc * sld + (va[q] ? 16 * q : 0)];
            const float y = xp[lc * xld + (vb[q] ? 16 * q : 0)];
            const unsigned ma = (vl && va[q]) ? 0xffffffffu : 0u, mb = (vl && vb[q]) ? 0xffffffffu : 0u;
            ra[q] = __uint_as_float(__float_as_uint(x) & ma);
            rb[q] = __uint_as_float(__float_as_uint(y) & mb);
        }
    };
    load(lb, a, b);
    for (int l0 = lb; l0 < le; l0 += 4) {
        float an[4], bn[4];
        load(l0 + 4, an, bn);
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = an[q];
            b[q] = bn[q];
        }
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + 16 * bi + 4 * kr + r;
            if (i >= n) continue;
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const int j = j0 + 16 * bj + c16;
                if (j >= n) continue;
                if (part) {
                    part[((int64_t)blockIdx.z * n + i) * n + j] = acc[bi][bj][r];
                } else {
                    float* g = G + (int64_t)i * n + j;
                    *g = accumulate ? *g + alpha * acc[bi][bj][r] : alpha * acc[bi][bj][r];
                }
            }
        }
}

// Sum of the contraction slices of k_gw_mfma in a fixed order.
__global__ void __launch_bounds__(256) k_gw_reduce(const float* __restrict__ part, int splits, int64_t nn, float alpha,
                                                   float* __restrict__ G, int accumulate) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
        float v = part[e];
        for (int z = 1; z < splits; ++z) v += part[z * nn + e];
        G[e] = accumulate ? G[e] + alpha * v : alpha * v;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_transpose(const T* __restrict__ W, T* __restrict__ Wt, int n, int64_t ld) {
    __shared__ T tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    for (int r = ty; r < 64; r += 4) {
        const int i = i0 + r, j = j0 + tx;
        tile[r][tx] = (i < n && j < n) ? W[(int64_t)i * ld + j] : T(0);
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int j = j0 + r, i = i0 + tx;
        if (j < n && i < n) Wt[(int64_t)j * ld + i] = tile[tx][r];
    }
}

// AoS ([S][n][3]) -> SoA ([S][3][ld]) into m and the current stage input.
template <typename T>
__global__ void k_load_state(const T* __restrict__ aos, T* __restrict__ m, T* __restrict__ x, int n, int64_t ld) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= n) return;
    for (int c = 0; c < 3; ++c) {
        const T v = aos[((int64_t)s * n + i) * 3 + c];
        m[((int64_t)s * 3 + c) * ld + i] = v;
        x[((int64_t)s * 3 + c) * ld + i] = v;
    }
}

// Outputs: dL/dm0 ([S][n][3]) and dL/dw_in (n x n_in, summed over the
// streams in order) from the accumulators.
template <typename T>
__global__ void k_adj_outputs(const T* __restrict__ mbar, const double* __restrict__ gwin, T* __restrict__ g_m0,
                              T* __restrict__ g_win, int n, int n_in, int S, int64_t ld) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (g_m0)
        for (int s = 0; s < S; ++s)
            for (int c = 0; c < 3; ++c) g_m0[((int64_t)s * n + i) * 3 + c] = mbar[((int64_t)s * 3 + c) * ld + i];
    if (g_win)
        for (int q = 0; q < n_in; ++q) {
            double v = 0.0;
            for (int s = 0; s < S; ++s) v += gwin[((int64_t)q * S + s) * ld + i];
            g_win[(int64_t)i * n_in + q] = (T)v;
        }
}

// Sum of the per-node scalar partials ([4][S][ld]) in a fixed order (one workgroup).
__global__ void __launch_bounds__(256) k_adj_scalars(const double* __restrict__ gacc, int n, int S, int64_t ld,
                                                     double* __restrict__ out) {
    __shared__ double part[256];
    const int64_t total = (int64_t)S * n;
    for (int q = 0; q < 4; ++q) {
        double v = 0.0;
        for (int64_t e = threadIdx.x; e < total; e += 256) {
            const int64_t s = e / n, i = e - s * n;
            v += gacc[((int64_t)q * S + s) * ld + i];
        }
        part[threadIdx.x] = v;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = part[0];
        __syncthreads();
    }
}

// Launch shapes of the two streaming kernels (rows of W per wave x unroll
// of the column loop); STO_ADJ_ROWS / STO_ADJ_UNROLL choose one for
// measurements.  Otherwise 1 row with unroll 4 below 4096 nodes (more waves
// for a small matrix: at N = 10^3 FP64 the adjoint took 99.7 ms against
// 117.2 with 2 x 2; one row split over the four waves of a workgroup was
// slower still, 111.4) and 2 rows with unroll 2 above (at N = 10^4 FP32,
// 202 ms against 227 with 1 x 4).
int env_int(const char* name, int dflt) {
    const char* v = getenv(name);
    return v ? atoi(v) : dflt;
}

// sticky |= the abort word of the last persistent launch (whose own word
// is cleared at the start of every launch).
__global__ void k_keep_abort(const int* word, int* sticky) {
    if (threadIdx.x == 0 && *word) *sticky = 1;
}

template <typename T>
void adj_shape(int n, int* rows, int* unroll) {
    static const int r = env_int("STO_ADJ_ROWS", 0), u = env_int("STO_ADJ_UNROLL", 0);
    *rows = n < 4096 ? 1 : 2;
    *unroll = n < 4096 ? 4 : 2;
    const int ok[][2] = {{1, 4}, {2, 2}, {2, 4}, {4, 1}, {4, 2}};
    for (const auto& v : ok)
        if (v[0] == r && v[1] == u) {
            *rows = r;
            *unroll = u;
        }
}

template <typename T, bool XYZ>
void launch_fwd(int rows, int unroll, hipStream_t st, const AdjDev<T>& d, const Coef<T>& k, int kk, int stage,
                int trace) {
    const dim3 grid((d.n + 4 * rows - 1) / (4 * rows)), block(256);
#define ADJ_FWD(RR, UU)                                                                                  \
    if (rows == RR && unroll == UU) {                                                                    \
        hipLaunchKernelGGL((k_fwd_trace<T, XYZ, RR, UU>), grid, block, 0, st, d, k, kk, stage, stage & 1, \
                           trace);                                                                       \
        return;                                                                                          \
    }
    ADJ_FWD(1, 4)
    ADJ_FWD(2, 2)
    ADJ_FWD(2, 4)
    ADJ_FWD(4, 1)
    ADJ_FWD(4, 2)
#undef ADJ_FWD
}

template <typename T, bool XYZ>
void launch_rev(int rows, int unroll, hipStream_t st, const AdjDev<T>& d, const Coef<T>& k, int kk, int stage) {
    const dim3 grid((d.n + 4 * rows - 1) / (4 * rows)), block(256);
#define ADJ_REV(RR, UU)                                                                            \
    if (rows == RR && unroll == UU) {                                                              \
        hipLaunchKernelGGL((k_adj_stage<T, XYZ, RR, UU>), grid, block, 0, st, d, k, kk, stage); \
        return;                                                                                    \
    }
    ADJ_REV(1, 4)
    ADJ_REV(2, 2)
    ADJ_REV(2, 4)
    ADJ_REV(4, 1)
    ADJ_REV(4, 2)
#undef ADJ_REV
}

struct DevAlloc {
    std::vector<void*> ptrs;
    ~DevAlloc() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename P>
    hipError_t get(P** out, size_t bytes) {
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) return e;
        ptrs.push_back(p);
        *out = static_cast<P*>(p);
        return hipSuccess;
    }
};

#define ADJ_TRY(x)                         \
    do {                                   \
        hipError_t e_ = (x);               \
        if (e_ != hipSuccess) return e_;   \
    } while (0)

template <typename T, bool XYZ>
hipError_t adjoint_impl(const AdjArgs<T>& a) {
    constexpr int C = XYZ ? 3 : 1;
    const hipStream_t st = a.stream;
    int rows = 2, unroll = 2;
    const int n = a.n, NS = a.streams;
    adj_shape<T>(n, &rows, &unroll);
    const int64_t ld = a.ld, NSTEP = a.steps;
    const int64_t K = std::max<int64_t>(1, std::min<int64_t>(a.seg_steps, NSTEP));
    const int64_t nseg = (NSTEP + K - 1) / K;
    const size_t vec = (size_t)3 * ld * NS * sizeof(T);   // one state of all streams
    const size_t per_stage = (size_t)NS * ld * sizeof(T);  // one component of all streams
    DevAlloc mem;
    AdjDev<T> d{};
    d.W = a.W;
    d.Wt = a.Wt;
    d.w_in = a.w_in;
    d.bad = a.bad;
    d.g_rec = a.g_rec;
    d.g_fin = a.g_fin;
    d.u = a.u;
    d.rec = nullptr;
    d.n = n;
    d.n_in = a.n_in;
    d.substeps = a.substeps;
    d.renorm = a.renorm;
    d.S = NS;
    d.ld = ld;
    d.steps = NSTEP;
    T* cps = nullptr;
    ADJ_TRY(mem.get(&d.m, vec));
    ADJ_TRY(mem.get(&d.ms[0], vec));
    ADJ_TRY(mem.get(&d.ms[1], vec));
    ADJ_TRY(mem.get(&d.acc, vec));
    ADJ_TRY(mem.get(&d.abar, vec));
    ADJ_TRY(mem.get(&d.mbar, vec));
    ADJ_TRY(mem.get(&d.loc, vec));
    if (!a.records) ADJ_TRY(mem.get(&cps, vec * (size_t)nseg));
    ADJ_TRY(mem.get(&d.xt, (size_t)K * 4 * 3 * per_stage));
    ADJ_TRY(mem.get(&d.wx, (size_t)K * 4 * C * per_stage));
    ADJ_TRY(mem.get(&d.st, (size_t)K * 4 * C * per_stage));
    ADJ_TRY(mem.get(&d.pn, (size_t)K * per_stage));
    ADJ_TRY(mem.get(&d.gacc, (size_t)4 * NS * ld * sizeof(double)));
    ADJ_TRY(mem.get(&d.gwin, (size_t)std::max(1, a.n_in) * NS * ld * sizeof(double)));
    // zero everything whose padding is read (stage inputs, coupling adjoints)
    // and every accumulator
    for (T* p : {d.m, d.ms[0], d.ms[1], d.acc, d.abar, d.mbar, d.loc}) ADJ_TRY(hipMemsetAsync(p, 0, vec, st));
    ADJ_TRY(hipMemsetAsync(d.st, 0, (size_t)K * 4 * C * per_stage, st));
    ADJ_TRY(hipMemsetAsync(d.gacc, 0, (size_t)4 * NS * ld * sizeof(double), st));
    ADJ_TRY(hipMemsetAsync(d.gwin, 0, (size_t)std::max(1, a.n_in) * NS * ld * sizeof(double), st));

    // FP32 dL/dW: the contraction is split into slices when the output has
    // too few 128 x 128 tiles to fill the GPU (small n, long segments); at
    // most 64 slices, or STO_GW_SPLITS (1 to 256) for measurements
    const int gw_tiles = ((n + 127) / 128) * ((n + 127) / 128);
    const int gw_max = std::min(256, std::max(1, env_int("STO_GW_SPLITS", 64)));
    auto gw_splits = [&](int L) { return std::max(1, std::min({gw_max, 2048 / gw_tiles, L / 256})); };
    float* gw_part = nullptr;
    if (sizeof(T) == 4 && a.g_W) {
        const int smax = gw_splits((int)(K * 4 * NS * C));
        if (smax > 1) ADJ_TRY(mem.get(&gw_part, (size_t)smax * n * n * sizeof(float)));
    }
    const dim3 pgrid((n + 255) / 256, NS), pblock(256);
    const Coef<T> k = a.k;
    // one forward / reversed stage: streamed mat-vecs for one stream, the
    // FP32 MFMA product of all streams otherwise
    auto fwd_stage = [&](int kk, int stage, int trace) {
        if (NS == 1) {
            launch_fwd<T, XYZ>(rows, unroll, st, d, k, kk, stage, trace);
        } else if constexpr (sizeof(T) == 4) {
            launch_batch_fwd(d, k, kk, stage, stage & 1, trace, XYZ, st);
        }
    };
    auto rev_stage = [&](int kk, int stage) {
        if (NS == 1) {
            launch_rev<T, XYZ>(rows, unroll, st, d, k, kk, stage);
        } else if constexpr (sizeof(T) == 4) {
            launch_batch_rev(d, k, kk, stage, XYZ, st);
        }
    };
    // S streams in FP32 with segments of whole samples: the forward runs on
    // the persistent multi-stream kernel (the arithmetic of the plain
    // multi-stream run), one cooperative launch per segment, writing the
    // stage trace where the reverse needs it
    // The reversed stages of a segment run the same way (k_multi_rev) when
    // that kernel is co-resident too; STO_MULTI_REVERSE=0 keeps them on the
    // per-stage kernels, for measurements.
    bool use_multi = false, use_multi_rev = false;
    float* xchg = nullptr;
    int* msync = nullptr;   // [0, 64): the launches' words; [64]: sticky abort
    if constexpr (sizeof(T) == 4) {
        use_multi = NS > 1 && K % a.substeps == 0 && multi_fits(n, NS, XYZ, nullptr, nullptr) &&
                    multi_segment_fits(n, NS, XYZ);
        use_multi_rev = use_multi && env_int("STO_MULTI_REVERSE", 1) != 0 && multi_reverse_fits(n, NS, XYZ, a.n_in);
        if (use_multi) {
            ADJ_TRY(mem.get(&xchg, (size_t)3 * C * NS * ld * sizeof(float)));
            ADJ_TRY(mem.get(&msync, 512));
            ADJ_TRY(hipMemsetAsync(msync, 0, 512, st));
        }
    }
    // One stream whose W fits the CUs' LDS, with segments of whole samples:
    // the recompute and the reversed stages of every segment each run in one
    // cooperative launch of the resident kernels (STO_RES_ADJOINT=0 keeps
    // them on the per-stage kernels, for measurements).
    bool use_res = false;
    T* rxchg = nullptr;
    if (NS == 1 && K % a.substeps == 0 && env_int("STO_RES_ADJOINT", 1) != 0 &&
        resident_adjoint_fits(n, (int)sizeof(T), XYZ, a.n_in)) {
        use_res = true;
        ADJ_TRY(mem.get(&rxchg, (size_t)3 * C * ld * sizeof(T)));
        ADJ_TRY(mem.get(&msync, 512));
        ADJ_TRY(hipMemsetAsync(msync, 0, 512, st));
    }
    auto keep_abort = [&]() -> hipError_t {
        hipLaunchKernelGGL(k_keep_abort, dim3(1), dim3(64), 0, st, msync + kSyncAbortWord, msync + 64);
        return hipGetLastError();
    };
    // forward over local steps [0, kn) of the segment starting at j0; the
    // state is in m and ms[0] (cur = 0 between steps)
    int used = 0;   // ADJ_* kernel families run
    auto forward = [&](int64_t j0, int64_t kn, int trace) -> hipError_t {
        d.j0 = j0;
        used |= (use_multi || use_res) ? ADJ_FWD_PERSISTENT : ADJ_FWD_STAGE;
        if (use_res) {
            DevState<T> ds{};
            ds.W = a.W;
            ds.w_in = a.w_in;
            ds.m = d.m;
            ds.ms[0] = d.ms[0];
            ds.ms[1] = d.ms[1];
            ds.acc = d.acc;
            ds.xchg = rxchg;
            ds.bad = a.bad;
            ds.sync = msync;
            ds.n = n;
            ds.n_in = a.n_in;
            ds.ld = ld;
            RunSpec rs{};
            rs.u = a.u + (j0 / a.substeps) * a.n_in;
            rs.states = nullptr;
            rs.samples = (int)(kn / a.substeps);
            rs.substeps = a.substeps;
            rs.cur = 0;
            rs.renorm = a.renorm;
            rs.xyz = XYZ;
            rs.stream = st;
            if (trace) {
                const ResTrace<T> tr{d.xt, d.wx, d.pn};
                ADJ_TRY(run_resident_traced<T>(ds, k, rs, tr, (int)(j0 / a.substeps)));
            } else {
                ADJ_TRY(run_resident<T>(ds, k, rs));
            }
            return keep_abort();
        }
        if constexpr (sizeof(T) == 4) {
            if (use_multi) {
                DevState<float> ds{};
                ds.W = a.W;
                ds.w_in = a.w_in;
                ds.m = d.m;
                ds.xchg = xchg;
                ds.bad = a.bad;
                ds.sync = msync;
                ds.n = n;
                ds.n_in = a.n_in;
                ds.ld = ld;
                RunSpec rs{};
                rs.u = a.u + (j0 / a.substeps) * NS * a.n_in;
                rs.states = nullptr;
                rs.samples = (int)(kn / a.substeps);
                rs.substeps = a.substeps;
                rs.cur = 0;
                rs.renorm = a.renorm;
                rs.xyz = XYZ;
                rs.stream = st;
                const MultiTrace tr{trace ? d.xt : nullptr, d.wx, d.pn};
                ADJ_TRY(run_multi_segment(ds, k, rs, NS, (int)(j0 / a.substeps), tr));
                ADJ_TRY(keep_abort());
                ADJ_TRY(hipMemcpyAsync(d.ms[0], d.m, vec, hipMemcpyDeviceToDevice, st));
                return hipGetLastError();
            }
        }
        for (int64_t kk = 0; kk < kn; ++kk)
            for (int stage = 0; stage < 4; ++stage) fwd_stage((int)kk, stage, trace);
        return hipGetLastError();
    };
    if (NSTEP > 0) {
        hipLaunchKernelGGL(k_load_state<T>, pgrid, pblock, 0, st, a.m_start, d.m, d.ms[0], n, ld);
        ADJ_TRY(hipGetLastError());
    }
    // pass 1: checkpoints; the last segment is traced directly.  With the
    // run's records the state at the start of segment g > 0 is the record
    // of sample g K / substeps - 1, and pass 1 is not needed.
    if (!a.records) {
        for (int64_t g = 0; g < nseg; ++g) {
            const int64_t j0 = g * K, kn = std::min(K, NSTEP - j0);
            ADJ_TRY(hipMemcpyAsync(cps + (size_t)g * 3 * ld * NS, d.m, vec, hipMemcpyDeviceToDevice, st));
            ADJ_TRY(forward(j0, kn, g == nseg - 1));
        }
    }
    int gw_started = 0;
    for (int64_t g = nseg - 1; g >= 0; --g) {
        const int64_t j0 = g * K, kn = std::min(K, NSTEP - j0);
        if (a.records) {
            const T* src = g == 0 ? a.m_start : a.records + (j0 / a.substeps - 1) * (int64_t)NS * n * 3;
            hipLaunchKernelGGL(k_load_state<T>, pgrid, pblock, 0, st, src, d.m, d.ms[0], n, ld);
            ADJ_TRY(hipGetLastError());
            ADJ_TRY(forward(j0, kn, 1));
        } else if (g < nseg - 1) {
            ADJ_TRY(hipMemcpyAsync(d.m, cps + (size_t)g * 3 * ld * NS, vec, hipMemcpyDeviceToDevice, st));
            ADJ_TRY(hipMemcpyAsync(d.ms[0], d.m, vec, hipMemcpyDeviceToDevice, st));
            ADJ_TRY(forward(j0, kn, 1));
        }
        d.j0 = j0;
        hipLaunchKernelGGL((k_adj_prep<T, XYZ>), pgrid, pblock, 0, st, d, k, (int)(kn - 1));
        bool reversed = false;
        if (use_res) {
            ADJ_TRY(hipGetLastError());
            ADJ_TRY(run_resident_reverse<T>(d, k, (int)kn, XYZ, rxchg, msync, st));
            ADJ_TRY(keep_abort());
            reversed = true;
        }
        if constexpr (sizeof(T) == 4) {
            if (use_multi_rev) {
                ADJ_TRY(hipGetLastError());
                ADJ_TRY(run_multi_reverse(d, k, (int)kn, XYZ, xchg, msync, st));
                ADJ_TRY(keep_abort());
                reversed = true;
            }
        }
        if (!reversed)
            for (int64_t kk = kn - 1; kk >= 0; --kk)
                for (int stage = 3; stage >= 0; --stage) rev_stage((int)kk, stage);
        used |= reversed ? ADJ_REV_PERSISTENT : ADJ_REV_STAGE;
        ADJ_TRY(hipGetLastError());
        if (a.g_W) {
            // rows of the panels: (step, stage, stream, component), pitch ld
            const int L = (int)(kn * 4 * NS * C);
            const int64_t xld = XYZ ? ld : 3 * ld;
            if constexpr (sizeof(T) == 4) {
                const int splits = gw_part ? gw_splits(L) : 1;
                const int lchunk = ((L + splits - 1) / splits + 3) / 4 * 4;
                const int z = (L + lchunk - 1) / lchunk;
                const dim3 ggrid((n + 127) / 128, (n + 127) / 128, z);
                hipLaunchKernelGGL(k_gw_mfma, ggrid, dim3(256), 0, st, d.st, ld, d.xt, xld, L, n, ld, k.a_cp, a.g_W,
                                   gw_started, lchunk, z > 1 ? gw_part : nullptr);
                if (z > 1) {
                    const int64_t nn = (int64_t)n * n;
                    hipLaunchKernelGGL(k_gw_reduce, dim3((unsigned)std::min<int64_t>((nn + 255) / 256, 4096)),
                                       dim3(256), 0, st, gw_part, z, nn, k.a_cp, a.g_W, gw_started);
                }
            } else {
                const dim3 ggrid((n + 63) / 64, (n + 63) / 64);
                hipLaunchKernelGGL(k_gw<T>, ggrid, dim3(256), 0, st, d.st, ld, d.xt, xld, L, n, k.a_cp, a.g_W,
                                   gw_started);
            }
            ADJ_TRY(hipGetLastError());
            gw_started = 1;
        }
    }
    if (a.g_W && !gw_started) ADJ_TRY(hipMemsetAsync(a.g_W, 0, (size_t)n * n * sizeof(T), st));
    if (NSTEP == 0) {
        // no step: dL/dm0 is the final-state gradient
        const size_t mb = (size_t)NS * n * 3 * sizeof(T);
        if (a.g_fin && a.g_m0)
            ADJ_TRY(hipMemcpyAsync(a.g_m0, a.g_fin, mb, hipMemcpyDeviceToDevice, st));
        else if (a.g_m0)
            ADJ_TRY(hipMemsetAsync(a.g_m0, 0, mb, st));
        if (a.g_win) ADJ_TRY(hipMemsetAsync(a.g_win, 0, (size_t)n * a.n_in * sizeof(T), st));
    } else if (a.g_m0 || a.g_win) {
        hipLaunchKernelGGL(k_adj_outputs<T>, dim3((n + 255) / 256), pblock, 0, st, d.mbar, d.gwin, a.g_m0, a.g_win,
                           n, a.n_in, NS, ld);
        ADJ_TRY(hipGetLastError());
    }
    if (a.g_scal) {
        hipLaunchKernelGGL(k_adj_scalars, dim3(1), dim3(256), 0, st, d.gacc, n, NS, ld, a.g_scal);
        ADJ_TRY(hipGetLastError());
    }
    if (a.kernels) *a.kernels = used;
    // the workspace is freed on return: wait for the work that uses it
    int aborted = 0;
    if (msync) ADJ_TRY(hipMemcpyAsync(&aborted, msync + 64, sizeof(int), hipMemcpyDeviceToHost, st));
    ADJ_TRY(hipStreamSynchronize(st));
    // a persistent launch whose exchange timed out left its results incomplete
    return aborted ? hipErrorLaunchTimeOut : hipSuccess;
}

}  // namespace

int64_t adjoint_trace_bytes_per_step(int64_t ld, int elem_bytes, int xyz, int streams) {
    const int C = xyz ? 3 : 1;
    return (int64_t)(4 * (3 + 2 * C) + 1) * ld * elem_bytes * streams;
}

template <typename T>
hipError_t transpose_matrix(const T* W, T* Wt, int n, int64_t ld, hipStream_t st) {
    const dim3 grid((n + 63) / 64, (n + 63) / 64);
    hipLaunchKernelGGL(k_transpose<T>, grid, dim3(256), 0, st, W, Wt, n, ld);
    return hipGetLastError();
}

template <typename T>
hipError_t adjoint_run(const AdjArgs<T>& a) {
    return a.xyz ? adjoint_impl<T, true>(a) : adjoint_impl<T, false>(a);
}

template hipError_t transpose_matrix<double>(const double*, double*, int, int64_t, hipStream_t);
template hipError_t transpose_matrix<float>(const float*, float*, int, int64_t, hipStream_t);
template hipError_t adjoint_run<double>(const AdjArgs<double>&);
template hipError_t adjoint_run<float>(const AdjArgs<float>&);

}  // namespace sto
