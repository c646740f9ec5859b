// RK4 stage kernel for N coupled spin-torque oscillators on gfx950.
//
// One RK4 stage evaluates, for every node k, the coupling contraction
// c_k = a_cp sum_i W_ki m_i^x over the stage input (paper, Eq. (coup); the
// only O(N^2) term, Sec. 3.1 and 3.3), then the pointwise right-hand side of
// Eq. (gov) and the classic RK4 stage bookkeeping (Sec. 3.2).
//
//   k_stage  (STREAM path)  one launch per RK4 stage for any N.  Each wave
//            owns R rows of W and streams them from HBM with 16-byte
//            non-temporal loads; the stage input vector is read through the
//            caches (it is N elements, shared by all rows).  The row sums are
//            reduced across the wave and the RK4 epilogue is fused, so every
//            stage is exactly one pass over W.
//
// The file also holds the streaming-read bandwidth probe.

#include <algorithm>
#include <climits>

#include "sto_internal.hpp"

namespace sto {

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

template <typename T> struct Vec;
template <> struct Vec<double> { using type = dvec2; static constexpr int n = 2; };
template <> struct Vec<float> { using type = fvec4; static constexpr int n = 4; };

// ---------------------------------------------------------------------------
// Shared epilogue: RHS of Eq. (gov) + RK4 stage update for node `row`.
// ---------------------------------------------------------------------------
template <typename T, bool XYZ>
__device__ __forceinline__ void stage_epilogue(const DevState<T>& d, const Coef<T>& k, int row,
                                               T dot_x, T dot_y, T dot_z, T hin, const T* xin,
                                               T* xout, int stage, int renorm, T* record,
                                               int sample) {
    const int64_t ld = d.ld;
    T sx = xin[row], sy = xin[ld + row], sz = xin[2 * ld + row];
    T cx = k.a_cp * dot_x;
    T cy = XYZ ? k.a_cp * dot_y : T(0);
    T cz = XYZ ? k.a_cp * dot_z : T(0);
    T fx, fy, fz;
    llg_rhs<T, XYZ>(k, sx, sy, sz, cx, cy, cz, hin, fx, fy, fz);
    T mx = d.m[row], my = d.m[ld + row], mz = d.m[2 * ld + row];
    T ax = T(0), ay = T(0), az = T(0);
    if (stage > 0) {
        ax = d.acc[row];
        ay = d.acc[ld + row];
        az = d.acc[2 * ld + row];
    }
    T nx = rk4_update(k, stage, mx, ax, fx);
    T ny = rk4_update(k, stage, my, ay, fy);
    T nz = rk4_update(k, stage, mz, az, fz);
    if (stage == 3) {
        if (renorm) renormalize(nx, ny, nz);
        d.m[row] = nx;
        d.m[ld + row] = ny;
        d.m[2 * ld + row] = nz;
        if (record) {
            record[3 * (int64_t)row + 0] = nx;
            record[3 * (int64_t)row + 1] = ny;
            record[3 * (int64_t)row + 2] = nz;
        }
        if (!finite3(nx, ny, nz)) atomicMin(d.bad, sample);
    } else {
        d.acc[row] = ax;
        d.acc[ld + row] = ay;
        d.acc[2 * ld + row] = az;
    }
    xout[row] = nx;
    xout[ld + row] = ny;
    xout[2 * ld + row] = nz;
}

// ---------------------------------------------------------------------------
// STREAM path: one RK4 stage.
// ---------------------------------------------------------------------------
template <typename T, bool XYZ, int R, bool NT, int U>
__global__ void __launch_bounds__(256) k_stage(DevState<T> d, Coef<T> k, const double* __restrict__ u_s,
                                               T* __restrict__ record, int sample, int stage, int cur,
                                               int renorm, int reverse) {
    using A = Acc<T>;
    using AT = typename A::type;
    using V = typename Vec<T>::type;
    constexpr int VN = Vec<T>::n;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // On alternate stages the row blocks are visited last-to-first, so the
    // rows streamed at the end of one stage (still in the memory-side cache)
    // are the first ones the next stage reads.
    const int block = reverse ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x;
    const int row0 = (block * 4 + wave) * R;
    const int n = d.n;
    if (row0 >= n) return;   // wave-uniform
    const int64_t ld = d.ld;
    const T* __restrict__ xin = d.ms[cur];
    T* __restrict__ xout = d.ms[cur ^ 1];

    const T* wrow[R];
#pragma unroll
    for (int r = 0; r < R; ++r) wrow[r] = d.W + (int64_t)min(row0 + r, n - 1) * ld;

    AT ax[R], ay[R], az[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ax[r] = ay[r] = az[r] = A::zero();

#pragma unroll U
    for (int64_t c = (int64_t)lane * VN; c < ld; c += 64 * VN) {
        V xv = *reinterpret_cast<const V*>(xin + c);
        V yv, zv;
        if (XYZ) {
            yv = *reinterpret_cast<const V*>(xin + ld + c);
            zv = *reinterpret_cast<const V*>(xin + 2 * ld + c);
        }
        V wv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const V* p = reinterpret_cast<const V*>(wrow[r] + c);
            wv[r] = NT ? __builtin_nontemporal_load(p) : *p;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int e = 0; e < VN; ++e) {
                A::fma(ax[r], wv[r][e], xv[e]);
                if (XYZ) {
                    A::fma(ay[r], wv[r][e], yv[e]);
                    A::fma(az[r], wv[r][e], zv[e]);
                }
            }
        }
    }
    T dx = T(0), dy = T(0), dz = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        AT sx = group_reduce<T>(ax[r], 64);
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
    if (lane < R && row < n) {
        T hin = input_field(k, d.w_in + (int64_t)row * d.n_in, u_s, d.n_in);
        stage_epilogue<T, XYZ>(d, k, row, dx, dy, dz, hin, xin, xout, stage, renorm, record, sample);
    }
}

template <typename T, bool XYZ, bool NT, int R, int U>
static void launch_stage(hipStream_t st, const DevState<T>& d, const Coef<T>& k, const double* u_s, T* rec, int s,
                         int stage, int c, int renorm, int reverse) {
    dim3 grid((d.n + 4 * R - 1) / (4 * R));
    hipLaunchKernelGGL((k_stage<T, XYZ, R, NT, U>), grid, dim3(256), 0, st, d, k, u_s, rec, s, stage, c, renorm,
                       reverse);
}

// Variants of the stream kernel: rows per wave R and column-loop unroll U.
template <typename T, bool XYZ, bool NT>
static void launch_stage_rv(int rows, int unroll, hipStream_t st, const DevState<T>& d, const Coef<T>& k,
                            const double* u_s, T* rec, int s, int stage, int c, int renorm, int reverse) {
#define STO_STAGE_CASE(RR, UU)                                                                   \
    if (rows == RR && unroll == UU) {                                                            \
        launch_stage<T, XYZ, NT, RR, UU>(st, d, k, u_s, rec, s, stage, c, renorm, reverse); \
        return;                                                                                  \
    }
    STO_STAGE_CASE(1, 4)
    STO_STAGE_CASE(2, 2)
    STO_STAGE_CASE(2, 4)
    STO_STAGE_CASE(4, 1)
    STO_STAGE_CASE(4, 2)
    STO_STAGE_CASE(4, 4)
    STO_STAGE_CASE(8, 1)
    STO_STAGE_CASE(8, 2)
#undef STO_STAGE_CASE
    launch_stage<T, XYZ, NT, sizeof(T) == 8 ? 2 : 4, 2>(st, d, k, u_s, rec, s, stage, c, renorm, reverse);
}

// Non-temporal loads of W unless W fits the 256 MB memory-side cache with
// room to spare for little else: between 96 and 256 MB, cached loads keep
// much of W there from one stage to the next (N = 5,000 FP64, 200 MB: 126.9
// against 145.0 us per RK4 step), while smaller matrices (50 MB: 47.2
// against 43.9) and larger ones (400 MB: 250.3 against 237.4) stream faster
// with non-temporal loads.
static bool stream_nt(int64_t w_bytes, int forced) {
    if (forced >= 0) return forced != 0;
    return !(w_bytes > (int64_t)96 << 20 && w_bytes <= (int64_t)256 << 20);
}

template <typename T>
hipError_t run_stream(const DevState<T>& d, const Coef<T>& k, const RunSpec& r) {
    const Tune& t = tune();
    int rows = 2, unroll = 2;
    stream_shape((int)sizeof(T), d.n, &rows, &unroll);
    const bool nt = stream_nt((int64_t)d.n * d.ld * (int64_t)sizeof(T), t.stream_nontemporal);
    T* states = static_cast<T*>(r.states);
    int cur = r.cur;
    int64_t sigma = 0;
    for (int s = 0; s < r.samples; ++s) {
        const double* u_s = r.u + (int64_t)s * d.n_in;
        for (int sub = 0; sub < r.substeps; ++sub) {
            for (int stage = 0; stage < 4; ++stage, ++sigma) {
                T* rec = (states && stage == 3 && sub == r.substeps - 1)
                             ? states + (int64_t)s * d.n * 3 : nullptr;
                const int c = cur ^ (stage & 1);
                const int rev = t.stream_alternate ? (int)(sigma & 1) : 0;
                if (r.xyz) {
                    if (nt) launch_stage_rv<T, true, true>(rows, unroll, r.stream, d, k, u_s, rec, s, stage, c, r.renorm, rev);
                    else launch_stage_rv<T, true, false>(rows, unroll, r.stream, d, k, u_s, rec, s, stage, c, r.renorm, rev);
                } else {
                    if (nt) launch_stage_rv<T, false, true>(rows, unroll, r.stream, d, k, u_s, rec, s, stage, c, r.renorm, rev);
                    else launch_stage_rv<T, false, false>(rows, unroll, r.stream, d, k, u_s, rec, s, stage, c, r.renorm, rev);
                }
            }
        }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagnostic: attainable HBM read bandwidth (plain streaming read).
// ---------------------------------------------------------------------------
template <int L>
__global__ void __launch_bounds__(256) k_read_probe(const fvec4* __restrict__ src, int64_t nvec,
                                                    float* __restrict__ sink) {
    fvec4 acc = {0.f, 0.f, 0.f, 0.f};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i + (L - 1) * stride < nvec; i += L * stride) {
        fvec4 v[L];
#pragma unroll
        for (int q = 0; q < L; ++q) v[q] = __builtin_nontemporal_load(src + i + q * stride);
#pragma unroll
        for (int q = 0; q < L; ++q) acc += v[q];
    }
    for (; i < nvec; i += stride) acc += __builtin_nontemporal_load(src + i);
    const float v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (v == 12345.678f) sink[threadIdx.x] = v;   // keeps the loads alive; never true for zeros
}

// Each wave streams one contiguous segment (the access pattern of the
// coupling kernel, whose waves each read whole rows).
template <int L>
__global__ void __launch_bounds__(256) k_read_probe_seg(const fvec4* __restrict__ src, int64_t nvec,
                                                        int64_t seg, float* __restrict__ sink) {
    fvec4 acc = {0.f, 0.f, 0.f, 0.f};
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t b = wave * seg;
    const int64_t e = b + seg < nvec ? b + seg : nvec;
    int64_t i = b + lane;
    for (; i + (L - 1) * 64 < e; i += L * 64) {
        fvec4 v[L];
#pragma unroll
        for (int q = 0; q < L; ++q) v[q] = __builtin_nontemporal_load(src + i + q * 64);
#pragma unroll
        for (int q = 0; q < L; ++q) acc += v[q];
    }
    for (; i < e; i += 64) acc += __builtin_nontemporal_load(src + i);
    const float v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (v == 12345.678f) sink[threadIdx.x] = v;
}

// Best of a few launch shapes: grid-stride with 4 or 8 loads in flight per
// thread at 4, 8 or 16 workgroups per CU, and contiguous per-wave segments.
hipError_t read_bandwidth(int64_t bytes, int reps, double* gbs) {
    void* buf = nullptr;
    float* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const int64_t nvec = bytes / 16;
    hipError_t e = hipMalloc(&buf, nvec * 16);
    if (e == hipSuccess) e = hipMalloc(&sink, 256 * sizeof(float));
    if (e == hipSuccess) e = hipMemset(buf, 0, nvec * 16);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int dev = 0, cus = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    double best = 0.0;
    const int per_cu[] = {4, 8, 16};
    for (int lf = 0; lf < 4 && e == hipSuccess; ++lf) {
        for (int pc : per_cu) {
            const dim3 grid(cus * pc), block(256);
            const int64_t waves = (int64_t)cus * pc * 4;
            const int64_t seg = (nvec + waves - 1) / waves;
            auto launch = [&]() {
                if (lf == 0) hipLaunchKernelGGL(k_read_probe<4>, grid, block, 0, nullptr, (const fvec4*)buf, nvec, sink);
                else if (lf == 1) hipLaunchKernelGGL(k_read_probe<8>, grid, block, 0, nullptr, (const fvec4*)buf, nvec, sink);
                else if (lf == 2)
                    hipLaunchKernelGGL(k_read_probe_seg<4>, grid, block, 0, nullptr, (const fvec4*)buf, nvec, seg, sink);
                else
                    hipLaunchKernelGGL(k_read_probe_seg<8>, grid, block, 0, nullptr, (const fvec4*)buf, nvec, seg, sink);
            };
            launch();   // warm-up
            e = hipEventRecord(e0, nullptr);
            for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
            if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms > 0.f) best = std::max(best, (double)nvec * 16 * reps / (ms * 1e-3) / 1e9);
            if (e == hipSuccess) e = hipGetLastError();
        }
    }
    if (e == hipSuccess) *gbs = best;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (buf) (void)hipFree(buf);
    if (sink) (void)hipFree(sink);
    return e;
}

template hipError_t run_stream<double>(const DevState<double>&, const Coef<double>&, const RunSpec&);
template hipError_t run_stream<float>(const DevState<float>&, const Coef<float>&, const RunSpec&);

}  // namespace sto
