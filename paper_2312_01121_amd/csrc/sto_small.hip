// SMALL path for N coupled spin-torque oscillators on gfx950: one
// workgroup runs the whole trajectory.  W and the stage input live in LDS,
// each node's state, stage input and RK4 accumulator live in registers, and
// L lanes share one node's row sum of the coupling contraction (paper,
// Eq. (coup)), followed by the right-hand side of Eq. (gov) and the classic
// RK4 bookkeeping (Sec. 3.2).  No launch and no global memory traffic per
// step beyond the records.

#include <algorithm>
#include <climits>
#include <cstdlib>

#include "sto_internal.hpp"

namespace sto {

// ---------------------------------------------------------------------------
// SMALL path: the whole trajectory in one workgroup.
// ---------------------------------------------------------------------------
// L: lanes per node (a compile-time constant, so that the butterfly of the
// row sums has no run-time branches).
template <typename T, bool XYZ, int L>
__global__ void __launch_bounds__(1024) k_small(DevState<T> d, Coef<T> k, const double* __restrict__ u,
                                               T* __restrict__ states, int samples, int substeps,
                                               int cur, int renorm) {
    using A = Acc<T>;
    using AT = typename A::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = d.n;
    const int64_t ld = d.ld;
    T* wsh = reinterpret_cast<T*>(smem_raw);       // n x n
    T* xs = wsh + (int64_t)n * n;                   // [2][3][n]
    const int tid = threadIdx.x;
    const int node = tid / L;
    const int l = tid - node * L;
    const bool active = node < n;
    const int kk = active ? node : n - 1;

    for (int i = tid; i < n * n; i += blockDim.x) {
        int row = i / n;
        wsh[i] = d.W[(int64_t)row * ld + (i - row * n)];
    }
    T mx = d.m[kk], my = d.m[ld + kk], mz = d.m[2 * ld + kk];
    if (active && l == 0) {
        xs[kk] = mx;
        xs[n + kk] = my;
        xs[2 * n + kk] = mz;
    }
    __syncthreads();

    T sx = mx, sy = my, sz = mz;
    T ax = T(0), ay = T(0), az = T(0);
    int b = 0;
    const T* wr = wsh + (int64_t)kk * n;
    for (int s = 0; s < samples; ++s) {
        const T hin = input_field(k, d.w_in + (int64_t)kk * d.n_in, u + (int64_t)s * d.n_in, d.n_in);
        for (int sub = 0; sub < substeps; ++sub) {
            for (int stage = 0; stage < 4; ++stage) {
                const T* xb = xs + b * 3 * n;
                // two independent accumulation chains per lane (even and odd
                // terms), joined before the butterfly
                AT vx = A::zero(), vy = A::zero(), vz = A::zero();
                AT wx = A::zero(), wy = A::zero(), wz = A::zero();
                int j = l;
                for (; j + L < n; j += 2 * L) {
                    const T w0 = wr[j], w1 = wr[j + L];
                    A::fma(vx, w0, xb[j]);
                    A::fma(wx, w1, xb[j + L]);
                    if (XYZ) {
                        A::fma(vy, w0, xb[n + j]);
                        A::fma(wy, w1, xb[n + j + L]);
                        A::fma(vz, w0, xb[2 * n + j]);
                        A::fma(wz, w1, xb[2 * n + j + L]);
                    }
                }
                if (j < n) {
                    const T w0 = wr[j];
                    A::fma(vx, w0, xb[j]);
                    if (XYZ) {
                        A::fma(vy, w0, xb[n + j]);
                        A::fma(vz, w0, xb[2 * n + j]);
                    }
                }
                vx = A::add(vx, wx);
                if (XYZ) {
                    vy = A::add(vy, wy);
                    vz = A::add(vz, wz);
                }
                vx = group_reduce<T>(vx, L);
                T cx = k.a_cp * A::round(vx), cy = T(0), cz = T(0);
                if (XYZ) {
                    vy = group_reduce<T>(vy, L);
                    vz = group_reduce<T>(vz, L);
                    cy = k.a_cp * A::round(vy);
                    cz = k.a_cp * A::round(vz);
                }
                T fx, fy, fz;
                llg_rhs<T, XYZ>(k, sx, sy, sz, cx, cy, cz, hin, fx, fy, fz);
                T nx = rk4_update(k, stage, mx, ax, fx);
                T ny = rk4_update(k, stage, my, ay, fy);
                T nz = rk4_update(k, stage, mz, az, fz);
                if (stage == 3) {
                    if (renorm) renormalize(nx, ny, nz);
                    mx = nx;
                    my = ny;
                    mz = nz;
                }
                sx = nx;
                sy = ny;
                sz = nz;
                if (active && l == 0) {
                    T* xo = xs + (b ^ 1) * 3 * n;
                    xo[kk] = nx;
                    xo[n + kk] = ny;
                    xo[2 * n + kk] = nz;
                }
                b ^= 1;
                __syncthreads();
            }
        }
        if (active && l == 0) {
            if (states) {
                T* rec = states + ((int64_t)s * n + kk) * 3;
                rec[0] = mx;
                rec[1] = my;
                rec[2] = mz;
            }
            if (!finite3(mx, my, mz)) atomicMin(d.bad, s);
        }
    }
    if (active && l == 0) {
        d.m[kk] = mx;
        d.m[ld + kk] = my;
        d.m[2 * ld + kk] = mz;
        T* xc = d.ms[cur];
        xc[kk] = mx;
        xc[ld + kk] = my;
        xc[2 * ld + kk] = mz;
    }
}

static size_t small_lds_bytes(int n, int elem) { return ((size_t)n * n + 6 * (size_t)n) * elem; }
static const size_t kLdsMax = 160 * 1024;

int small_max_n(int elem_bytes, int /*xyz*/) {
    int n = 1;
    while (n + 1 <= 1024 && small_lds_bytes(n + 1, elem_bytes) <= kLdsMax) ++n;
    return n;
}

// Lanes per node.  FP64: a table measured per node count (us per RK4 step
// at N = 1, 2, 4, 8, 10, 16, 24, 32, 48, 64, 100 with the lane counts that
// give 1, 2, 4 and 8 terms per lane): N lanes (one term each) won at N = 4, 8
// and 16, 4 lanes at N = 10, and 8 lanes from N = 24 up, where more lanes
// mean more than 512 threads and slower barriers.  Each entry covers n up to
// the midpoint to the next measured size.  FP32: the largest power of two
// with at least 4 terms per lane.  Both at most 64 lanes and 1,024 threads in
// all.  STO_SMALL_TERMS sets the terms per lane for measurements.
struct SmallLanes {
    int n_max, lanes;
};
constexpr SmallLanes kSmallLanesF64[] = {{3, 2}, {6, 4}, {9, 8}, {13, 4}, {20, 16}, {1 << 30, 8}};

static int small_lanes(int n, int elem_bytes) {
    const char* env = getenv("STO_SMALL_TERMS");
    int L = 1;
    if (env && atoi(env) > 0) {
        const int terms = atoi(env);
        while (L * 2 <= 64 && L * 2 * terms <= n && L * 2 * n <= 1024) L *= 2;
        return L;
    }
    if (elem_bytes == 8) {
        for (const SmallLanes& e : kSmallLanesF64)
            if (n <= e.n_max) {
                L = e.lanes;
                break;
            }
        while (L > 1 && (L > n || L * n > 1024)) L >>= 1;
        return L;
    }
    while (L * 2 <= 64 && L * 2 * 4 <= n && L * 2 * n <= 1024) L *= 2;
    return L;
}

template <typename T, bool XYZ, int L>
static hipError_t launch_small(const DevState<T>& d, const Coef<T>& k, const RunSpec& r, int block, size_t lds) {
    const void* fn = reinterpret_cast<const void*>(&k_small<T, XYZ, L>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_small<T, XYZ, L>), dim3(1), dim3(block), lds, r.stream, d, k, r.u,
                       static_cast<T*>(r.states), r.samples, r.substeps, r.cur, r.renorm);
    return hipGetLastError();
}

template <typename T, bool XYZ>
static hipError_t launch_small_l(int L, const DevState<T>& d, const Coef<T>& k, const RunSpec& r, int block,
                                 size_t lds) {
    switch (L) {
        case 1: return launch_small<T, XYZ, 1>(d, k, r, block, lds);
        case 2: return launch_small<T, XYZ, 2>(d, k, r, block, lds);
        case 4: return launch_small<T, XYZ, 4>(d, k, r, block, lds);
        case 8: return launch_small<T, XYZ, 8>(d, k, r, block, lds);
        case 16: return launch_small<T, XYZ, 16>(d, k, r, block, lds);
        case 32: return launch_small<T, XYZ, 32>(d, k, r, block, lds);
        case 64: return launch_small<T, XYZ, 64>(d, k, r, block, lds);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t run_small(const DevState<T>& d, const Coef<T>& k, const RunSpec& r) {
    const int n = d.n;
    const int L = small_lanes(n, (int)sizeof(T));
    const int block = (L * n + 63) / 64 * 64;
    size_t lds = small_lds_bytes(n, sizeof(T));
    if (L * n > block || block > 1024 || lds > kLdsMax) return hipErrorInvalidValue;
    return r.xyz ? launch_small_l<T, true>(L, d, k, r, block, lds) : launch_small_l<T, false>(L, d, k, r, block, lds);
}

template hipError_t run_small<double>(const DevState<double>&, const Coef<double>&, const RunSpec&);
template hipError_t run_small<float>(const DevState<float>&, const Coef<float>&, const RunSpec&);

}  // namespace sto
