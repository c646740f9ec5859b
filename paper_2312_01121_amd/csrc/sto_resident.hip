// RESIDENT path: the whole trajectory in one cooperative launch, with the
// coupling matrix split across the LDS of all co-resident workgroups.
//
// Workgroup g owns a contiguous block of rows of W (paper, Eq. (coup)) and
// keeps it in LDS for the entire run; the state, stage input and RK4
// accumulator of its rows live in registers.  Every RK4 stage needs the
// whole stage input m^x of all nodes (Sec. 3.3: the coupling is W^cp x), so
// stages are separated by a grid-wide barrier: each workgroup publishes its
// rows of the next stage input to global memory, crosses the barrier, and
// stages the full vector into LDS.
//
// The barrier is a counter plus a generation word in global memory with
// agent-scope release/acquire.  Its wait loop is bounded: after a spin
// limit it raises a sticky abort flag and every workgroup leaves the
// kernel, so a grid that is not co-resident ends with an error instead of
// a hang.  The cooperative launch itself refuses grids that cannot be
// co-resident.

#include <climits>

#include "sto_internal.hpp"

namespace sto {

namespace {

constexpr int kBlock = 256;              // 4 waves
constexpr int kWaves = kBlock / 64;
constexpr int kMaxRowsPerWave = 4;       // rows per workgroup <= 16
constexpr int kSpinLimit = 1 << 24;      // ~0.5 s of s_sleep(1) polls
constexpr size_t kLdsMax = 160 * 1024 - 256;   // leave room for the static barrier word

// Barrier words (int offsets into DevState::sync, 256 bytes zeroed before
// every launch): arrive counter, generation, abort flag on separate lines.
constexpr int kArrive = 0, kGen = 16, kAbort = kSyncAbortWord;

__device__ bool grid_barrier(int* sync, int nblocks, int& gen, int* ok_lds) {
    __threadfence();       // release this thread's global writes at agent scope
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const int target = gen + 1;
        const int arrived = __hip_atomic_fetch_add(sync + kArrive, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(sync + kArrive, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(sync + kGen, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            int spins = 0;
            while (__hip_atomic_load(sync + kGen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (__hip_atomic_load(sync + kAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
                if (++spins > kSpinLimit) {
                    __hip_atomic_store(sync + kAbort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __threadfence();   // acquire: later loads of this workgroup see the other groups' writes
        gen = target;
        *ok_lds = ok;
    }
    __syncthreads();
    return *ok_lds != 0;
}

template <typename T, bool XYZ>
__global__ void __launch_bounds__(kBlock) k_resident(DevState<T> d, Coef<T> k, const double* __restrict__ u,
                                                     T* __restrict__ states, int samples, int substeps, int cur,
                                                     int renorm, int rows_per_block, int wld) {
    using A = Acc<T>;
    using AT = typename A::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int ok_lds;
    const int n = d.n;
    const int64_t ld = d.ld;
    T* wsh = reinterpret_cast<T*>(smem_raw);                    // rows_per_block x wld
    T* xs = wsh + (int64_t)rows_per_block * wld;                // [3][n] stage input
    const int row_begin = blockIdx.x * rows_per_block;
    const int nrows = max(0, min(rows_per_block, n - row_begin));
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;

    for (int i = threadIdx.x; i < nrows * n; i += kBlock) {
        const int r = i / n;
        const int c = i - r * n;
        wsh[(int64_t)r * wld + c] = d.W[(int64_t)(row_begin + r) * ld + c];
    }

    // Registers of the rows this wave owns (rows wave, wave + 4, ...); every
    // lane keeps a copy, lane 0 publishes.
    T mx[kMaxRowsPerWave], my[kMaxRowsPerWave], mz[kMaxRowsPerWave];
    T ax[kMaxRowsPerWave], ay[kMaxRowsPerWave], az[kMaxRowsPerWave];
    T sx[kMaxRowsPerWave], sy[kMaxRowsPerWave], sz[kMaxRowsPerWave];
    T hin[kMaxRowsPerWave];
#pragma unroll
    for (int q = 0; q < kMaxRowsPerWave; ++q) {
        const int r = wave + q * kWaves;
        const int row = row_begin + min(r, max(nrows - 1, 0));
        const int rr = min(row, n - 1);
        mx[q] = sx[q] = d.m[rr];
        my[q] = sy[q] = d.m[ld + rr];
        mz[q] = sz[q] = d.m[2 * ld + rr];
        ax[q] = ay[q] = az[q] = T(0);
        hin[q] = T(0);
    }

    int gen = 0;
    int b = cur;
    for (int s = 0; s < samples; ++s) {
#pragma unroll
        for (int q = 0; q < kMaxRowsPerWave; ++q) {
            const int r = wave + q * kWaves;
            if (r < nrows)
                hin[q] = input_field(k, d.w_in + (int64_t)(row_begin + r) * d.n_in, u + (int64_t)s * d.n_in, d.n_in);
        }
        for (int sub = 0; sub < substeps; ++sub) {
            for (int stage = 0; stage < 4; ++stage) {
                // stage the current stage input (all nodes) into LDS
                const T* xin = d.ms[b];
                for (int i = threadIdx.x; i < n; i += kBlock) {
                    xs[i] = xin[i];
                    if (XYZ) {
                        xs[n + i] = xin[ld + i];
                        xs[2 * n + i] = xin[2 * ld + i];
                    }
                }
                __syncthreads();
                T* xout = d.ms[b ^ 1];
#pragma unroll
                for (int q = 0; q < kMaxRowsPerWave; ++q) {
                    const int r = wave + q * kWaves;
                    if (r >= nrows) break;   // wave-uniform
                    const T* wr = wsh + (int64_t)r * wld;
                    AT vx = A::zero(), vy = A::zero(), vz = A::zero();
                    for (int j = lane; j < n; j += 64) {
                        const T w = wr[j];
                        A::fma(vx, w, xs[j]);
                        if (XYZ) {
                            A::fma(vy, w, xs[n + j]);
                            A::fma(vz, w, xs[2 * n + j]);
                        }
                    }
                    vx = group_reduce<T>(vx, 64);
                    T cx = k.a_cp * A::round(vx), cy = T(0), cz = T(0);
                    if (XYZ) {
                        vy = group_reduce<T>(vy, 64);
                        vz = group_reduce<T>(vz, 64);
                        cy = k.a_cp * A::round(vy);
                        cz = k.a_cp * A::round(vz);
                    }
                    T fx, fy, fz;
                    llg_rhs<T, XYZ>(k, sx[q], sy[q], sz[q], cx, cy, cz, hin[q], fx, fy, fz);
                    T nx = rk4_update(k, stage, mx[q], ax[q], fx);
                    T ny = rk4_update(k, stage, my[q], ay[q], fy);
                    T nz = rk4_update(k, stage, mz[q], az[q], fz);
                    if (stage == 3) {
                        if (renorm) renormalize(nx, ny, nz);
                        mx[q] = nx;
                        my[q] = ny;
                        mz[q] = nz;
                    }
                    sx[q] = nx;
                    sy[q] = ny;
                    sz[q] = nz;
                    if (lane == 0) {
                        const int row = row_begin + r;
                        xout[row] = nx;
                        xout[ld + row] = ny;
                        xout[2 * ld + row] = nz;
                    }
                }
                b ^= 1;
                if (!grid_barrier(d.sync, gridDim.x, gen, &ok_lds)) return;
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < kMaxRowsPerWave; ++q) {
                const int r = wave + q * kWaves;
                if (r >= nrows) break;
                const int row = row_begin + r;
                if (states) {
                    T* rec = states + ((int64_t)s * n + row) * 3;
                    rec[0] = mx[q];
                    rec[1] = my[q];
                    rec[2] = mz[q];
                }
                if (!finite3(mx[q], my[q], mz[q])) atomicMin(d.bad, s);
            }
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < kMaxRowsPerWave; ++q) {
            const int r = wave + q * kWaves;
            if (r >= nrows) break;
            const int row = row_begin + r;
            d.m[row] = mx[q];
            d.m[ld + row] = my[q];
            d.m[2 * ld + row] = mz[q];
        }
    }
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

int64_t wld_of(int n) { return (n + 3) / 4 * 4; }

size_t resident_lds(int n, int rows_per_block, int elem) {
    return ((size_t)rows_per_block * wld_of(n) + 3 * (size_t)n) * elem;
}

}  // namespace

bool resident_fits(int n, int elem_bytes, int /*xyz*/, int* grid_out) {
    const int cus = device_cus();
    if (cus <= 0 || n < 2) return false;
    const int rpb = (n + cus - 1) / cus;
    if (rpb > kWaves * kMaxRowsPerWave) return false;
    if (resident_lds(n, rpb, elem_bytes) > kLdsMax) return false;
    if (grid_out) *grid_out = (n + rpb - 1) / rpb;
    return true;
}

template <typename T>
hipError_t run_resident(const DevState<T>& d, const Coef<T>& k, const RunSpec& r) {
    int grid = 0;
    if (!resident_fits(d.n, sizeof(T), r.xyz, &grid)) return hipErrorInvalidValue;
    const int rpb = (d.n + grid - 1) / grid;
    int wld = (int)wld_of(d.n);
    const size_t lds = resident_lds(d.n, rpb, sizeof(T));
    hipError_t e = hipMemsetAsync(d.sync, 0, 256, r.stream);
    if (e != hipSuccess) return e;
    DevState<T> dd = d;
    Coef<T> kk = k;
    const double* u = r.u;
    T* states = static_cast<T*>(r.states);
    int samples = r.samples, substeps = r.substeps, cur = r.cur, renorm = r.renorm, rows = rpb;
    void* args[] = {&dd, &kk, &u, &states, &samples, &substeps, &cur, &renorm, &rows, &wld};
    const void* fn = r.xyz ? reinterpret_cast<const void*>(&k_resident<T, true>)
                           : reinterpret_cast<const void*>(&k_resident<T, false>);
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args, (unsigned)lds, r.stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template hipError_t run_resident<double>(const DevState<double>&, const Coef<double>&, const RunSpec&);
template hipError_t run_resident<float>(const DevState<float>&, const Coef<float>&, const RunSpec&);

}  // namespace sto
