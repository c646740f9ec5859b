// SWEEP path: many independent reservoirs of uneven size and differing
// constants (a parameter sweep, the use case of paper Sec. 1 and 2), driven
// by one shared input series, stepped together.
//
// One launch evaluates one RK4 stage of every reservoir.  Work is split into
// wave tasks (a table built on the host), each covering consecutive rows of
// one reservoir: the wave is split into lane groups of G lanes, G the
// largest power of two that the reservoir's row pitch fills with 16-byte
// vectors (at most 64), and each group streams R rows of that reservoir's
// coupling matrix with non-temporal loads against the reservoir's stage
// input.  Short rows therefore do not leave most of a wave idle.  The row
// sums are reduced within the group, and R lanes of each group apply the
// reservoir's own right-hand side of Eq. (gov) and the RK4 bookkeeping
// (Sec. 3.2), exactly as the single-reservoir stream kernel does.  The sum
// of N_r^2 matrix elements is read once per stage, so the launch is bound by
// HBM bandwidth.

#include <climits>
#include <cstdlib>

#include "sto_internal.hpp"
#include "sto_sweep.hpp"

namespace sto {

namespace {

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <typename T> struct SVec;
template <> struct SVec<double> { using type = dvec2; static constexpr int n = 2; };
template <> struct SVec<float> { using type = fvec4; static constexpr int n = 4; };

// Lanes per row group for a reservoir of row pitch ld: the largest power of
// two <= min(64, ld / VN), so that rows shorter than 64 vectors do not leave
// most of a wave idle.  A wave task then holds 64 / G groups of R rows.
__host__ __device__ inline int group_lanes(int64_t ld, int vn) {
    int g = 64;
    while (g > 1 && (int64_t)g * vn > ld) g >>= 1;
    return g;
}

template <typename T, int R, int U>
__global__ void __launch_bounds__(256) k_sweep_stage(SweepDev<T> d, const double* __restrict__ u_s, int sample,
                                                     int stage, int cur, int record, int renorm) {
    using A = Acc<T>;
    using AT = typename A::type;
    using V = typename SVec<T>::type;
    constexpr int VN = SVec<T>::n;
    const int lane = threadIdx.x & 63;
    const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (task >= d.tasks) return;   // wave-uniform
    const SweepTask tk = d.task[task];
    const int n = tk.n;
    const int64_t ld = tk.ld;
    const int G = group_lanes(ld, VN);   // wave-uniform
    const int gl = lane & (G - 1);
    const int rowg = tk.row + (lane / G) * R;   // first row of this lane's group
    const T* W = d.W + tk.woff;
    T* m = d.m + tk.soff;
    T* acc = d.acc + tk.soff;
    const T* xin = d.ms[cur] + tk.soff;
    T* xout = d.ms[cur ^ 1] + tk.soff;
    const int row = rowg + gl;
    const bool own = gl < R && row < n;
    const SweepRes res = d.res[tk.res];
    const Coef<T> k = d.coef[tk.res];

    // the epilogue's state inputs do not depend on the row sums: load them
    // before the coupling pass so that their latency overlaps it
    T sx = T(0), sy = T(0), sz = T(0), mx = T(0), my = T(0), mz = T(0), ax = T(0), ay = T(0), az = T(0);
    if (own) {
        sx = xin[row];
        sy = xin[ld + row];
        sz = xin[2 * ld + row];
        mx = m[row];
        my = m[ld + row];
        mz = m[2 * ld + row];
        if (stage > 0) {
            ax = acc[row];
            ay = acc[ld + row];
            az = acc[2 * ld + row];
        }
    }

    const T* wrow[R];
#pragma unroll
    for (int r = 0; r < R; ++r) wrow[r] = W + (int64_t)min(rowg + r, n - 1) * ld;
    AT av[R];
#pragma unroll
    for (int r = 0; r < R; ++r) av[r] = A::zero();
#pragma unroll U
    for (int64_t c = (int64_t)gl * VN; c < ld; c += (int64_t)G * VN) {
        const V xv = *reinterpret_cast<const V*>(xin + c);
        V wv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) wv[r] = __builtin_nontemporal_load(reinterpret_cast<const V*>(wrow[r] + c));
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int e = 0; e < VN; ++e) A::fma(av[r], wv[r][e], xv[e]);
    }
    T dot = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const AT s = group_reduce<T>(av[r], G);
        if (gl == r) dot = A::round(s);
    }
    if (!own) return;
    const T hin = input_field(k, d.w_in + res.winoff + (int64_t)row * d.n_in, u_s, d.n_in);
    T fx, fy, fz;
    llg_rhs<T, false>(k, sx, sy, sz, k.a_cp * dot, T(0), T(0), hin, fx, fy, fz);
    T nx = rk4_update(k, stage, mx, ax, fx);
    T ny = rk4_update(k, stage, my, ay, fy);
    T nz = rk4_update(k, stage, mz, az, fz);
    if (stage == 3) {
        if (renorm) renormalize(nx, ny, nz);
        m[row] = nx;
        m[ld + row] = ny;
        m[2 * ld + row] = nz;
        if (record && d.states) {
            T* rec = d.states + (d.rec_samples * res.noff + (int64_t)sample * n + row) * 3;
            rec[0] = nx;
            rec[1] = ny;
            rec[2] = nz;
        }
        if (!finite3(nx, ny, nz)) atomicMin(d.bad, sample);
    } else {
        acc[row] = ax;
        acc[ld + row] = ay;
        acc[2 * ld + row] = az;
    }
    xout[row] = nx;
    xout[ld + row] = ny;
    xout[2 * ld + row] = nz;
}

}  // namespace

// Rows per lane group (R): 8, measured fastest on a 256-reservoir sweep
// (361.9 us per RK4 step against 368.6 with 4 and 415 with 2; visiting the
// tasks last-to-first on alternate stages measured slower, 369.2).
// STO_SWEEP_ROWS (2, 4 or 8) overrides it for measurements; it is read once
// per process, so the task table and the kernel always agree.
int sweep_rows_per_task(int elem_bytes) {
    (void)elem_bytes;
    static const int rows = [] {
        const char* v = getenv("STO_SWEEP_ROWS");
        const int r = v ? atoi(v) : 8;
        return (r == 2 || r == 4) ? r : 8;
    }();
    return rows;
}

// Rows of one reservoir covered by one wave task: R rows per lane group
// times the groups in a wave.
int sweep_task_rows(int64_t ld, int elem_bytes) {
    return sweep_rows_per_task(elem_bytes) * (64 / group_lanes(ld, 16 / elem_bytes));
}

template <typename T>
hipError_t run_sweep(const SweepDev<T>& d, const RunSpec& r) {
    constexpr int U = sizeof(T) == 8 ? 4 : 2;
    const int R = sweep_rows_per_task((int)sizeof(T));
    const dim3 grid((d.tasks + 3) / 4), block(256);
    for (int s = 0; s < r.samples; ++s) {
        const double* u_s = r.u + (int64_t)s * d.n_in;
        for (int sub = 0; sub < r.substeps; ++sub)
            for (int stage = 0; stage < 4; ++stage) {
                const int rec = stage == 3 && sub == r.substeps - 1;
                const int c = r.cur ^ (stage & 1);
                if (R == 4)
                    hipLaunchKernelGGL((k_sweep_stage<T, 4, U>), grid, block, 0, r.stream, d, u_s, s, stage, c, rec,
                                       r.renorm);
                else if (R == 8)
                    hipLaunchKernelGGL((k_sweep_stage<T, 8, U>), grid, block, 0, r.stream, d, u_s, s, stage, c, rec,
                                       r.renorm);
                else
                    hipLaunchKernelGGL((k_sweep_stage<T, 2, U>), grid, block, 0, r.stream, d, u_s, s, stage, c, rec,
                                       r.renorm);
            }
    }
    return hipGetLastError();
}

template hipError_t run_sweep<double>(const SweepDev<double>&, const RunSpec&);
template hipError_t run_sweep<float>(const SweepDev<float>&, const RunSpec&);

}  // namespace sto
