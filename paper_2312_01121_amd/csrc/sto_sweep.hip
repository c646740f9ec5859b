// SWEEP path: many independent reservoirs of uneven size and differing
// constants (a parameter sweep, the use case of paper Sec. 1 and 2), driven
// by one shared input series, stepped together.
//
// One launch evaluates one RK4 stage of every reservoir.  Work is split into
// wave tasks (a table built on the host), each covering consecutive rows of
// one reservoir: the wave is split into lane groups of G lanes, G the
// largest power of two that the reservoir's row pitch fills with 16-byte
// vectors (at most 64), so that short rows do not leave most of a wave idle,
// and each group streams R rows (2, 4 or 8) of that reservoir's coupling
// matrix with non-temporal loads against the reservoir's stage input.  R
// and the row pitch come per reservoir size from a table measured on a
// mixed sweep (a shorter pitch streams fewer padding bytes); every
// reservoir starts on a 256-byte boundary.  The row sums are reduced within
// the group, and R lanes of each group apply the reservoir's own right-hand
// side of Eq. (gov) and the RK4 bookkeeping (Sec. 3.2), exactly as the
// single-reservoir stream kernel does.  The sum of N_r^2 matrix elements is
// read once per stage, so the launch is bound by HBM bandwidth.
//
// The index of the sample being stepped lives in device memory and a
// one-thread kernel advances it after each sample, so the launches of every
// sample are identical: the host captures those of a few samples once into
// a HIP graph and replays it.

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>

#include "sto_internal.hpp"
#include "sto_sweep.hpp"
#include "sweep_tune.hpp"

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

// One wave task: R rows per lane group.  The sample being stepped comes
// from the device counter, so that the launches of one sample are the same
// for every sample (and can be replayed from a graph).
template <typename T, int R, int U>
__device__ __forceinline__ void sweep_task(const SweepDev<T>& d, const SweepTask& tk, const double* __restrict__ u,
                                           int sample, int stage, int cur, int record, int renorm) {
    using A = Acc<T>;
    using AT = typename A::type;
    using V = typename SVec<T>::type;
    constexpr int VN = SVec<T>::n;
    const int lane = threadIdx.x & 63;
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
    // only the vectors that start below n: the row padding is zero, and
    // leaving it unread saves its HBM traffic
#pragma unroll U
    for (int64_t c = (int64_t)gl * VN; c < n; c += (int64_t)G * VN) {
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
    const T hin = input_field(k, d.w_in + res.winoff + (int64_t)row * d.n_in, u + (int64_t)sample * d.n_in, d.n_in);
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

// One RK4 stage of every reservoir; each wave runs one task with the task's
// rows per lane group (wave-uniform).
template <typename T, int U>
__global__ void __launch_bounds__(256) k_sweep_stage(SweepDev<T> d, const double* __restrict__ u, int stage, int cur,
                                                     int record, int renorm) {
    const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (task >= d.tasks) return;   // wave-uniform
    const SweepTask tk = d.task[task];
    if (tk.n == 0) return;   // padding of the XCD-aware task order (wave-uniform)
    const int sample = *d.sample;
    switch (tk.rpg) {
        case 2: sweep_task<T, 2, U>(d, tk, u, sample, stage, cur, record, renorm); break;
        case 4: sweep_task<T, 4, U>(d, tk, u, sample, stage, cur, record, renorm); break;
        default: sweep_task<T, 8, U>(d, tk, u, sample, stage, cur, record, renorm); break;
    }
}

__global__ void k_sweep_set(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_sweep_next(int* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p += 1;
}

int env_int(const char* name) {
    const char* v = getenv(name);
    return v && *v ? atoi(v) : 0;
}

// The launches of `samples` samples (4 per RK4 step, then the sample counter).
template <typename T>
void issue(const SweepDev<T>& d, const RunSpec& r, int samples, hipStream_t st) {
    constexpr int U = sizeof(T) == 8 ? 4 : 2;
    const dim3 grid((d.tasks + 3) / 4), block(256);
    for (int s = 0; s < samples; ++s) {
        for (int sub = 0; sub < r.substeps; ++sub)
            for (int stage = 0; stage < 4; ++stage) {
                const int rec = stage == 3 && sub == r.substeps - 1;
                const int c = r.cur ^ (stage & 1);
                hipLaunchKernelGGL((k_sweep_stage<T, U>), grid, block, 0, st, d, r.u, stage, c, rec, r.renorm);
            }
        hipLaunchKernelGGL(k_sweep_next, dim3(1), dim3(64), 0, st, d.sample);
    }
}

// Rows per lane group and row pitch (elements) of the reservoirs of n nodes.
void sweep_shape(int elem_bytes, int n, int* rows_per_group, int* pitch) {
    const int env_rows = env_int("STO_SWEEP_ROWS"), env_pitch = env_int("STO_SWEEP_PITCH");
    int rpg = 8, p = 64;
    bool found = false;
    // STO_SWEEP_TABLE="n_max:rows:pitch,...", scanned like the table, replaces
    // it for both element types (the autotuner's candidates)
    if (const char* t = getenv("STO_SWEEP_TABLE")) {
        while (*t && !found) {
            int nm = 0, r = 0, pp = 0, used = 0;
            if (sscanf(t, "%d:%d:%d%n", &nm, &r, &pp, &used) != 3) break;
            if (n <= nm) {
                rpg = r;
                p = pp;
                found = true;
            }
            t += used;
            if (*t == ',') ++t;
        }
        found = true;   // a given table replaces the compiled one even where it has no entry
    }
    for (const SweepTuneEntry& e : kSweepTune) {
        if (found) break;
        if (e.elem_bytes == elem_bytes && n <= e.n_max) {
            rpg = e.rows;
            p = e.pitch;
            found = true;
        }
    }
    if (rpg != 2 && rpg != 4 && rpg != 8) rpg = 8;
    if (env_rows == 2 || env_rows == 4 || env_rows == 8) rpg = env_rows;
    if (env_pitch > 0) p = env_pitch;
    const int vn = 16 / elem_bytes;   // the pitch keeps every row 16-byte aligned
    p = std::max(vn, (p + vn - 1) / vn * vn);
    *rows_per_group = rpg;
    *pitch = p;
}

}  // namespace

SweepLayout sweep_layout(int elem_bytes, int count, const int64_t* n, int n_in) {
    SweepLayout L;
    const int64_t vn = 16 / elem_bytes, align = 256 / elem_bytes;
    int64_t woff = 0, soff = 0;
    for (int r = 0; r < count; ++r) {
        SweepRes x;
        int rpg = 8, pitch = 64;
        sweep_shape(elem_bytes, (int)n[r], &rpg, &pitch);
        x.n = (int)n[r];
        x.pad = 0;
        // a lane group holds at least as many lanes as rows (lane q of a
        // group finishes row q): the pitch holds at least rpg 16-byte vectors
        x.ld = (std::max<int64_t>(n[r], rpg * vn) + pitch - 1) / pitch * pitch;
        x.woff = woff;
        x.soff = soff;
        x.winoff = L.win_elems;
        x.noff = L.nodes;
        L.res.push_back(x);
        // every reservoir starts on a 256-byte boundary, so that a short row
        // pitch of one reservoir does not misalign the cache lines of every
        // reservoir after it
        woff = (woff + n[r] * x.ld + align - 1) / align * align;
        soff = (soff + 3 * x.ld + align - 1) / align * align;
        L.win_elems += n[r] * n_in;
        L.nodes += n[r];
    }
    L.w_elems = woff;
    L.s_elems = soff;

    // Wave tasks: a task covers rpg rows per lane group times the groups in
    // a wave.  The workgroups of a launch go to the chip's XCDs in turn
    // (workgroup b to XCD b mod 8), each XCD with its own L2.  With the
    // XCD-aware order every reservoir is given whole to one XCD, so its
    // stage input and state are fetched into one L2 only: reservoirs are
    // dealt to the XCDs largest first, each to the least loaded (bytes of W),
    // and workgroup k*8 + x runs the k-th four tasks of XCD x (empty tasks
    // pad the shorter lists).  Within an XCD, and in the plain order, tasks
    // follow the reservoir order (largest first was measured slower: the
    // small tasks then form the tail).
    std::vector<std::vector<SweepTask>> per(count);
    for (int r = 0; r < count; ++r) {
        const SweepRes& x = L.res[r];
        int rpg = 8, pitch = 64;
        sweep_shape(elem_bytes, x.n, &rpg, &pitch);
        const int rows = rpg * (64 / group_lanes(x.ld, (int)vn));
        for (int row = 0; row < x.n; row += rows) per[r].push_back({x.woff, x.soff, (int)x.ld, x.n, r, row, rpg, 0});
    }
    const char* xcd_env = getenv("STO_SWEEP_XCD");
    const bool xcd = !(xcd_env && *xcd_env == '0');
    if (!xcd) {
        for (int r = 0; r < count; ++r) L.tasks.insert(L.tasks.end(), per[r].begin(), per[r].end());
        return L;
    }
    constexpr int kXcds = 8, kTasksPerBlock = 4;
    std::vector<int> order(count);
    for (int r = 0; r < count; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return L.res[a].n * L.res[a].ld > L.res[b].n * L.res[b].ld; });
    std::vector<std::vector<int>> bin(kXcds);
    std::vector<int64_t> load(kXcds, 0);
    for (int r : order) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        bin[x].push_back(r);
        load[x] += L.res[r].n * L.res[r].ld;
    }
    std::vector<std::vector<SweepTask>> list(kXcds);
    size_t blocks = 0;
    for (int x = 0; x < kXcds; ++x) {
        std::sort(bin[x].begin(), bin[x].end());
        for (int r : bin[x]) list[x].insert(list[x].end(), per[r].begin(), per[r].end());
        blocks = std::max(blocks, (list[x].size() + kTasksPerBlock - 1) / kTasksPerBlock);
    }
    const SweepTask empty{0, 0, 0, 0, 0, 0, 8, 0};
    L.tasks.assign(blocks * kXcds * kTasksPerBlock, empty);
    for (int x = 0; x < kXcds; ++x)
        for (size_t i = 0; i < list[x].size(); ++i) {
            const size_t k = i / kTasksPerBlock, w = i % kTasksPerBlock;
            L.tasks[(k * kXcds + x) * kTasksPerBlock + w] = list[x][i];
        }
    return L;
}

template <typename T>
hipError_t run_sweep(const SweepDev<T>& d, const RunSpec& r, hipStream_t capture, int graph_samples,
                     hipGraph_t* graph, hipGraphExec_t* exec) {
    hipLaunchKernelGGL(k_sweep_set, dim3(1), dim3(64), 0, r.stream, d.sample, 0);
    int done = 0;
    if (capture && graph_samples > 0 && r.samples >= graph_samples) {
        hipError_t e = hipStreamBeginCapture(capture, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return e;
        issue<T>(d, r, graph_samples, capture);
        e = hipStreamEndCapture(capture, graph);
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return e;
        for (; done + graph_samples <= r.samples; done += graph_samples) {
            e = hipGraphLaunch(*exec, r.stream);
            if (e != hipSuccess) return e;
        }
    }
    issue<T>(d, r, r.samples - done, r.stream);
    return hipGetLastError();
}

template hipError_t run_sweep<double>(const SweepDev<double>&, const RunSpec&, hipStream_t, int, hipGraph_t*,
                                      hipGraphExec_t*);
template hipError_t run_sweep<float>(const SweepDev<float>&, const RunSpec&, hipStream_t, int, hipGraph_t*,
                                     hipGraphExec_t*);

}  // namespace sto
