// Many ridge readouts at once: `count` record sets, each with its target
// series (the reservoirs of a sweep, or the S streams of one multi-stream
// reservoir), each fitted as readout.hip fits one -- design matrix
// [features, 1], normal equations in the primal (rows >= cols) or dual
// form, Cholesky factorisation, substitution, NMSE, all in FP64 -- but with
// every kernel covering all items: their design and Gram matrices sit side
// by side in device memory, and the number of launches does not grow with
// the number of items.
//
// The Cholesky factorisation G = L L^T is blocked.  For each panel of kNB
// columns, one workgroup per item factors the diagonal block in LDS and
// solves the rows below it against that block (L21 = A21 L11^-T); the
// trailing lower triangle is then updated by the rank-kNB product
// A22 -= L21 L21^T over 16 x 16 tiles listed across all items.  That is two
// launches per panel, where the column-at-a-time factorisation of
// readout_solve takes two per column.

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "readout_batch.hpp"

namespace sto {

namespace {

constexpr int kNB = 32;   // panel width of the blocked Cholesky
constexpr int kT = 16;    // tile edge of the Gram and trailing-update kernels

struct RItem {
    const void* rec;    // record of the item's first fitted row
    int64_t stride;     // elements between consecutive records
    const double* y;    // targets of the fitted rows
    double* w;          // weights out (cols)
    int64_t phi;        // offset (doubles) of the design matrix, rows x cols
    int64_t c;          // offset of the Gram matrix, m x m (lower triangle used)
    int64_t rhs;        // offset of the right-hand side, then the solution (m)
    int n, cols, m, primal;
};

// The item owning flat tile b: start[q] <= b < start[q + 1] (start has
// count + 1 entries, start[0] = 0; items without tiles have empty ranges).
__device__ __forceinline__ int item_of(const int64_t* start, int count, int64_t b) {
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Lower-triangle tile t, counted row by row over tj <= ti, as (ti, tj).
__device__ __forceinline__ void tri_tile(int64_t t, int& ti, int& tj) {
    int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)(r + 1) * (r + 2) / 2 <= t) ++r;
    while ((int64_t)r * (r + 1) / 2 > t) --r;
    ti = r;
    tj = (int)(t - (int64_t)r * (r + 1) / 2);
}

// Design matrices: phi_i[r][j] = feature j of record r, last column 1.
// Raises bad[2 q + 1] if a feature or target of item q is not finite.
template <typename R>
__global__ void k_bgather(const RItem* __restrict__ items, int rows, int features, double* __restrict__ phi_base,
                          int* bad) {
    const int q = blockIdx.y;
    const RItem it = items[q];
    const double* y = it.y;
    const R* rec = static_cast<const R*>(it.rec);
    double* phi = phi_base + it.phi;
    const int cols = it.cols;
    const int64_t total = (int64_t)rows * cols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / cols);
        const int j = (int)(i - (int64_t)r * cols);
        double v = 1.0;
        if (j < cols - 1) v = (double)rec[(int64_t)r * it.stride + (features ? j : 3 * j)];
        if (!__builtin_isfinite(v) || (j == cols - 1 && !__builtin_isfinite(y[r]))) atomicExch(bad + 2 * q + 1, 1);
        phi[i] = v;
    }
}

// Lower-triangle 16 x 16 tiles of every item's Gram matrix plus lambda I:
// Phi^T Phi (primal) or Phi Phi^T (dual).  Loads are coalesced along the
// rows of Phi in both forms.
__global__ void __launch_bounds__(256) k_bgram(const RItem* __restrict__ items, const int64_t* __restrict__ start,
                                               int count, int rows, double lam, const double* __restrict__ phi_base,
                                               double* __restrict__ c_base) {
    __shared__ double a[kT][kT + 1];
    __shared__ double b[kT][kT + 1];
    const int q = item_of(start, count, blockIdx.x);
    const RItem it = items[q];
    int ti, tj;
    tri_tile(blockIdx.x - start[q], ti, tj);
    const double* X = phi_base + it.phi;
    const int m = it.m, cols = it.cols;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int i = ti * kT + ty, j = tj * kT + tx;
    double s = 0.0;
    if (it.primal) {
        // C[i][j] = sum over rows t of X[t][i] X[t][j]; a[t][x] = X[t0 + t][16 ti + x]
        for (int t0 = 0; t0 < rows; t0 += kT) {
            const int t = t0 + ty;
            a[ty][tx] = (t < rows && ti * kT + tx < m) ? X[(int64_t)t * cols + ti * kT + tx] : 0.0;
            b[ty][tx] = (t < rows && tj * kT + tx < m) ? X[(int64_t)t * cols + tj * kT + tx] : 0.0;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kT; ++k) s = __builtin_fma(a[k][ty], b[k][tx], s);
            __syncthreads();
        }
    } else {
        // C[i][j] = sum over columns t of X[i][t] X[j][t]; a[y][t] = X[16 ti + y][t0 + t]
        for (int t0 = 0; t0 < cols; t0 += kT) {
            const int t = t0 + tx;
            a[ty][tx] = (ti * kT + ty < m && t < cols) ? X[(int64_t)(ti * kT + ty) * cols + t] : 0.0;
            b[ty][tx] = (tj * kT + ty < m && t < cols) ? X[(int64_t)(tj * kT + ty) * cols + t] : 0.0;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kT; ++k) s = __builtin_fma(a[ty][k], b[tx][k], s);
            __syncthreads();
        }
    }
    if (i < m && j < m && j <= i) c_base[it.c + (int64_t)i * m + j] = s + (i == j ? lam : 0.0);
}

// mode 0: right-hand side, Phi^T y (primal) or y (dual).
// mode 1: weights from the solution a, a itself (primal) or Phi^T a (dual).
__global__ void k_bvec(const RItem* __restrict__ items, int rows, const double* __restrict__ phi_base,
                       double* __restrict__ rhs_base, int mode, const int* bad) {
    const int q = blockIdx.y;
    const RItem it = items[q];
    const double* y = it.y;
    if (mode == 1 && (bad[2 * q] | bad[2 * q + 1])) return;
    const double* phi = phi_base + it.phi;
    double* rhs = rhs_base + it.rhs;
    const int len = mode == 0 ? it.m : it.cols;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < len; j += gridDim.x * blockDim.x) {
        const double* v = mode == 0 ? y : rhs;
        const bool product = mode == 0 ? it.primal : !it.primal;
        double s;
        if (product) {
            s = 0.0;
            for (int r = 0; r < rows; ++r) s = __builtin_fma(phi[(int64_t)r * it.cols + j], v[r], s);
        } else {
            s = v[j];
        }
        if (mode == 0) rhs[j] = s;
        else it.w[j] = s;
    }
}

// Panel j0 of every item's factorisation: the diagonal block in LDS, then
// the rows below it.  Raises bad[2 q] when item q is not positive definite.
__global__ void __launch_bounds__(256) k_bpanel(const RItem* __restrict__ items, double* __restrict__ c_base, int j0,
                                                int* bad) {
    __shared__ double L[kNB][kNB + 1];
    const int q = blockIdx.x;
    const RItem it = items[q];
    const int m = it.m;
    if (j0 >= m || (bad[2 * q] | bad[2 * q + 1])) return;   // block-uniform
    double* C = c_base + it.c;
    const int jb = min(kNB, m - j0);
    const int t = threadIdx.x;
    for (int e = t; e < jb * jb; e += blockDim.x) {
        const int a = e / jb, b = e - a * jb;
        L[a][b] = b <= a ? C[(int64_t)(j0 + a) * m + j0 + b] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < jb; ++k) {
        const double d = L[k][k];
        if (!(d > 0.0)) {   // every thread read the same d: all leave together
            if (t == 0) atomicExch(bad + 2 * q, 1);
            return;
        }
        const double lkk = __builtin_sqrt(d);
        __syncthreads();   // L[k][k] read by all before it is overwritten
        if (t == 0) L[k][k] = lkk;
        for (int a = k + 1 + t; a < jb; a += blockDim.x) L[a][k] = L[a][k] / lkk;
        __syncthreads();
        const int r = jb - k - 1;
        for (int e = t; e < r * r; e += blockDim.x) {
            const int a = k + 1 + e / r, b = k + 1 + e % r;
            if (b <= a) L[a][b] -= L[a][k] * L[b][k];
        }
        __syncthreads();
    }
    for (int e = t; e < jb * jb; e += blockDim.x) {
        const int a = e / jb, b = e - a * jb;
        if (b <= a) C[(int64_t)(j0 + a) * m + j0 + b] = L[a][b];
    }
    // rows below the block: x L11^T = a, x_b = (a_b - sum_{k<b} x_k L_bk) / L_bb
    for (int row = j0 + jb + t; row < m; row += blockDim.x) {
        double* cr = C + (int64_t)row * m + j0;
        double x[kNB];
#pragma unroll
        for (int b = 0; b < kNB; ++b) x[b] = b < jb ? cr[b] : 0.0;
#pragma unroll
        for (int b = 0; b < kNB; ++b) {
            if (b < jb) {
                double s = x[b];
#pragma unroll
                for (int k = 0; k < b; ++k) s -= x[k] * L[b][k];
                x[b] = s / L[b][b];
            }
        }
#pragma unroll
        for (int b = 0; b < kNB; ++b)
            if (b < jb) cr[b] = x[b];
    }
}

// Trailing update after panel j0: A22 -= L21 L21^T on the lower triangle,
// one 16 x 16 tile per workgroup, tiles of all items listed by `start`.
__global__ void __launch_bounds__(256) k_bupdate(const RItem* __restrict__ items, const int64_t* __restrict__ start,
                                                 int count, double* __restrict__ c_base, int j0, const int* bad) {
    __shared__ double La[kT][kNB + 1];
    __shared__ double Lb[kT][kNB + 1];
    const int q = item_of(start, count, blockIdx.x);
    if (bad[2 * q] | bad[2 * q + 1]) return;   // block-uniform
    const RItem it = items[q];
    const int m = it.m;
    const int jb = min(kNB, m - j0);
    const int r0 = j0 + jb;   // first trailing row and column
    int ti, tj;
    tri_tile(blockIdx.x - start[q], ti, tj);
    double* C = c_base + it.c;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kT + tx;
    for (int e = tid; e < kT * kNB; e += kT * kT) {
        const int y = e / kNB, k = e - y * kNB;
        const int ra = r0 + ti * kT + y, rb = r0 + tj * kT + y;
        La[y][k] = (ra < m && k < jb) ? C[(int64_t)ra * m + j0 + k] : 0.0;
        Lb[y][k] = (rb < m && k < jb) ? C[(int64_t)rb * m + j0 + k] : 0.0;
    }
    __syncthreads();
    const int i = r0 + ti * kT + ty, j = r0 + tj * kT + tx;
    if (i < m && j < m && j <= i) {
        double s = 0.0;
        for (int k = 0; k < jb; ++k) s = __builtin_fma(La[ty][k], Lb[tx][k], s);
        C[(int64_t)i * m + j] -= s;
    }
}

// L z = b, then L^T x = z, in place in the item's right-hand side; one
// workgroup per item.
__global__ void k_bsolve(const RItem* __restrict__ items, const double* __restrict__ c_base,
                         double* __restrict__ rhs_base, const int* bad) {
    const int q = blockIdx.x;
    const RItem it = items[q];
    if (bad[2 * q] | bad[2 * q + 1]) return;   // block-uniform
    const double* L = c_base + it.c;
    double* b = rhs_base + it.rhs;
    const int m = it.m;
    for (int j = 0; j < m; ++j) {
        __syncthreads();
        const double zj = b[j] / L[(int64_t)j * m + j];
        __syncthreads();
        if (threadIdx.x == 0) b[j] = zj;
        for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) b[i] -= L[(int64_t)i * m + j] * zj;
    }
    for (int j = m - 1; j >= 0; --j) {
        __syncthreads();
        const double xj = b[j] / L[(int64_t)j * m + j];
        __syncthreads();
        if (threadIdx.x == 0) b[j] = xj;
        for (int i = threadIdx.x; i < j; i += blockDim.x) b[i] -= L[(int64_t)j * m + i] * xj;
    }
}

// Residuals y - Phi w of every fitted row, one wave per row (its columns
// read along the row, the products summed by a butterfly in a fixed order).
__global__ void __launch_bounds__(256) k_bresid(const RItem* __restrict__ items, int rows,
                                                const double* __restrict__ phi_base, double* __restrict__ res_base,
                                                const int* bad) {
    const int q = blockIdx.y;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= rows || (bad[2 * q] | bad[2 * q + 1])) return;   // wave-uniform
    const RItem it = items[q];
    const double* row = phi_base + it.phi + (int64_t)r * it.cols;
    double p = 0.0;
    for (int j = lane; j < it.cols; j += 64) p = __builtin_fma(row[j], it.w[j], p);
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) p += __shfl_xor(p, m, 64);
    if (lane == 0) res_base[(int64_t)q * rows + r] = it.y[r] - p;
}

// sums[2 q] = sum of squared residuals, sums[2 q + 1] = sum of (y - mean y)^2.
__global__ void __launch_bounds__(1024) k_bnmse(const RItem* __restrict__ items, int rows,
                                                const double* __restrict__ res_base, double* sums, const int* bad) {
    __shared__ double red[1024];
    const int q = blockIdx.x;
    const RItem it = items[q];
    if (bad[2 * q] | bad[2 * q + 1]) return;   // block-uniform
    const double* y = it.y;
    const double* res = res_base + (int64_t)q * rows;
    auto block_sum = [&](double v) {
        red[threadIdx.x] = v;
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        const double r = red[0];
        __syncthreads();
        return r;
    };
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) s += y[r];
    const double ybar = block_sum(s) / rows;
    double rr = 0.0, dd = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        const double e = res[r];
        const double d = y[r] - ybar;
        rr += e * e;
        dd += d * d;
    }
    const double srr = block_sum(rr);
    const double sdd = block_sum(dd);
    if (threadIdx.x == 0) {
        sums[2 * q] = srr;
        sums[2 * q + 1] = sdd;
    }
}

}  // namespace

namespace {

__global__ void k_zero_ints(int* p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Items, tile lists and the workspace layout of one batched readout.
struct Plan {
    std::vector<RItem> items;
    std::vector<int64_t> gstart, ustart;
    int panels = 0, max_m = 0, max_cols = 0;
    // byte offsets of the device buffers in one workspace, and its size
    size_t o_items = 0, o_gstart = 0, o_ustart = 0, o_phi = 0, o_c = 0, o_rhs = 0, o_res = 0, o_sums = 0,
           o_bad = 0, bytes = 0;
};

Plan make_plan(int count, const void* const* rec, const int64_t* stride, int rows, const int64_t* n, int features,
               const double* const* y, double* const* w_dev) {
    Plan pl;
    pl.items.resize(count);
    int64_t phi_total = 0, c_total = 0, rhs_total = 0;
    for (int q = 0; q < count; ++q) {
        RItem& it = pl.items[q];
        it.rec = rec[q];
        it.stride = stride[q];
        it.y = y[q];
        it.w = w_dev[q];
        it.n = (int)n[q];
        it.cols = (features ? 3 * it.n : it.n) + 1;
        it.primal = rows >= it.cols;
        it.m = it.primal ? it.cols : rows;
        it.phi = phi_total;
        it.c = c_total;
        it.rhs = rhs_total;
        phi_total += (int64_t)rows * it.cols;
        c_total += (int64_t)it.m * it.m;
        rhs_total += std::max(it.m, it.cols);
        pl.max_m = std::max(pl.max_m, it.m);
        pl.max_cols = std::max(pl.max_cols, it.cols);
    }
    // tile lists: the Gram matrices, and the trailing update after each panel
    pl.panels = (pl.max_m + kNB - 1) / kNB;
    pl.gstart.assign(count + 1, 0);
    pl.ustart.assign((size_t)pl.panels * (count + 1), 0);
    auto tri = [](int64_t edge) {
        const int64_t nt = (edge + kT - 1) / kT;
        return nt * (nt + 1) / 2;
    };
    for (int q = 0; q < count; ++q) pl.gstart[q + 1] = pl.gstart[q] + tri(pl.items[q].m);
    for (int p = 0; p < pl.panels; ++p) {
        int64_t* us = &pl.ustart[(size_t)p * (count + 1)];
        for (int q = 0; q < count; ++q) {
            const int j0 = p * kNB, m = pl.items[q].m;
            const int rem = j0 < m ? m - std::min(m, j0 + kNB) : 0;
            us[q + 1] = us[q] + tri(rem);
        }
    }
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t at = off;
        off += align256(std::max<size_t>(b, 1));
        return at;
    };
    pl.o_items = take(sizeof(RItem) * count);
    pl.o_gstart = take(8 * pl.gstart.size());
    pl.o_ustart = take(8 * pl.ustart.size());
    pl.o_phi = take((size_t)phi_total * 8);
    pl.o_c = take((size_t)c_total * 8);
    pl.o_rhs = take((size_t)rhs_total * 8);
    pl.o_res = take((size_t)count * rows * 8);
    pl.o_sums = take((size_t)count * 16);
    pl.o_bad = take((size_t)count * 2 * sizeof(int));
    pl.bytes = off;
    return pl;
}

// The fit itself, every device buffer carved out of the workspace ws.
int solve_in(const Plan& pl, void* ws, int count, int rec_f32, int rows, int features, double lam,
             double* nmse_host, hipStream_t stream, const char** err, int* bad_item) {
    char* base = static_cast<char*>(ws);
    RItem* items_d = reinterpret_cast<RItem*>(base + pl.o_items);
    int64_t* gstart_d = reinterpret_cast<int64_t*>(base + pl.o_gstart);
    int64_t* ustart_d = reinterpret_cast<int64_t*>(base + pl.o_ustart);
    double* phi = reinterpret_cast<double*>(base + pl.o_phi);
    double* C = reinterpret_cast<double*>(base + pl.o_c);
    double* rhs = reinterpret_cast<double*>(base + pl.o_rhs);
    double* res = reinterpret_cast<double*>(base + pl.o_res);
    double* sums = reinterpret_cast<double*>(base + pl.o_sums);
    int* bad = reinterpret_cast<int*>(base + pl.o_bad);
    int rc = 0;
    auto check = [&](hipError_t e) {
        if (e != hipSuccess && rc == 0) {
            rc = 2;
            if (err) *err = hipGetErrorString(e);
        }
        return e == hipSuccess;
    };
    std::vector<int> hbad(2 * count, 0);
    std::vector<double> hsums(2 * count, 0.0);
    const int max_m = pl.max_m, max_cols = pl.max_cols, panels = pl.panels;
    const std::vector<int64_t>& ustart = pl.ustart;
    hipLaunchKernelGGL(k_zero_ints, dim3((2 * count + 255) / 256), dim3(256), 0, stream, bad, 2 * count);
    if (check(hipGetLastError()) &&
        check(hipMemcpyAsync(items_d, pl.items.data(), sizeof(RItem) * count, hipMemcpyHostToDevice, stream)) &&
        check(hipMemcpyAsync(gstart_d, pl.gstart.data(), 8 * pl.gstart.size(), hipMemcpyHostToDevice, stream)) &&
        (ustart.empty() ||
         check(hipMemcpyAsync(ustart_d, ustart.data(), 8 * ustart.size(), hipMemcpyHostToDevice, stream)))) {
        const dim3 per_item(256, count);
        if (rec_f32)
            hipLaunchKernelGGL(k_bgather<float>, per_item, dim3(256), 0, stream, items_d, rows, features, phi, bad);
        else
            hipLaunchKernelGGL(k_bgather<double>, per_item, dim3(256), 0, stream, items_d, rows, features, phi, bad);
        hipLaunchKernelGGL(k_bgram, dim3((unsigned)pl.gstart[count]), dim3(kT, kT), 0, stream, items_d, gstart_d,
                           count, rows, lam, phi, C);
        hipLaunchKernelGGL(k_bvec, dim3((max_m + 255) / 256, count), dim3(256), 0, stream, items_d, rows, phi, rhs, 0,
                           bad);
        for (int p = 0; p < panels; ++p) {
            hipLaunchKernelGGL(k_bpanel, dim3(count), dim3(256), 0, stream, items_d, C, p * kNB, bad);
            const int64_t tiles = ustart[(size_t)p * (count + 1) + count];
            if (tiles > 0)
                hipLaunchKernelGGL(k_bupdate, dim3((unsigned)tiles), dim3(kT, kT), 0, stream, items_d,
                                   ustart_d + (size_t)p * (count + 1), count, C, p * kNB, bad);
        }
        hipLaunchKernelGGL(k_bsolve, dim3(count), dim3(1024), 0, stream, items_d, C, rhs, bad);
        hipLaunchKernelGGL(k_bvec, dim3((max_cols + 255) / 256, count), dim3(256), 0, stream, items_d, rows, phi, rhs,
                           1, bad);
        hipLaunchKernelGGL(k_bresid, dim3((rows + 3) / 4, count), dim3(256), 0, stream, items_d, rows, phi, res, bad);
        hipLaunchKernelGGL(k_bnmse, dim3(count), dim3(1024), 0, stream, items_d, rows, res, sums, bad);
        check(hipGetLastError());
        check(hipMemcpyAsync(hbad.data(), bad, (size_t)count * 2 * sizeof(int), hipMemcpyDeviceToHost, stream));
        check(hipMemcpyAsync(hsums.data(), sums, (size_t)count * 16, hipMemcpyDeviceToHost, stream));
        check(hipStreamSynchronize(stream));
    }
    if (rc == 0) {
        for (int q = 0; q < count && rc == 0; ++q) {
            if (hbad[2 * q + 1]) {
                rc = 3;
                *bad_item = q;
                if (err) *err = "non-finite record or target";
            } else if (hbad[2 * q]) {
                rc = 1;
                *bad_item = q;
                if (err) *err = "normal-equation matrix is not positive definite";
            }
        }
        if (rc == 0)
            for (int q = 0; q < count; ++q) nmse_host[q] = hsums[2 * q] / hsums[2 * q + 1];
    }
    return rc;
}

// Workspace of the allocation-free readout: one array per device, resolved
// to a device address once per device (the name itself is a host-side
// stand-in and is never passed to a kernel).
__device__ __align__(256) unsigned char scratch[kReadoutScratchBytes];

struct ScratchAddr {
    void* ptr = nullptr;
    bool resolved = false;
};
std::mutex g_scratch_mu;
ScratchAddr g_scratch[64];

}  // namespace

int readout_solve_batch(int count, const void* const* rec, const int64_t* stride, int rec_f32, int rows,
                        const int64_t* n, int features, const double* const* y, double lam, double* const* w_dev,
                        double* nmse_host, hipStream_t stream, const char** err, int* bad_item) {
    *bad_item = -1;
    const Plan pl = make_plan(count, rec, stride, rows, n, features, y, w_dev);
    void* ws = nullptr;
    hipError_t e = hipMalloc(&ws, pl.bytes);
    if (e != hipSuccess) {
        if (err) *err = hipGetErrorString(e);
        return 2;
    }
    const int rc = solve_in(pl, ws, count, rec_f32, rows, features, lam, nmse_host, stream, err, bad_item);
    (void)hipFree(ws);
    return rc;
}

size_t readout_workspace_bytes(int count, const int64_t* n, int rows, int features) {
    std::vector<const void*> rec(count, nullptr);
    std::vector<int64_t> stride(count, 0);
    std::vector<const double*> y(count, nullptr);
    std::vector<double*> w(count, nullptr);
    return make_plan(count, rec.data(), stride.data(), rows, n, features, y.data(), w.data()).bytes;
}

hipError_t readout_scratch_address(void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev].resolved) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev].ptr = p;
        g_scratch[dev].resolved = true;
    }
    *ptr = g_scratch[dev].ptr;
    return hipSuccess;
}

int readout_solve_scratch(const void* rec, int rec_f32, int rows, int64_t n, int features, const double* y,
                          double lam, double* w_dev, double* nmse_host, hipStream_t stream, const char** err) {
    const int64_t stride = 3 * n;
    int bad_item = -1;
    const Plan pl = make_plan(1, &rec, &stride, rows, &n, features, &y, &w_dev);
    if (pl.bytes > kReadoutScratchBytes) {
        if (err) *err = "workspace exceeds the static scratch";
        return 4;
    }
    void* ws = nullptr;
    hipError_t e = readout_scratch_address(&ws);
    if (e != hipSuccess) {
        if (err) *err = hipGetErrorString(e);
        return 2;
    }
    return solve_in(pl, ws, 1, rec_f32, rows, features, lam, nmse_host, stream, err, &bad_item);
}

}  // namespace sto
