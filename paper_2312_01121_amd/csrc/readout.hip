// Ridge-regression readout in FP64 on the GPU.
//
// The paper trains only the readout of the reservoir (Sec. 1) and uses the
// N node states as its features (Sec. 3.1); the fit here is ridge
// regression.  Steps (all kernels below):
//   1. gather the design matrix Phi = [features of each record, 1];
//   2. the Gram matrix Phi^T Phi (primal, rows >= cols) or Phi Phi^T (dual),
//      plus lambda on the diagonal, and the right-hand side;
//   3. Cholesky factorisation G = L L^T, one column per step (right-looking);
//   4. forward and back substitution; the dual form maps a to w = Phi^T a;
//   5. residual y - Phi w and NMSE = sum r^2 / sum (y - mean y)^2.

#include <algorithm>
#include <cmath>

#include "sto_adjoint.hpp"
#include "sto_internal.hpp"

namespace sto {

namespace {

constexpr int TILE = 16;

// features: 0 = m^x of every node, 1 = all three components; rec is
// rows x n x 3 (AoS records, FP32 or FP64), phi is rows x cols row-major in
// FP64.  Raises *bad if a feature or target is not finite.
template <typename R>
__global__ void k_gather(const R* __restrict__ rec, int rows, int n, int features, const double* __restrict__ y,
                         double* __restrict__ phi, int* bad) {
    const int cols = (features ? 3 * n : n) + 1;
    const int64_t total = (int64_t)rows * cols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / cols);
        const int j = (int)(i - (int64_t)r * cols);
        double v;
        if (j == cols - 1) v = 1.0;
        else if (features) v = (double)rec[(int64_t)r * 3 * n + j];
        else v = (double)rec[((int64_t)r * n + j) * 3];
        if (!__builtin_isfinite(v) || (j == cols - 1 && !__builtin_isfinite(y[r]))) atomicExch(bad, 1);
        phi[i] = v;
    }
}

// C (m x m) = X^T X + lam I where X is k x m (TRANS = true, i.e. entries
// X[r*m + i]), or C = X X^T + lam I where X is m x k (TRANS = false).
template <bool TRANS>
__global__ void k_gram(const double* __restrict__ X, int m, int k, double lam, double* __restrict__ C) {
    __shared__ double a[TILE][TILE + 1];
    __shared__ double b[TILE][TILE + 1];
    const int i = blockIdx.y * TILE + threadIdx.y;   // row of C
    const int j = blockIdx.x * TILE + threadIdx.x;   // column of C
    double s = 0.0;
    for (int t0 = 0; t0 < k; t0 += TILE) {
        // a[y][x] = Xop(i_block + y, t0 + x); b[y][x] = Xop(j_block + y, t0 + x)
        const int ia = blockIdx.y * TILE + threadIdx.y, ta = t0 + threadIdx.x;
        const int jb = blockIdx.x * TILE + threadIdx.y;
        if (TRANS) {
            a[threadIdx.y][threadIdx.x] = (ia < m && ta < k) ? X[(int64_t)ta * m + ia] : 0.0;
            b[threadIdx.y][threadIdx.x] = (jb < m && ta < k) ? X[(int64_t)ta * m + jb] : 0.0;
        } else {
            a[threadIdx.y][threadIdx.x] = (ia < m && ta < k) ? X[(int64_t)ia * k + ta] : 0.0;
            b[threadIdx.y][threadIdx.x] = (jb < m && ta < k) ? X[(int64_t)jb * k + ta] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < TILE; ++t) s = __builtin_fma(a[threadIdx.y][t], b[threadIdx.x][t], s);
        __syncthreads();
    }
    if (i < m && j < m) C[(int64_t)i * m + j] = s + (i == j ? lam : 0.0);
}

// out (len m) = X^T v where X is k x m row-major (v has length k).
__global__ void k_gemv_t(const double* __restrict__ X, int k, int m, const double* __restrict__ v,
                         double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double s = 0.0;
    for (int r = 0; r < k; ++r) s = __builtin_fma(X[(int64_t)r * m + j], v[r], s);
    out[j] = s;
}

// Column j of the right-looking Cholesky: L_jj = sqrt(C_jj), L_ij = C_ij / L_jj.
// One workgroup: every thread reads C_jj before thread 0 overwrites it.
__global__ void k_chol_col(double* C, int m, int j, int* flag) {
    if (*flag) return;
    const double d = C[(int64_t)j * m + j];
    __syncthreads();
    if (!(d > 0.0)) {
        if (threadIdx.x == 0) atomicExch(flag, 1);
        return;
    }
    const double ljj = __builtin_sqrt(d);
    for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x)
        C[(int64_t)i * m + j] = C[(int64_t)i * m + j] / ljj;
    if (threadIdx.x == 0) C[(int64_t)j * m + j] = ljj;
}

// Trailing update C_ik -= L_ij L_kj for j < k <= i < m (lower triangle).
__global__ void k_chol_update(double* C, int m, int j, const int* flag) {
    if (*flag) return;
    const int k = j + 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int i = j + 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (k >= m || i >= m || k > i) return;
    C[(int64_t)i * m + k] -= C[(int64_t)i * m + j] * C[(int64_t)k * m + j];
}

// Solve L z = b then L^T x = z in place (x overwrites b); one workgroup.
__global__ void k_chol_solve(const double* __restrict__ L, int m, double* b) {
    for (int j = 0; j < m; ++j) {           // forward: column-oriented
        __syncthreads();
        const double zj = b[j] / L[(int64_t)j * m + j];
        __syncthreads();
        if (threadIdx.x == 0) b[j] = zj;
        for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) b[i] -= L[(int64_t)i * m + j] * zj;
    }
    for (int j = m - 1; j >= 0; --j) {      // backward with L^T: row j of L^T is column j of L
        __syncthreads();
        const double xj = b[j] / L[(int64_t)j * m + j];
        __syncthreads();
        if (threadIdx.x == 0) b[j] = xj;
        for (int i = threadIdx.x; i < j; i += blockDim.x) b[i] -= L[(int64_t)j * m + i] * xj;
    }
}

// Residual and NMSE in one workgroup: out[0] = sum r^2, out[1] = sum (y - ybar)^2.
__global__ void k_nmse(const double* __restrict__ phi, int rows, int cols, const double* __restrict__ w,
                       const double* __restrict__ y, double* out) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) s += y[r];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double ybar = red[0] / rows;
    __syncthreads();
    double rr = 0.0, dd = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        double p = 0.0;
        for (int j = 0; j < cols; ++j) p = __builtin_fma(phi[(int64_t)r * cols + j], w[j], p);
        const double e = y[r] - p;
        const double d = y[r] - ybar;
        rr += e * e;
        dd += d * d;
    }
    red[threadIdx.x] = rr;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
    __syncthreads();
    red[threadIdx.x] = dd;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[1] = red[0];
}

// Gradient of the ridge objective at its optimum (readout_grad).
// Residual r = Phi w - y of one fitted row per workgroup, in FP64.
template <typename R>
__global__ void __launch_bounds__(256) k_residual(const R* __restrict__ rec, int rows, int n, int features,
                                                  const double* __restrict__ y, const double* __restrict__ w,
                                                  double* __restrict__ res) {
    __shared__ double part[256];
    const int row = blockIdx.x;
    if (row >= rows) return;   // uniform per workgroup
    const int f = features ? 3 * n : n;
    const R* x = rec + (int64_t)row * n * 3;
    double s = 0.0;
    for (int j = threadIdx.x; j < f; j += 256) s += (double)(features ? x[j] : x[3 * (int64_t)j]) * w[j];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) res[row] = (part[0] + w[f]) - y[row];
}

// grad[t][k][c] = (2/rows) r[t - washout] w[feature of (k, c)] for fitted
// rows and feature components, zero elsewhere.
template <typename R>
__global__ void k_readout_grad(const double* __restrict__ res, const double* __restrict__ w, int T, int washout,
                               int n, int features, R* __restrict__ grad) {
    const int64_t total = (int64_t)T * n * 3;
    const double scale = 2.0 / (double)(T - washout);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(e / ((int64_t)n * 3));
        const int kc = (int)(e - (int64_t)t * n * 3);
        double g = 0.0;
        if (t >= washout) {
            if (features) g = scale * res[t - washout] * w[kc];
            else if (kc % 3 == 0) g = scale * res[t - washout] * w[kc / 3];
        }
        grad[e] = (R)g;
    }
}

// J = (sum r^2 + lambda sum w^2) / rows, summed in a fixed order (one workgroup).
__global__ void __launch_bounds__(256) k_ridge_objective(const double* __restrict__ res, int rows,
                                                         const double* __restrict__ w, int cols, double lambda,
                                                         double* __restrict__ out) {
    __shared__ double part[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < rows; i += 256) a += res[i] * res[i];
    for (int i = threadIdx.x; i < cols; i += 256) b += w[i] * w[i];
    part[threadIdx.x] = a + lambda * b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0] / (double)rows;
}

}  // namespace

int readout_solve(const void* rec_dev, int rec_f32, int rows, int n, int features, const double* y_dev,
                  double lam, double* w_dev, double* nmse_host, hipStream_t stream, const char** err) {
    const int cols = (features ? 3 * n : n) + 1;
    const bool primal = rows >= cols;
    const int m = primal ? cols : rows;
    double *phi = nullptr, *C = nullptr, *rhs = nullptr, *sums = nullptr;
    int* flag = nullptr;   // [0]: not positive definite, [1]: non-finite input
    int rc = 0;
    auto check = [&](hipError_t e) {
        if (e != hipSuccess && rc == 0) {
            rc = 2;
            if (err) *err = hipGetErrorString(e);
        }
        return e == hipSuccess;
    };
    if (check(hipMalloc(&phi, (size_t)rows * cols * 8)) && check(hipMalloc(&C, (size_t)m * m * 8)) &&
        check(hipMalloc(&rhs, (size_t)m * 8)) && check(hipMalloc(&sums, 16)) &&
        check(hipMalloc(&flag, 2 * sizeof(int))) && check(hipMemsetAsync(flag, 0, 2 * sizeof(int), stream))) {
        if (rec_f32)
            hipLaunchKernelGGL(k_gather<float>, dim3(1024), dim3(256), 0, stream, static_cast<const float*>(rec_dev),
                               rows, n, features, y_dev, phi, flag + 1);
        else
            hipLaunchKernelGGL(k_gather<double>, dim3(1024), dim3(256), 0, stream,
                               static_cast<const double*>(rec_dev), rows, n, features, y_dev, phi, flag + 1);
        dim3 tb(TILE, TILE), tg((m + TILE - 1) / TILE, (m + TILE - 1) / TILE);
        if (primal) {
            hipLaunchKernelGGL(k_gram<true>, tg, tb, 0, stream, phi, m, rows, lam, C);
            hipLaunchKernelGGL(k_gemv_t, dim3((cols + 255) / 256), dim3(256), 0, stream, phi, rows, cols, y_dev, rhs);
        } else {
            hipLaunchKernelGGL(k_gram<false>, tg, tb, 0, stream, phi, m, cols, lam, C);
            check(hipMemcpyAsync(rhs, y_dev, (size_t)rows * 8, hipMemcpyDeviceToDevice, stream));
        }
        for (int j = 0; j < m && rc == 0; ++j) {
            hipLaunchKernelGGL(k_chol_col, dim3(1), dim3(256), 0, stream, C, m, j, flag);
            const int rem = m - j - 1;
            if (rem > 0) {
                dim3 ub(16, 16), ug((rem + 15) / 16, (rem + 15) / 16);
                hipLaunchKernelGGL(k_chol_update, ug, ub, 0, stream, C, m, j, flag);
            }
        }
        int hflag[2] = {0, 0};
        check(hipGetLastError());
        check(hipMemcpyAsync(hflag, flag, 2 * sizeof(int), hipMemcpyDeviceToHost, stream));
        check(hipStreamSynchronize(stream));
        if (rc == 0 && hflag[1]) {
            rc = 3;
            if (err) *err = "non-finite record or target";
        }
        if (rc == 0 && hflag[0]) {
            rc = 1;
            if (err) *err = "normal-equation matrix is not positive definite";
        }
        if (rc == 0) {
            hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(1024), 0, stream, C, m, rhs);
            if (primal)
                check(hipMemcpyAsync(w_dev, rhs, (size_t)cols * 8, hipMemcpyDeviceToDevice, stream));
            else
                hipLaunchKernelGGL(k_gemv_t, dim3((cols + 255) / 256), dim3(256), 0, stream, phi, rows, cols, rhs,
                                   w_dev);
            hipLaunchKernelGGL(k_nmse, dim3(1), dim3(1024), 0, stream, phi, rows, cols, w_dev, y_dev, sums);
            double hs[2] = {0.0, 0.0};
            check(hipGetLastError());
            check(hipMemcpyAsync(hs, sums, 16, hipMemcpyDeviceToHost, stream));
            check(hipStreamSynchronize(stream));
            if (rc == 0) *nmse_host = hs[0] / hs[1];
        }
    }
    for (void* p : {(void*)phi, (void*)C, (void*)rhs, (void*)sums, (void*)flag})
        if (p) (void)hipFree(p);
    return rc;
}

hipError_t readout_grad(const void* rec_dev, int rec_f32, int T, int washout, int n, int features,
                        const double* y_dev, const double* w_dev, double lambda, void* grad_dev, double* loss_host,
                        hipStream_t stream) {
    const int rows = T - washout;
    const int cols = (features ? 3 * n : n) + 1;
    double* work = nullptr;   // residuals, then the objective
    hipError_t e = hipMalloc(&work, sizeof(double) * (rows + 1));
    if (e != hipSuccess) return e;
    const size_t elem = rec_f32 ? 4 : 8;
    const void* fitted = static_cast<const char*>(rec_dev) + (size_t)washout * n * 3 * elem;
    const int64_t total = (int64_t)T * n * 3;
    const dim3 ggrid((unsigned)std::min<int64_t>((total + 255) / 256, 4096));
    if (rec_f32) {
        hipLaunchKernelGGL(k_residual<float>, dim3(rows), dim3(256), 0, stream, static_cast<const float*>(fitted),
                           rows, n, features, y_dev + washout, w_dev, work);
        hipLaunchKernelGGL(k_readout_grad<float>, ggrid, dim3(256), 0, stream, work, w_dev, T, washout, n, features,
                           static_cast<float*>(grad_dev));
    } else {
        hipLaunchKernelGGL(k_residual<double>, dim3(rows), dim3(256), 0, stream, static_cast<const double*>(fitted),
                           rows, n, features, y_dev + washout, w_dev, work);
        hipLaunchKernelGGL(k_readout_grad<double>, ggrid, dim3(256), 0, stream, work, w_dev, T, washout, n, features,
                           static_cast<double*>(grad_dev));
    }
    hipLaunchKernelGGL(k_ridge_objective, dim3(1), dim3(256), 0, stream, work, rows, w_dev, cols, lambda, work + rows);
    e = hipGetLastError();
    if (e == hipSuccess && loss_host)
        e = hipMemcpyAsync(loss_host, work + rows, sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    hipError_t f = hipFree(work);
    return e != hipSuccess ? e : f;
}

}  // namespace sto
