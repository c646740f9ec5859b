// Ridge-regression readout in FP64 on the GPU.
//
// The paper trains only the readout of the reservoir (Sec. 1) and uses the
// N node states as its features (Sec. 3.1); the fit here is ridge
// regression: the design matrix Phi = [features of each record, 1], the
// normal equations in the primal (rows >= cols) or dual form, Cholesky
// factorisation, substitution and NMSE.  One record set is fitted by the
// batched implementation (readout_batch.hip) with a batch of one; this file
// holds the gradient of the ridge objective at its optimum.

#include <algorithm>
#include <cmath>

#include "readout_batch.hpp"
#include "sto_adjoint.hpp"
#include "sto_internal.hpp"

namespace sto {

namespace {

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
    const int64_t stride = 3 * (int64_t)n, nn = n;
    int bad_item = -1;
    return readout_solve_batch(1, &rec_dev, &stride, rec_f32, rows, &nn, features, &y_dev, lam, &w_dev, nmse_host,
                               stream, err, &bad_item);
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
