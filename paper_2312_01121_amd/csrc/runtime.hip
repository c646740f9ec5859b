// Host runtime behind include/sto_reservoir.h: validation, device buffers,
// path selection and error reporting.  Every numerical step runs in the HIP
// kernels of sto_kernels.hip, sto_resident.hip and readout.hip.

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/sto_reservoir.h"
#include "sto_internal.hpp"

namespace {

thread_local std::string g_err;

sto_status fail(sto_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

sto_status hip_fail(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory)
        return fail(STO_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(STO_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                         \
    do {                                            \
        hipError_t _e = (call);                     \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

bool finite_all(const double* p, int64_t count) {
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int env_flag(const char* name, int dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v) != 0;
}

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

}  // namespace

namespace sto {
const Tune& tune() {
    static const Tune t = {env_flag("STO_STREAM_ALTERNATE", 0), env_flag("STO_STREAM_NT", 1),
                           env_int("STO_STREAM_ROWS", 0), env_int("STO_STREAM_UNROLL", 0)};
    return t;
}
}  // namespace sto

struct sto_reservoir {
    int64_t n = 0, n_in = 0, ld = 0;
    sto_params prm{};
    int dtype = STO_F64;
    int path = STO_PATH_STREAM;
    int resident_grid = 0;
    size_t elem = 8;
    void* W = nullptr;
    void* w_in = nullptr;
    void* m = nullptr;
    void* ms[2] = {nullptr, nullptr};
    void* acc = nullptr;
    void* xchg = nullptr;
    int* bad = nullptr;
    int* sync = nullptr;
    int cur = 0;
    hipStream_t stream = nullptr;
    // scratch for the host-buffer entry point
    double* u_dev = nullptr;
    size_t u_cap = 0;
    void* states_dev = nullptr;
    size_t states_cap = 0;
};

namespace {

template <typename T>
sto::Coef<T> make_coef(const sto_params& p) {
    sto::Coef<T> k;
    const double d = 1.0 + p.alpha * p.alpha;
    k.h_appl = (T)p.h_appl;
    k.h_k = (T)p.h_k;
    k.h_s = (T)p.h_s;
    k.lam = (T)p.lambda_stt;
    k.px = (T)p.p[0];
    k.py = (T)p.p[1];
    k.pz = (T)p.p[2];
    k.a_cp = (T)p.a_cp;
    k.a_in = (T)p.a_in;
    k.c1 = (T)(1.0 / d);
    k.c2 = (T)(p.alpha / d);
    k.h2 = (T)(p.dt / 2.0);
    k.h1 = (T)p.dt;
    k.h6 = (T)(p.dt / 6.0);
    return k;
}

template <typename T>
sto::DevState<T> dev_state(const sto_reservoir* r) {
    sto::DevState<T> d;
    d.W = static_cast<const T*>(r->W);
    d.w_in = static_cast<const T*>(r->w_in);
    d.m = static_cast<T*>(r->m);
    d.ms[0] = static_cast<T*>(r->ms[0]);
    d.ms[1] = static_cast<T*>(r->ms[1]);
    d.acc = static_cast<T*>(r->acc);
    d.xchg = static_cast<T*>(r->xchg);
    d.bad = r->bad;
    d.sync = r->sync;
    d.n = (int)r->n;
    d.n_in = (int)r->n_in;
    d.ld = r->ld;
    return d;
}

void free_all(sto_reservoir* r) {
    void* ptrs[] = {r->W, r->w_in, r->m, r->ms[0], r->ms[1], r->acc, r->xchg, r->bad, r->sync, r->u_dev, r->states_dev};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (r->stream) (void)hipStreamDestroy(r->stream);
}

// Upload an n x cols host matrix of doubles into a device matrix of rows x
// ld elements of the handle's type (zero padding beyond cols).
sto_status upload_matrix(sto_reservoir* r, void* dst, const double* src, int64_t rows, int64_t cols,
                         int64_t ld) {
    if (r->dtype == STO_F64) {
        HIP_TRY(hipMemcpy2D(dst, ld * sizeof(double), src, cols * sizeof(double), cols * sizeof(double),
                            rows, hipMemcpyHostToDevice),
                "upload");
        return STO_OK;
    }
    // FP32: convert in row blocks to bound the host staging memory
    const int64_t block_rows = std::max<int64_t>(1, (64 << 20) / (cols * 4));
    std::vector<float> tmp;
    try {
        tmp.resize((size_t)std::min(rows, block_rows) * cols);
    } catch (const std::bad_alloc&) {
        return fail(STO_E_NOMEM, "host staging buffer");
    }
    for (int64_t r0 = 0; r0 < rows; r0 += block_rows) {
        int64_t nr = std::min(block_rows, rows - r0);
        for (int64_t i = 0; i < nr * cols; ++i) tmp[i] = (float)src[r0 * cols + i];
        HIP_TRY(hipMemcpy2D(static_cast<float*>(dst) + r0 * ld, ld * sizeof(float), tmp.data(),
                            cols * sizeof(float), cols * sizeof(float), nr, hipMemcpyHostToDevice),
                "upload");
    }
    return STO_OK;
}

// Write an AoS host state into m and the current stage-input buffer.
sto_status upload_state(sto_reservoir* r, const double* m_aos) {
    const int64_t n = r->n, ld = r->ld;
    std::vector<double> soa((size_t)3 * ld, 0.0);
    for (int64_t k = 0; k < n; ++k)
        for (int c = 0; c < 3; ++c) soa[c * ld + k] = m_aos[3 * k + c];
    if (r->dtype == STO_F64) {
        HIP_TRY(hipMemcpy(r->m, soa.data(), 3 * ld * 8, hipMemcpyHostToDevice), "state upload");
        HIP_TRY(hipMemcpy(r->ms[r->cur], soa.data(), 3 * ld * 8, hipMemcpyHostToDevice), "state upload");
    } else {
        std::vector<float> f(soa.begin(), soa.end());
        HIP_TRY(hipMemcpy(r->m, f.data(), 3 * ld * 4, hipMemcpyHostToDevice), "state upload");
        HIP_TRY(hipMemcpy(r->ms[r->cur], f.data(), 3 * ld * 4, hipMemcpyHostToDevice), "state upload");
    }
    return STO_OK;
}

sto_status validate_params(const sto_params* p) {
    if (!p) return fail(STO_E_INVALID, "params is NULL");
    const double v[] = {p->alpha, p->h_appl, p->h_k, p->h_s, p->lambda_stt, p->p[0],
                        p->p[1],  p->p[2],   p->a_cp, p->a_in, p->dt};
    for (double x : v)
        if (!std::isfinite(x)) return fail(STO_E_INVALID, "non-finite parameter");
    if (!(p->dt > 0.0)) return fail(STO_E_INVALID, "dt must be > 0");
    if (p->substeps < 1) return fail(STO_E_INVALID, "substeps must be >= 1");
    if (p->dtype != STO_F64 && p->dtype != STO_F32) return fail(STO_E_INVALID, "unknown dtype %d", p->dtype);
    if (p->coupling != STO_COUPLE_X && p->coupling != STO_COUPLE_XYZ)
        return fail(STO_E_INVALID, "unknown coupling %d", p->coupling);
    if (p->path < STO_PATH_AUTO || p->path > STO_PATH_STREAM)
        return fail(STO_E_INVALID, "unknown path %d", p->path);
    if (p->renormalize != 0 && p->renormalize != 1) return fail(STO_E_INVALID, "renormalize must be 0 or 1");
    if (p->reserved != 0) return fail(STO_E_INVALID, "reserved must be 0");
    return STO_OK;
}

template <typename T>
hipError_t dispatch(sto_reservoir* r, const double* u_dev, int samples, void* states_dev, hipStream_t s) {
    sto::DevState<T> d = dev_state<T>(r);
    sto::Coef<T> k = make_coef<T>(r->prm);
    sto::RunSpec spec;
    spec.u = u_dev;
    spec.states = states_dev;
    spec.samples = samples;
    spec.substeps = r->prm.substeps;
    spec.cur = r->cur;
    spec.renorm = r->prm.renormalize;
    spec.xyz = r->prm.coupling == STO_COUPLE_XYZ;
    spec.stream = s;
    switch (r->path) {
        case STO_PATH_SMALL: return sto::run_small<T>(d, k, spec);
        case STO_PATH_RESIDENT: return sto::run_resident<T>(d, k, spec);
        default: return sto::run_stream<T>(d, k, spec);
    }
}

sto_status run_device_impl(sto_reservoir* r, const double* u_dev, int64_t steps, void* states_dev,
                           hipStream_t stream) {
    if (!r) return fail(STO_E_INVALID, "handle is NULL");
    if (steps < 0 || steps % r->prm.substeps != 0)
        return fail(STO_E_INVALID, "steps (%lld) must be a non-negative multiple of substeps (%d)",
                    (long long)steps, r->prm.substeps);
    const int64_t samples = steps / r->prm.substeps;
    if (samples == 0) return STO_OK;
    if (samples > INT_MAX) return fail(STO_E_INVALID, "too many samples");
    if (!u_dev) return fail(STO_E_INVALID, "u is NULL");
    const int none = INT_MAX;
    HIP_TRY(hipMemcpyAsync(r->bad, &none, sizeof(int), hipMemcpyHostToDevice, stream), "flag reset");
    hipError_t e = r->dtype == STO_F64
                       ? dispatch<double>(r, u_dev, (int)samples, states_dev, stream)
                       : dispatch<float>(r, u_dev, (int)samples, states_dev, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    int bad = none, abort_word = 0;
    HIP_TRY(hipMemcpyAsync(&bad, r->bad, sizeof(int), hipMemcpyDeviceToHost, stream), "flag read");
    if (r->path == STO_PATH_RESIDENT)
        HIP_TRY(hipMemcpyAsync(&abort_word, r->sync + sto::kSyncAbortWord, sizeof(int), hipMemcpyDeviceToHost,
                               stream),
                "flag read");
    HIP_TRY(hipStreamSynchronize(stream), "run");
    if (abort_word)
        return fail(STO_E_DEVICE, "grid barrier timed out: the resident kernel's workgroups were not co-resident");
    if (bad != none)
        return fail(STO_E_NONFINITE, "state not finite after sample %d", bad);
    return STO_OK;
}

sto_status readout_check(int64_t T, int64_t n, int64_t washout, double lambda, int32_t features) {
    if (T < 1 || n < 1) return fail(STO_E_INVALID, "T and n must be >= 1");
    if (washout < 0 || washout >= T) return fail(STO_E_INVALID, "washout must be in [0, T)");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(STO_E_INVALID, "lambda must be >= 0");
    if (features != 0 && features != 1) return fail(STO_E_INVALID, "features must be 0 or 1");
    const int64_t rows = T - washout;
    const int64_t cols = (features ? 3 * n : n) + 1;
    if (rows > 65536 || cols > 65536) return fail(STO_E_UNSUPPORTED, "readout larger than 65536 rows or columns");
    return STO_OK;
}

sto_status readout_status(int rc, const char* err) {
    if (rc == 1) return fail(STO_E_INVALID, "readout: %s", err ? err : "not positive definite");
    if (rc == 3) return fail(STO_E_NONFINITE, "readout: %s", err ? err : "non-finite input");
    return fail(STO_E_DEVICE, "readout: %s", err ? err : "device error");
}

}  // namespace

extern "C" {

const char* sto_last_error(void) { return g_err.c_str(); }

sto_status sto_read_bandwidth(int64_t bytes, int32_t reps, double* gbs_out) {
    if (!gbs_out || bytes < (1 << 20) || reps < 1) return fail(STO_E_INVALID, "bytes >= 1 MiB, reps >= 1, gbs_out");
    hipError_t e = sto::read_bandwidth(bytes, reps, gbs_out);
    if (e != hipSuccess) return hip_fail(e, "read bandwidth probe");
    return STO_OK;
}

sto_status reservoir_create(int64_t n, int64_t n_in, const sto_params* prm, const double* W,
                            const double* w_in, const double* m0, sto_reservoir** out) {
    if (!out) return fail(STO_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > (int64_t)INT_MAX / 4) return fail(STO_E_INVALID, "n out of range: %lld", (long long)n);
    if (n_in < 1 || n_in > 65536) return fail(STO_E_INVALID, "n_in out of range: %lld", (long long)n_in);
    sto_status st = validate_params(prm);
    if (st != STO_OK) return st;
    if (!W || !w_in || !m0) return fail(STO_E_INVALID, "W, w_in and m0 must be non-NULL");
    if (!finite_all(W, n * n) || !finite_all(w_in, n * n_in) || !finite_all(m0, 3 * n))
        return fail(STO_E_NONFINITE, "non-finite input array");
    for (int64_t k = 0; k < n; ++k) {
        const double* v = m0 + 3 * k;
        double nn = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (std::fabs(nn - 1.0) > 1e-12) return fail(STO_E_INVALID, "|m0[%lld]| = %.17g is not 1", (long long)k, nn);
    }

    sto_reservoir* r = new (std::nothrow) sto_reservoir();
    if (!r) return fail(STO_E_NOMEM, "handle");
    r->n = n;
    r->n_in = n_in;
    r->prm = *prm;
    r->dtype = prm->dtype;
    r->elem = prm->dtype == STO_F64 ? 8 : 4;
    r->ld = round_up(n, 64);
    const int xyz = prm->coupling == STO_COUPLE_XYZ;

    // path selection
    int path = prm->path;
    int grid = 0;
    const int small_n = sto::small_max_n((int)r->elem, xyz);
    if (path == STO_PATH_AUTO) {
        if (n <= small_n) path = STO_PATH_SMALL;
        else if (sto::resident_fits((int)n, (int)r->elem, xyz, &grid)) path = STO_PATH_RESIDENT;
        else path = STO_PATH_STREAM;
    } else if (path == STO_PATH_SMALL && n > small_n) {
        delete r;
        return fail(STO_E_UNSUPPORTED, "small path holds n <= %d", small_n);
    } else if (path == STO_PATH_RESIDENT && !sto::resident_fits((int)n, (int)r->elem, xyz, &grid)) {
        delete r;
        return fail(STO_E_UNSUPPORTED, "resident path cannot hold n = %lld", (long long)n);
    }
    r->path = path;
    r->resident_grid = grid;

    auto cleanup = [&](sto_status s) {
        free_all(r);
        delete r;
        return s;
    };
    hipError_t e;
#define ALLOC(ptr, bytes)                                          \
    e = hipMalloc(&(ptr), (bytes));                                \
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipMalloc")); \
    e = hipMemset((ptr), 0, (bytes));                              \
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipMemset"));
    const size_t vec = (size_t)3 * r->ld * r->elem;
    ALLOC(r->W, (size_t)n * r->ld * r->elem);
    ALLOC(r->w_in, (size_t)n * n_in * r->elem);
    ALLOC(r->m, vec);
    ALLOC(r->ms[0], vec);
    ALLOC(r->ms[1], vec);
    ALLOC(r->acc, vec);
    if (path == STO_PATH_RESIDENT) {
        ALLOC(r->xchg, 3 * vec);
    }
    ALLOC(r->bad, sizeof(int));
    ALLOC(r->sync, 256);
#undef ALLOC
    e = hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipStreamCreate"));

    st = upload_matrix(r, r->W, W, n, n, r->ld);
    if (st != STO_OK) return cleanup(st);
    st = upload_matrix(r, r->w_in, w_in, n, n_in, n_in);
    if (st != STO_OK) return cleanup(st);
    st = upload_state(r, m0);
    if (st != STO_OK) return cleanup(st);
    *out = r;
    return STO_OK;
}

void reservoir_destroy(sto_reservoir* r) {
    if (!r) return;
    if (r->stream) (void)hipStreamSynchronize(r->stream);
    free_all(r);
    delete r;
}

int32_t reservoir_path(const sto_reservoir* r) { return r ? r->path : -1; }

sto_status reservoir_run_device(sto_reservoir* r, const void* u_dev, int64_t steps, void* states_dev,
                                void* hip_stream) {
    return run_device_impl(r, static_cast<const double*>(u_dev), steps, states_dev,
                           static_cast<hipStream_t>(hip_stream));
}

sto_status reservoir_run(sto_reservoir* r, const double* u, int64_t steps, double* states) {
    if (!r) return fail(STO_E_INVALID, "handle is NULL");
    if (steps < 0 || steps % r->prm.substeps != 0)
        return fail(STO_E_INVALID, "steps (%lld) must be a non-negative multiple of substeps (%d)",
                    (long long)steps, r->prm.substeps);
    const int64_t samples = steps / r->prm.substeps;
    if (samples == 0) return STO_OK;
    if (!u) return fail(STO_E_INVALID, "u is NULL");
    if (!finite_all(u, samples * r->n_in)) return fail(STO_E_NONFINITE, "non-finite input u");
    const size_t ub = (size_t)samples * r->n_in * sizeof(double);
    if (ub > r->u_cap) {
        if (r->u_dev) (void)hipFree(r->u_dev);
        r->u_dev = nullptr;
        r->u_cap = 0;
        HIP_TRY(hipMalloc(&r->u_dev, ub), "hipMalloc u");
        r->u_cap = ub;
    }
    const size_t sb = (size_t)samples * r->n * 3 * r->elem;
    if (states && sb > r->states_cap) {
        if (r->states_dev) (void)hipFree(r->states_dev);
        r->states_dev = nullptr;
        r->states_cap = 0;
        HIP_TRY(hipMalloc(&r->states_dev, sb), "hipMalloc states");
        r->states_cap = sb;
    }
    HIP_TRY(hipMemcpyAsync(r->u_dev, u, ub, hipMemcpyHostToDevice, r->stream), "u upload");
    sto_status st = run_device_impl(r, r->u_dev, steps, states ? r->states_dev : nullptr, r->stream);
    if (states && (st == STO_OK || st == STO_E_NONFINITE)) {
        std::string msg = g_err;
        if (r->dtype == STO_F64) {
            HIP_TRY(hipMemcpy(states, r->states_dev, sb, hipMemcpyDeviceToHost), "states download");
        } else {
            std::vector<float> f((size_t)samples * r->n * 3);
            HIP_TRY(hipMemcpy(f.data(), r->states_dev, sb, hipMemcpyDeviceToHost), "states download");
            for (size_t i = 0; i < f.size(); ++i) states[i] = f[i];
        }
        g_err = msg;
    }
    return st;
}

sto_status reservoir_get_state(const sto_reservoir* r, double* m) {
    if (!r || !m) return fail(STO_E_INVALID, "NULL argument");
    const int64_t n = r->n, ld = r->ld;
    HIP_TRY(hipStreamSynchronize(r->stream), "sync");
    std::vector<double> soa((size_t)3 * ld);
    if (r->dtype == STO_F64) {
        HIP_TRY(hipMemcpy(soa.data(), r->m, 3 * ld * 8, hipMemcpyDeviceToHost), "state download");
    } else {
        std::vector<float> f((size_t)3 * ld);
        HIP_TRY(hipMemcpy(f.data(), r->m, 3 * ld * 4, hipMemcpyDeviceToHost), "state download");
        for (size_t i = 0; i < f.size(); ++i) soa[i] = f[i];
    }
    for (int64_t k = 0; k < n; ++k)
        for (int c = 0; c < 3; ++c) m[3 * k + c] = soa[c * ld + k];
    return STO_OK;
}

sto_status reservoir_set_state(sto_reservoir* r, const double* m) {
    if (!r || !m) return fail(STO_E_INVALID, "NULL argument");
    if (!finite_all(m, 3 * r->n)) return fail(STO_E_NONFINITE, "non-finite state");
    HIP_TRY(hipStreamSynchronize(r->stream), "sync");
    return upload_state(r, m);
}

sto_status readout_fit(const double* states, int64_t T, int64_t n, const double* y, int64_t washout,
                       double lambda, int32_t features, double* w_out, double* nmse_out) {
    if (!states || !y || !w_out || !nmse_out) return fail(STO_E_INVALID, "NULL argument");
    sto_status st = readout_check(T, n, washout, lambda, features);
    if (st != STO_OK) return st;
    const int64_t rows = T - washout;
    const int64_t F = features ? 3 * n : n;
    const int64_t cols = F + 1;
    if (!finite_all(states + washout * n * 3, rows * n * 3) || !finite_all(y + washout, rows))
        return fail(STO_E_NONFINITE, "non-finite states or targets");
    double *rec_dev = nullptr, *y_dev = nullptr, *w_dev = nullptr;
    auto release = [&]() {
        if (rec_dev) (void)hipFree(rec_dev);
        if (y_dev) (void)hipFree(y_dev);
        if (w_dev) (void)hipFree(w_dev);
    };
    hipError_t e;
    const size_t rec_bytes = (size_t)rows * n * 3 * 8;
    if ((e = hipMalloc(&rec_dev, rec_bytes)) != hipSuccess || (e = hipMalloc(&y_dev, rows * 8)) != hipSuccess ||
        (e = hipMalloc(&w_dev, cols * 8)) != hipSuccess) {
        release();
        return hip_fail(e, "hipMalloc readout");
    }
    if ((e = hipMemcpy(rec_dev, states + washout * n * 3, rec_bytes, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(y_dev, y + washout, rows * 8, hipMemcpyHostToDevice)) != hipSuccess) {
        release();
        return hip_fail(e, "readout upload");
    }
    const char* err = nullptr;
    int rc = sto::readout_solve(rec_dev, 0, (int)rows, (int)n, features, y_dev, lambda, w_dev, nmse_out, nullptr,
                                &err);
    if (rc == 0) e = hipMemcpy(w_out, w_dev, cols * 8, hipMemcpyDeviceToHost);
    release();
    if (rc != 0) return readout_status(rc, err);
    if (e != hipSuccess) return hip_fail(e, "readout download");
    return STO_OK;
}

sto_status readout_fit_device(const void* states_dev, int32_t dtype, int64_t T, int64_t n, const void* y_dev,
                              int64_t washout, double lambda, int32_t features, void* w_out_dev, double* nmse_out,
                              void* hip_stream) {
    if (!states_dev || !y_dev || !w_out_dev || !nmse_out) return fail(STO_E_INVALID, "NULL argument");
    if (dtype != STO_F64 && dtype != STO_F32) return fail(STO_E_INVALID, "unknown dtype %d", dtype);
    sto_status st = readout_check(T, n, washout, lambda, features);
    if (st != STO_OK) return st;
    const int64_t rows = T - washout;
    const size_t elem = dtype == STO_F64 ? 8 : 4;
    const void* rec = static_cast<const char*>(states_dev) + (size_t)washout * n * 3 * elem;
    const double* y = static_cast<const double*>(y_dev) + washout;
    const char* err = nullptr;
    int rc = sto::readout_solve(rec, dtype == STO_F32, (int)rows, (int)n, features, y, lambda,
                                static_cast<double*>(w_out_dev), nmse_out, static_cast<hipStream_t>(hip_stream), &err);
    return rc == 0 ? STO_OK : readout_status(rc, err);
}

}  // extern "C"
