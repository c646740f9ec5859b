// Host runtime behind include/sto_reservoir.h: validation, device buffers,
// path selection and error reporting.  Every numerical step runs in the HIP
// kernels of sto_kernels.hip, sto_small.hip, sto_resident.hip, sto_multi.hip,
// sto_sweep.hip and readout.hip.

#include <algorithm>
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
#include "sto_adjoint.hpp"
#include "readout_batch.hpp"
#include "sto_internal.hpp"
#include "sto_load.hpp"
#include "sto_sweep.hpp"
#include "stream_tune.hpp"

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
static Tune& tune_mut() {
    // STO_STREAM_NT: 1 non-temporal loads of W, 0 cached loads, unset: by the
    // size of W (the stream kernel's choice)
    static Tune t = {env_flag("STO_STREAM_ALTERNATE", 0), env_int("STO_STREAM_NT", -1), env_int("STO_STREAM_ROWS", 0),
                     env_int("STO_STREAM_UNROLL", 0)};
    return t;
}
const Tune& tune() { return tune_mut(); }

bool set_stream_variant(int rows, int unroll) {
    static const int ok[][2] = {{0, 0}, {1, 4}, {2, 2}, {2, 4}, {4, 1}, {4, 2}, {4, 4}, {8, 1}, {8, 2}};
    for (const auto& v : ok)
        if (v[0] == rows && v[1] == unroll) {
            tune_mut().stream_rows = rows;
            tune_mut().stream_unroll = unroll;
            return true;
        }
    return false;
}

void stream_shape(int elem_bytes, int n, int* rows, int* unroll) {
    const Tune& t = tune();
    if (t.stream_rows > 0 && t.stream_unroll > 0) {
        *rows = t.stream_rows;
        *unroll = t.stream_unroll;
        return;
    }
    *rows = 2;
    *unroll = elem_bytes == 8 ? 4 : 2;
    for (const StreamTuneEntry& e : kStreamTune)
        if (e.elem_bytes == elem_bytes && n <= e.n_max) {
            *rows = e.rows;
            *unroll = e.unroll;
            return;
        }
}
}  // namespace sto

struct sto_reservoir {
    int64_t n = 0, n_in = 0, ld = 0, streams = 1;
    sto_params prm{};
    int dtype = STO_F64;
    int path = STO_PATH_STREAM;
    int resident_grid = 0;
    size_t elem = 8;
    void* W = nullptr;
    void* Wt = nullptr;     // transpose of W, made by the first adjoint call
    void* w_in = nullptr;
    void* m = nullptr;
    void* ms[2] = {nullptr, nullptr};
    void* acc = nullptr;
    void* xchg = nullptr;
    int* bad = nullptr;
    int* sync = nullptr;
    int cur = 0;
    hipStream_t stream = nullptr;
    int adjoint_kernels = 0;   // kernel families of the last adjoint call
    // phase trace of the persistent paths (reservoir_trace_phases)
    unsigned long long* trace = nullptr;
    int64_t trace_stages = 0;
    int64_t trace_groups = 0;
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
    void* ptrs[] = {r->W, r->Wt, r->w_in, r->m, r->ms[0], r->ms[1], r->acc, r->xchg, r->bad, r->sync, r->u_dev,
                    r->states_dev, r->trace};
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

// Write an AoS host state ([stream][node][xyz]) into m and, for the
// single-stream paths, the current stage-input buffer.
sto_status upload_state(sto_reservoir* r, const double* m_aos) {
    const int64_t n = r->n, ld = r->ld, S = r->streams;
    std::vector<double> soa((size_t)3 * ld * S, 0.0);
    for (int64_t st = 0; st < S; ++st)
        for (int64_t k = 0; k < n; ++k)
            for (int c = 0; c < 3; ++c) soa[(st * 3 + c) * ld + k] = m_aos[(st * n + k) * 3 + c];
    const size_t count = soa.size();
    if (r->dtype == STO_F64) {
        HIP_TRY(hipMemcpy(r->m, soa.data(), count * 8, hipMemcpyHostToDevice), "state upload");
        if (S == 1 || r->path == STO_PATH_BATCH)
            HIP_TRY(hipMemcpy(r->ms[r->cur], soa.data(), count * 8, hipMemcpyHostToDevice), "state upload");
    } else {
        std::vector<float> f(soa.begin(), soa.end());
        HIP_TRY(hipMemcpy(r->m, f.data(), count * 4, hipMemcpyHostToDevice), "state upload");
        if (S == 1 || r->path == STO_PATH_BATCH)
            HIP_TRY(hipMemcpy(r->ms[r->cur], f.data(), count * 4, hipMemcpyHostToDevice), "state upload");
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
    if (p->path < STO_PATH_AUTO || p->path > STO_PATH_BATCH)
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
    spec.trace = r->trace;
    spec.trace_stages = (int)r->trace_stages;
    spec.trace_groups = (int)r->trace_groups;
    switch (r->path) {
        case STO_PATH_SMALL: return sto::run_small<T>(d, k, spec);
        case STO_PATH_RESIDENT: return sto::run_resident<T>(d, k, spec);
        case STO_PATH_MULTI:
            if constexpr (sizeof(T) == 4) return sto::run_multi(d, k, spec, (int)r->streams);
            return hipErrorInvalidValue;
        case STO_PATH_BATCH:
            if constexpr (sizeof(T) == 4) {
                sto::BatchRun b;
                b.W = d.W;
                b.Wt = static_cast<const float*>(r->Wt);
                b.w_in = d.w_in;
                b.m = d.m;
                b.ms[0] = d.ms[0];
                b.ms[1] = d.ms[1];
                b.acc = d.acc;
                b.bad = d.bad;
                b.u = u_dev;
                b.states = static_cast<float*>(states_dev);
                b.k = k;
                b.n = d.n;
                b.n_in = d.n_in;
                b.streams = (int)r->streams;
                b.substeps = spec.substeps;
                b.renorm = spec.renorm;
                b.xyz = spec.xyz;
                b.samples = samples;
                b.cur = r->cur;
                b.ld = d.ld;
                b.stream = s;
                return sto::run_batch(b);
            }
            return hipErrorInvalidValue;
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
    if (r->path == STO_PATH_RESIDENT || r->path == STO_PATH_MULTI)
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

// The transpose of W (zero padding), made once per handle: the adjoint's
// reversed stages and the BATCH path read it.
sto_status ensure_transpose(sto_reservoir* r, hipStream_t stream) {
    if (r->Wt) return STO_OK;
    const size_t wb = (size_t)r->n * r->ld * r->elem;
    HIP_TRY(hipMalloc(&r->Wt, wb), "hipMalloc W^T");
    HIP_TRY(hipMemsetAsync(r->Wt, 0, wb, stream), "W^T clear");
    hipError_t e = r->dtype == STO_F64
                       ? sto::transpose_matrix<double>(static_cast<const double*>(r->W), static_cast<double*>(r->Wt),
                                                       (int)r->n, r->ld, stream)
                       : sto::transpose_matrix<float>(static_cast<const float*>(r->W), static_cast<float*>(r->Wt),
                                                      (int)r->n, r->ld, stream);
    if (e != hipSuccess) {
        (void)hipFree(r->Wt);
        r->Wt = nullptr;
        return hip_fail(e, "transpose");
    }
    return STO_OK;
}

// Workspace budget of the adjoint's stage trace when the caller lets the
// library choose the segment length.
constexpr int64_t kAdjointTraceBudget = int64_t(4) << 30;

template <typename T>
sto_status adjoint_dispatch(sto_reservoir* r, const void* m_start, const double* u, int64_t steps, const void* g_rec,
                            const void* g_fin, void* g_W, void* g_win, void* g_m0, double* g_scal, int64_t seg,
                            const void* records, hipStream_t stream) {
    sto::AdjArgs<T> a;
    a.W = static_cast<const T*>(r->W);
    a.Wt = static_cast<const T*>(r->Wt);
    a.w_in = static_cast<const T*>(r->w_in);
    a.n = (int)r->n;
    a.n_in = (int)r->n_in;
    a.streams = (int)r->streams;
    a.ld = r->ld;
    a.k = make_coef<T>(r->prm);
    a.substeps = r->prm.substeps;
    a.renorm = r->prm.renormalize;
    a.xyz = r->prm.coupling == STO_COUPLE_XYZ;
    a.u = u;
    a.steps = steps;
    a.m_start = static_cast<const T*>(m_start);
    a.g_rec = static_cast<const T*>(g_rec);
    a.g_fin = static_cast<const T*>(g_fin);
    a.records = static_cast<const T*>(records);
    a.g_W = static_cast<T*>(g_W);
    a.g_win = static_cast<T*>(g_win);
    a.g_m0 = static_cast<T*>(g_m0);
    a.g_scal = g_scal;
    a.seg_steps = seg;
    a.bad = r->bad;
    a.stream = stream;
    a.kernels = &r->adjoint_kernels;
    hipError_t e = sto::adjoint_run<T>(a);
    if (e == hipErrorLaunchTimeOut)
        return fail(STO_E_DEVICE,
                    "adjoint: the stage exchange of a persistent kernel timed out (its workgroups were not "
                    "co-resident)");
    if (e != hipSuccess) return hip_fail(e, "adjoint");
    return STO_OK;
}

// records: the run's records as the segments' checkpoints, or nullptr (the
// checkpoints then come from a forward pass of the adjoint's own).
sto_status adjoint_device_impl(sto_reservoir* r, const void* m_start, const void* u_dev, int64_t steps,
                               const void* g_rec, const void* g_fin, void* g_W, void* g_win, void* g_m0,
                               double* g_scal, int64_t checkpoint_every, const void* records, hipStream_t stream) {
    if (!r) return fail(STO_E_INVALID, "handle is NULL");
    if (steps < 0 || steps % r->prm.substeps != 0)
        return fail(STO_E_INVALID, "steps (%lld) must be a non-negative multiple of substeps (%d)",
                    (long long)steps, r->prm.substeps);
    if (steps / r->prm.substeps > INT_MAX) return fail(STO_E_INVALID, "too many samples");
    if (!m_start) return fail(STO_E_INVALID, "m_start is NULL");
    if (steps > 0 && !u_dev) return fail(STO_E_INVALID, "u is NULL");
    if (checkpoint_every < 0) return fail(STO_E_INVALID, "checkpoint_every must be >= 0");
    const int64_t sub = r->prm.substeps;
    if (records && checkpoint_every % sub != 0)
        return fail(STO_E_INVALID,
                    "checkpoint_every (%lld) must be a multiple of substeps (%lld) when the records are the "
                    "checkpoints",
                    (long long)checkpoint_every, (long long)sub);
    int64_t seg = checkpoint_every;
    if (seg == 0) {
        const int64_t per = sto::adjoint_trace_bytes_per_step(r->ld, (int)r->elem, r->prm.coupling == STO_COUPLE_XYZ,
                                                              (int)r->streams);
        seg = std::max<int64_t>(1, std::min<int64_t>(std::max<int64_t>(steps, 1), kAdjointTraceBudget / per));
        // records are states at sample boundaries: whole samples per segment
        if (records) seg = std::max<int64_t>(sub, seg / sub * sub);
    }
    {
        sto_status ts = ensure_transpose(r, stream);
        if (ts != STO_OK) return ts;
    }
    const int none = INT_MAX;
    HIP_TRY(hipMemcpyAsync(r->bad, &none, sizeof(int), hipMemcpyHostToDevice, stream), "flag reset");
    const double* u = static_cast<const double*>(u_dev);
    sto_status st = r->dtype == STO_F64
                        ? adjoint_dispatch<double>(r, m_start, u, steps, g_rec, g_fin, g_W, g_win, g_m0, g_scal, seg,
                                                   records, stream)
                        : adjoint_dispatch<float>(r, m_start, u, steps, g_rec, g_fin, g_W, g_win, g_m0, g_scal, seg,
                                                  records, stream);
    if (st != STO_OK) return st;
    int bad = none;
    HIP_TRY(hipMemcpyAsync(&bad, r->bad, sizeof(int), hipMemcpyDeviceToHost, stream), "flag read");
    HIP_TRY(hipStreamSynchronize(stream), "adjoint");
    if (bad != none) return fail(STO_E_NONFINITE, "state not finite after sample %d", bad);
    return STO_OK;
}

// Device copy of a host array of doubles in the handle's type.
sto_status to_device(const sto_reservoir* r, const double* h, int64_t count, void** out) {
    *out = nullptr;
    if (!h) return STO_OK;
    const size_t bytes = (size_t)std::max<int64_t>(count, 1) * r->elem;
    HIP_TRY(hipMalloc(out, bytes), "hipMalloc");
    if (r->dtype == STO_F64) {
        HIP_TRY(hipMemcpy(*out, h, (size_t)count * 8, hipMemcpyHostToDevice), "upload");
    } else {
        std::vector<float> f(h, h + count);
        HIP_TRY(hipMemcpy(*out, f.data(), (size_t)count * 4, hipMemcpyHostToDevice), "upload");
    }
    return STO_OK;
}

sto_status from_device(const sto_reservoir* r, const void* d, int64_t count, double* h) {
    if (!h) return STO_OK;
    if (r->dtype == STO_F64) {
        HIP_TRY(hipMemcpy(h, d, (size_t)count * 8, hipMemcpyDeviceToHost), "download");
    } else {
        std::vector<float> f((size_t)count);
        HIP_TRY(hipMemcpy(f.data(), d, (size_t)count * 4, hipMemcpyDeviceToHost), "download");
        for (int64_t i = 0; i < count; ++i) h[i] = f[i];
    }
    return STO_OK;
}

}  // namespace

struct sto_sweep {
    int count = 0;
    int64_t n_in = 0, nodes = 0;
    int dtype = STO_F64;
    size_t elem = 8;
    int substeps = 1, renorm = 0;
    std::vector<sto::SweepRes> res;
    void* W = nullptr;
    void* w_in = nullptr;
    void* m = nullptr;
    void* ms[2] = {nullptr, nullptr};
    void* acc = nullptr;
    void* res_dev = nullptr;
    void* coef_dev = nullptr;
    void* task_dev = nullptr;
    int tasks = 0;
    int* bad = nullptr;
    int* sample = nullptr;         // device: the input sample being stepped
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr; // stream the graph of the stage launches is captured on
    double* u_dev = nullptr;
    size_t u_cap = 0;
    void* states_dev = nullptr;
    size_t states_cap = 0;
};

namespace {

void sweep_free(sto_sweep* s) {
    void* ptrs[] = {s->W, s->w_in, s->m, s->ms[0], s->ms[1], s->acc, s->res_dev, s->coef_dev, s->task_dev, s->bad,
                    s->sample, s->u_dev, s->states_dev};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->capture) (void)hipStreamDestroy(s->capture);
}

// Copy a rows x cols host matrix of doubles into the device at dst (element
// pitch ld, the handle's element type).
sto_status sweep_upload(int dtype, void* dst, const double* src, int64_t rows, int64_t cols, int64_t ld) {
    if (dtype == STO_F64) {
        HIP_TRY(hipMemcpy2D(dst, ld * 8, src, cols * 8, cols * 8, rows, hipMemcpyHostToDevice), "sweep upload");
        return STO_OK;
    }
    std::vector<float> tmp((size_t)rows * cols);
    for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (float)src[i];
    HIP_TRY(hipMemcpy2D(dst, ld * 4, tmp.data(), cols * 4, cols * 4, rows, hipMemcpyHostToDevice), "sweep upload");
    return STO_OK;
}

template <typename T>
sto::SweepDev<T> sweep_dev(const sto_sweep* s, void* states, int64_t samples) {
    sto::SweepDev<T> d;
    d.W = static_cast<const T*>(s->W);
    d.w_in = static_cast<const T*>(s->w_in);
    d.m = static_cast<T*>(s->m);
    d.ms[0] = static_cast<T*>(s->ms[0]);
    d.ms[1] = static_cast<T*>(s->ms[1]);
    d.acc = static_cast<T*>(s->acc);
    d.states = static_cast<T*>(states);
    d.bad = s->bad;
    d.res = static_cast<const sto::SweepRes*>(s->res_dev);
    d.coef = static_cast<const sto::Coef<T>*>(s->coef_dev);
    d.task = static_cast<const sto::SweepTask*>(s->task_dev);
    d.tasks = s->tasks;
    d.n_in = (int)s->n_in;
    d.rec_samples = samples;
    d.sample = s->sample;
    return d;
}

sto_status sweep_run_impl(sto_sweep* s, const double* u_dev, int64_t steps, void* states_dev, hipStream_t stream) {
    if (!s) return fail(STO_E_INVALID, "handle is NULL");
    if (steps < 0 || steps % s->substeps != 0)
        return fail(STO_E_INVALID, "steps (%lld) must be a non-negative multiple of substeps (%d)", (long long)steps,
                    s->substeps);
    const int64_t samples = steps / s->substeps;
    if (samples == 0) return STO_OK;
    if (samples > INT_MAX) return fail(STO_E_INVALID, "too many samples");
    if (!u_dev) return fail(STO_E_INVALID, "u is NULL");
    const int none = INT_MAX;
    HIP_TRY(hipMemcpyAsync(s->bad, &none, sizeof(int), hipMemcpyHostToDevice, stream), "flag reset");
    sto::RunSpec spec;
    spec.u = u_dev;
    spec.states = states_dev;
    spec.samples = (int)samples;
    spec.substeps = s->substeps;
    spec.cur = 0;
    spec.renorm = s->renorm;
    spec.xyz = 0;
    spec.stream = stream;
    // the launches of a few samples are captured once into a graph and
    // replayed (STO_SWEEP_GRAPH=0: every launch issued directly; the sample
    // count per graph from STO_SWEEP_GRAPH_SAMPLES, default 8)
    const int graph_on = env_flag("STO_SWEEP_GRAPH", 1);
    const int graph_samples = std::max(1, env_int("STO_SWEEP_GRAPH_SAMPLES", 8));
    if (graph_on && !s->capture)
        HIP_TRY(hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking), "hipStreamCreate");
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = s->dtype == STO_F64
                       ? sto::run_sweep<double>(sweep_dev<double>(s, states_dev, samples), spec,
                                                graph_on ? s->capture : nullptr, graph_samples, &graph, &exec)
                       : sto::run_sweep<float>(sweep_dev<float>(s, states_dev, samples), spec,
                                               graph_on ? s->capture : nullptr, graph_samples, &graph, &exec);
    auto drop_graph = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    };
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(stream);
        drop_graph();
        return hip_fail(e, "kernel launch");
    }
    int bad = none;
    e = hipMemcpyAsync(&bad, s->bad, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    drop_graph();
    if (e != hipSuccess) return hip_fail(e, "run");
    if (bad != none) return fail(STO_E_NONFINITE, "state not finite after sample %d", bad);
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

sto_status sto_set_stream_variant(int32_t rows, int32_t unroll) {
    if (!sto::set_stream_variant(rows, unroll))
        return fail(STO_E_INVALID, "no compiled stream variant with rows=%d unroll=%d", rows, unroll);
    return STO_OK;
}

sto_status sto_read_bandwidth(int64_t bytes, int32_t reps, double* gbs_out) {
    if (!gbs_out || bytes < (1 << 20) || reps < 1) return fail(STO_E_INVALID, "bytes >= 1 MiB, reps >= 1, gbs_out");
    hipError_t e = sto::read_bandwidth(bytes, reps, gbs_out);
    if (e != hipSuccess) return hip_fail(e, "read bandwidth probe");
    return STO_OK;
}

sto_status reservoir_create(int64_t n, int64_t n_in, const sto_params* prm, const double* W,
                            const double* w_in, const double* m0, sto_reservoir** out) {
    return reservoir_create_streams(n, n_in, 1, prm, W, w_in, m0, out);
}

int64_t reservoir_streams(const sto_reservoir* r) { return r ? r->streams : -1; }

}  // extern "C"

namespace {

// Checks the sizes and constants, chooses the path and allocates a handle
// whose device arrays are all zero (W, w_in and the state still to load).
sto_status create_empty(int64_t n, int64_t n_in, int64_t streams, const sto_params* prm, sto_reservoir** out) {
    if (!out) return fail(STO_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > (int64_t)INT_MAX / 4) return fail(STO_E_INVALID, "n out of range: %lld", (long long)n);
    if (streams < 1 || streams > 65536) return fail(STO_E_INVALID, "streams out of range: %lld", (long long)streams);
    if (n_in < 1 || n_in > 65536) return fail(STO_E_INVALID, "n_in out of range: %lld", (long long)n_in);
    sto_status st = validate_params(prm);
    if (st != STO_OK) return st;

    sto_reservoir* r = new (std::nothrow) sto_reservoir();
    if (!r) return fail(STO_E_NOMEM, "handle");
    r->n = n;
    r->n_in = n_in;
    r->prm = *prm;
    r->dtype = prm->dtype;
    r->elem = prm->dtype == STO_F64 ? 8 : 4;
    r->ld = round_up(n, 64);
    r->streams = streams;
    const int xyz = prm->coupling == STO_COUPLE_XYZ;

    // path selection
    int path = prm->path;
    int grid = 0;
    const int small_n = sto::small_max_n((int)r->elem, xyz);
    if (streams > 1 || path == STO_PATH_MULTI || path == STO_PATH_BATCH) {
        // the persistent multi-stream kernel when it can run the reservoir,
        // else one launch per stage (both couplings, any n)
        const bool multi_ok = sto::multi_fits((int)n, (int)streams, xyz, nullptr, nullptr);
        const char* why = nullptr;
        if (prm->dtype != STO_F32) why = "the multi-stream paths compute in FP32";
        else if (path == STO_PATH_MULTI && !multi_ok)
            why = "n x streams does not fit the persistent multi-stream kernel (n <= 1024, all tiles co-resident)";
        else if (path != STO_PATH_AUTO && path != STO_PATH_MULTI && path != STO_PATH_BATCH)
            why = "streams > 1 runs only the multi-stream paths";
        if (why) {
            delete r;
            return fail(STO_E_UNSUPPORTED, "%s", why);
        }
        if (path == STO_PATH_AUTO) path = multi_ok ? STO_PATH_MULTI : STO_PATH_BATCH;
    } else if (path == STO_PATH_AUTO) {
        // the measured path table where it has an entry for n (each path
        // only where it can hold n), else by capacity
        const int tuned = sto::tuned_path((int)r->elem, xyz, (int)n, nullptr, nullptr);
        const bool resident_ok = sto::resident_fits((int)n, (int)r->elem, xyz, &grid);
        if (tuned == STO_PATH_SMALL && n <= small_n) path = STO_PATH_SMALL;
        else if (tuned == STO_PATH_RESIDENT && resident_ok) path = STO_PATH_RESIDENT;
        else if (tuned == STO_PATH_STREAM) path = STO_PATH_STREAM;
        else if (n <= small_n) path = STO_PATH_SMALL;
        else if (resident_ok) path = STO_PATH_RESIDENT;
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
    const size_t svec = path == STO_PATH_BATCH ? vec * streams : vec;   // stage buffers of all streams
    ALLOC(r->m, vec * streams);
    ALLOC(r->ms[0], svec);
    ALLOC(r->ms[1], svec);
    ALLOC(r->acc, svec);
    if (path == STO_PATH_RESIDENT) {
        ALLOC(r->xchg, 3 * vec);
    } else if (path == STO_PATH_MULTI) {
        ALLOC(r->xchg, 3 * (size_t)(xyz ? 3 : 1) * streams * r->ld * r->elem);
    }
    ALLOC(r->bad, sizeof(int));
    ALLOC(r->sync, 256);
#undef ALLOC
    e = hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipStreamCreate"));
    *out = r;
    return STO_OK;
}

void destroy_handle(sto_reservoir* r) {
    if (!r) return;
    if (r->stream) (void)hipStreamSynchronize(r->stream);
    free_all(r);
    delete r;
}

// The BATCH path reads W^T on every run: made when W is first set.
sto_status batch_transpose(sto_reservoir* r) {
    if (r->path != STO_PATH_BATCH) return STO_OK;
    sto_status st = ensure_transpose(r, r->stream);
    if (st == STO_OK && hipStreamSynchronize(r->stream) != hipSuccess) st = fail(STO_E_DEVICE, "transpose");
    return st;
}

template <typename T>
hipError_t load_arrays(sto_reservoir* r, const double* W, const double* w_in, const double* m, int check_norm,
                       hipStream_t stream) {
    hipError_t e = hipSuccess;
    if (W) {
        e = sto::load_matrix<T>(W, r->n, r->n, static_cast<T*>(r->W), r->ld, r->bad, stream);
        // a transpose made before (adjoint, BATCH path) follows W
        if (e == hipSuccess && r->Wt)
            e = sto::transpose_matrix<T>(static_cast<const T*>(r->W), static_cast<T*>(r->Wt), (int)r->n, r->ld,
                                         stream);
    }
    if (e == hipSuccess && w_in)
        e = sto::load_matrix<T>(w_in, r->n, r->n_in, static_cast<T*>(r->w_in), r->n_in, r->bad, stream);
    if (e == hipSuccess && m) {
        T* ms = r->streams == 1 || r->path == STO_PATH_BATCH ? static_cast<T*>(r->ms[r->cur]) : nullptr;
        e = sto::load_state<T>(m, r->n, r->streams, r->ld, static_cast<T*>(r->m), ms, check_norm, r->bad, stream);
    }
    return e;
}

sto_status load_device_impl(sto_reservoir* r, const double* W, const double* w_in, const double* m,
                            const sto_params* prm, int check_norm, hipStream_t stream) {
    if (!r) return fail(STO_E_INVALID, "handle is NULL");
    if (prm) {
        sto_status st = validate_params(prm);
        if (st != STO_OK) return st;
        const sto_params& o = r->prm;
        if (prm->dtype != o.dtype || prm->coupling != o.coupling || prm->substeps != o.substeps ||
            prm->renormalize != o.renormalize || prm->path != o.path)
            return fail(STO_E_INVALID,
                        "params may change only the constants of the equation: dtype, coupling, substeps, "
                        "renormalize and path must stay those of the handle");
    }
    HIP_TRY(hipStreamSynchronize(r->stream), "sync");
    int flags = 0;
    if (W || w_in || m) {
        HIP_TRY(hipMemsetAsync(r->bad, 0, sizeof(int), stream), "flag reset");
        hipError_t e = r->dtype == STO_F64 ? load_arrays<double>(r, W, w_in, m, check_norm, stream)
                                           : load_arrays<float>(r, W, w_in, m, check_norm, stream);
        if (e != hipSuccess) return hip_fail(e, "load");
        HIP_TRY(hipMemcpyAsync(&flags, r->bad, sizeof(int), hipMemcpyDeviceToHost, stream), "flag read");
        HIP_TRY(hipStreamSynchronize(stream), "load");
    }
    if (flags & sto::kLoadNonFinite) return fail(STO_E_NONFINITE, "non-finite input array");
    if (flags & sto::kLoadOffSphere) return fail(STO_E_INVALID, "an initial magnetisation is not of unit length");
    if (prm) r->prm = *prm;
    return STO_OK;
}

}  // namespace

extern "C" {

sto_status reservoir_create_streams(int64_t n, int64_t n_in, int64_t streams, const sto_params* prm,
                                    const double* W, const double* w_in, const double* m0, sto_reservoir** out) {
    if (!out) return fail(STO_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!W || !w_in || !m0) return fail(STO_E_INVALID, "W, w_in and m0 must be non-NULL");
    if (n >= 1 && n_in >= 1 && streams >= 1 && n <= (int64_t)INT_MAX / 4 && n_in <= 65536 && streams <= 65536) {
        if (!finite_all(W, n * n) || !finite_all(w_in, n * n_in) || !finite_all(m0, 3 * n * streams))
            return fail(STO_E_NONFINITE, "non-finite input array");
        for (int64_t k = 0; k < n * streams; ++k) {
            const double* v = m0 + 3 * k;
            double nn = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (std::fabs(nn - 1.0) > 1e-12)
                return fail(STO_E_INVALID, "|m0[%lld]| = %.17g is not 1", (long long)k, nn);
        }
    }
    sto_reservoir* r = nullptr;
    sto_status st = create_empty(n, n_in, streams, prm, &r);
    if (st != STO_OK) return st;
    st = upload_matrix(r, r->W, W, n, n, r->ld);
    if (st == STO_OK) st = upload_matrix(r, r->w_in, w_in, n, n_in, n_in);
    if (st == STO_OK) st = upload_state(r, m0);
    if (st == STO_OK) st = batch_transpose(r);
    if (st != STO_OK) {
        destroy_handle(r);
        return st;
    }
    *out = r;
    return STO_OK;
}

sto_status reservoir_create_device(int64_t n, int64_t n_in, int64_t streams, const sto_params* prm,
                                   const double* W_dev, const double* w_in_dev, const double* m0_dev,
                                   void* hip_stream, sto_reservoir** out) {
    if (!out) return fail(STO_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!W_dev || !w_in_dev || !m0_dev) return fail(STO_E_INVALID, "W, w_in and m0 must be non-NULL");
    sto_reservoir* r = nullptr;
    sto_status st = create_empty(n, n_in, streams, prm, &r);
    if (st != STO_OK) return st;
    st = load_device_impl(r, W_dev, w_in_dev, m0_dev, nullptr, 1, static_cast<hipStream_t>(hip_stream));
    if (st == STO_OK) st = batch_transpose(r);
    if (st != STO_OK) {
        destroy_handle(r);
        return st;
    }
    *out = r;
    return STO_OK;
}

sto_status reservoir_load_device(sto_reservoir* r, const double* W_dev, const double* w_in_dev,
                                 const double* m_dev, const sto_params* prm, void* hip_stream) {
    return load_device_impl(r, W_dev, w_in_dev, m_dev, prm, 0, static_cast<hipStream_t>(hip_stream));
}


int32_t reservoir_adjoint_kernels(const sto_reservoir* r) { return r ? r->adjoint_kernels : -1; }

sto_status reservoir_trace_phases(sto_reservoir* r, int64_t stages) {
    if (!r) return fail(STO_E_INVALID, "handle is NULL");
    if (stages < 0 || stages > (1 << 20)) return fail(STO_E_INVALID, "stages out of range: %lld", (long long)stages);
    if (r->trace) {
        HIP_TRY(hipStreamSynchronize(r->stream), "trace");
        HIP_TRY(hipFree(r->trace), "hipFree trace");
        r->trace = nullptr;
    }
    r->trace_stages = r->trace_groups = 0;
    if (stages == 0) return STO_OK;
    const int xyz = r->prm.coupling == STO_COUPLE_XYZ;
    int groups = 0;
    if (r->path == STO_PATH_RESIDENT) {
        int split = 1;   // the run's own shape, two waves per row included
        if (!sto::resident_shape((int)r->n, (int)r->elem, xyz, &groups, nullptr, nullptr, &split))
            return fail(STO_E_UNSUPPORTED, "resident shape does not fit");
    } else if (r->path == STO_PATH_MULTI) {
        int gx = 0, gy = 0;
        if (!sto::multi_fits((int)r->n, (int)r->streams, xyz, &gx, &gy))
            return fail(STO_E_UNSUPPORTED, "multi-stream shape does not fit");
        groups = gx * gy;
    } else {
        return fail(STO_E_UNSUPPORTED, "phase traces exist for the resident and multi-stream paths only");
    }
    const size_t bytes = (size_t)groups * stages * 4 * sizeof(unsigned long long);
    HIP_TRY(hipMalloc(&r->trace, bytes), "hipMalloc trace");
    HIP_TRY(hipMemset(r->trace, 0, bytes), "hipMemset trace");
    r->trace_stages = stages;
    r->trace_groups = groups;
    return STO_OK;
}

sto_status reservoir_phase_times(const sto_reservoir* r, uint64_t* out, int64_t capacity, int64_t* groups,
                                 int64_t* stages, int64_t* clock_khz) {
    if (!r) return fail(STO_E_INVALID, "handle is NULL");
    if (!groups || !stages || !clock_khz) return fail(STO_E_INVALID, "groups, stages and clock_khz are required");
    *groups = r->trace_groups;
    *stages = r->trace_stages;
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "wall clock rate");
    *clock_khz = khz;
    const int64_t count = r->trace_groups * r->trace_stages * 4;
    if (count == 0 || !out) return STO_OK;   // out NULL: a query of the sizes
    if (capacity < count) return fail(STO_E_INVALID, "out must hold %lld values", (long long)count);
    HIP_TRY(hipStreamSynchronize(r->stream), "trace");
    HIP_TRY(hipDeviceSynchronize(), "trace");
    HIP_TRY(hipMemcpy(out, r->trace, (size_t)count * sizeof(uint64_t), hipMemcpyDeviceToHost), "trace copy");
    return STO_OK;
}

void reservoir_destroy(sto_reservoir* r) { destroy_handle(r); }

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
    if (!finite_all(u, samples * r->streams * r->n_in)) return fail(STO_E_NONFINITE, "non-finite input u");
    const size_t ub = (size_t)samples * r->streams * r->n_in * sizeof(double);
    if (ub > r->u_cap) {
        if (r->u_dev) (void)hipFree(r->u_dev);
        r->u_dev = nullptr;
        r->u_cap = 0;
        HIP_TRY(hipMalloc(&r->u_dev, ub), "hipMalloc u");
        r->u_cap = ub;
    }
    const size_t sb = (size_t)samples * r->streams * r->n * 3 * r->elem;
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
            std::vector<float> f((size_t)samples * r->streams * r->n * 3);
            HIP_TRY(hipMemcpy(f.data(), r->states_dev, sb, hipMemcpyDeviceToHost), "states download");
            for (size_t i = 0; i < f.size(); ++i) states[i] = f[i];
        }
        g_err = msg;
    }
    return st;
}

sto_status reservoir_adjoint_device(sto_reservoir* r, const void* m_start_dev, const void* u_dev, int64_t steps,
                                    const void* grad_states_dev, const void* grad_final_dev, void* grad_W_dev,
                                    void* grad_w_in_dev, void* grad_m0_dev, double* grad_scalars_dev,
                                    int64_t checkpoint_every, void* hip_stream) {
    return adjoint_device_impl(r, m_start_dev, u_dev, steps, grad_states_dev, grad_final_dev, grad_W_dev,
                               grad_w_in_dev, grad_m0_dev, grad_scalars_dev, checkpoint_every, nullptr,
                               static_cast<hipStream_t>(hip_stream));
}

sto_status reservoir_adjoint_records_device(sto_reservoir* r, const void* m_start_dev, const void* u_dev,
                                            int64_t steps, const void* records_dev, const void* grad_states_dev,
                                            const void* grad_final_dev, void* grad_W_dev, void* grad_w_in_dev,
                                            void* grad_m0_dev, double* grad_scalars_dev, int64_t checkpoint_every,
                                            void* hip_stream) {
    if (!records_dev) return fail(STO_E_INVALID, "records is NULL");
    return adjoint_device_impl(r, m_start_dev, u_dev, steps, grad_states_dev, grad_final_dev, grad_W_dev,
                               grad_w_in_dev, grad_m0_dev, grad_scalars_dev, checkpoint_every, records_dev,
                               static_cast<hipStream_t>(hip_stream));
}

sto_status reservoir_adjoint(sto_reservoir* r, const double* m_start, const double* u, int64_t steps,
                             const double* grad_states, const double* grad_final, double* grad_W, double* grad_w_in,
                             double* grad_m0, double* grad_scalars, int64_t checkpoint_every) {
    if (!r) return fail(STO_E_INVALID, "handle is NULL");
    if (steps < 0 || steps % r->prm.substeps != 0)
        return fail(STO_E_INVALID, "steps (%lld) must be a non-negative multiple of substeps (%d)",
                    (long long)steps, r->prm.substeps);
    if (!m_start) return fail(STO_E_INVALID, "m_start is NULL");
    const int64_t samples = steps / r->prm.substeps, n = r->n, S = r->streams;
    if (samples > 0 && !u) return fail(STO_E_INVALID, "u is NULL");
    if (!finite_all(m_start, 3 * n * S) || (samples > 0 && !finite_all(u, samples * S * r->n_in)) ||
        (grad_states && !finite_all(grad_states, samples * S * n * 3)) ||
        (grad_final && !finite_all(grad_final, 3 * n * S)))
        return fail(STO_E_NONFINITE, "non-finite input");
    void *m_d = nullptr, *gr_d = nullptr, *gf_d = nullptr, *gw_d = nullptr, *gwin_d = nullptr, *gm_d = nullptr;
    double *u_d = nullptr, *gs_d = nullptr;
    auto release = [&]() {
        void* ptrs[] = {m_d, gr_d, gf_d, gw_d, gwin_d, gm_d, u_d, gs_d};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
    };
    sto_status st = to_device(r, m_start, 3 * n * S, &m_d);
    if (st == STO_OK) st = to_device(r, grad_states, samples * S * n * 3, &gr_d);
    if (st == STO_OK) st = to_device(r, grad_final, 3 * n * S, &gf_d);
    if (st == STO_OK && samples > 0) {
        if (hipMalloc(&u_d, (size_t)samples * S * r->n_in * 8) != hipSuccess ||
            hipMemcpy(u_d, u, (size_t)samples * S * r->n_in * 8, hipMemcpyHostToDevice) != hipSuccess)
            st = fail(STO_E_DEVICE, "u upload");
    }
    if (st == STO_OK && grad_W && hipMalloc(&gw_d, (size_t)n * n * r->elem) != hipSuccess)
        st = fail(STO_E_NOMEM, "hipMalloc dL/dW");
    if (st == STO_OK && grad_w_in && hipMalloc(&gwin_d, (size_t)n * r->n_in * r->elem) != hipSuccess)
        st = fail(STO_E_NOMEM, "hipMalloc dL/dw_in");
    if (st == STO_OK && grad_m0 && hipMalloc(&gm_d, (size_t)S * n * 3 * r->elem) != hipSuccess)
        st = fail(STO_E_NOMEM, "hipMalloc dL/dm0");
    if (st == STO_OK && grad_scalars && hipMalloc(&gs_d, 4 * sizeof(double)) != hipSuccess)
        st = fail(STO_E_NOMEM, "hipMalloc scalars");
    if (st == STO_OK)
        st = adjoint_device_impl(r, m_d, u_d, steps, gr_d, gf_d, gw_d, gwin_d, gm_d, gs_d, checkpoint_every,
                                 nullptr, r->stream);
    if (st == STO_OK) st = from_device(r, gw_d, n * n, grad_W);
    if (st == STO_OK) st = from_device(r, gwin_d, n * r->n_in, grad_w_in);
    if (st == STO_OK) st = from_device(r, gm_d, S * n * 3, grad_m0);
    if (st == STO_OK && grad_scalars && hipMemcpy(grad_scalars, gs_d, 4 * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        st = fail(STO_E_DEVICE, "download");
    release();
    return st;
}

sto_status readout_grad_device(const void* states_dev, int32_t dtype, int64_t T, int64_t n, const void* y_dev,
                               int64_t washout, double lambda, int32_t features, const void* w_dev, void* grad_dev,
                               double* loss_out, void* hip_stream) {
    if (!states_dev || !y_dev || !w_dev || !grad_dev) return fail(STO_E_INVALID, "NULL argument");
    if (dtype != STO_F64 && dtype != STO_F32) return fail(STO_E_INVALID, "unknown dtype %d", dtype);
    sto_status st = readout_check(T, n, washout, lambda, features);
    if (st != STO_OK) return st;
    hipError_t e = sto::readout_grad(states_dev, dtype == STO_F32, (int)T, (int)washout, (int)n, features,
                                     static_cast<const double*>(y_dev), static_cast<const double*>(w_dev), lambda,
                                     grad_dev, loss_out, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "readout gradient");
    return STO_OK;
}

sto_status reservoir_get_state(const sto_reservoir* r, double* m) {
    if (!r || !m) return fail(STO_E_INVALID, "NULL argument");
    const int64_t n = r->n, ld = r->ld, S = r->streams;
    HIP_TRY(hipStreamSynchronize(r->stream), "sync");
    std::vector<double> soa((size_t)3 * ld * S);
    if (r->dtype == STO_F64) {
        HIP_TRY(hipMemcpy(soa.data(), r->m, soa.size() * 8, hipMemcpyDeviceToHost), "state download");
    } else {
        std::vector<float> f(soa.size());
        HIP_TRY(hipMemcpy(f.data(), r->m, f.size() * 4, hipMemcpyDeviceToHost), "state download");
        for (size_t i = 0; i < f.size(); ++i) soa[i] = f[i];
    }
    for (int64_t st = 0; st < S; ++st)
        for (int64_t k = 0; k < n; ++k)
            for (int c = 0; c < 3; ++c) m[(st * n + k) * 3 + c] = soa[(st * 3 + c) * ld + k];
    return STO_OK;
}

sto_status reservoir_set_state(sto_reservoir* r, const double* m) {
    if (!r || !m) return fail(STO_E_INVALID, "NULL argument");
    if (!finite_all(m, 3 * r->n * r->streams)) return fail(STO_E_NONFINITE, "non-finite state");
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


sto_status readout_fit_device_noalloc(const void* states_dev, int32_t dtype, int64_t T, int64_t n, const void* y_dev,
                                      int64_t washout, double lambda, int32_t features, void* w_out_dev,
                                      double* nmse_out, void* hip_stream) {
    if (!states_dev || !y_dev || !w_out_dev || !nmse_out) return fail(STO_E_INVALID, "NULL argument");
    if (dtype != STO_F64 && dtype != STO_F32) return fail(STO_E_INVALID, "unknown dtype %d", dtype);
    sto_status st = readout_check(T, n, washout, lambda, features);
    if (st != STO_OK) return st;
    const int64_t rows = T - washout;
    const size_t need = sto::readout_workspace_bytes(1, &n, (int)rows, features);
    if (need > sto::kReadoutScratchBytes)
        return fail(STO_E_UNSUPPORTED,
                    "readout of %lld rows x %lld nodes needs %zu bytes of workspace; the allocation-free fit "
                    "holds at most %zu (use readout_fit_device)",
                    (long long)rows, (long long)n, need, sto::kReadoutScratchBytes);
    const size_t elem = dtype == STO_F64 ? 8 : 4;
    const void* rec = static_cast<const char*>(states_dev) + (size_t)washout * n * 3 * elem;
    const double* y = static_cast<const double*>(y_dev) + washout;
    const char* err = nullptr;
    int rc = sto::readout_solve_scratch(rec, dtype == STO_F32, (int)rows, n, features, y, lambda,
                                        static_cast<double*>(w_out_dev), nmse_out,
                                        static_cast<hipStream_t>(hip_stream), &err);
    if (rc == 4) return fail(STO_E_UNSUPPORTED, "readout: %s", err ? err : "workspace exceeds the scratch");
    return rc == 0 ? STO_OK : readout_status(rc, err);
}

sto_status readout_fit_batch_device(int32_t count, const void* const* states_dev, const int64_t* row_stride,
                                    int32_t dtype, int64_t T, const int64_t* n, const void* const* y_dev, int64_t washout,
                                    double lambda, int32_t features, double* const* w_out_dev, double* nmse_out,
                                    void* hip_stream) {
    if (count < 1 || !states_dev || !n || !y_dev || !w_out_dev || !nmse_out)
        return fail(STO_E_INVALID, "count >= 1 and non-NULL arguments");
    if (count > 65535) return fail(STO_E_INVALID, "at most 65535 record sets per call");
    if (dtype != STO_F64 && dtype != STO_F32) return fail(STO_E_INVALID, "unknown dtype %d", dtype);
    const size_t elem = dtype == STO_F64 ? 8 : 4;
    std::vector<const void*> rec(count);
    std::vector<const double*> y(count);
    std::vector<int64_t> stride(count);
    for (int32_t q = 0; q < count; ++q) {
        sto_status st = readout_check(T, n[q], washout, lambda, features);
        if (st != STO_OK) return st;
        if (!states_dev[q] || !w_out_dev[q] || !y_dev[q]) return fail(STO_E_INVALID, "item %d: NULL pointer", q);
        stride[q] = row_stride && row_stride[q] ? row_stride[q] : 3 * n[q];
        if (stride[q] < 3 * n[q]) return fail(STO_E_INVALID, "item %d: row_stride below 3 n", q);
        rec[q] = static_cast<const char*>(states_dev[q]) + (size_t)washout * stride[q] * elem;
        y[q] = static_cast<const double*>(y_dev[q]) + washout;
    }
    const char* err = nullptr;
    int bad = -1;
    int rc = sto::readout_solve_batch(count, rec.data(), stride.data(), dtype == STO_F32, (int)(T - washout), n,
                                      features, y.data(), lambda, w_out_dev, nmse_out,
                                      static_cast<hipStream_t>(hip_stream), &err, &bad);
    if (rc == 0) return STO_OK;
    if (rc == 1) return fail(STO_E_INVALID, "readout of item %d: %s", bad, err ? err : "not positive definite");
    if (rc == 3) return fail(STO_E_NONFINITE, "readout of item %d: %s", bad, err ? err : "non-finite input");
    return fail(STO_E_DEVICE, "readout: %s", err ? err : "device error");
}

sto_status sweep_create(int32_t count, const int64_t* n, int64_t n_in, const sto_params* prm, const double* const* W,
                        const double* const* w_in, const double* const* m0, sto_sweep** out) {
    if (!out) return fail(STO_E_INVALID, "out is NULL");
    *out = nullptr;
    if (count < 1 || !n || !prm || !W || !w_in || !m0) return fail(STO_E_INVALID, "count >= 1 and non-NULL arrays");
    if (n_in < 1 || n_in > 65536) return fail(STO_E_INVALID, "n_in out of range");
    for (int r = 0; r < count; ++r) {
        sto_status st = validate_params(prm + r);
        if (st != STO_OK) return st;
        if (n[r] < 1 || n[r] > 65536) return fail(STO_E_INVALID, "n[%d] out of range", r);
        if (prm[r].dtype != prm[0].dtype || prm[r].substeps != prm[0].substeps ||
            prm[r].renormalize != prm[0].renormalize || prm[r].coupling != prm[0].coupling)
            return fail(STO_E_INVALID, "dtype, substeps, renormalize and coupling must agree (reservoir %d)", r);
        if (prm[r].coupling != STO_COUPLE_X) return fail(STO_E_UNSUPPORTED, "sweeps couple m^x only");
        if (!W[r] || !w_in[r] || !m0[r]) return fail(STO_E_INVALID, "NULL array of reservoir %d", r);
        if (!finite_all(W[r], n[r] * n[r]) || !finite_all(w_in[r], n[r] * n_in) || !finite_all(m0[r], 3 * n[r]))
            return fail(STO_E_NONFINITE, "non-finite input array (reservoir %d)", r);
        for (int64_t k = 0; k < n[r]; ++k) {
            const double* v = m0[r] + 3 * k;
            if (std::fabs(std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - 1.0) > 1e-12)
                return fail(STO_E_INVALID, "|m0| != 1 (reservoir %d, node %lld)", r, (long long)k);
        }
    }
    sto_sweep* s = new (std::nothrow) sto_sweep();
    if (!s) return fail(STO_E_NOMEM, "handle");
    s->count = count;
    s->n_in = n_in;
    s->dtype = prm[0].dtype;
    s->elem = s->dtype == STO_F64 ? 8 : 4;
    s->substeps = prm[0].substeps;
    s->renorm = prm[0].renormalize;
    sto::SweepLayout lay = sto::sweep_layout((int)s->elem, count, n, n_in);
    s->res = lay.res;
    std::vector<sto::SweepTask>& tasks = lay.tasks;
    const int64_t woff = lay.w_elems, soff = lay.s_elems, winoff = lay.win_elems;
    s->nodes = lay.nodes;
    s->tasks = (int)tasks.size();
    auto cleanup = [&](sto_status st) {
        sweep_free(s);
        delete s;
        return st;
    };
    hipError_t e;
#define SALLOC(ptr, bytes)                                         \
    e = hipMalloc(&(ptr), (bytes));                                \
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipMalloc")); \
    e = hipMemset((ptr), 0, (bytes));                              \
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipMemset"));
    SALLOC(s->W, (size_t)woff * s->elem);
    SALLOC(s->w_in, (size_t)winoff * s->elem);
    SALLOC(s->m, (size_t)soff * s->elem);
    SALLOC(s->ms[0], (size_t)soff * s->elem);
    SALLOC(s->ms[1], (size_t)soff * s->elem);
    SALLOC(s->acc, (size_t)soff * s->elem);
    SALLOC(s->res_dev, sizeof(sto::SweepRes) * count);
    SALLOC(s->coef_dev, (s->dtype == STO_F64 ? sizeof(sto::Coef<double>) : sizeof(sto::Coef<float>)) * count);
    SALLOC(s->task_dev, sizeof(sto::SweepTask) * tasks.size());
    SALLOC(s->bad, sizeof(int));
    SALLOC(s->sample, sizeof(int));
#undef SALLOC
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipStreamCreate"));
    for (int r = 0; r < count; ++r) {
        const sto::SweepRes& x = s->res[r];
        sto_status st = sweep_upload(s->dtype, static_cast<char*>(s->W) + x.woff * s->elem, W[r], n[r], n[r], x.ld);
        if (st == STO_OK)
            st = sweep_upload(s->dtype, static_cast<char*>(s->w_in) + x.winoff * s->elem, w_in[r], n[r], n_in, n_in);
        if (st == STO_OK) {
            // state: AoS -> SoA (x, y, z blocks of ld), into m and ms[0]
            std::vector<double> soa((size_t)3 * x.ld, 0.0);
            for (int64_t k = 0; k < n[r]; ++k)
                for (int c = 0; c < 3; ++c) soa[c * x.ld + k] = m0[r][3 * k + c];
            for (void* dst : {s->m, s->ms[0]})
                if (st == STO_OK)
                    st = sweep_upload(s->dtype, static_cast<char*>(dst) + x.soff * s->elem, soa.data(), 1, 3 * x.ld,
                                      3 * x.ld);
        }
        if (st != STO_OK) return cleanup(st);
    }
    if (s->dtype == STO_F64) {
        std::vector<sto::Coef<double>> c;
        for (int r = 0; r < count; ++r) c.push_back(make_coef<double>(prm[r]));
        e = hipMemcpy(s->coef_dev, c.data(), sizeof(c[0]) * count, hipMemcpyHostToDevice);
    } else {
        std::vector<sto::Coef<float>> c;
        for (int r = 0; r < count; ++r) c.push_back(make_coef<float>(prm[r]));
        e = hipMemcpy(s->coef_dev, c.data(), sizeof(c[0]) * count, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(s->res_dev, s->res.data(), sizeof(sto::SweepRes) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->task_dev, tasks.data(), sizeof(sto::SweepTask) * tasks.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(hip_fail(e, "sweep upload"));
    *out = s;
    return STO_OK;
}

int64_t sweep_nodes(const sto_sweep* s) { return s ? s->nodes : -1; }

void sweep_destroy(sto_sweep* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    sweep_free(s);
    delete s;
}

sto_status sweep_run_device(sto_sweep* s, const void* u_dev, int64_t steps, void* states_dev, void* hip_stream) {
    return sweep_run_impl(s, static_cast<const double*>(u_dev), steps, states_dev, static_cast<hipStream_t>(hip_stream));
}

sto_status sweep_run(sto_sweep* s, const double* u, int64_t steps, double* states) {
    if (!s) return fail(STO_E_INVALID, "handle is NULL");
    if (steps < 0 || steps % s->substeps != 0)
        return fail(STO_E_INVALID, "steps (%lld) must be a non-negative multiple of substeps (%d)", (long long)steps,
                    s->substeps);
    const int64_t samples = steps / s->substeps;
    if (samples == 0) return STO_OK;
    if (!u) return fail(STO_E_INVALID, "u is NULL");
    if (!finite_all(u, samples * s->n_in)) return fail(STO_E_NONFINITE, "non-finite input u");
    const size_t ub = (size_t)samples * s->n_in * 8;
    if (ub > s->u_cap) {
        if (s->u_dev) (void)hipFree(s->u_dev);
        s->u_dev = nullptr;
        s->u_cap = 0;
        HIP_TRY(hipMalloc(&s->u_dev, ub), "hipMalloc u");
        s->u_cap = ub;
    }
    const size_t sb = (size_t)samples * s->nodes * 3 * s->elem;
    if (states && sb > s->states_cap) {
        if (s->states_dev) (void)hipFree(s->states_dev);
        s->states_dev = nullptr;
        s->states_cap = 0;
        HIP_TRY(hipMalloc(&s->states_dev, sb), "hipMalloc states");
        s->states_cap = sb;
    }
    HIP_TRY(hipMemcpyAsync(s->u_dev, u, ub, hipMemcpyHostToDevice, s->stream), "u upload");
    sto_status st = sweep_run_impl(s, s->u_dev, steps, states ? s->states_dev : nullptr, s->stream);
    if (states && (st == STO_OK || st == STO_E_NONFINITE)) {
        std::string msg = g_err;
        if (s->dtype == STO_F64) {
            HIP_TRY(hipMemcpy(states, s->states_dev, sb, hipMemcpyDeviceToHost), "states download");
        } else {
            std::vector<float> f((size_t)samples * s->nodes * 3);
            HIP_TRY(hipMemcpy(f.data(), s->states_dev, sb, hipMemcpyDeviceToHost), "states download");
            for (size_t i = 0; i < f.size(); ++i) states[i] = f[i];
        }
        g_err = msg;
    }
    return st;
}

sto_status sweep_get_state(const sto_sweep* s, double* m) {
    if (!s || !m) return fail(STO_E_INVALID, "NULL argument");
    HIP_TRY(hipStreamSynchronize(s->stream), "sync");
    for (int r = 0; r < s->count; ++r) {
        const sto::SweepRes& x = s->res[r];
        std::vector<double> soa((size_t)3 * x.ld);
        if (s->dtype == STO_F64) {
            HIP_TRY(hipMemcpy(soa.data(), static_cast<char*>(s->m) + x.soff * 8, soa.size() * 8, hipMemcpyDeviceToHost),
                    "state download");
        } else {
            std::vector<float> f(soa.size());
            HIP_TRY(hipMemcpy(f.data(), static_cast<char*>(s->m) + x.soff * 4, f.size() * 4, hipMemcpyDeviceToHost),
                    "state download");
            for (size_t i = 0; i < f.size(); ++i) soa[i] = f[i];
        }
        for (int64_t k = 0; k < x.n; ++k)
            for (int c = 0; c < 3; ++c) m[(x.noff + k) * 3 + c] = soa[c * x.ld + k];
    }
    return STO_OK;
}

}  // extern "C"
