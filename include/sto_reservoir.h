/*
 * sto_reservoir.h -- C ABI of the MI355X coupled spin-torque-oscillator
 * reservoir library (libsto_reservoir.so, HIP for gfx950).
 *
 * The library integrates N coupled macrospins with the Landau-Lifshitz-
 * Gilbert equation plus Slonczewski spin-transfer torque (paper, Sec. 3.1,
 * Eq. (gov)), coupled through a dense N x N matrix (Eq. (coup)) and driven
 * by an input series (Eq. (in)), with classic fourth-order Runge-Kutta at a
 * fixed step (Sec. 3.2).  It records the 3N-dimensional state once per input
 * sample (the N node states are the reservoir nodes, Sec. 3.1) and fits a
 * ridge-regression readout (the paper trains only the readout, Sec. 1).
 *
 * Conventions for every entry point:
 *   - The return value is an sto_status; 0 is success.  No exception or
 *     C++ object crosses this boundary.  After a non-OK status,
 *     sto_last_error() returns a message for the calling thread.
 *   - Host pointers are plain CPU memory; "device" pointers are HIP device
 *     memory on the current device.  The caller owns every buffer it
 *     passes; the library never frees caller memory.
 *   - Matrices are row-major, states are array-of-structures (x, y, z) per
 *     node, records are [sample][node][component].
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef STO_RESERVOIR_H
#define STO_RESERVOIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STO_OK = 0,
    STO_E_INVALID = -1,      /* bad argument (size, pointer, value)          */
    STO_E_NOMEM = -2,        /* device or host allocation failed             */
    STO_E_DEVICE = -3,       /* a HIP call failed                            */
    STO_E_NONFINITE = -4,    /* the state became NaN or infinite             */
    STO_E_UNSUPPORTED = -5   /* valid request the library does not provide   */
} sto_status;

typedef enum { STO_F64 = 0, STO_F32 = 1 } sto_dtype;

/* STO_COUPLE_X is Eq. (coup): only m^x couples, into e_x.
 * STO_COUPLE_XYZ couples all three components into the matching field
 * components (an isotropic variant the paper does not use). */
typedef enum { STO_COUPLE_X = 0, STO_COUPLE_XYZ = 1 } sto_coupling;

/* Kernel family.  AUTO picks by size; the others force one family (for
 * testing each at any size where it applies). */
typedef enum {
    STO_PATH_AUTO = 0,
    STO_PATH_SMALL = 1,     /* one workgroup holds W and the state; all steps in one launch */
    STO_PATH_RESIDENT = 2,  /* W split across the CUs' LDS; all steps in one cooperative launch */
    STO_PATH_STREAM = 3,    /* W streamed from HBM once per RK4 stage, one launch per stage */
    STO_PATH_MULTI = 4,     /* S input streams share W: the coupling of all streams is one FP32
                               MFMA matrix product per stage; all steps in one cooperative launch;
                               both couplings, n <= 1024 */
    STO_PATH_BATCH = 5      /* S input streams share W: the same FP32 MFMA product, one launch per
                               RK4 stage; both couplings, any n (chosen for S > 1 when
                               STO_PATH_MULTI cannot run the reservoir) */
} sto_path;

/*
 * Constants of Eq. (gov) in dimensionless form: time in units of t0 = 1 ns,
 * fields in units of 1/(gamma t0) (56.689 Oe for gamma = 1.764e7 rad/(Oe s)).
 * With b the total field of Eq. (gov) in that unit,
 *   dm_k/dtau = -1/(1+alpha^2) m_k x b_k - alpha/(1+alpha^2) m_k x (m_k x b_k),
 *   b_k = (h_appl + h_k m_k^z) e_z + a_cp (W m^x)_k e_x + a_in (w_in u)_k e_x
 *         + h_s / (1 + lambda_stt m_k . p) * (p x m_k).
 * h_k is gamma t0 (H_K - 4 pi M); h_s is gamma t0 hbar eta I / (2 e M V).
 */
typedef struct {
    double alpha;        /* Gilbert damping                                    */
    double h_appl;       /* applied field                                      */
    double h_k;          /* anisotropy minus demagnetisation field             */
    double h_s;          /* spin-torque field amplitude                        */
    double lambda_stt;   /* spin-torque asymmetry                              */
    double p[3];         /* pinned-layer direction                             */
    double a_cp;         /* coupling amplitude                                 */
    double a_in;         /* input amplitude                                    */
    double dt;           /* RK4 step (0.01 = 1e-11 s)                          */
    int32_t substeps;    /* RK4 steps per input sample (>= 1)                  */
    int32_t renormalize; /* 1: m_k <- m_k/|m_k| after every step (default 0)   */
    int32_t dtype;       /* sto_dtype of the device arithmetic and storage     */
    int32_t coupling;    /* sto_coupling                                       */
    int32_t path;        /* sto_path                                           */
    int32_t reserved;    /* must be 0                                          */
} sto_params;

typedef struct sto_reservoir sto_reservoir;

/*
 * reservoir_create -- build a reservoir on the current HIP device.
 *   n      number of oscillators (nodes), n >= 1
 *   n_in   number of input channels, n_in >= 1
 *   prm    constants (copied); dt > 0, substeps >= 1, finite values
 *   W      host, n*n doubles, coupling matrix (Eq. (coup)), used as given
 *          (its diagonal is not forced to zero)
 *   w_in   host, n*n_in doubles, input weights (Eq. (in))
 *   m0     host, n*3 doubles, initial unit magnetisations (|m0_k| = 1
 *          within 1e-12, else STO_E_INVALID)
 *   out    receives the handle
 * The handle owns device copies of W, w_in and the state, converted to
 * prm->dtype.  Errors: STO_E_INVALID, STO_E_NOMEM, STO_E_DEVICE,
 * STO_E_UNSUPPORTED (a forced path that cannot hold this size).
 */
sto_status reservoir_create(int64_t n, int64_t n_in, const sto_params *prm,
                            const double *W, const double *w_in, const double *m0,
                            sto_reservoir **out);

/*
 * reservoir_create_streams -- a reservoir driven by S independent input
 * streams at once: S copies of the same oscillators (one W, w_in and set of
 * constants), each with its own state and input series.  The coupling of
 * all streams is the product of W with the N x S block of stage inputs
 * (Eq. (coup) applied to every stream).
 *   streams  S >= 1; S == 1 is reservoir_create
 *   m0       host, S*n*3 doubles, [stream][node][xyz]
 * For S > 1 prm->dtype must be STO_F32 (STO_E_UNSUPPORTED otherwise) and the
 * handle runs STO_PATH_MULTI when it can (either coupling, n <= 1024, all
 * tiles co-resident), else STO_PATH_BATCH; prm->path may ask for either
 * (STO_E_UNSUPPORTED if STO_PATH_MULTI cannot run it).  For such a handle, u
 * and states of the run calls gain a stream axis: u is [sample][stream][n_in]
 * and states [sample][stream][node][xyz]; get/set_state use [stream][node][xyz].
 */
sto_status reservoir_create_streams(int64_t n, int64_t n_in, int64_t streams, const sto_params *prm,
                                    const double *W, const double *w_in, const double *m0,
                                    sto_reservoir **out);

/*
 * reservoir_create_device -- reservoir_create_streams from device buffers of
 * doubles on the current HIP device (the same model, Sec. 3.1, Eq. (gov),
 * (coup) and (in)); nothing passes through host memory.
 *   W_dev       device, n*n doubles, row-major (Eq. (coup))
 *   w_in_dev    device, n*n_in doubles (Eq. (in))
 *   m0_dev      device, S*n*3 doubles, [stream][node][xyz], unit vectors
 *               (within 1e-12, else STO_E_INVALID)
 *   hip_stream  hipStream_t the copies are enqueued on (NULL: the null
 *               stream); the call returns after it has finished them
 * The buffers are read, not kept.  Errors: those of
 * reservoir_create_streams; STO_E_NONFINITE for a non-finite value.
 */
sto_status reservoir_create_device(int64_t n, int64_t n_in, int64_t streams, const sto_params *prm,
                                   const double *W_dev, const double *w_in_dev, const double *m0_dev,
                                   void *hip_stream, sto_reservoir **out);

/*
 * reservoir_load_device -- replace the coupling matrix, the input weights,
 * the state and the constants of an existing handle, from device buffers of
 * doubles, without building a new handle (a gradient-based tuning loop of
 * the model of Sec. 3.1 changes W, w_in and the constants between runs).
 *   W_dev       device, n*n doubles, row-major; NULL keeps W
 *   w_in_dev    device, n*n_in doubles; NULL keeps w_in
 *   m_dev       device, S*n*3 doubles, [stream][node][xyz]: the state the
 *               next run starts from (checked for finiteness only, as
 *               reservoir_set_state); NULL keeps the state
 *   prm         host; NULL keeps the constants.  Only the constants of the
 *               equation may differ from the handle's (alpha, h_appl, h_k,
 *               h_s, lambda_stt, p, a_cp, a_in, dt); dtype, coupling,
 *               substeps, renormalize and path must be those the handle was
 *               created with (STO_E_INVALID otherwise)
 *   hip_stream  hipStream_t to enqueue on (NULL: the null stream); the
 *               call returns after it has finished
 * Conversion to the handle's dtype and layout runs on the device (one pass
 * over each array); a transpose of W the handle keeps follows the new W.
 * Errors: STO_E_INVALID, STO_E_NONFINITE (a non-finite value: the arrays
 * named are then partly loaded and must be loaded again before a run; the
 * constants are not changed), STO_E_DEVICE.
 */
sto_status reservoir_load_device(sto_reservoir *r, const double *W_dev, const double *w_in_dev,
                                 const double *m_dev, const sto_params *prm, void *hip_stream);

/*
 * reservoir_run -- integrate steps RK4 steps from the current state.
 *   u       host, (steps/substeps) * n_in doubles, one input vector per
 *           sample, held for substeps steps (all four stages of a step see
 *           the same sample)
 *   steps   multiple of substeps (else STO_E_INVALID); 0 is a no-op
 *   states  host, (steps/substeps) * n * 3 doubles, receives the state after
 *           the last step of every sample; may be NULL
 * Runs continue from the state the previous run ended in: running u[:a]
 * then u[a:] gives bitwise the same records as running u.  Blocks until
 * done.  On STO_E_NONFINITE the records before the first sample whose state
 * is not finite are valid, and sto_last_error() names that sample.
 */
sto_status reservoir_run(sto_reservoir *r, const double *u, int64_t steps, double *states);

/*
 * reservoir_run_device -- as reservoir_run, on device buffers and a stream.
 *   u_dev       device, (steps/substeps) * n_in doubles
 *   states_dev  device, (steps/substeps) * n * 3 elements of the handle's
 *               dtype (double or float); may be NULL
 *   hip_stream  hipStream_t to enqueue on (NULL: the null stream)
 * Work is enqueued on hip_stream; the call returns after the stream has
 * finished the run so that a non-finite state can be reported.
 */
sto_status reservoir_run_device(sto_reservoir *r, const void *u_dev, int64_t steps,
                                void *states_dev, void *hip_stream);

/*
 * reservoir_adjoint_device -- gradients of a loss on the records of a run:
 * the exact derivative of the discrete RK4 map of Eq. (gov) with the
 * coupling of Eq. (coup) and the input field of Eq. (in) (paper, Sec. 3.1
 * and 3.2), by reverse-mode differentiation of every RK4 stage.  The paper
 * has no adjoint; the derivatives are those of its integrator.
 *
 * The run is recomputed from m_start over u (the handle's current state is
 * neither used nor changed), and L enters only through its gradient.  For a
 * handle of S input streams (reservoir_create_streams) every per-stream
 * array below gains the stream axis as in the run calls, and the gradients
 * of the shared W, w_in and constants sum over the streams.
 *   m_start_dev      device, S*n*3 elements of the handle's dtype, AoS: the
 *                    state the run starts from
 *   u_dev            device, (steps/substeps)*S*n_in doubles: the run's inputs
 *   steps            RK4 steps, a non-negative multiple of substeps
 *   grad_states_dev  device, (steps/substeps)*S*n*3 dtype: dL/d(record), the
 *                    records being those reservoir_run writes; NULL: zero
 *   grad_final_dev   device, S*n*3 dtype: dL/d(state after the run); NULL: zero
 * Outputs (device, overwritten; each may be NULL to skip it):
 *   grad_W_dev       n*n dtype, row-major, no padding: dL/dW
 *   grad_w_in_dev    n*n_in dtype: dL/dw_in
 *   grad_m0_dev      S*n*3 dtype, AoS: dL/dm_start
 *   grad_scalars_dev 4 doubles: dL/da_cp, dL/da_in, dL/dh_s, dL/dh_appl
 *                    (the dimensionless constants of sto_params)
 *   checkpoint_every RK4 steps per recomputed segment; 0: the library
 *                    chooses (the whole run when its stage trace fits a 4 GiB
 *                    workspace).  Smaller segments use less memory and
 *                    recompute more of the forward.
 *   hip_stream       hipStream_t to enqueue on (NULL: the null stream)
 * The forward is run from m_start and a state checkpoint kept at the start of
 * every segment; each segment is recomputed with its stage trace and
 * reversed.  With one stream each stage is a streamed mat-vec with W or
 * W^T; with S streams it is one FP32 MFMA product for all streams.  The call
 * allocates its workspace (about checkpoint_every * (4*(3+2C)+1) * S * ld
 * elements, C = 1 or 3 coupled components, ld = n rounded up to 64) plus
 * one transpose of W kept by the handle, and returns after the stream has
 * finished.  FP32 handles compute the adjoint in FP32 (the scalar sums in
 * FP64).
 * Errors: STO_E_INVALID (arguments), STO_E_NONFINITE (the recomputed state
 * is not finite; the message names the sample), STO_E_NOMEM, STO_E_DEVICE.
 */
sto_status reservoir_adjoint_device(sto_reservoir *r, const void *m_start_dev, const void *u_dev, int64_t steps,
                                    const void *grad_states_dev, const void *grad_final_dev, void *grad_W_dev,
                                    void *grad_w_in_dev, void *grad_m0_dev, double *grad_scalars_dev,
                                    int64_t checkpoint_every, void *hip_stream);

/*
 * reservoir_adjoint_records_device -- reservoir_adjoint_device for a run
 * whose records the caller still holds (the differentiated map and the
 * arguments are the same; Sec. 3.1 and 3.2 as above).  A record is the state
 * after the last step of a sample, so with segments of whole samples the
 * state at the start of segment g > 0 is the record of sample
 * g*checkpoint_every/substeps - 1, and the adjoint takes its checkpoints
 * from the records instead of running the forward once more before the
 * recompute of every segment.
 *   records_dev      device, (steps/substeps)*S*n*3 elements of the handle's
 *                    dtype: the records reservoir_run_device wrote for this
 *                    m_start, u and handle (same parameters and path); not
 *                    checked, and gradients of other records are those of a
 *                    different trajectory.  Read only.
 *   checkpoint_every a multiple of substeps (else STO_E_INVALID); 0: the
 *                    library chooses, as above, rounded down to whole samples
 * Every other argument, the workspace and the errors are those of
 * reservoir_adjoint_device; records_dev NULL is STO_E_INVALID.
 */
sto_status reservoir_adjoint_records_device(sto_reservoir *r, const void *m_start_dev, const void *u_dev,
                                            int64_t steps, const void *records_dev, const void *grad_states_dev,
                                            const void *grad_final_dev, void *grad_W_dev, void *grad_w_in_dev,
                                            void *grad_m0_dev, double *grad_scalars_dev, int64_t checkpoint_every,
                                            void *hip_stream);

/*
 * reservoir_adjoint -- reservoir_adjoint_device on host arrays of doubles
 * (m_start S*n*3, u (steps/substeps)*S*n_in, grad_states, grad_final, and
 * the outputs grad_W n*n, grad_w_in n*n_in, grad_m0 S*n*3, grad_scalars 4),
 * on the handle's stream.  Inputs are checked for finiteness
 * (STO_E_NONFINITE).
 */
sto_status reservoir_adjoint(sto_reservoir *r, const double *m_start, const double *u, int64_t steps,
                             const double *grad_states, const double *grad_final, double *grad_W,
                             double *grad_w_in, double *grad_m0, double *grad_scalars,
                             int64_t checkpoint_every);

/* reservoir_get_state / reservoir_set_state -- copy the current state
 * (host, n*3 doubles, AoS) out of / into the handle.  set_state checks
 * finiteness only; it does not renormalise. */
sto_status reservoir_get_state(const sto_reservoir *r, double *m);
sto_status reservoir_set_state(sto_reservoir *r, const double *m);

/* reservoir_streams -- S of the handle (1 for reservoir_create), or -1 for NULL. */
int64_t reservoir_streams(const sto_reservoir *r);

/* reservoir_path -- the sto_path the handle runs (never STO_PATH_AUTO). */
int32_t reservoir_path(const sto_reservoir *r);

/*
 * reservoir_trace_phases -- diagnostic of the persistent paths
 * (STO_PATH_RESIDENT, STO_PATH_MULTI), which exchange the stage inputs of
 * every RK4 stage (paper, Sec. 3.3: the coupling W^cp x needs all of x)
 * through global memory.  stages > 0 arms a trace: every later run of the
 * handle has wave 0 of each workgroup stamp the device's constant-rate
 * clock at four points of each of its first `stages` RK4 stages, counted
 * from the start of that run: 0 stage start, 1 stage input gathered, 2 own
 * rows computed, 3 own rows published.  stages == 0 frees the trace.  The
 * handle owns the trace buffer (groups * stages * 4 * 8 bytes).
 * Errors: STO_E_INVALID, STO_E_UNSUPPORTED (any other path), STO_E_NOMEM.
 *
 * reservoir_phase_times -- copies the stamps of the last run into out
 * (host, groups * stages * 4 values, [group][stage][point]; capacity is its
 * length; NULL only queries the sizes) after the handle's stream has
 * finished.  Fills *groups and
 * *stages (0 when no trace is armed) and *clock_khz, the clock's rate.
 * A stamp of 0 was not reached (a stage beyond the run's last).
 */
sto_status reservoir_trace_phases(sto_reservoir *r, int64_t stages);

/*
 * reservoir_adjoint_kernels -- which kernel families the handle's last
 * adjoint call (reservoir_adjoint*) ran, as a bit mask: 1 forward passes
 * with one launch per RK4 stage, 2 forward passes in one persistent launch
 * per segment, 4 reversed stages with one launch per stage, 8 reversed
 * stages in one persistent launch per segment.  0 before the first adjoint
 * call, -1 for a NULL handle.  Lets a caller (and the tests) see whether the
 * persistent kernels ran or the call fell back to the per-stage ones.
 */
int32_t reservoir_adjoint_kernels(const sto_reservoir *r);
sto_status reservoir_phase_times(const sto_reservoir *r, uint64_t *out, int64_t capacity, int64_t *groups,
                                 int64_t *stages, int64_t *clock_khz);

/* reservoir_destroy -- free the handle and its device memory; NULL is a no-op. */
void reservoir_destroy(sto_reservoir *r);

/*
 * Parameter sweeps: many independent reservoirs of uneven size and their own
 * constants (the parameter-space exploration the paper motivates, Sec. 1
 * and 2), driven by one shared input series and stepped together on the GPU.
 */
typedef struct sto_sweep sto_sweep;

/*
 * sweep_create -- build `count` reservoirs on the current device.
 *   n[r]     nodes of reservoir r (>= 1)
 *   n_in     input channels, shared (the input series is shared)
 *   prm[r]   constants of reservoir r; dtype, coupling, substeps and
 *            renormalize must agree across r (STO_E_INVALID otherwise);
 *            coupling must be STO_COUPLE_X (STO_E_UNSUPPORTED otherwise);
 *            path is ignored
 *   W[r], w_in[r], m0[r]  host arrays as in reservoir_create
 * The handle owns device copies of every matrix and state.
 */
sto_status sweep_create(int32_t count, const int64_t *n, int64_t n_in, const sto_params *prm,
                        const double *const *W, const double *const *w_in, const double *const *m0,
                        sto_sweep **out);

/* sweep_nodes -- total nodes (sum of n[r]), or -1 for NULL. */
int64_t sweep_nodes(const sto_sweep *s);

/*
 * sweep_run / sweep_run_device -- integrate every reservoir steps RK4 steps.
 *   u       (steps/substeps) * n_in doubles, the shared input series (host
 *           for sweep_run, device for sweep_run_device)
 *   states  (steps/substeps) * sum(n) * 3 elements or NULL, laid out
 *           [reservoir][sample][node][xyz]: reservoir r's records are one
 *           contiguous block starting at samples * (n[0] + ... + n[r-1]) * 3
 *           (doubles on the host; the handle's dtype on the device)
 *   hip_stream  as in reservoir_run_device
 * Continuation, blocking and STO_E_NONFINITE behave as in reservoir_run.
 */
sto_status sweep_run(sto_sweep *s, const double *u, int64_t steps, double *states);
sto_status sweep_run_device(sto_sweep *s, const void *u_dev, int64_t steps, void *states_dev,
                            void *hip_stream);

/* sweep_get_state -- current states, host, sum(n)*3 doubles, reservoirs in order. */
sto_status sweep_get_state(const sto_sweep *s, double *m);

/* sweep_destroy -- free the handle; NULL is a no-op. */
void sweep_destroy(sto_sweep *s);

/*
 * readout_fit -- ridge-regression readout, computed in FP64 on the GPU.
 *   states    host, T * n * 3 doubles (the records of a run)
 *   y         host, T doubles, target per record
 *   washout   rows n < washout are skipped; 0 <= washout < T
 *   lambda    ridge penalty (>= 0) on every weight, bias included
 *   features  0: m^x of every node; 1: all three components
 *   w_out     host, F + 1 doubles (F = n or 3n): weights, bias last
 *   nmse_out  host, 1 double: sum (y - Phi w)^2 / sum (y - mean y)^2 over
 *             the fitted rows
 * Solves (Phi^T Phi + lambda I) w = Phi^T y by Cholesky when the fitted
 * rows are at least the columns, else the equivalent dual system
 * (Phi Phi^T + lambda I) a = y, w = Phi^T a.  Errors: STO_E_INVALID (also
 * when the system is not positive definite), STO_E_NONFINITE (NaN inputs),
 * STO_E_NOMEM, STO_E_DEVICE.
 */
sto_status readout_fit(const double *states, int64_t T, int64_t n, const double *y,
                       int64_t washout, double lambda, int32_t features,
                       double *w_out, double *nmse_out);

/*
 * readout_fit_device -- readout_fit on device buffers, in FP64 on the GPU.
 *   states_dev  device, T * n * 3 elements of type dtype (sto_dtype), e.g.
 *               the records written by reservoir_run_device
 *   dtype       element type of states_dev
 *   y_dev       device, T doubles
 *   w_out_dev   device, F + 1 doubles (weights, bias last)
 *   nmse_out    host, 1 double
 *   hip_stream  hipStream_t to enqueue on (NULL: the null stream); the call
 *               returns after the stream has finished the fit
 * Same system, arguments and errors as readout_fit; non-finite records or
 * targets are detected on the device (STO_E_NONFINITE).
 */
sto_status readout_fit_device(const void *states_dev, int32_t dtype, int64_t T, int64_t n,
                              const void *y_dev, int64_t washout, double lambda, int32_t features,
                              void *w_out_dev, double *nmse_out, void *hip_stream);

/*
 * readout_fit_device_noalloc -- readout_fit_device for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same kernels and results,
 * with the fit's whole workspace (design matrix, Gram matrix, tile lists,
 * residuals, flags) in the library's static device array of 96 MiB, of
 * which each GPU the library runs on holds one copy until the process
 * ends.  The call makes no hipMalloc or hipFree.  Arguments, results and
 * errors as readout_fit_device, plus STO_E_UNSUPPORTED when the workspace,
 * about 8 ((T - washout) (F + 1) + m^2) bytes with m = min(T - washout,
 * F + 1), would exceed the array (the message states both sizes; N = 1,000
 * over 9,000 fitted rows and N = 10,000 over 900 fit).  Every call on one
 * GPU shares that GPU's array and overwrites it: calls that overlap on one
 * GPU (several host threads or streams) race and must be serialised by the
 * caller.
 */
sto_status readout_fit_device_noalloc(const void *states_dev, int32_t dtype, int64_t T, int64_t n,
                                      const void *y_dev, int64_t washout, double lambda, int32_t features,
                                      void *w_out_dev, double *nmse_out, void *hip_stream);

/*
 * readout_fit_batch_device -- readout_fit_device for `count` record sets,
 * each with its own target series (which may be one shared buffer), fitted
 * together: the readouts of a sweep's reservoirs, or of the S streams of a
 * multi-stream reservoir.  Item q is
 * fitted exactly as readout_fit_device fits one record set; the kernels
 * cover all items at once, so the launch count does not grow with `count`.
 *   count       number of record sets, 1 ... 65535
 *   states_dev  host array of `count` device pointers: record t of item q
 *               (n[q] x 3 elements of dtype, AoS) starts at element
 *               t * row_stride[q] of states_dev[q]
 *   row_stride  host array of `count` strides in elements (>= 3 n[q]), or
 *               NULL (or 0 entries) for contiguous records, 3 n[q]; e.g.
 *               3 n S for stream q of a multi-stream reservoir's states
 *   dtype, T, washout, lambda, features  as readout_fit_device
 *   n           host array of `count` node counts
 *   y_dev       host array of `count` device pointers, T doubles each
 *   w_out_dev   host array of `count` device pointers, each F_q + 1 doubles
 *   nmse_out    host, `count` doubles
 *   hip_stream  hipStream_t to enqueue on; returns after the stream finished
 * Device memory of about 8 (T - washout) sum_q (F_q + 1) bytes for the
 * design matrices plus the Gram matrices is allocated for the call.
 * Errors as readout_fit_device; the message names the first item concerned.
 */
sto_status readout_fit_batch_device(int32_t count, const void *const *states_dev, const int64_t *row_stride,
                                    int32_t dtype, int64_t T, const int64_t *n, const void *const *y_dev,
                                    int64_t washout, double lambda, int32_t features,
                                    double *const *w_out_dev, double *nmse_out, void *hip_stream);

/*
 * readout_grad_device -- the ridge objective at its optimum and its gradient
 * with respect to the records, the loss to feed reservoir_adjoint_device.
 *   J = (|Phi w - y|^2 + lambda |w|^2) / T', T' = T - washout fitted rows,
 *   w the weights readout_fit_device returned for the same arguments.
 * w minimises the objective, so its derivative in w vanishes and
 * dJ/dPhi = (2/T') (Phi w - y) w^T exactly (envelope theorem); records
 * before the washout and components that are not features get zero.
 *   states_dev, dtype, T, n, y_dev, washout, lambda, features
 *               as readout_fit_device
 *   w_dev       device, F + 1 doubles: the fitted weights, bias last
 *   grad_dev    device, T*n*3 elements of dtype: dJ/d(records), overwritten
 *   loss_out    host, 1 double: J (may be NULL)
 *   hip_stream  hipStream_t to enqueue on; returns after the stream finished
 * Errors: STO_E_INVALID, STO_E_UNSUPPORTED (as readout_fit), STO_E_DEVICE.
 */
sto_status readout_grad_device(const void *states_dev, int32_t dtype, int64_t T, int64_t n, const void *y_dev,
                               int64_t washout, double lambda, int32_t features, const void *w_dev,
                               void *grad_dev, double *loss_out, void *hip_stream);

/*
 * sto_read_bandwidth -- diagnostic: HBM read bandwidth this device attains
 * with a plain streaming kernel (16-byte non-temporal loads over a buffer of
 * `bytes`, read `reps` times), in GB/s.  Used to report the roofline of the
 * coupling kernels against the attainable as well as the nominal peak.
 * Allocates and frees its own buffer.  Errors: STO_E_INVALID, STO_E_NOMEM,
 * STO_E_DEVICE.
 */
sto_status sto_read_bandwidth(int64_t bytes, int32_t reps, double *gbs_out);

/*
 * sto_set_stream_variant -- choose the launch shape of the streaming
 * kernels (STO_PATH_STREAM and sweeps) for this process: rows of W per wave
 * and unroll of the column loop.  (0, 0) restores the built-in table, which
 * the autotuner (paper_2312_01121_amd/autotune.py) writes from measurements.
 * Only compiled variants are accepted: rows x unroll in {1x4, 2x2, 2x4, 4x1,
 * 4x2, 4x4, 8x1, 8x2}; STO_E_INVALID otherwise.  Not synchronised with runs
 * in flight on other threads.
 */
sto_status sto_set_stream_variant(int32_t rows, int32_t unroll);

/* sto_last_error -- message of the last non-OK status on this thread
 * (empty string if none).  Valid until the next call on this thread. */
const char *sto_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STO_RESERVOIR_H */
