// Device-side pieces of the adjoint of the RK4 trajectory shared by the
// single-stream kernels (sto_adjoint.hip: streamed coupling mat-vecs) and
// the multi-stream kernels (sto_batch.hip: the coupling of all S input
// streams as one FP32 MFMA product): the workspace layout, the pointwise
// adjoint of Eq. (gov), the start of a reversed step, and the epilogues of a
// traced forward stage and of a reversed stage.
#pragma once

#include "sto_internal.hpp"

namespace sto {

// Device view of the adjoint workspace for S streams sharing one W.  Every
// per-stream array holds the streams one after the other; within a stream,
// component c of node k sits at c * ld + k.
template <typename T>
struct AdjDev {
    const T* W;      // n x ld
    const T* Wt;     // n x ld, the transpose of W
    const T* w_in;   // n x n_in (shared by the streams)
    T* m;            // forward state [S][3][ld]
    T* ms[2];        // forward stage inputs (ping-pong) [S][3][ld]
    T* acc;          // forward RK4 accumulator [S][3][ld]
    int* bad;
    T* xt;           // trace: stage inputs [K][4][S][3][ld]
    T* wx;           // trace: raw coupling sums (W x) [K][4][S][C][ld]
    T* st;           // adjoint of the coupling field per stage [K][4][S][C][ld]
    T* pn;           // trace: norm before renormalisation [K][S][ld]
    T* abar;         // [S][3][ld]  a of the step being reversed
    T* mbar;         // [S][3][ld]  running dL/dm of the step being reversed
    T* loc;          // [S][3][ld]  pointwise part of xbar of the stage being reversed
    double* gacc;    // [4][S][ld]  per-node d/da_cp, d/da_in, d/dh_s, d/dh_appl
    double* gwin;    // [n_in][S][ld]
    const T* g_rec;  // [samples][S][n][3]: dL/d(record), or null
    const T* g_fin;  // [S][n][3]: dL/d(final state), or null
    const double* u; // [samples][S][n_in]
    T* rec;          // plain forward runs: records [samples][S][n][3], or null
    int n, n_in, substeps, renorm, S;
    int64_t ld, steps, j0;   // j0: global index of the first step of the launch's segment
};

template <int C>
__host__ __device__ __forceinline__ int64_t adj_slot(int kk, int stage, int S, int64_t ld) {
    return ((int64_t)kk * 4 + stage) * S * C * ld;
}

// Unscaled input sum (w_in u)_row in the arithmetic type.
template <typename T>
__device__ __forceinline__ T input_dot(const T* w_in_row, const double* u_s, int n_in) {
    typename Acc<T>::type a = Acc<T>::zero();
    for (int j = 0; j < n_in; ++j) Acc<T>::fma(a, w_in_row[j], (T)u_s[j]);
    return Acc<T>::round(a);
}

// Pointwise adjoint of the right-hand side of Eq. (gov) at stage input m,
// coupling field c and input field hin, applied to v.  Returns
// g = v^T dF/dm with c held fixed, bb = v^T dF/db and hsp = v^T dF/dh_s.
template <typename T, bool XYZ>
__device__ __forceinline__ void llg_vjp(const Coef<T>& k, T mx, T my, T mz, T cx, T cy, T cz, T hin, T vx,
                                        T vy, T vz, T& gx, T& gy, T& gz, T& bbx, T& bby, T& bbz, T& hsp) {
    const T mp = (mx * k.px + my * k.py) + mz * k.pz;
    const T den = T(1) + k.lam * mp;
    const T hs = k.h_s / den;
    const T qx = k.py * mz - k.pz * my;
    const T qy = k.pz * mx - k.px * mz;
    const T qz = k.px * my - k.py * mx;
    const T hz = k.h_appl + k.h_k * mz;
    const T bx = (cx + hin) + hs * qx;
    const T by = XYZ ? cy + hs * qy : hs * qy;
    const T bz = XYZ ? (hz + cz) + hs * qz : hz + hs * qz;
    // mb = m x b
    const T ax = my * bz - mz * by;
    const T ay = mz * bx - mx * bz;
    const T az = mx * by - my * bx;
    // adjoint of mb: -c1 v - c2 (v x m)
    const T wmx = vy * mz - vz * my;
    const T wmy = vz * mx - vx * mz;
    const T wmz = vx * my - vy * mx;
    const T ex = (-k.c1) * vx - k.c2 * wmx;
    const T ey = (-k.c1) * vy - k.c2 * wmy;
    const T ez = (-k.c1) * vz - k.c2 * wmz;
    // through the m in m x (m x b): -c2 (mb x v); through m in m x b: b x ebar
    gx = (-k.c2) * (ay * vz - az * vy) + (by * ez - bz * ey);
    gy = (-k.c2) * (az * vx - ax * vz) + (bz * ex - bx * ez);
    gz = (-k.c2) * (ax * vy - ay * vx) + (bx * ey - by * ex);
    // adjoint of b: ebar x m
    bbx = ey * mz - ez * my;
    bby = ez * mx - ex * mz;
    bbz = ex * my - ey * mx;
    // b through m: h_k m_z, hs (p x m), hs(m . p)
    gz = gz + k.h_k * bbz;
    const T rx = bby * k.pz - bbz * k.py;
    const T ry = bbz * k.px - bbx * k.pz;
    const T rz = bbx * k.py - bby * k.px;
    const T hsbar = (bbx * qx + bby * qy) + bbz * qz;
    const T dh = hsbar * ((-k.lam) * hs / den);
    gx = gx + hs * rx + dh * k.px;
    gy = gy + hs * ry + dh * k.py;
    gz = gz + hs * rz + dh * k.pz;
    hsp = hsbar / den;
}

// Inputs of the pointwise adjoint of one stage at node i of stream s: the
// traced stage input, raw coupling sums and unscaled input sum.
template <typename T>
struct VjpIn {
    T mx, my, mz, wxx, wxy, wxz, raw;
    const double* u_s;
};

template <typename T, bool XYZ>
__device__ __forceinline__ VjpIn<T> vjp_load(const AdjDev<T>& d, int i, int s, int kk, int stage) {
    constexpr int C = XYZ ? 3 : 1;
    const int64_t ld = d.ld;
    const int S = d.S;
    const T* x = d.xt + adj_slot<3>(kk, stage, S, ld) + (int64_t)s * 3 * ld;
    const T* wx = d.wx + adj_slot<C>(kk, stage, S, ld) + (int64_t)s * C * ld;
    VjpIn<T> in;
    in.mx = x[i];
    in.my = x[ld + i];
    in.mz = x[2 * ld + i];
    in.wxx = wx[i];
    in.wxy = XYZ ? wx[ld + i] : T(0);
    in.wxz = XYZ ? wx[2 * ld + i] : T(0);
    const int64_t sample = (d.j0 + kk) / d.substeps;
    in.u_s = d.u + (sample * S + s) * d.n_in;
    in.raw = input_dot<T>(d.w_in + (int64_t)i * d.n_in, in.u_s, d.n_in);
    return in;
}

// Where the pointwise adjoint of a stage leaves the node's parameter
// partials (d/da_cp, d/da_in, d/dh_s, d/dh_appl and A_in b_x, the factor of
// dL/dw_in against the input u_s): added to gacc / gwin at once.
struct GlobalSink {
    template <typename T, typename V>
    __device__ __forceinline__ void add(const AdjDev<T>& d, int64_t gi, double pcp, double pin, double phs,
                                        double pap, double ab, const double* u_s, V, V, V) {
        const int64_t gs = (int64_t)d.S * d.ld;
        d.gacc[gi] += pcp;
        d.gacc[gs + gi] += pin;
        d.gacc[2 * gs + gi] += phs;
        d.gacc[3 * gs + gi] += pap;
        for (int q = 0; q < d.n_in; ++q) d.gwin[q * gs + gi] += ab * u_s[q];
    }
};

// Pointwise adjoint of stage `stage` of local step kk at node i of stream s,
// applied to v: stores the pointwise part of xbar (loc) and the coupling
// adjoint (st), and hands the node's parameter partials and the coupling
// adjoint to the sink.
template <typename T, bool XYZ, class Sink>
__device__ __forceinline__ void vjp_apply(const AdjDev<T>& d, const Coef<T>& k, int i, int s, int kk, int stage,
                                          const VjpIn<T>& in, T vx, T vy, T vz, Sink& sink) {
    constexpr int C = XYZ ? 3 : 1;
    const int64_t ld = d.ld;
    const int S = d.S;
    const T hin = k.a_in * in.raw;
    T gx, gy, gz, bx, by, bz, hsp;
    llg_vjp<T, XYZ>(k, in.mx, in.my, in.mz, k.a_cp * in.wxx, k.a_cp * in.wxy, k.a_cp * in.wxz, hin, vx, vy, vz, gx,
                    gy, gz, bx, by, bz, hsp);
    T* lc = d.loc + (int64_t)s * 3 * ld;
    lc[i] = gx;
    lc[ld + i] = gy;
    lc[2 * ld + i] = gz;
    T* sp = d.st + adj_slot<C>(kk, stage, S, ld) + (int64_t)s * C * ld;
    sp[i] = bx;
    if (XYZ) {
        sp[ld + i] = by;
        sp[2 * ld + i] = bz;
    }
    double pcp = (double)bx * (double)in.wxx;
    if (XYZ) pcp += (double)by * (double)in.wxy + (double)bz * (double)in.wxz;
    sink.add(d, (int64_t)s * ld + i, pcp, (double)bx * (double)in.raw, (double)hsp, (double)bz,
             (double)k.a_in * (double)bx, in.u_s, bx, by, bz);
}

template <typename T, bool XYZ, class Sink>
__device__ __forceinline__ void stage_vjp(const AdjDev<T>& d, const Coef<T>& k, int i, int s, int kk, int stage,
                                          T vx, T vy, T vz, Sink& sink) {
    vjp_apply<T, XYZ>(d, k, i, s, kk, stage, vjp_load<T, XYZ>(d, i, s, kk, stage), vx, vy, vz, sink);
}

// Inputs of prep_apply for local step kk at node i of stream s: the loss
// gradients on m_{j+1} (each read only where it applies), the state m_{j+1}
// after projection and its norm before it, and the inputs of the pointwise
// adjoint of the step's last stage; none depends on a coupling sum.
template <typename T>
struct PrepIn {
    T gr[3], gf[3], mh[3], pn;
    VjpIn<T> v;
};

// mhat: the state m_{j+1} (after projection) of stream s, [3][ld]; pn: the
// norm of m_{j+1} before projection.
template <typename T, bool XYZ>
__device__ __forceinline__ PrepIn<T> prep_load(const AdjDev<T>& d, int i, int s, int kk, const T* mhat, T pn) {
    const int64_t ld = d.ld;
    const int64_t jn = d.j0 + kk + 1;   // index of the state this step produces
    PrepIn<T> in;
    for (int c = 0; c < 3; ++c) in.gr[c] = in.gf[c] = in.mh[c] = T(0);
    if (d.g_rec && jn % d.substeps == 0) {
        const T* g = d.g_rec + (((jn / d.substeps - 1) * d.S + s) * d.n + i) * 3;
        for (int c = 0; c < 3; ++c) in.gr[c] = g[c];
    }
    if (d.g_fin && jn == d.steps) {
        const T* g = d.g_fin + ((int64_t)s * d.n + i) * 3;
        for (int c = 0; c < 3; ++c) in.gf[c] = g[c];
    }
    if (d.renorm)
        for (int c = 0; c < 3; ++c) in.mh[c] = mhat[c * ld + i];
    in.pn = pn;
    in.v = vjp_load<T, XYZ>(d, i, s, kk, 3);
    return in;
}

// Start reversing local step kk (global step j = j0 + kk) of stream s:
// a = dL/dm_{j+1} (carry plus the loss gradient on m_{j+1}), reversed
// through the optional projection; then the pointwise adjoint of its last
// stage.
template <typename T, bool XYZ, class Sink>
__device__ __forceinline__ void prep_apply(const AdjDev<T>& d, const Coef<T>& k, int i, int s, int kk,
                                           const PrepIn<T>& in, T cx, T cy, T cz, Sink& sink) {
    const int64_t ld = d.ld;
    const int64_t jn = d.j0 + kk + 1;
    T a[3] = {cx, cy, cz};
    if (d.g_rec && jn % d.substeps == 0)
        for (int c = 0; c < 3; ++c) a[c] += in.gr[c];
    if (d.g_fin && jn == d.steps)
        for (int c = 0; c < 3; ++c) a[c] += in.gf[c];
    if (d.renorm) {
        const T ux = in.mh[0], uy = in.mh[1], uz = in.mh[2];
        const T ao = (a[0] * ux + a[1] * uy) + a[2] * uz;
        a[0] = (a[0] - ao * ux) / in.pn;
        a[1] = (a[1] - ao * uy) / in.pn;
        a[2] = (a[2] - ao * uz) / in.pn;
    }
    const int64_t sb = (int64_t)s * 3 * ld;
    for (int c = 0; c < 3; ++c) {
        d.abar[sb + c * ld + i] = a[c];
        d.mbar[sb + c * ld + i] = a[c];
    }
    vjp_apply<T, XYZ>(d, k, i, s, kk, 3, in.v, k.h6 * a[0], k.h6 * a[1], k.h6 * a[2], sink);
}

template <typename T, bool XYZ, class Sink>
__device__ __forceinline__ void prep_step(const AdjDev<T>& d, const Coef<T>& k, int i, int s, int kk, const T* mhat,
                                          T pn, T cx, T cy, T cz, Sink& sink) {
    prep_apply<T, XYZ>(d, k, i, s, kk, prep_load<T, XYZ>(d, i, s, kk, mhat, pn), cx, cy, cz, sink);
}

// Inputs of a forward stage's epilogue at node i of stream s (stage input,
// state, RK4 accumulator, input field); none depends on the coupling sums,
// so the multi-stream kernels load them before the product.
template <typename T>
struct FwdIn {
    T sx, sy, sz, mx, my, mz, cx, cy, cz, hin;
};

template <typename T>
__device__ __forceinline__ FwdIn<T> fwd_load(const AdjDev<T>& d, const Coef<T>& k, int i, int s, int kk, int stage,
                                             int cur) {
    const int64_t ld = d.ld;
    const int64_t sb = (int64_t)s * 3 * ld;
    const T* xin = d.ms[cur] + sb;
    const T* m = d.m + sb;
    const T* acc = d.acc + sb;
    const int sample = (int)((d.j0 + kk) / d.substeps);
    FwdIn<T> in;
    in.hin = input_field(k, d.w_in + (int64_t)i * d.n_in, d.u + ((int64_t)sample * d.S + s) * d.n_in, d.n_in);
    in.sx = xin[i];
    in.sy = xin[ld + i];
    in.sz = xin[2 * ld + i];
    in.mx = m[i];
    in.my = m[ld + i];
    in.mz = m[2 * ld + i];
    in.cx = in.cy = in.cz = T(0);
    if (stage > 0) {
        in.cx = acc[i];
        in.cy = acc[ld + i];
        in.cz = acc[2 * ld + i];
    }
    return in;
}

// Epilogue of a forward stage for node i of stream s, given its inputs and
// the raw coupling sums (dx, dy, dz): the right-hand side of Eq. (gov), the
// RK4 stage update (the arithmetic of the plain stage kernels), the stage
// trace and, for plain runs, the record after the last step of a sample.
template <typename T, bool XYZ>
__device__ __forceinline__ void fwd_finish(const AdjDev<T>& d, const Coef<T>& k, int i, int s, int kk, int stage,
                                           int cur, int trace, const FwdIn<T>& in, T dx, T dy, T dz) {
    constexpr int C = XYZ ? 3 : 1;
    const int64_t ld = d.ld;
    const int64_t sb = (int64_t)s * 3 * ld;
    T* xout = d.ms[cur ^ 1] + sb;
    const int64_t j = d.j0 + kk;
    const int sample = (int)(j / d.substeps);
    if (trace) {
        T* x = d.xt + adj_slot<3>(kk, stage, d.S, ld) + sb;
        x[i] = in.sx;
        x[ld + i] = in.sy;
        x[2 * ld + i] = in.sz;
        T* w = d.wx + adj_slot<C>(kk, stage, d.S, ld) + (int64_t)s * C * ld;
        w[i] = dx;
        if (XYZ) {
            w[ld + i] = dy;
            w[2 * ld + i] = dz;
        }
    }
    T fx, fy, fz;
    llg_rhs<T, XYZ>(k, in.sx, in.sy, in.sz, k.a_cp * dx, XYZ ? k.a_cp * dy : T(0), XYZ ? k.a_cp * dz : T(0), in.hin,
                    fx, fy, fz);
    T* m = d.m + sb;
    T* acc = d.acc + sb;
    T cx = in.cx, cy = in.cy, cz = in.cz;
    T nx = rk4_update(k, stage, in.mx, cx, fx);
    T ny = rk4_update(k, stage, in.my, cy, fy);
    T nz = rk4_update(k, stage, in.mz, cz, fz);
    if (stage == 3) {
        if (d.renorm) {
            if (trace) {
                const double ex = nx, ey = ny, ez = nz;
                d.pn[((int64_t)kk * d.S + s) * ld + i] = (T)__builtin_sqrt((ex * ex + ey * ey) + ez * ez);
            }
            renormalize(nx, ny, nz);
        }
        m[i] = nx;
        m[ld + i] = ny;
        m[2 * ld + i] = nz;
        if (d.rec && (j + 1) % d.substeps == 0) {
            T* r = d.rec + (((int64_t)sample * d.S + s) * d.n + i) * 3;
            r[0] = nx;
            r[1] = ny;
            r[2] = nz;
        }
        if (!finite3(nx, ny, nz)) atomicMin(d.bad, sample);
    } else {
        acc[i] = cx;
        acc[ld + i] = cy;
        acc[2 * ld + i] = cz;
    }
    xout[i] = nx;
    xout[ld + i] = ny;
    xout[2 * ld + i] = nz;
}

template <typename T, bool XYZ>
__device__ __forceinline__ void fwd_epilogue(const AdjDev<T>& d, const Coef<T>& k, int i, int s, int kk, int stage,
                                             int cur, int trace, T dx, T dy, T dz) {
    fwd_finish<T, XYZ>(d, k, i, s, kk, stage, cur, trace, fwd_load<T>(d, k, i, s, kk, stage, cur), dx, dy, dz);
}

// Inputs of a reversed stage's epilogue at node i of stream s: the
// pointwise part of xbar, dL/dm so far, a, and (below the last stage) the
// inputs of the next stage's pointwise adjoint; none depends on the product.
template <typename T>
struct RevIn {
    T lc[3], mb[3], ab[3];
    PrepIn<T> p;   // p.v: the next stage's pointwise adjoint inputs; all of p when that stage starts the previous step
};

template <typename T, bool XYZ>
__device__ __forceinline__ RevIn<T> rev_load(const AdjDev<T>& d, int i, int s, int kk, int stage) {
    const int64_t ld = d.ld;
    const int64_t sb = (int64_t)s * 3 * ld;
    RevIn<T> in;
    for (int c = 0; c < 3; ++c) {
        in.lc[c] = d.loc[sb + c * ld + i];
        in.mb[c] = d.mbar[sb + c * ld + i];
        in.ab[c] = d.abar[sb + c * ld + i];
    }
    if (stage > 0) {
        in.p.v = vjp_load<T, XYZ>(d, i, s, kk, stage - 1);
    } else if (kk > 0) {
        // the first stage of step kk is reversed: the previous step starts,
        // and its output m_{j0+kk} is the traced first stage input of step kk
        const T* mhat = d.xt + adj_slot<3>(kk, 0, d.S, ld) + sb;
        const T pn = d.renorm ? d.pn[((int64_t)(kk - 1) * d.S + s) * ld + i] : T(1);
        in.p = prep_load<T, XYZ>(d, i, s, kk - 1, mhat, pn);
    }
    return in;
}

// Epilogue of a reversed stage for node i of stream s, given its inputs and
// t = (W^T bbar) of the stage: xbar = loc + a_cp t along the coupled
// components, dL/dm += xbar, then the pointwise adjoint of the next stage to
// reverse (or, after the first stage, the start of the previous step).
template <typename T, bool XYZ, class Sink>
__device__ __forceinline__ void rev_finish(const AdjDev<T>& d, const Coef<T>& k, int i, int s, int kk, int stage,
                                           const RevIn<T>& in, T tx, T ty, T tz, Sink& sink) {
    const int64_t ld = d.ld;
    const int64_t sb = (int64_t)s * 3 * ld;
    T xb[3] = {in.lc[0] + k.a_cp * tx, in.lc[1], in.lc[2]};
    if (XYZ) {
        xb[1] = xb[1] + k.a_cp * ty;
        xb[2] = xb[2] + k.a_cp * tz;
    }
    T mb[3];
    for (int c = 0; c < 3; ++c) {
        mb[c] = in.mb[c] + xb[c];
        d.mbar[sb + c * ld + i] = mb[c];
    }
    if (stage > 0) {
        // kbar of stage-1: its weight in m' times a, plus its step into this stage's input
        const T wgt = (stage - 1 == 0) ? k.h6 : T(2) * k.h6;
        const T hst = (stage == 3) ? k.h1 : k.h2;
        const T v0 = wgt * in.ab[0] + hst * xb[0];
        const T v1 = wgt * in.ab[1] + hst * xb[1];
        const T v2 = wgt * in.ab[2] + hst * xb[2];
        vjp_apply<T, XYZ>(d, k, i, s, kk, stage - 1, in.p.v, v0, v1, v2, sink);
    } else if (kk > 0) {
        // step j = j0 + kk is reversed: mbar = dL/dm_j.  Start step j - 1.
        prep_apply<T, XYZ>(d, k, i, s, kk - 1, in.p, mb[0], mb[1], mb[2], sink);
    }
}

template <typename T, bool XYZ>
__device__ __forceinline__ void rev_epilogue(const AdjDev<T>& d, const Coef<T>& k, int i, int s, int kk, int stage,
                                             T tx, T ty, T tz) {
    GlobalSink sink;
    rev_finish<T, XYZ>(d, k, i, s, kk, stage, rev_load<T, XYZ>(d, i, s, kk, stage), tx, ty, tz, sink);
}

// Launchers of the multi-stream (S > 1) stage kernels, FP32 (sto_batch.hip).
void launch_batch_fwd(const AdjDev<float>& d, const Coef<float>& k, int kk, int stage, int cur, int trace, int xyz,
                      hipStream_t st);
void launch_batch_rev(const AdjDev<float>& d, const Coef<float>& k, int kk, int stage, int xyz, hipStream_t st);

}  // namespace sto
