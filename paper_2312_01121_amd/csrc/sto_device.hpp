// Device helpers shared by the RK4 kernels: coefficients, the pointwise
// right-hand side of the LLG + spin-transfer-torque equation, the RK4 stage
// update, and the dot-product accumulators.
//
// Rounding contract (FP64).  The coupled, driven model is chaotic, so the
// FP64 path fixes its arithmetic completely:
//   * every coupling and input sum is accumulated in double-double
//     (error-free transformations: TwoProduct by fma, Knuth's TwoSum) and
//     rounded once, which gives the nearest double to the exact sum except
//     when the exact sum lies within ~n u^2 of a rounding boundary;
//   * every other operation is one IEEE double operation in the grouping
//     written below.  All HIP sources are compiled with -ffp-contract=off so
//     that no multiply-add is fused behind our back.
// FP32 accumulates plain fma in float and is checked to a tolerance.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sto {

template <typename T>
struct Coef {
    T h_appl, h_k, h_s, lam, px, py, pz;
    T a_cp, a_in;
    T c1, c2;          // 1/(1+alpha^2), alpha/(1+alpha^2)
    T h2, h1, h6;      // dt/2, dt, dt/6
};

// ---------------------------------------------------------------------------
// Accumulators
// ---------------------------------------------------------------------------
// Double-double running sum (s, c): s + c approximates the exact sum of the
// products added so far, with error ~ n u^2 sum |a_i b_i|.
struct DD {
    double s, c;
};

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void dd_fma(DD& acc, double a, double b) {
    double p = a * b;
    double pe = __builtin_fma(a, b, -p);   // exact: p + pe == a*b
    double s, e;
    two_sum(acc.s, p, s, e);
    acc.s = s;
    acc.c = acc.c + (e + pe);
}

__device__ __forceinline__ DD dd_add(DD x, DD y) {
    DD r;
    double e;
    two_sum(x.s, y.s, r.s, e);
    r.c = (x.c + y.c) + e;
    return r;
}

__device__ __forceinline__ double dd_round(DD x) { return x.s + x.c; }

template <typename T> struct Acc;
template <> struct Acc<double> {
    using type = DD;
    static __device__ __forceinline__ DD zero() { return DD{0.0, 0.0}; }
    static __device__ __forceinline__ void fma(DD& a, double w, double x) { dd_fma(a, w, x); }
    static __device__ __forceinline__ DD add(DD a, DD b) { return dd_add(a, b); }
    static __device__ __forceinline__ double round(DD a) { return dd_round(a); }
    static __device__ __forceinline__ DD shfl_xor(DD a, int mask, int width) {
        return DD{__shfl_xor(a.s, mask, width), __shfl_xor(a.c, mask, width)};
    }
};
template <> struct Acc<float> {
    using type = float;
    static __device__ __forceinline__ float zero() { return 0.0f; }
    static __device__ __forceinline__ void fma(float& a, float w, float x) { a = __builtin_fmaf(w, x, a); }
    static __device__ __forceinline__ float add(float a, float b) { return a + b; }
    static __device__ __forceinline__ float round(float a) { return a; }
    static __device__ __forceinline__ float shfl_xor(float a, int mask, int width) {
        return __shfl_xor(a, mask, width);
    }
};

// Lane exchange for the butterfly below, without an LDS round trip.  Inside
// a 16-lane row it is a DPP move: OFF = 1 and 2 are the xor partners (quad
// permutations); OFF = 4 and 8 are the row's half-mirror and mirror, which
// reach a lane of the partner group of 4 or 8 lanes (used only where every
// lane of a group already holds the same value).  OFF = 16 and 32 are the
// xor partners through gfx950's permlane swaps: swapping a value with itself
// leaves the partner's value in one of the two results (lanes with bit
// OFF set take the first).
template <int OFF>
__device__ __forceinline__ int lane_partner_i32(int v) {
    if constexpr (OFF == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (threadIdx.x & 16) ? r[0] : r[1];
    } else if constexpr (OFF == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (threadIdx.x & 32) ? r[0] : r[1];
    } else {
        static_assert(OFF == 1 || OFF == 2 || OFF == 4 || OFF == 8, "lane distance");
        constexpr int ctrl = OFF == 1 ? 0xB1 : OFF == 2 ? 0x4E : OFF == 4 ? 0x141 : 0x140;
        return __builtin_amdgcn_update_dpp(0, v, ctrl, 0xF, 0xF, false);
    }
}
template <int OFF>
__device__ __forceinline__ float lane_partner(float v) {
    return __builtin_bit_cast(float, lane_partner_i32<OFF>(__builtin_bit_cast(int, v)));
}
template <int OFF>
__device__ __forceinline__ double lane_partner(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned long long lo = (unsigned)lane_partner_i32<OFF>((int)(unsigned)b);
    const unsigned long long hi = (unsigned)lane_partner_i32<OFF>((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, lo | (hi << 32));
}
template <int OFF>
__device__ __forceinline__ DD lane_partner(DD v) {
    return DD{lane_partner<OFF>(v.s), lane_partner<OFF>(v.c)};
}

// Butterfly reduction over groups of `width` consecutive lanes (power of
// two, <= 64, wave-uniform, groups aligned to their width); every lane of
// the group ends with the group's total.  Partners at distance 1, 2, 4, 8,
// 16, 32 in that order: after each step every lane of a group holds the same
// value (the additions commute bitwise, in double-double too), so the whole
// wave's total is (r0 + r1) + (r2 + r3) of its four row totals.
template <typename T>
__device__ __forceinline__ typename Acc<T>::type group_reduce(typename Acc<T>::type v, int width) {
    using A = Acc<T>;
    if (width >= 2) v = A::add(v, lane_partner<1>(v));
    if (width >= 4) v = A::add(v, lane_partner<2>(v));
    if (width >= 8) v = A::add(v, lane_partner<4>(v));
    if (width >= 16) v = A::add(v, lane_partner<8>(v));
    if (width >= 32) v = A::add(v, lane_partner<16>(v));
    if (width >= 64) v = A::add(v, lane_partner<32>(v));
    return v;
}

// Plain sum over the 64 lanes of a wave (every lane ends with the total), in
// the butterfly order above.
template <typename T>
__device__ __forceinline__ T lane_sum(T v) {
    v += lane_partner<1>(v);
    v += lane_partner<2>(v);
    v += lane_partner<4>(v);
    v += lane_partner<8>(v);
    v += lane_partner<16>(v);
    v += lane_partner<32>(v);
    return v;
}

// ---------------------------------------------------------------------------
// Pointwise right-hand side, Eq. (gov), for one node.
//   (mx,my,mz)  stage input of the node
//   cx,cy,cz    coupling field a_cp * (W m)_k (cy = cz = 0 unless xyz)
//   hin         input field a_in * (w_in u)_k, along e_x
// ---------------------------------------------------------------------------
template <typename T, bool XYZ>
__device__ __forceinline__ void llg_rhs(const Coef<T>& k, T mx, T my, T mz, T cx, T cy, T cz,
                                        T hin, T& fx, T& fy, T& fz) {
    T mp = (mx * k.px + my * k.py) + mz * k.pz;
    T hs = k.h_s / (T(1) + k.lam * mp);
    // q = p x m
    T qx = k.py * mz - k.pz * my;
    T qy = k.pz * mx - k.px * mz;
    T qz = k.px * my - k.py * mx;
    T hz = k.h_appl + k.h_k * mz;
    T bx = (cx + hin) + hs * qx;
    T by, bz;
    if (XYZ) {
        by = cy + hs * qy;
        bz = (hz + cz) + hs * qz;
    } else {
        by = hs * qy;
        bz = hz + hs * qz;
    }
    // m x b
    T ax = my * bz - mz * by;
    T ay = mz * bx - mx * bz;
    T az = mx * by - my * bx;
    // m x (m x b)
    T dx = my * az - mz * ay;
    T dy = mz * ax - mx * az;
    T dz = mx * ay - my * ax;
    fx = (-k.c1) * ax - k.c2 * dx;
    fy = (-k.c1) * ay - k.c2 * dy;
    fz = (-k.c1) * az - k.c2 * dz;
}

// RK4 stage bookkeeping for one node and one component.
//   stage 0: acc = k1;          next = m + (dt/2) k1
//   stage 1: acc = acc + 2 k2;  next = m + (dt/2) k2
//   stage 2: acc = acc + 2 k3;  next = m + dt k3
//   stage 3: m' = m + (dt/6)(acc + k4); next = m'
// Returns the next stage input; on stage 3 it is also the new state.
template <typename T>
__device__ __forceinline__ T rk4_update(const Coef<T>& k, int stage, T m, T& acc, T f) {
    switch (stage) {
        case 0: acc = f; return m + k.h2 * f;
        case 1: acc = acc + T(2) * f; return m + k.h2 * f;
        case 2: acc = acc + T(2) * f; return m + k.h1 * f;
        default: return m + k.h6 * (acc + f);
    }
}

template <typename T>
__device__ __forceinline__ void renormalize(T& x, T& y, T& z) {
    T nrm = __builtin_sqrt((x * x + y * y) + z * z);
    x = x / nrm;
    y = y / nrm;
    z = z / nrm;
}
template <>
__device__ __forceinline__ void renormalize<float>(float& x, float& y, float& z) {
    // the FP32 path takes the norm in FP64
    double dx = x, dy = y, dz = z;
    double nrm = __builtin_sqrt((dx * dx + dy * dy) + dz * dz);
    x = (float)(dx / nrm);
    y = (float)(dy / nrm);
    z = (float)(dz / nrm);
}

template <typename T>
__device__ __forceinline__ bool finite3(T x, T y, T z) {
    return __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z);
}

// Input field a_in * sum_j w_in[j] u[j] for one node (u is FP64 on the device).
template <typename T>
__device__ __forceinline__ T input_field(const Coef<T>& k, const T* __restrict__ w_in_row,
                                         const double* __restrict__ u_s, int n_in) {
    typename Acc<T>::type a = Acc<T>::zero();
    for (int j = 0; j < n_in; ++j)
        Acc<T>::fma(a, w_in_row[j], (T)u_s[j]);
    return k.a_in * Acc<T>::round(a);
}

}  // namespace sto
