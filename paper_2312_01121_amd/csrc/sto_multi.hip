// MULTI path: S input streams drive S copies of one reservoir (one coupling
// matrix W, one set of constants, S states).  Per RK4 stage the coupling of
// all streams is one matrix product, C = a_cp * W X with X the N x S block of
// stage inputs m^x (paper, Eq. (coup); Sec. 3.3 writes the single-stream
// case as W^cp x), or the N x 3S block of all three components under the
// isotropic coupling, evaluated with FP32 MFMA (v_mfma_f32_16x16x4f32, FP32
// accumulation) and fused with the pointwise right-hand side of Eq. (gov)
// and the RK4 bookkeeping (Sec. 3.2).
//
// Tiling.  The columns of X are (stream, component) pairs.  Workgroup
// (bi, bj) owns the 16-row output tile of nodes 16 bi..16 bi + 15 against the
// 16 columns of SPW streams (16 streams of one component, or 5 streams of
// three components with the 16th column empty) for the whole run.  Its eight
// waves split the contraction dimension into eighths; each wave keeps its
// 16 rows x N/8 slice of W in registers as MFMA A operands (one element per
// lane per MFMA), reads the stage inputs of its columns from LDS as B
// operands, and the eight partial tiles are summed in LDS in a fixed order.
// One of the first 256 threads per (node, stream) pair then takes the pair's
// C coupling sums: its state, RK4 accumulator and stage input stay in
// registers.
//
// Exchange.  Stage inputs move through three rotating global buffers, laid
// out [component][stream][node], whose unpublished entries hold a sentinel
// bit pattern.  Each workgroup waits for the entries of its columns of the
// current buffer, re-arms its own entries of the buffer two stages ahead
// (every workgroup has finished reading that buffer: the gather just saw all
// outputs of the previous stage, each published after its workgroup's own
// gather), computes while those stores complete, waits for them and then
// publishes its outputs into the next buffer.  Every wait is bounded and
// raises a sticky abort flag when it expires.

#include <climits>
#include <cstdlib>

#include "sto_adjoint_dev.hpp"
#include "sto_internal.hpp"
#include "sto_multi.hpp"

namespace sto {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 512;
constexpr int kWaves = kBlock / 64;   // waves per workgroup, each a slice of the contraction
constexpr int kTile = 16;
// LDS row pitch of the gathered stage inputs: 17 (odd), so that the gather's
// writes (consecutive threads on consecutive nodes of one column) fall in
// distinct banks; the MFMA operand reads (16 columns of 4 nodes) then meet
// at most 2-way conflicts.
constexpr int kXP = kTile + 1;
constexpr int kSpinLimit = 1 << 20;
// 4-byte loads in flight per thread in the gather, at most.
constexpr int kMaxInFlight = 64;

// Streams per workgroup: the 16 columns hold SPW streams of C components.
template <bool XYZ> constexpr int streams_per_group() { return XYZ ? 5 : 16; }

// Wait until the stage inputs of the workgroup's columns are published and
// store them K-major in LDS: xs[k * kXP + js * C + c] for node k, local
// stream js and component c.  Component c of stream s, node k sits at
// xb[c * cstride + s * ld + k].  The columns are SPW C rows (js, c) of n
// entries; thread t covers entries t, t + 512, ... (KI of them) of every
// row, so all indices but its own column are compile-time constants.  Up to
// kMaxInFlight loads per thread are in flight in one round trip to memory.
template <int C, int SPW, int KI>
__device__ bool gather_multi(const float* xb, int64_t ld, int64_t cstride, int n, int s0, int ns, float* xs,
                             int* abort_flag) {
    constexpr int kRows = C * SPW;
    constexpr int kRpr = kRows < kMaxInFlight / KI ? kRows : kMaxInFlight / KI;   // rows per round
    constexpr int KQ = kRpr * KI;
    constexpr int kWords = (KQ + 31) / 32;
    const unsigned* src = reinterpret_cast<const unsigned*>(xb);
    const int t = threadIdx.x;
    bool ok = true;
    for (int r0 = 0; r0 < kRows && ok; r0 += kRpr) {
        unsigned v[KQ];
        unsigned todo[kWords];   // bit q: entry q of this round is still unpublished
#pragma unroll
        for (int w = 0; w < kWords; ++w) todo[w] = 0u;
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            const int row = r0 + q / KI, k = t + kBlock * (q % KI);
            if (row < kRows && row / C < ns && k < n) todo[q / 32] |= 1u << (q % 32);
        }
        auto pending = [&] {
            unsigned any = 0u;
#pragma unroll
            for (int w = 0; w < kWords; ++w) any |= todo[w];
            return any != 0u;
        };
        int rounds = 0;
        while (pending()) {
            // the addresses are recomputed in every poll round from a copy of
            // the base that the compiler cannot hoist, instead of holding KQ
            // 64-bit addresses in registers
            const unsigned* base = src + (int64_t)s0 * ld + t;
            asm volatile("" : "+v"(base));
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                if (todo[q / 32] & (1u << (q % 32))) {
                    const int row = r0 + q / KI, js = row / C, c = row % C;
                    v[q] = __hip_atomic_load(base + (c * cstride + (int64_t)js * ld + kBlock * (q % KI)),
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                if ((todo[q / 32] & (1u << (q % 32))) && v[q] != ~0u) {
                    const int row = r0 + q / KI, k = t + kBlock * (q % KI);
                    xs[k * kXP + row] = __builtin_bit_cast(float, v[q]);
                    todo[q / 32] &= ~(1u << (q % 32));
                }
            }
            if (pending() && (++rounds & 255) == 0) {
                if (rounds > kSpinLimit) {
                    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = false;
                    break;
                }
                if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = false;
                    break;
                }
            }
        }
    }
    return ok;
}

// KREG: MFMA steps per wave, >= ceil(N/32) (each step contracts 4 nodes;
// N <= 32 KREG).  XYZ: all three components coupled, else m^x only.  TRACE:
// write the stage trace of the adjoint (tr); sample0 offsets the sample
// index reported on a non-finite state.  RT: 16-node row tiles per
// workgroup (1 or 2), which share the gathered columns.
// One wave's partial product tile: acc[rt] += sum over t < KREG of the
// 16 x 4 slice A[rt][t] of the row tile times the 4 x 16 slice of the
// gathered columns (LDS, row stride kXP) at this wave's nodes 4t .. 4t + 3.
// The LDS reads of a group of up to GROUP steps are issued before its
// products, so one read latency covers the group.  Steps past the wave's share of the
// contraction have zero A and add nothing; their reads are clamped into the
// array.
template <int KREG, int RT, int GROUP>
__device__ __forceinline__ void wave_tile_product(const float (&areg)[RT][KREG], const float* xs, int node0, int kp,
                                                  int lane, f4 (&acc)[RT]) {
    constexpr int G = KREG < GROUP ? KREG : GROUP;
#pragma unroll
    for (int t0 = 0; t0 < KREG; t0 += G) {
        float b[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int kk = min(node0 + 4 * (t0 + g) + (lane >> 4), kp - 1);
            b[g] = xs[kk * kXP + (lane & 15)];
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(areg[rt][t0 + g], b[g], acc[rt], 0, 0, 0);
    }
}

// PHASE (an instance of its own, so that the others carry no trace code):
// thread 0 of every workgroup stamps the device's constant-rate clock at
// four points of each of the first phase_stages stages (start, columns
// gathered, own pairs computed, published).
template <bool PHASE>
__device__ __forceinline__ void multi_stamp(unsigned long long* phase, int phase_stages, int sigma, int point) {
    if constexpr (PHASE) {
        if (sigma < phase_stages && threadIdx.x == 0)
            phase[(((size_t)blockIdx.y * gridDim.x + blockIdx.x) * phase_stages + sigma) * 4 + point] = wall_clock64();
    }
}

template <int KREG, bool XYZ, bool TRACE, int RT, bool PHASE>
__global__ void __launch_bounds__(kBlock) k_multi(DevState<float> d, Coef<float> k, const double* __restrict__ u,
                                                  float* __restrict__ states, int streams, int samples,
                                                  int substeps, int renorm, int sample0, MultiTrace tr,
                                                  unsigned long long* phase, int phase_stages) {
    constexpr int C = XYZ ? 3 : 1;
    constexpr int SPW = streams_per_group<XYZ>();
    constexpr int KI = KREG <= 16 ? 1 : KREG / 16;   // gather entries per row and thread: 512 KI >= 32 KREG >= N
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int ok_lds;
    const int n = d.n;
    const int64_t ld = d.ld;
    const int kp = (n + 31) / 32 * 32;                           // contraction length padded to 32
    float* xs = reinterpret_cast<float*>(smem_raw);              // [kp][kXP]
    float* cs = xs + (int64_t)kp * kXP;                          // [RT][kWaves][16][16] partial tiles
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row0 = blockIdx.x * kTile * RT;
    const int s0 = blockIdx.y * SPW;
    const int ns = min(SPW, streams - s0);
    int* abort_flag = d.sync + kSyncAbortWord;
    if (threadIdx.x == 0) ok_lds = 1;
    for (int i = threadIdx.x; i < kp * kXP; i += kBlock) xs[i] = 0.0f;   // padded nodes and columns stay 0

    // A operands: this wave's eighth of the contraction for the tile's rows.
    const int kq = kp / kWaves;                                  // nodes per wave (multiple of 4)
    const int steps = kq / 4;
    float areg[RT][KREG];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int r = row0 + rt * kTile + (lane & 15);
#pragma unroll
        for (int t = 0; t < KREG; ++t) {
            const int kk = wave * kq + 4 * t + (lane >> 4);
            areg[rt][t] = (t < steps && r < n && kk < n) ? d.W[(int64_t)r * ld + kk] : 0.0f;
        }
    }

    // the (node, stream) pair of this thread: row tile tt, output row ti,
    // first column tj of the stream's C columns
    const int tt = threadIdx.x >> 8, ti = (threadIdx.x >> 4) & 15, tj = threadIdx.x & 15;
    const int js = tj / C;
    const int node = row0 + tt * kTile + ti;
    const int strm = s0 + js;
    const bool mine = tt < RT && tj % C == 0 && js < ns && node < n;
    const int nd = min(node, n - 1), sd = min(strm, streams - 1);
    const float* m_in = d.m + (int64_t)sd * 3 * ld;
    float mx = m_in[nd], my = m_in[ld + nd], mz = m_in[2 * ld + nd];
    float sx = mx, sy = my, sz = mz, ax = 0.f, ay = 0.f, az = 0.f;
    float* xbuf = d.xchg;                                        // [3 buffers][C][streams][ld]
    const int64_t cstride = (int64_t)streams * ld;               // one component of one buffer
    const int64_t bstride = C * cstride;                         // one buffer

    int sigma = 0;
    for (int s = 0; s < samples; ++s) {
        const float hin =
            input_field(k, d.w_in + (int64_t)nd * d.n_in, u + ((int64_t)s * streams + sd) * d.n_in, d.n_in);
        for (int sub = 0; sub < substeps; ++sub) {
            for (int stage = 0; stage < 4; ++stage, ++sigma) {
                float* xin = xbuf + (int64_t)(sigma % 3) * bstride;
                float* xout = xbuf + (int64_t)((sigma + 1) % 3) * bstride;
                float* xold = xbuf + (int64_t)((sigma + 2) % 3) * bstride;
                __syncthreads();
                multi_stamp<PHASE>(phase, phase_stages, sigma, 0);
                if (!gather_multi<C, SPW, KI>(xin, ld, cstride, n, s0, ns, xs, abort_flag)) ok_lds = 0;
                __syncthreads();
                if (ok_lds == 0) return;
                multi_stamp<PHASE>(phase, phase_stages, sigma, 1);
                // re-arm this pair's entries of the buffer two stages ahead now;
                // the stores complete while the stage is computed
                if (mine) {
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        __hip_atomic_store(reinterpret_cast<unsigned*>(xold + c * cstride + (int64_t)strm * ld + node),
                                           ~0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                // partial tile of this wave: D[i][col] = sum over its nodes of
                // W[row0+i][k] X[k][col]
                f4 acc[RT];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) acc[rt] = f4{0.f, 0.f, 0.f, 0.f};
                wave_tile_product<KREG, RT, 8>(areg, xs, wave * kq, kp, lane, acc);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        cs[((rt * kWaves + wave) * kTile + 4 * (lane >> 4) + r) * kTile + (lane & 15)] = acc[rt][r];
                __syncthreads();
                float dot[C];
                const int tc = min(tt, RT - 1);   // stays in the partial tiles for threads that own no pair
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int col = min(tj + c, kTile - 1);
                    float v = cs[((tc * kWaves + 0) * kTile + ti) * kTile + col];
#pragma unroll
                    for (int w = 1; w < kWaves; ++w) v += cs[((tc * kWaves + w) * kTile + ti) * kTile + col];
                    dot[c] = v;
                }
                // the re-arm stores must complete before the publish below;
                // the trace stores need not
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                if constexpr (TRACE) {
                    if (mine) {
                        const int64_t slot = ((int64_t)(s * substeps + sub) * 4 + stage) * streams + strm;
                        float* x = tr.xt + slot * 3 * ld;
                        x[node] = sx;
                        x[ld + node] = sy;
                        x[2 * ld + node] = sz;
                        float* w = tr.wx + slot * C * ld;
#pragma unroll
                        for (int c = 0; c < C; ++c) w[c * ld + node] = dot[c];
                    }
                }
                float fx, fy, fz;
                if constexpr (XYZ)
                    llg_rhs<float, true>(k, sx, sy, sz, k.a_cp * dot[0], k.a_cp * dot[1], k.a_cp * dot[2], hin, fx,
                                         fy, fz);
                else
                    llg_rhs<float, false>(k, sx, sy, sz, k.a_cp * dot[0], 0.f, 0.f, hin, fx, fy, fz);
                float nx = rk4_update(k, stage, mx, ax, fx);
                float ny = rk4_update(k, stage, my, ay, fy);
                float nz = rk4_update(k, stage, mz, az, fz);
                if (stage == 3) {
                    if (renorm) {
                        if constexpr (TRACE) {
                            if (mine) {
                                const double ex = nx, ey = ny, ez = nz;
                                tr.pn[((int64_t)(s * substeps + sub) * streams + strm) * ld + node] =
                                    (float)__builtin_sqrt((ex * ex + ey * ey) + ez * ez);
                            }
                        }
                        renormalize(nx, ny, nz);
                    }
                    mx = nx;
                    my = ny;
                    mz = nz;
                }
                sx = nx;
                sy = ny;
                sz = nz;
                multi_stamp<PHASE>(phase, phase_stages, sigma, 2);
                if (mine) {
                    const int64_t o = (int64_t)strm * ld + node;
                    __hip_atomic_store(xout + o, nx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if constexpr (XYZ) {
                        __hip_atomic_store(xout + cstride + o, ny, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(xout + 2 * cstride + o, nz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                multi_stamp<PHASE>(phase, phase_stages, sigma, 3);
            }
        }
        if (mine) {
            if (states) {
                float* rec = states + (((int64_t)s * streams + strm) * n + node) * 3;
                rec[0] = mx;
                rec[1] = my;
                rec[2] = mz;
            }
            if (!finite3(mx, my, mz)) atomicMin(d.bad, sample0 + s);
        }
    }
    if (mine) {
        float* mo = d.m + (int64_t)strm * 3 * ld;
        mo[node] = mx;
        mo[ld + node] = my;
        mo[2 * ld + node] = mz;
    }
}

// Parameter partials of one (node, stream) pair summed in registers over a
// segment (up to kRegIn input channels) and added to gacc / gwin once at the
// end; the last coupling adjoint the epilogue produced is kept for the
// exchange.
constexpr int kRegIn = 4;

struct RegSink {
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    double w[kRegIn] = {0.0, 0.0, 0.0, 0.0};
    float b[3] = {0.f, 0.f, 0.f};
    __device__ __forceinline__ void add(const AdjDev<float>& d, int64_t, double pcp, double pin, double phs,
                                        double pap, double ab, const double* u_s, float bx, float by, float bz) {
        g[0] += pcp;
        g[1] += pin;
        g[2] += phs;
        g[3] += pap;
#pragma unroll
        for (int q = 0; q < kRegIn; ++q)
            if (q < d.n_in) w[q] += ab * u_s[q];
        b[0] = bx;
        b[1] = by;
        b[2] = bz;
    }
    __device__ __forceinline__ void flush(const AdjDev<float>& d, int64_t gi) {
        const int64_t gs = (int64_t)d.S * d.ld;
#pragma unroll
        for (int c = 0; c < 4; ++c) d.gacc[c * gs + gi] += g[c];
#pragma unroll
        for (int q = 0; q < kRegIn; ++q)
            if (q < d.n_in) d.gwin[q * gs + gi] += w[q];
    }
};

// Reversed stages of one adjoint segment in one cooperative launch: per
// stage t = W^T bbar for all streams (the exchange and the RT row tiles per
// workgroup of k_multi, with the transpose of W as the A operands), then
// each pair's adjoint epilogue (rev_load / rev_finish, as the per-stage
// kernels run it).  Each pair's epilogue inputs are loaded before the
// gather, so their latency hides behind the wait for the other workgroups;
// its parameter partials stay in registers until the end.  The epilogue
// leaves the next stage's bbar in the trace of coupling adjoints and
// publishes it through the rotating buffers.  Stages run from (kn - 1, 3)
// down to (0, 0); buffer 0 starts with the bbar of (kn - 1, 3).
template <int KREG, bool XYZ, int RT>
__global__ void __launch_bounds__(kBlock) k_multi_rev(AdjDev<float> d, Coef<float> k, float* __restrict__ xbuf,
                                                      int* sync, int kn) {
    constexpr int C = XYZ ? 3 : 1;
    constexpr int SPW = streams_per_group<XYZ>();
    constexpr int KI = KREG <= 16 ? 1 : KREG / 16;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int ok_lds;
    const int n = d.n;
    const int64_t ld = d.ld;
    const int streams = d.S;
    const int kp = (n + 31) / 32 * 32;
    float* xs = reinterpret_cast<float*>(smem_raw);              // [kp][kXP]
    float* cs = xs + (int64_t)kp * kXP;                          // [RT][kWaves][16][16]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row0 = blockIdx.x * kTile * RT;
    const int s0 = blockIdx.y * SPW;
    const int ns = min(SPW, streams - s0);
    int* abort_flag = sync + kSyncAbortWord;
    if (threadIdx.x == 0) ok_lds = 1;
    for (int i = threadIdx.x; i < kp * kXP; i += kBlock) xs[i] = 0.0f;

    const int kq = kp / kWaves;
    const int steps = kq / 4;
    float areg[RT][KREG];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int r = row0 + rt * kTile + (lane & 15);
#pragma unroll
        for (int t = 0; t < KREG; ++t) {
            const int kk = wave * kq + 4 * t + (lane >> 4);
            areg[rt][t] = (t < steps && r < n && kk < n) ? d.Wt[(int64_t)r * ld + kk] : 0.0f;
        }
    }
    // the pair of this thread: row tile tt, row ti, first column tj
    const int tt = threadIdx.x >> 8, ti = (threadIdx.x >> 4) & 15, tj = threadIdx.x & 15;
    const int js = tj / C;
    const int node = row0 + tt * kTile + ti;
    const int strm = s0 + js;
    const bool mine = tt < RT && tj % C == 0 && js < ns && node < n;
    const int64_t cstride = (int64_t)streams * ld;
    const int64_t bstride = C * cstride;
    RegSink sink;

    int sigma = 0;
    for (int kk = kn - 1; kk >= 0; --kk) {
        for (int stage = 3; stage >= 0; --stage, ++sigma) {
            const float* xin = xbuf + (int64_t)(sigma % 3) * bstride;
            float* xout = xbuf + (int64_t)((sigma + 1) % 3) * bstride;
            float* xold = xbuf + (int64_t)((sigma + 2) % 3) * bstride;
            // the epilogue's inputs depend neither on the product nor on the
            // other workgroups: load them before waiting for the exchange
            RevIn<float> in{};
            if (mine) in = rev_load<float, XYZ>(d, node, strm, kk, stage);
            __syncthreads();
            if (!gather_multi<C, SPW, KI>(xin, ld, cstride, n, s0, ns, xs, abort_flag)) ok_lds = 0;
            __syncthreads();
            if (ok_lds == 0) return;
            if (mine) {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    __hip_atomic_store(reinterpret_cast<unsigned*>(xold + c * cstride + (int64_t)strm * ld + node), ~0u,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            f4 acc[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[rt] = f4{0.f, 0.f, 0.f, 0.f};
            if constexpr (KREG >= 32) {
                // the reverse holds more registers: at KREG = 32 grouped reads
                // spill, so each step reads its slice just before its product
#pragma unroll
                for (int t = 0; t < KREG; ++t) {
                    if (t < steps) {
                        const int kr = wave * kq + 4 * t + (lane >> 4);
                        const float b = xs[kr * kXP + (lane & 15)];
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt)
                            acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(areg[rt][t], b, acc[rt], 0, 0, 0);
                    }
                }
            } else {
                wave_tile_product<KREG, RT, 8>(areg, xs, wave * kq, kp, lane, acc);
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    cs[((rt * kWaves + wave) * kTile + 4 * (lane >> 4) + r) * kTile + (lane & 15)] = acc[rt][r];
            __syncthreads();
            float t3[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int col = min(tj + c, kTile - 1);
                float v = 0.f;
#pragma unroll
                for (int w = 0; w < kWaves; ++w) v += cs[((min(tt, RT - 1) * kWaves + w) * kTile + ti) * kTile + col];
                t3[c] = v;
            }
            // the re-arm stores must complete before the publish below; the
            // epilogue's own stores need not
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (mine) {
                rev_finish<float, XYZ>(d, k, node, strm, kk, stage, in, t3[0], t3[1], t3[2], sink);
                if (kk > 0 || stage > 0) {
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        __hip_atomic_store(xout + c * cstride + (int64_t)strm * ld + node, sink.b[c], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
    if (mine) sink.flush(d, (int64_t)strm * ld + node);
}

// Buffer 0 <- the bbar slot [stream][C][ld] rearranged as [C][stream][ld];
// buffers 1 and 2 <- sentinel.
__global__ void k_multi_rev_prologue(const float* slot, float* xchg, int streams, int64_t ld, int C) {
    const int64_t per = (int64_t)streams * ld;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * C * per;
         i += (int64_t)gridDim.x * blockDim.x) {
        unsigned v = ~0u;
        if (i < C * per) {
            const int64_t c = i / per, r = i - c * per;
            const int64_t st = r / ld, node = r - st * ld;
            v = __builtin_bit_cast(unsigned, slot[(st * C + c) * ld + node]);
        }
        reinterpret_cast<unsigned*>(xchg)[i] = v;
    }
}

__global__ void k_multi_prologue(const float* m, float* xchg, int streams, int64_t ld, int C) {
    // buffer 0 <- the coupled components of every stream ([C][streams][ld]);
    // buffers 1 and 2 <- sentinel
    const int64_t per = (int64_t)streams * ld;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * C * per;
         i += (int64_t)gridDim.x * blockDim.x) {
        unsigned v = ~0u;
        if (i < C * per) {
            const int64_t c = i / per, r = i - c * per;
            const int64_t st = r / ld, node = r - st * ld;
            v = __builtin_bit_cast(unsigned, m[st * 3 * ld + c * ld + node]);
        }
        reinterpret_cast<unsigned*>(xchg)[i] = v;
    }
}

constexpr int kMaxKreg = 32;   // N <= 1024

int kreg_for(int n) {
    const int need = ((n + 31) / 32 * 32) / 32;
    for (int kr : {4, 8, 16, 32})
        if (kr >= need) return kr;
    return 0;
}

template <int KREG>
const void* multi_rev_kernel(int xyz, int rt) {
    if (rt == 2)
        return xyz ? reinterpret_cast<const void*>(&k_multi_rev<KREG, true, 2>)
                   : reinterpret_cast<const void*>(&k_multi_rev<KREG, false, 2>);
    return xyz ? reinterpret_cast<const void*>(&k_multi_rev<KREG, true, 1>)
               : reinterpret_cast<const void*>(&k_multi_rev<KREG, false, 1>);
}

// trace: 0 forward, 1 forward with the adjoint's trace, 3 forward with the
// phase stamps.
template <int KREG, int RT>
const void* multi_kernel(int xyz, int trace) {
    if (trace == 1)
        return xyz ? reinterpret_cast<const void*>(&k_multi<KREG, true, true, RT, false>)
                   : reinterpret_cast<const void*>(&k_multi<KREG, false, true, RT, false>);
    if (trace == 3)
        return xyz ? reinterpret_cast<const void*>(&k_multi<KREG, true, false, RT, true>)
                   : reinterpret_cast<const void*>(&k_multi<KREG, false, false, RT, true>);
    return xyz ? reinterpret_cast<const void*>(&k_multi<KREG, true, false, RT, false>)
               : reinterpret_cast<const void*>(&k_multi<KREG, false, false, RT, false>);
}

template <int KREG>
const void* multi_kernel(int xyz, int trace, int rt) {
    return rt == 2 ? multi_kernel<KREG, 2>(xyz, trace) : multi_kernel<KREG, 1>(xyz, trace);
}

}  // namespace

namespace {

// LDS of a kernel instance: the columns and one partial tile per wave and
// row tile.
size_t lds_bytes(int n, int rt) {
    const int kp = (n + 31) / 32 * 32;
    return ((size_t)kp * kXP + rt * kWaves * kTile * kTile) * sizeof(float);
}

}  // namespace

namespace {

// The kernel instance for n nodes and rt row tiles, with its dynamic LDS
// limit raised to what it needs; nullptr when n is out of range.
// trace: 0 forward, 1 forward with the adjoint's trace, 2 reversed stages,
// 3 forward with the phase stamps.
const void* multi_fn(int n, int xyz, int trace, int rt) {
    const void* fn = nullptr;
    switch (kreg_for(n)) {
        case 4: fn = trace == 2 ? multi_rev_kernel<4>(xyz, rt) : multi_kernel<4>(xyz, trace, rt); break;
        case 8: fn = trace == 2 ? multi_rev_kernel<8>(xyz, rt) : multi_kernel<8>(xyz, trace, rt); break;
        case 16: fn = trace == 2 ? multi_rev_kernel<16>(xyz, rt) : multi_kernel<16>(xyz, trace, rt); break;
        case 32: fn = trace == 2 ? multi_rev_kernel<32>(xyz, rt) : multi_kernel<32>(xyz, trace, rt); break;
        default: return nullptr;
    }
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes(n, rt)) != hipSuccess)
        return nullptr;
    return fn;
}

int stream_groups(int streams, int xyz) {
    const int spw = xyz ? streams_per_group<true>() : streams_per_group<false>();
    return (streams + spw - 1) / spw;
}

}  // namespace

namespace {

// A launch of one kernel instance: row tiles per workgroup, grid, LDS.
struct Shape {
    const void* fn;
    int rt, gx, gy;
    size_t lds;
};

// Whether every workgroup of the instance with rt row tiles can be
// co-resident (the cooperative launch needs all of them): the LDS fits and
// the grid is within the occupancy the runtime reports for it.
bool fits_rt(int n, int streams, int xyz, int trace, int rt, Shape* sh) {
    const int rows = kTile * rt;
    const int gx = (n + rows - 1) / rows, gy = stream_groups(streams, xyz);
    const size_t lds = lds_bytes(n, rt);
    if (lds + 64 > 160 * 1024) return false;
    const void* fn = multi_fn(n, xyz, trace, rt);
    if (!fn) return false;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, lds) != hipSuccess) return false;
    if (per_cu < 1 || (int64_t)gx * gy > (int64_t)cus * per_cu) return false;
    if (sh) *sh = Shape{fn, rt, gx, gy, lds};
    return true;
}

// The launch shape of an instance, or false when none is co-resident.  Two
// row tiles per workgroup when a grid of one-tile workgroups would need more
// than one per CU (the tiles then share one gather of the columns: at 64
// streams x N = 512 with isotropic coupling 18.2 us per RK4 step against
// 24.4), else one (with m^x coupling, 128 one-tile workgroups took 16.8 us
// per step and 64 two-tile ones 18.8); the same for the reverse.
// STO_MULTI_TILES=1 or 2 chooses for measurements.
bool fits(int n, int streams, int xyz, int trace, Shape* sh) {
    if (n < 1 || streams < 1 || n > 32 * kMaxKreg) return false;
    const char* env = getenv("STO_MULTI_TILES");
    const int forced = env ? atoi(env) : 0;
    if (forced == 1 || forced == 2) return fits_rt(n, streams, xyz, trace, forced, sh);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    const int64_t one = (int64_t)((n + kTile - 1) / kTile) * stream_groups(streams, xyz);
    const int first = one > cus ? 2 : 1;
    return fits_rt(n, streams, xyz, trace, first, sh) || fits_rt(n, streams, xyz, trace, 3 - first, sh);
}

hipError_t launch_multi(const DevState<float>& d, const Coef<float>& k, const RunSpec& r, int streams, int sample0,
                        const MultiTrace& tr) {
    // the instance with the phase stamps when a trace was armed for its grid
    Shape sh{};
    if (!fits(d.n, streams, r.xyz, tr.xt != nullptr, &sh)) return hipErrorInvalidValue;
    bool stamp = false;
    if (!tr.xt && r.trace) {
        Shape ph{};
        if (fits(d.n, streams, r.xyz, 3, &ph) && r.trace_groups >= ph.gx * ph.gy) {
            sh = ph;
            stamp = true;
        }
    }
    hipError_t e = hipMemsetAsync(d.sync, 0, 256, r.stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_multi_prologue, dim3(64), dim3(256), 0, r.stream, (const float*)d.m, d.xchg, streams, d.ld,
                       r.xyz ? 3 : 1);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    DevState<float> dd = d;
    Coef<float> kk = k;
    const double* u = r.u;
    float* states = static_cast<float*>(r.states);
    int st = streams, samples = r.samples, substeps = r.substeps, renorm = r.renorm, s0 = sample0;
    MultiTrace t = tr;
    unsigned long long* phase = stamp ? r.trace : nullptr;
    int phase_stages = stamp ? r.trace_stages : 0;
    void* args[] = {&dd, &kk, &u, &states, &st, &samples, &substeps, &renorm, &s0, &t, &phase, &phase_stages};
    e = hipLaunchCooperativeKernel(sh.fn, dim3(sh.gx, sh.gy), dim3(kBlock), args, (unsigned)sh.lds, r.stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace

bool multi_fits(int n, int streams, int xyz, int* grid_x, int* grid_y) {
    Shape sh{};
    if (!fits(n, streams, xyz, 0, &sh)) return false;
    if (grid_x) *grid_x = sh.gx;
    if (grid_y) *grid_y = sh.gy;
    return true;
}

bool multi_segment_fits(int n, int streams, int xyz) { return fits(n, streams, xyz, 1, nullptr); }

bool multi_reverse_fits(int n, int streams, int xyz, int n_in) {
    return n_in >= 1 && n_in <= kRegIn && fits(n, streams, xyz, 2, nullptr);
}

hipError_t run_multi(const DevState<float>& d, const Coef<float>& k, const RunSpec& r, int streams) {
    return launch_multi(d, k, r, streams, 0, MultiTrace{nullptr, nullptr, nullptr});
}

hipError_t run_multi_segment(const DevState<float>& d, const Coef<float>& k, const RunSpec& r, int streams,
                             int sample0, const MultiTrace& tr) {
    return launch_multi(d, k, r, streams, sample0, tr);
}

}  // namespace sto

namespace sto {

hipError_t run_multi_reverse(const AdjDev<float>& d, const Coef<float>& k, int kn, int xyz, float* xchg, int* sync,
                             hipStream_t stream) {
    Shape sh{};
    if (d.n_in < 1 || d.n_in > kRegIn || !fits(d.n, d.S, xyz, 2, &sh)) return hipErrorInvalidValue;
    const int C = xyz ? 3 : 1;
    hipError_t e = hipMemsetAsync(sync, 0, 256, stream);
    if (e != hipSuccess) return e;
    const float* slot = d.st + (xyz ? adj_slot<3>(kn - 1, 3, d.S, d.ld) : adj_slot<1>(kn - 1, 3, d.S, d.ld));
    hipLaunchKernelGGL(k_multi_rev_prologue, dim3(64), dim3(256), 0, stream, slot, xchg, d.S, d.ld, C);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    AdjDev<float> dd = d;
    Coef<float> kk = k;
    float* xb = xchg;
    int* sy = sync;
    int knn = kn;
    void* args[] = {&dd, &kk, &xb, &sy, &knn};
    e = hipLaunchCooperativeKernel(sh.fn, dim3(sh.gx, sh.gy), dim3(kBlock), args, (unsigned)sh.lds, stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace sto
