// RESIDENT path: the whole trajectory in one cooperative launch, with the
// coupling matrix split across the LDS of all co-resident workgroups.
//
// Workgroup g owns a contiguous block of rows of W (paper, Eq. (coup)) and
// keeps it in LDS for the entire run; the state, stage input and RK4
// accumulator of its rows live in registers.  Every RK4 stage needs the
// whole stage input m^x of all nodes (Sec. 3.3: the coupling is W^cp x), so
// the stage inputs are exchanged through global memory every stage.
//
// Exchange without a grid barrier.  The stage inputs live in three rotating
// buffers.  The input of stage s is buffer s % 3.  An entry that has not been
// published yet holds a sentinel bit pattern (all ones: a NaN with a payload
// that IEEE arithmetic never generates, and the library rejects non-finite
// inputs).  A workgroup
//   1. polls every entry of buffer s % 3 until none is the sentinel, copying
//      the values into LDS (this is the only wait: data and synchronisation
//      arrive in the same load);
//   2. re-arms its rows of buffer (s + 2) % 3 with the sentinel (every
//      workgroup finished reading that buffer, the input of stage s - 1,
//      before it published its stage s - 1 output, all of which step 1 has
//      seen);
//   3. computes its rows of stage s while those stores complete;
//   4. waits for the re-arm stores to complete, and only then publishes its
//      rows of buffer (s + 1) % 3.
// All exchange loads and stores are agent-scope atomics, which on gfx950 are
// coherent across the XCDs without an L2 writeback: the ordering of step 2
// before step 4 is the store-completion wait of the publishing wave, and a
// reader that sees a published value issues its later loads after it.
// Agent-scope release fences per workgroup (L2 writebacks) cost ~70 ns each
// and serialise, so a counter barrier over 256 workgroups costs 20-35 us;
// this exchange costs about one memory round trip.  With STAGGER, step 1
// keeps two polls of every entry in flight, the second issued part of a
// round trip after the first, so a value published between two polls is
// seen sooner.
//
// Every wait is bounded: after a spin limit a workgroup raises a sticky
// abort flag, and every workgroup that sees it leaves the kernel, so a grid
// that is not co-resident ends with an error instead of a hang.  The
// cooperative launch itself refuses grids that cannot be co-resident.
//
// Launch shape: BLOCK threads (4, 8 or 16 waves) and rows_per_block rows of
// W per workgroup, at most 4 rows per wave (1 with 16 waves).  The default
// is 4 waves and ceil(n / CUs) rows.  With SPLIT = 2 or 4 that many waves share each row,
// each summing its share of the columns; their wave totals meet in LDS, which
// shortens the dependent chain of a row's sum at the cost of one barrier per
// row.  With a trace buffer, wave 0 of every workgroup stamps the device's
// constant-rate clock at four points of each of the first trace_stages
// stages (stage start, gather done, own rows computed, own rows published),
// for the phase breakdown of the exchange.

#include <algorithm>
#include <climits>

#include "path_tune.hpp"
#include "sto_adjoint_dev.hpp"
#include "sto_internal.hpp"
#include "sto_resident.hpp"

namespace sto {

namespace {

// rows per wave: up to 4 with 4 or 8 waves; one with 16 waves, whose
// register budget (128 per lane) holds one row's state without spilling
constexpr int max_rows_per_wave(int block) { return block >= 1024 ? 1 : 4; }
constexpr int kSpinLimit = 1 << 20;      // poll rounds (one memory round trip each)
constexpr int kStaggerUnrolled = 6;      // staggered poll pairs issued as straight-line code
constexpr int kPollStaggerF64 = 4;       // sleep units between the two polls (measured)
constexpr int kPollStaggerF32 = 4;
constexpr size_t kLdsMax = 160 * 1024;

template <typename T> struct Bits;
template <> struct Bits<double> { using type = unsigned long long; };
template <> struct Bits<float> { using type = unsigned int; };

template <typename T>
__device__ __forceinline__ typename Bits<T>::type sentinel() {
    return ~typename Bits<T>::type(0);
}

template <typename T>
__device__ __forceinline__ void publish(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void rearm(T* p) {
    using B = typename Bits<T>::type;
    __hip_atomic_store(reinterpret_cast<B*>(p), sentinel<T>(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Staggered polling of up to K entries per thread (entries i0 + q * BLOCK +
// thread): two loads of each entry are kept in flight, the second issued
// `stagger` sleep units (64 clocks each) after the first, so a published
// entry is seen after part of a round trip instead of after a whole one.
// Out-of-range entries load the last valid one and are ignored.
template <typename T, int BLOCK, int K>
__device__ bool gather_staggered(const typename Bits<T>::type* s, T* dst, int i0, int n, int* abort_flag,
                                 int stagger) {
    using B = typename Bits<T>::type;
    B a[K], b[K];
    bool got[K];
    int idx[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int i = i0 + q * BLOCK + (int)threadIdx.x;
        got[q] = i >= n;
        idx[q] = min(i, n - 1);
    }
    // take the entries a poll returned; true while some are still pending
    auto absorb = [&](const B (&v)[K]) {
        bool pending = false;
#pragma unroll
        for (int q = 0; q < K; ++q)
            if (!got[q]) {
                if (v[q] == sentinel<T>()) pending = true;
                else {
                    dst[idx[q]] = __builtin_bit_cast(T, v[q]);
                    got[q] = true;
                }
            }
        return pending;
    };
    // every lane issues every poll and the loop exits wave-uniformly, so
    // the compiler can keep the other poll in flight while one is checked
#pragma unroll
    for (int q = 0; q < K; ++q) a[q] = __hip_atomic_load(s + idx[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int k = 0; k < stagger; ++k) __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (int q = 0; q < K; ++q) b[q] = __hip_atomic_load(s + idx[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the first polls unrolled: straight-line code lets the compiler wait
    // for exactly the poll it checks (in a loop it waits for both)
#pragma unroll
    for (int r = 0; r < kStaggerUnrolled; ++r) {
        if (!__any(absorb(a))) return true;
#pragma unroll
        for (int q = 0; q < K; ++q) a[q] = __hip_atomic_load(s + idx[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!__any(absorb(b))) return true;
#pragma unroll
        for (int q = 0; q < K; ++q) b[q] = __hip_atomic_load(s + idx[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int rounds = 1;; ++rounds) {
        if (!__any(absorb(a))) return true;
#pragma unroll
        for (int q = 0; q < K; ++q) a[q] = __hip_atomic_load(s + idx[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!__any(absorb(b))) return true;
#pragma unroll
        for (int q = 0; q < K; ++q) b[q] = __hip_atomic_load(s + idx[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((rounds & 127) == 0) {
            if (rounds > kSpinLimit / 2) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        }
    }
}

// Wait until the n entries of src are published and copy them to LDS.
// Returns false if the wait was abandoned (spin limit or abort flag).
// STAGGER: two polls of every entry in flight (above) when n <= 2 * BLOCK
// and stagger > 0.
template <typename T, int BLOCK, bool STAGGER>
__device__ bool gather_stage_input(const T* src, T* dst, int n, int* abort_flag, int stagger) {
    using B = typename Bits<T>::type;
    const B* s = reinterpret_cast<const B*>(src);
    bool ok = true;
    if constexpr (STAGGER) {
        if (stagger > 0 && n <= 2 * BLOCK) {
            if (n <= BLOCK) return gather_staggered<T, BLOCK, 1>(s, dst, 0, n, abort_flag, stagger);
            return gather_staggered<T, BLOCK, 2>(s, dst, 0, n, abort_flag, stagger);
        }
    }
    for (int i0 = 0; i0 < n; i0 += 4 * BLOCK) {
        B v[4];
        bool pending = true;
        int rounds = 0;
        while (pending) {
            pending = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + q * BLOCK + threadIdx.x;
                v[q] = i < n ? __hip_atomic_load(s + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : B(0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + q * BLOCK + threadIdx.x;
                if (i < n) {
                    if (v[q] == sentinel<T>()) pending = true;
                    else dst[i] = __builtin_bit_cast(T, v[q]);
                }
            }
            if (pending && (++rounds & 255) == 0) {
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
        if (!ok) break;
    }
    return ok;
}

__device__ __forceinline__ void stamp(unsigned long long* trace, int trace_stages, int sigma, int point) {
    if (trace && sigma < trace_stages && threadIdx.x == 0)
        trace[((size_t)blockIdx.x * trace_stages + sigma) * 4 + point] = wall_clock64();
}

// TRACE: the adjoint's recompute of one segment; every stage also writes
// its input (xt), its raw coupling sums before a_cp (wx) and, at the last
// stage of a step, the norm before the projection (pn), in the layout of
// the adjoint's workspace ([step][stage][component][ld]; pn [step][ld]).
template <typename T, bool XYZ, int BLOCK, bool TRACE, int SPLIT, bool STAGGER = false>
__global__ void __launch_bounds__(BLOCK) k_resident(DevState<T> d, Coef<T> k, const double* __restrict__ u,
                                                    T* __restrict__ states, int samples, int substeps,
                                                    int cur, int renorm, int rows_per_block, int wld,
                                                    unsigned long long* trace, int trace_stages,
                                                    ResTrace<T> tr, int sample0, int stagger) {
    constexpr int kBlock = BLOCK;
    constexpr int kWaves = BLOCK / 64;
    constexpr int kMaxRowsPerWave = max_rows_per_wave(BLOCK);
    using A = Acc<T>;
    using AT = typename A::type;
    constexpr int C = XYZ ? 3 : 1;                           // exchanged components
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int ok_lds;
    const int n = d.n;
    const int64_t ld = d.ld;
    T* wsh = reinterpret_cast<T*>(smem_raw);                    // rows_per_block x wld
    T* xs = wsh + (int64_t)rows_per_block * wld;                // [C][n] stage input
    const int row_begin = blockIdx.x * rows_per_block;
    const int nrows = max(0, min(rows_per_block, n - row_begin));
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // SPLIT waves share each row: wave grp + p * kGroups sums the p-th share
    // of the columns; part 0 re-arms, publishes and records
    constexpr int kGroups = kWaves / SPLIT;
    const int grp = wave % kGroups;
    const int part = wave / kGroups;
    T* xbuf = d.xchg;                                           // [3][C][ld]
    int* abort_flag = d.sync + kSyncAbortWord;
    if (threadIdx.x == 0) ok_lds = 1;

    for (int i = threadIdx.x; i < nrows * n; i += kBlock) {
        const int r = i / n;
        const int c = i - r * n;
        wsh[(int64_t)r * wld + c] = d.W[(int64_t)(row_begin + r) * ld + c];
    }

    // Registers of the rows this wave owns (rows wave, wave + 4, ...); every
    // lane keeps a copy, lane 0 publishes.
    T mx[kMaxRowsPerWave], my[kMaxRowsPerWave], mz[kMaxRowsPerWave];
    T ax[kMaxRowsPerWave], ay[kMaxRowsPerWave], az[kMaxRowsPerWave];
    T sx[kMaxRowsPerWave], sy[kMaxRowsPerWave], sz[kMaxRowsPerWave];
    T hin[kMaxRowsPerWave];
#pragma unroll
    for (int q = 0; q < kMaxRowsPerWave; ++q) {
        const int r = grp + q * kGroups;
        const int rr = min(row_begin + min(r, max(nrows - 1, 0)), n - 1);
        mx[q] = sx[q] = d.m[rr];
        my[q] = sy[q] = d.m[ld + rr];
        mz[q] = sz[q] = d.m[2 * ld + rr];
        ax[q] = ay[q] = az[q] = T(0);
        hin[q] = T(0);
    }

    int sigma = 0;   // stage counter: the input of stage sigma is xbuf[sigma % 3]
    for (int s = 0; s < samples; ++s) {
#pragma unroll
        for (int q = 0; q < kMaxRowsPerWave; ++q) {
            const int r = grp + q * kGroups;
            if (r < nrows)
                hin[q] = input_field(k, d.w_in + (int64_t)(row_begin + r) * d.n_in, u + (int64_t)s * d.n_in, d.n_in);
        }
        for (int sub = 0; sub < substeps; ++sub) {
            for (int stage = 0; stage < 4; ++stage, ++sigma) {
                T* xin = xbuf + (int64_t)(sigma % 3) * C * ld;
                T* xout = xbuf + (int64_t)((sigma + 1) % 3) * C * ld;
                T* xold = xbuf + (int64_t)((sigma + 2) % 3) * C * ld;
                __syncthreads();   // every wave is done with xs of the previous stage
                stamp(trace, trace_stages, sigma, 0);
                bool ok = true;
#pragma unroll
                for (int c = 0; c < C; ++c)
                    ok = ok && gather_stage_input<T, BLOCK, STAGGER>(xin + c * ld, xs + c * n, n, abort_flag, stagger);
                if (!ok) ok_lds = 0;
                __syncthreads();
                if (ok_lds == 0) return;
                stamp(trace, trace_stages, sigma, 1);
                // step 3 early: re-arm this wave's rows of the buffer two
                // stages ahead as soon as the gather is done (every workgroup
                // finished reading it: the gather saw all outputs of the
                // previous stage), so the stores complete during the compute
                if (lane == 0 && part == 0) {
#pragma unroll
                    for (int q = 0; q < kMaxRowsPerWave; ++q) {
                        const int r = grp + q * kGroups;
                        if (r >= nrows) break;
                        const int row = row_begin + r;
                        rearm(xold + row);
                        if (XYZ) {
                            rearm(xold + ld + row);
                            rearm(xold + 2 * ld + row);
                        }
                    }
                }
                // right-hand side, RK4 update and (stage 3) projection of row q
                // from its coupling sums
                auto finish_row = [&](int q, int r, int64_t kk, T cx, T cy, T cz) {
                    T fx, fy, fz;
                    llg_rhs<T, XYZ>(k, sx[q], sy[q], sz[q], cx, cy, cz, hin[q], fx, fy, fz);
                    T nx = rk4_update(k, stage, mx[q], ax[q], fx);
                    T ny = rk4_update(k, stage, my[q], ay[q], fy);
                    T nz = rk4_update(k, stage, mz[q], az[q], fz);
                    if (stage == 3) {
                        if (TRACE && renorm && lane == 0 && part == 0) {
                            const double ex = nx, ey = ny, ez = nz;
                            tr.pn[kk * ld + row_begin + r] = (T)__builtin_sqrt((ex * ex + ey * ey) + ez * ez);
                        }
                        if (renorm) renormalize(nx, ny, nz);
                        mx[q] = nx;
                        my[q] = ny;
                        mz[q] = nz;
                    }
                    sx[q] = nx;
                    sy[q] = ny;
                    sz[q] = nz;
                };
                if constexpr (SPLIT > 1) {
                    // each wave sums its share of the columns (pairs 64 lanes
                    // apart, two chains per lane) and reduces it over the
                    // wave; the shares meet in LDS and every wave of the row
                    // finishes it (part 0's results are the ones kept)
                    __shared__ AT psum[SPLIT][kGroups][kMaxRowsPerWave][C];
                    const int qn = (nrows + kGroups - 1) / kGroups;   // block-uniform
#pragma unroll
                    for (int q = 0; q < kMaxRowsPerWave; ++q) {
                        if (q >= qn) break;   // every wave reaches the barrier below
                        const int r = grp + q * kGroups;
                        const bool has = r < nrows;   // wave-uniform
                        const int64_t kk = (int64_t)s * substeps + sub;
                        if (has) {
                            if (TRACE && lane == 0 && part == 0) {
                                T* x = tr.xt + (kk * 4 + stage) * 3 * ld;
                                x[row_begin + r] = sx[q];
                                x[ld + row_begin + r] = sy[q];
                                x[2 * ld + row_begin + r] = sz[q];
                            }
                            const T* wr = wsh + (int64_t)r * wld;
                            AT vx = A::zero(), vy = A::zero(), vz = A::zero();
                            AT ux = A::zero(), uy = A::zero(), uz = A::zero();
                            int j = lane + 64 * part;
                            for (; j + 64 * SPLIT < n; j += 128 * SPLIT) {
                                const T w0 = wr[j], w1 = wr[j + 64 * SPLIT];
                                A::fma(vx, w0, xs[j]);
                                A::fma(ux, w1, xs[j + 64 * SPLIT]);
                                if (XYZ) {
                                    A::fma(vy, w0, xs[n + j]);
                                    A::fma(uy, w1, xs[n + j + 64 * SPLIT]);
                                    A::fma(vz, w0, xs[2 * n + j]);
                                    A::fma(uz, w1, xs[2 * n + j + 64 * SPLIT]);
                                }
                            }
                            if (j < n) {
                                const T w0 = wr[j];
                                A::fma(vx, w0, xs[j]);
                                if (XYZ) {
                                    A::fma(vy, w0, xs[n + j]);
                                    A::fma(vz, w0, xs[2 * n + j]);
                                }
                            }
                            vx = group_reduce<T>(A::add(vx, ux), 64);
                            if (XYZ) {
                                vy = group_reduce<T>(A::add(vy, uy), 64);
                                vz = group_reduce<T>(A::add(vz, uz), 64);
                            }
                            if (lane == 0) {
                                psum[part][grp][q][0] = vx;
                                if (XYZ) {
                                    psum[part][grp][q][C - 2] = vy;
                                    psum[part][grp][q][C - 1] = vz;
                                }
                            }
                        }
                        __syncthreads();
                        if (has) {
                            AT tx = psum[0][grp][q][0], ty = A::zero(), tz = A::zero();
#pragma unroll
                            for (int p = 1; p < SPLIT; ++p) tx = A::add(tx, psum[p][grp][q][0]);
                            if (XYZ) {
                                ty = psum[0][grp][q][C - 2];
                                tz = psum[0][grp][q][C - 1];
#pragma unroll
                                for (int p = 1; p < SPLIT; ++p) {
                                    ty = A::add(ty, psum[p][grp][q][C - 2]);
                                    tz = A::add(tz, psum[p][grp][q][C - 1]);
                                }
                            }
                            const T cx = k.a_cp * A::round(tx);
                            const T cy = XYZ ? k.a_cp * A::round(ty) : T(0);
                            const T cz = XYZ ? k.a_cp * A::round(tz) : T(0);
                            if (TRACE && lane == 0 && part == 0) {
                                T* w = tr.wx + (kk * 4 + stage) * C * ld;
                                w[row_begin + r] = A::round(tx);
                                if (XYZ) {
                                    w[ld + row_begin + r] = A::round(ty);
                                    w[2 * ld + row_begin + r] = A::round(tz);
                                }
                            }
                            finish_row(q, r, kk, cx, cy, cz);
                        }
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < kMaxRowsPerWave; ++q) {
                        const int r = grp + q * kGroups;
                        if (r >= nrows) break;   // wave-uniform
                        const T* wr = wsh + (int64_t)r * wld;
                        const int64_t kk = (int64_t)s * substeps + sub;   // step of this launch
                        if (TRACE && lane == 0) {
                            T* x = tr.xt + (kk * 4 + stage) * 3 * ld;
                            x[row_begin + r] = sx[q];
                            x[ld + row_begin + r] = sy[q];
                            x[2 * ld + row_begin + r] = sz[q];
                        }
                        // two independent accumulation chains per lane (columns
                        // j and j + 64 of each 128), joined before the butterfly
                        // (measured: four chains are slower)
                        AT vx = A::zero(), vy = A::zero(), vz = A::zero();
                        AT ux = A::zero(), uy = A::zero(), uz = A::zero();
                        int j = lane;
                        for (; j + 64 < n; j += 128) {
                            const T w0 = wr[j], w1 = wr[j + 64];
                            A::fma(vx, w0, xs[j]);
                            A::fma(ux, w1, xs[j + 64]);
                            if (XYZ) {
                                A::fma(vy, w0, xs[n + j]);
                                A::fma(uy, w1, xs[n + j + 64]);
                                A::fma(vz, w0, xs[2 * n + j]);
                                A::fma(uz, w1, xs[2 * n + j + 64]);
                            }
                        }
                        if (j < n) {
                            const T w0 = wr[j];
                            A::fma(vx, w0, xs[j]);
                            if (XYZ) {
                                A::fma(vy, w0, xs[n + j]);
                                A::fma(vz, w0, xs[2 * n + j]);
                            }
                        }
                        vx = A::add(vx, ux);
                        if (XYZ) {
                            vy = A::add(vy, uy);
                            vz = A::add(vz, uz);
                        }
                        vx = group_reduce<T>(vx, 64);
                        T cx = k.a_cp * A::round(vx), cy = T(0), cz = T(0);
                        if (XYZ) {
                            vy = group_reduce<T>(vy, 64);
                            vz = group_reduce<T>(vz, 64);
                            cy = k.a_cp * A::round(vy);
                            cz = k.a_cp * A::round(vz);
                        }
                        if (TRACE && lane == 0) {
                            T* w = tr.wx + (kk * 4 + stage) * C * ld;
                            w[row_begin + r] = A::round(vx);
                            if (XYZ) {
                                w[ld + row_begin + r] = A::round(vy);
                                w[2 * ld + row_begin + r] = A::round(vz);
                            }
                        }
                        finish_row(q, r, kk, cx, cy, cz);
                    }
                }
                stamp(trace, trace_stages, sigma, 2);
                // step 4: publish this wave's rows once the re-arm stores have
                // completed (one wait for all rows; the clobber keeps the
                // compiler from moving the stores across it)
                if (lane == 0 && part == 0) {
                    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
                    for (int q = 0; q < kMaxRowsPerWave; ++q) {
                        const int r = grp + q * kGroups;
                        if (r >= nrows) break;
                        const int row = row_begin + r;
                        publish(xout + row, sx[q]);
                        if (XYZ) {
                            publish(xout + ld + row, sy[q]);
                            publish(xout + 2 * ld + row, sz[q]);
                        }
                    }
                }
                stamp(trace, trace_stages, sigma, 3);
            }
        }
        if (lane == 0 && part == 0) {
#pragma unroll
            for (int q = 0; q < kMaxRowsPerWave; ++q) {
                const int r = grp + q * kGroups;
                if (r >= nrows) break;
                const int row = row_begin + r;
                if (states) {
                    T* rec = states + ((int64_t)s * n + row) * 3;
                    rec[0] = mx[q];
                    rec[1] = my[q];
                    rec[2] = mz[q];
                }
                if (!finite3(mx[q], my[q], mz[q])) atomicMin(d.bad, sample0 + s);
            }
        }
    }
    if (lane == 0 && part == 0) {
        T* xc = d.ms[cur];
#pragma unroll
        for (int q = 0; q < kMaxRowsPerWave; ++q) {
            const int r = grp + q * kGroups;
            if (r >= nrows) break;
            const int row = row_begin + r;
            d.m[row] = xc[row] = mx[q];
            d.m[ld + row] = xc[ld + row] = my[q];
            d.m[2 * ld + row] = xc[2 * ld + row] = mz[q];
        }
    }
}

// Clears count words (a fill kernel rather than a memset node).
__global__ void k_zero_words(int* p, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}

__global__ void k_resident_prologue(const void* ms_cur, void* xchg, int64_t elems_per_buffer, int elem,
                                    int64_t copy_elems) {
    // buffer 0 <- current stage input (the state); buffers 1 and 2 <- sentinel
    const int64_t total = 3 * elems_per_buffer;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (elem == 8) {
            unsigned long long* x = static_cast<unsigned long long*>(xchg);
            x[i] = i < copy_elems ? static_cast<const unsigned long long*>(ms_cur)[i] : ~0ull;
        } else {
            unsigned int* x = static_cast<unsigned int*>(xchg);
            x[i] = i < copy_elems ? static_cast<const unsigned int*>(ms_cur)[i] : ~0u;
        }
    }
}

// Parameter partials of one node over a reversed segment, in registers
// (FP64), added to the per-node sums once at the end; captures the next
// stage's coupling adjoint for the exchange.
constexpr int kRevIn = 4;   // input channels summed in registers

template <typename T>
struct ResSink {
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    double w[kRevIn] = {0.0, 0.0, 0.0, 0.0};
    T b[3] = {T(0), T(0), T(0)};
    __device__ __forceinline__ void add(const AdjDev<T>& d, int64_t, double pcp, double pin, double phs, double pap,
                                        double ab, const double* u_s, T bx, T by, T bz) {
        g[0] += pcp;
        g[1] += pin;
        g[2] += phs;
        g[3] += pap;
#pragma unroll
        for (int q = 0; q < kRevIn; ++q)
            if (q < d.n_in) w[q] += ab * u_s[q];
        b[0] = bx;
        b[1] = by;
        b[2] = bz;
    }
    __device__ __forceinline__ void flush(const AdjDev<T>& d, int64_t gi) {
        const int64_t gs = d.ld;
#pragma unroll
        for (int c = 0; c < 4; ++c) d.gacc[c * gs + gi] += g[c];
#pragma unroll
        for (int q = 0; q < kRevIn; ++q)
            if (q < d.n_in) d.gwin[q * gs + gi] += w[q];
    }
};

// The reversed stages of one adjoint segment of a single stream in one
// cooperative launch.  Workgroup g keeps its rows of W^T in LDS; per stage
// every workgroup gathers the stage's coupling adjoint bbar of all nodes
// through the rotating sentinel buffers (the exchange of k_resident), each
// wave forms t = W^T bbar for its rows (plain fma, two chains per lane, a
// butterfly sum), and lane q of the wave runs the adjoint epilogue of its
// row q (rev_load / rev_finish, as the per-stage kernel k_adj_stage runs
// it).  The epilogue's inputs are loaded before the gather; its parameter
// partials stay in registers until the end of the segment; the next stage's
// bbar it computes is published.  Buffer 0 starts with the bbar of
// (kn - 1, 3).
template <typename T, bool XYZ, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_resident_rev(AdjDev<T> d, Coef<T> k, T* __restrict__ xbuf, int* sync,
                                                        int kn, int rows_per_block, int wld) {
    constexpr int kWaves = BLOCK / 64;
    constexpr int kMaxRowsPerWave = max_rows_per_wave(BLOCK);
    constexpr int C = XYZ ? 3 : 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int ok_lds;
    const int n = d.n;
    const int64_t ld = d.ld;
    T* wsh = reinterpret_cast<T*>(smem_raw);                    // rows_per_block x wld: rows of W^T
    T* xs = wsh + (int64_t)rows_per_block * wld;                // [C][n] coupling adjoint
    const int row_begin = blockIdx.x * rows_per_block;
    const int nrows = max(0, min(rows_per_block, n - row_begin));
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int* abort_flag = sync + kSyncAbortWord;
    if (threadIdx.x == 0) ok_lds = 1;
    for (int i = threadIdx.x; i < nrows * n; i += BLOCK) {
        const int r = i / n;
        const int c = i - r * n;
        wsh[(int64_t)r * wld + c] = d.Wt[(int64_t)(row_begin + r) * ld + c];
    }
    // lane q < kMaxRowsPerWave owns the epilogue of the wave's row q
    const int myr = wave + lane * kWaves;
    const bool mine = lane < kMaxRowsPerWave && myr < nrows;
    const int node = row_begin + myr;
    ResSink<T> sink;

    int sigma = 0;
    for (int kk = kn - 1; kk >= 0; --kk) {
        for (int stage = 3; stage >= 0; --stage, ++sigma) {
            const T* xin = xbuf + (int64_t)(sigma % 3) * C * ld;
            T* xout = xbuf + (int64_t)((sigma + 1) % 3) * C * ld;
            T* xold = xbuf + (int64_t)((sigma + 2) % 3) * C * ld;
            RevIn<T> in{};
            if (mine) in = rev_load<T, XYZ>(d, node, 0, kk, stage);
            __syncthreads();
            bool ok = true;
#pragma unroll
            for (int c = 0; c < C; ++c)
                ok = ok && gather_stage_input<T, BLOCK, false>(xin + c * ld, xs + c * n, n, abort_flag, 0);
            if (!ok) ok_lds = 0;
            __syncthreads();
            if (ok_lds == 0) return;
            if (mine) {
#pragma unroll
                for (int c = 0; c < C; ++c) rearm(xold + c * ld + node);
            }
            T t[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int q = 0; q < kMaxRowsPerWave; ++q) {
                const int r = wave + q * kWaves;
                if (r >= nrows) break;   // wave-uniform
                const T* wr = wsh + (int64_t)r * wld;
                T vx = T(0), vy = T(0), vz = T(0), ux = T(0), uy = T(0), uz = T(0);
                int j = lane;
                for (; j + 64 < n; j += 128) {
                    const T w0 = wr[j], w1 = wr[j + 64];
                    vx = __builtin_fma(w0, xs[j], vx);
                    ux = __builtin_fma(w1, xs[j + 64], ux);
                    if (XYZ) {
                        vy = __builtin_fma(w0, xs[n + j], vy);
                        uy = __builtin_fma(w1, xs[n + j + 64], uy);
                        vz = __builtin_fma(w0, xs[2 * n + j], vz);
                        uz = __builtin_fma(w1, xs[2 * n + j + 64], uz);
                    }
                }
                if (j < n) {
                    const T w0 = wr[j];
                    vx = __builtin_fma(w0, xs[j], vx);
                    if (XYZ) {
                        vy = __builtin_fma(w0, xs[n + j], vy);
                        vz = __builtin_fma(w0, xs[2 * n + j], vz);
                    }
                }
                vx = lane_sum<T>(vx + ux);
                if (XYZ) {
                    vy = lane_sum<T>(vy + uy);
                    vz = lane_sum<T>(vz + uz);
                }
                if (lane == q) {
                    t[0] = vx;
                    t[1] = vy;
                    t[2] = vz;
                }
            }
            // the re-arm stores must complete before the publish below; the
            // epilogue's own stores need not
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (mine) {
                rev_finish<T, XYZ>(d, k, node, 0, kk, stage, in, t[0], t[1], t[2], sink);
                if (kk > 0 || stage > 0) {
#pragma unroll
                    for (int c = 0; c < C; ++c) publish(xout + c * ld + node, sink.b[c]);
                }
            }
        }
    }
    if (mine) sink.flush(d, node);
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

int64_t wld_of(int n) { return (n + 3) / 4 * 4; }

size_t resident_lds(int n, int rows_per_block, int elem, int xyz) {
    return ((size_t)rows_per_block * wld_of(n) + (xyz ? 3 : 1) * (size_t)n) * elem;
}

// variant 0: plain run; 1: the adjoint's traced recompute; 2: its reverse;
// 3, 4: plain and traced with two waves per row; 5, 6: with four (8 or 16
// waves only); 7-10: 3-6 with staggered polls (16 waves only)
template <typename T, bool XYZ, int BLOCK>
const void* resident_fn_v(int variant) {
    if (variant == 1) return reinterpret_cast<const void*>(&k_resident<T, XYZ, BLOCK, true, 1>);
    if (variant == 2) {
        // the reverse never runs with 16 waves (reverse_block)
        if constexpr (BLOCK <= 512) return reinterpret_cast<const void*>(&k_resident_rev<T, XYZ, BLOCK>);
        return nullptr;
    }
    if (variant == 3) return reinterpret_cast<const void*>(&k_resident<T, XYZ, BLOCK, false, 2>);
    if (variant == 4) return reinterpret_cast<const void*>(&k_resident<T, XYZ, BLOCK, true, 2>);
    if constexpr (BLOCK >= 512) {
        if (variant == 5) return reinterpret_cast<const void*>(&k_resident<T, XYZ, BLOCK, false, 4>);
        if (variant == 6) return reinterpret_cast<const void*>(&k_resident<T, XYZ, BLOCK, true, 4>);
    }
    if constexpr (BLOCK == 1024) {
        if (variant == 7) return reinterpret_cast<const void*>(&k_resident<T, XYZ, BLOCK, false, 2, true>);
        if (variant == 8) return reinterpret_cast<const void*>(&k_resident<T, XYZ, BLOCK, true, 2, true>);
        if (variant == 9) return reinterpret_cast<const void*>(&k_resident<T, XYZ, BLOCK, false, 4, true>);
        if (variant == 10) return reinterpret_cast<const void*>(&k_resident<T, XYZ, BLOCK, true, 4, true>);
    }
    if (variant >= 5) return nullptr;
    return reinterpret_cast<const void*>(&k_resident<T, XYZ, BLOCK, false, 1>);
}

// the forward variant for waves per row `split`, plain or traced, with
// staggered polls (7-10: 16 waves, two or four waves per row only)
int split_variant(int split, bool traced, bool staggered = false) {
    if (staggered && split == 4) return traced ? 10 : 9;
    if (staggered && split == 2) return traced ? 8 : 7;
    if (split == 4) return traced ? 6 : 5;
    if (split == 2) return traced ? 4 : 3;
    return traced ? 1 : 0;
}

template <typename T, bool XYZ>
const void* resident_fn(int block, int variant) {
    switch (block) {
        case 256: return resident_fn_v<T, XYZ, 256>(variant);
        case 512: return resident_fn_v<T, XYZ, 512>(variant);
        case 1024: return resident_fn_v<T, XYZ, 1024>(variant);
        default: return nullptr;
    }
}

const void* resident_kernel(int elem, int xyz, int block, int variant = 0) {
    if (elem == 8) return xyz ? resident_fn<double, true>(block, variant) : resident_fn<double, false>(block, variant);
    return xyz ? resident_fn<float, true>(block, variant) : resident_fn<float, false>(block, variant);
}

// Whether the kernel variant runs a grid of `grid` workgroups of `block`
// threads with `lds` bytes co-resident on the CUs.
bool co_resident(const void* fn, int block, size_t lds, int grid, int cus) {
    if (!fn) return false;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return false;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess) return false;
    return (int64_t)per_cu * cus >= grid;
}

int env_int(const char* name) {
    const char* v = getenv(name);
    return v && *v ? atoi(v) : 0;
}

// Sleep units (64 clocks) between the two polls of the gather kept in
// flight, for the shapes that have a staggered instance (16 waves, two or
// four waves per row); 0 polls one load at a time.  The adjoint's reverse
// keeps single polls (staggered ones measured no faster there: 117.8
// against 118.0 ms for the sto1k FP64 adjoint).  Measured at N = 1,000
// (us per RK4 step): FP64 13.1 -> 11.9, FP32 9.9 -> 8.6, within 1 % for 3
// to 5 units.  STO_POLL_STAGGER overrides it (0 turns it off).
int poll_stagger(int elem_bytes) {
    const char* v = getenv("STO_POLL_STAGGER");
    if (v && *v) return std::min(std::max(atoi(v), 0), 64);
    return elem_bytes == 8 ? kPollStaggerF64 : kPollStaggerF32;
}

// Whether (waves, rpb, split) runs n nodes: rows per wave, LDS,
// co-residency.  split = 2 runs each row on two waves (half the columns
// each), so a workgroup holds half as many rows per wave.
bool shape_fits(int n, int elem_bytes, int xyz, int waves, int rpb, int split, int cus, int* grid_out) {
    const int block = 64 * waves;
    if (split != 1 && split != 2 && split != 4) return false;
    if (split > waves) return false;
    if (rpb < 1 || rpb > waves / split * max_rows_per_wave(block)) return false;
    const size_t lds = resident_lds(n, rpb, elem_bytes, xyz);
    if (lds + 64 + (split > 1 ? 2048 : 0) > kLdsMax) return false;   // the split's static LDS
    const int grid = (n + rpb - 1) / rpb;
    if (!co_resident(resident_kernel(elem_bytes, xyz, block, split_variant(split, false)), block, lds, grid, cus))
        return false;
    *grid_out = grid;
    return true;
}

}  // namespace

int tuned_path(int elem_bytes, int xyz, int n, int* waves, int* rpb, int* split) {
    for (const PathTuneEntry& e : kPathTune)
        if (e.elem_bytes == elem_bytes && e.xyz == (xyz ? 1 : 0) && n <= e.n_max) {
            if (waves) *waves = e.waves;
            if (rpb) *rpb = e.rpb;
            if (split) *split = e.split;
            return e.path;
        }
    return 0;
}

// Launch shape of the resident kernel for n: rows per workgroup, threads per
// workgroup and grid.  The measured shape of the path table for n when it
// fits, else 4 waves and ceil(n / CUs) rows (at most one workgroup per CU).
// STO_RESIDENT_RPB (rows per workgroup) and STO_RESIDENT_WAVES (4, 8 or 16)
// override both for measurements.  False if no shape fits (LDS, rows per
// wave) or its workgroups cannot all be co-resident.
bool resident_shape(int n, int elem_bytes, int xyz, int* grid_out, int* rpb_out, int* block_out, int* split_out) {
    const int cus = device_cus();
    if (cus <= 0 || n < 2) return false;
    const int env_waves = env_int("STO_RESIDENT_WAVES"), env_rpb = env_int("STO_RESIDENT_RPB");
    // a caller that cannot run the two-waves-per-row kernel (the adjoint's
    // traced and reversed kernels) passes no split_out and gets a shape of
    // one wave per row
    const bool allow_split = split_out != nullptr;
    const int env_split = allow_split ? env_int("STO_RESIDENT_SPLIT") : 0;
    const int def_rpb = (n + cus - 1) / cus;
    int cand[2][3];
    int nc = 0;
    if (env_waves > 0 || env_rpb > 0 || env_split > 0) {
        const int w = (env_waves == 8 || env_waves == 16) ? env_waves : 4;
        cand[nc][0] = w;
        cand[nc][1] = env_rpb > 0 ? env_rpb : def_rpb;
        cand[nc++][2] = (env_split == 2 || env_split == 4) ? env_split : 1;
    } else {
        int tw = 0, tr = 0, ts = 1;
        if (tuned_path(elem_bytes, xyz, n, &tw, &tr, &ts) == 2 && (tw == 4 || tw == 8 || tw == 16) &&
            (ts == 1 || allow_split)) {
            cand[nc][0] = tw;
            cand[nc][1] = tr > 0 ? tr : def_rpb;
            cand[nc++][2] = (ts == 2 || ts == 4) ? ts : 1;
        }
        cand[nc][0] = 4;
        cand[nc][1] = def_rpb;
        cand[nc++][2] = 1;
    }
    for (int c = 0; c < nc; ++c) {
        int grid = 0;
        if (shape_fits(n, elem_bytes, xyz, cand[c][0], cand[c][1], cand[c][2], cus, &grid)) {
            if (grid_out) *grid_out = grid;
            if (rpb_out) *rpb_out = cand[c][1];
            if (block_out) *block_out = 64 * cand[c][0];
            if (split_out) *split_out = cand[c][2];
            return true;
        }
    }
    return false;
}

bool resident_fits(int n, int elem_bytes, int xyz, int* grid_out) {
    int split = 1;   // the shape a run takes
    return resident_shape(n, elem_bytes, xyz, grid_out, nullptr, nullptr, &split);
}

template <typename T>
hipError_t run_resident(const DevState<T>& d, const Coef<T>& k, const RunSpec& r) {
    int grid = 0, rpb = 0, block = 0, split = 1;
    if (!resident_shape(d.n, sizeof(T), r.xyz, &grid, &rpb, &block, &split)) return hipErrorInvalidValue;
    int wld = (int)wld_of(d.n);
    const size_t lds = resident_lds(d.n, rpb, sizeof(T), r.xyz);
    const int C = r.xyz ? 3 : 1;
    hipError_t e = hipMemsetAsync(d.sync, 0, 256, r.stream);
    if (e != hipSuccess) return e;
    // the exchange buffers hold C components of ld entries each; the x, y, z
    // components of ms[cur] are contiguous blocks of ld, so the first C*ld
    // entries of ms[cur] are exactly buffer 0
    hipLaunchKernelGGL(k_resident_prologue, dim3(64), dim3(256), 0, r.stream, (const void*)d.ms[r.cur],
                       (void*)d.xchg, (int64_t)C * d.ld, (int)sizeof(T), (int64_t)C * d.ld);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    DevState<T> dd = d;
    Coef<T> kk = k;
    const double* u = r.u;
    T* states = static_cast<T*>(r.states);
    int samples = r.samples, substeps = r.substeps, cur = r.cur, renorm = r.renorm;
    // a trace armed for fewer workgroups than this launch has is not written
    unsigned long long* trace = r.trace && r.trace_groups >= grid ? r.trace : nullptr;
    int trace_stages = trace ? r.trace_stages : 0;
    ResTrace<T> tr{nullptr, nullptr, nullptr};
    int sample0 = 0;
    int stagger = block == 1024 && split > 1 ? poll_stagger((int)sizeof(T)) : 0;
    void* args[] = {&dd, &kk, &u, &states, &samples, &substeps, &cur, &renorm, &rpb, &wld, &trace, &trace_stages,
                    &tr, &sample0, &stagger};
    const void* fn = resident_kernel(sizeof(T), r.xyz, block, split_variant(split, false, stagger > 0));
    if (stagger > 0 && !co_resident(fn, block, lds, grid, device_cus())) {
        stagger = 0;
        fn = resident_kernel(sizeof(T), r.xyz, block, split_variant(split, false));
    }
    e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, (unsigned)lds, r.stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template hipError_t run_resident<double>(const DevState<double>&, const Coef<double>&, const RunSpec&);
template hipError_t run_resident<float>(const DevState<float>&, const Coef<float>&, const RunSpec&);

// The reverse keeps each row's epilogue inputs in registers; with 16 waves
// (128 registers per lane) they would spill, so it runs the same rows with
// 8 waves (at most 2 rows per wave).
int reverse_block(int block) { return block >= 1024 ? 512 : block; }

bool resident_adjoint_fits(int n, int elem_bytes, int xyz, int n_in) {
    if (n_in > kRevIn) return false;
    const int cus = device_cus();
    int grid = 0, rpb = 0, block = 0, split = 1;
    // the traced recompute runs the plain forward's shape
    if (!resident_shape(n, elem_bytes, xyz, &grid, &rpb, &block, &split)) return false;
    if (!co_resident(resident_kernel(elem_bytes, xyz, block, split_variant(split, true)), block,
                     resident_lds(n, rpb, elem_bytes, xyz), grid, cus))
        return false;
    // the reverse runs a shape of one wave per row
    if (!resident_shape(n, elem_bytes, xyz, &grid, &rpb, &block)) return false;
    const size_t lds = resident_lds(n, rpb, elem_bytes, xyz);
    return co_resident(resident_kernel(elem_bytes, xyz, reverse_block(block), 2), reverse_block(block), lds, grid,
                       cus);
}

template <typename T>
hipError_t run_resident_traced(const DevState<T>& d, const Coef<T>& k, const RunSpec& r, const ResTrace<T>& tr,
                               int sample0) {
    int grid = 0, rpb = 0, block = 0, split = 1;
    // the plain forward's shape, two waves per row included (the trace is in
    // node order, independent of the shape)
    if (!resident_shape(d.n, sizeof(T), r.xyz, &grid, &rpb, &block, &split)) return hipErrorInvalidValue;
    int wld = (int)wld_of(d.n);
    const size_t lds = resident_lds(d.n, rpb, sizeof(T), r.xyz);
    const int C = r.xyz ? 3 : 1;
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, r.stream, d.sync, 64);
    hipLaunchKernelGGL(k_resident_prologue, dim3(64), dim3(256), 0, r.stream, (const void*)d.ms[r.cur],
                       (void*)d.xchg, (int64_t)C * d.ld, (int)sizeof(T), (int64_t)C * d.ld);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    DevState<T> dd = d;
    Coef<T> kk = k;
    const double* u = r.u;
    T* states = nullptr;
    int samples = r.samples, substeps = r.substeps, cur = r.cur, renorm = r.renorm;
    unsigned long long* trace = nullptr;
    int trace_stages = 0;
    ResTrace<T> t = tr;
    int s0 = sample0;
    int stagger = block == 1024 && split > 1 ? poll_stagger((int)sizeof(T)) : 0;
    void* args[] = {&dd, &kk, &u, &states, &samples, &substeps, &cur, &renorm, &rpb, &wld, &trace, &trace_stages,
                    &t, &s0, &stagger};
    const void* fn = resident_kernel(sizeof(T), r.xyz, block, split_variant(split, true, stagger > 0));
    if (stagger > 0 && !co_resident(fn, block, lds, grid, device_cus())) {
        stagger = 0;
        fn = resident_kernel(sizeof(T), r.xyz, block, split_variant(split, true));
    }
    if (!co_resident(fn, block, lds, grid, device_cus())) return hipErrorInvalidValue;
    e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, (unsigned)lds, r.stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <typename T>
hipError_t run_resident_reverse(const AdjDev<T>& d, const Coef<T>& k, int kn, int xyz, T* xbuf, int* sync,
                                hipStream_t st) {
    int grid = 0, rpb = 0, block = 0;
    if (!resident_shape(d.n, sizeof(T), xyz, &grid, &rpb, &block)) return hipErrorInvalidValue;
    int wld = (int)wld_of(d.n);
    const size_t lds = resident_lds(d.n, rpb, sizeof(T), xyz);
    const int C = xyz ? 3 : 1;
    const T* first = d.st + (int64_t)(kn - 1) * 4 * C * d.ld + (int64_t)3 * C * d.ld;   // slot (kn - 1, 3)
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, sync, 64);
    hipLaunchKernelGGL(k_resident_prologue, dim3(64), dim3(256), 0, st, (const void*)first, (void*)xbuf,
                       (int64_t)C * d.ld, (int)sizeof(T), (int64_t)C * d.ld);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    AdjDev<T> dd = d;
    Coef<T> kc = k;
    T* xb = xbuf;
    int* sy = sync;
    int kn_ = kn;
    void* args[] = {&dd, &kc, &xb, &sy, &kn_, &rpb, &wld};
    const int rb = reverse_block(block);
    const void* fn = resident_kernel(sizeof(T), xyz, rb, 2);
    if (!co_resident(fn, rb, lds, grid, device_cus())) return hipErrorInvalidValue;
    e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(rb), args, (unsigned)lds, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template hipError_t run_resident_traced<double>(const DevState<double>&, const Coef<double>&, const RunSpec&,
                                                const ResTrace<double>&, int);
template hipError_t run_resident_traced<float>(const DevState<float>&, const Coef<float>&, const RunSpec&,
                                               const ResTrace<float>&, int);
template hipError_t run_resident_reverse<double>(const AdjDev<double>&, const Coef<double>&, int, int, double*, int*,
                                                 hipStream_t);
template hipError_t run_resident_reverse<float>(const AdjDev<float>&, const Coef<float>&, int, int, float*, int*,
                                                hipStream_t);

}  // namespace sto
