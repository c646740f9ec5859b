// MULTI path: S input streams drive S copies of one reservoir (one coupling
// matrix W, one set of constants, S states).  Per RK4 stage the coupling of
// all streams is one matrix product, C = a_cp * W X with X the N x S block of
// stage inputs m^x (paper, Eq. (coup); Sec. 3.3 writes the single-stream
// case as W^cp x), evaluated with FP32 MFMA (v_mfma_f32_16x16x4f32, FP32
// accumulation) and fused with the pointwise right-hand side of Eq. (gov)
// and the RK4 bookkeeping (Sec. 3.2).
//
// Tiling.  Workgroup (bi, bj) owns the 16 x 16 output tile of nodes
// 16 bi..16 bi + 15 and streams 16 bj..16 bj + 15 for the whole run.  Its four
// waves split the contraction dimension into quarters; each wave keeps its
// 16 rows x N/4 slice of W in registers as MFMA A operands (one element per
// lane per MFMA), reads the stage inputs of its 16 streams from LDS as B
// operands, and the four partial tiles are summed in LDS in a fixed order.
// Thread t then owns the pair (node 16 bi + t/16, stream 16 bj + t%16): its
// state, RK4 accumulator and stage input stay in registers.
//
// Stage inputs are exchanged through three rotating global buffers, laid out
// [stream][node], whose unpublished entries hold a sentinel bit pattern; the
// protocol (poll, re-arm two stages ahead, compute while those stores
// complete, wait for them, publish) is the one of the resident kernel.  Every wait is bounded and
// raises a sticky abort flag when it expires.

#include <climits>

#include "sto_internal.hpp"

namespace sto {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
constexpr int kTile = 16;
constexpr int kSpinLimit = 1 << 20;

// Wait until the stage inputs of the workgroup's streams are published and
// store them K-major in LDS: xs[k * 16 + j] for node k and local stream j.
// Each thread keeps Q loads in flight per round, so a round trip to memory
// covers Q * 256 entries.
constexpr int kQ = 16;
__device__ bool gather_multi(const float* xb, int64_t ld, int n, int s0, int ns, float* xs, int* abort_flag) {
    const unsigned* src = reinterpret_cast<const unsigned*>(xb);
    const int total = ns * n;
    bool ok = true;
    for (int e0 = 0; e0 < total && ok; e0 += kQ * kBlock) {
        unsigned v[kQ];
        unsigned todo = 0;   // bit q: entry q of this round is still unpublished
#pragma unroll
        for (int q = 0; q < kQ; ++q)
            if (e0 + q * kBlock + (int)threadIdx.x < total) todo |= 1u << q;
        int rounds = 0;
        while (todo) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                if (todo & (1u << q)) {
                    const int e = e0 + q * kBlock + threadIdx.x;
                    const int j = e / n, k = e - j * n;
                    v[q] = __hip_atomic_load(src + (int64_t)(s0 + j) * ld + k, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
                }
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                if ((todo & (1u << q)) && v[q] != ~0u) {
                    const int e = e0 + q * kBlock + threadIdx.x;
                    const int j = e / n, k = e - j * n;
                    xs[k * kTile + j] = __builtin_bit_cast(float, v[q]);
                    todo &= ~(1u << q);
                }
            }
            if (todo && (++rounds & 255) == 0) {
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

// KREG: MFMA steps per wave, >= ceil(N/16) (each step contracts 4 nodes).
template <int KREG>
__global__ void __launch_bounds__(kBlock) k_multi(DevState<float> d, Coef<float> k, const double* __restrict__ u,
                                                  float* __restrict__ states, int streams, int samples,
                                                  int substeps, int renorm) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int ok_lds;
    const int n = d.n;
    const int64_t ld = d.ld;
    const int kp = (n + kTile - 1) / kTile * kTile;             // contraction length padded to 16
    float* xs = reinterpret_cast<float*>(smem_raw);              // [kp][16]
    float* cs = xs + (int64_t)kp * kTile;                        // [4 waves][16][16] partial tiles
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row0 = blockIdx.x * kTile;
    const int s0 = blockIdx.y * kTile;
    const int ns = min(kTile, streams - s0);
    int* abort_flag = d.sync + kSyncAbortWord;
    if (threadIdx.x == 0) ok_lds = 1;
    for (int i = threadIdx.x; i < kp * kTile; i += kBlock) xs[i] = 0.0f;   // padded nodes/streams stay 0

    // A operands: this wave's quarter of the contraction for the tile's rows.
    const int kq = kp / 4;                                       // nodes per wave (multiple of 4)
    const int steps = kq / 4;
    float areg[KREG];
    {
        const int r = row0 + (lane & 15);
#pragma unroll
        for (int t = 0; t < KREG; ++t) {
            const int kk = wave * kq + 4 * t + (lane >> 4);
            areg[t] = (t < steps && r < n && kk < n) ? d.W[(int64_t)r * ld + kk] : 0.0f;
        }
    }

    // the (node, stream) pair of this thread
    const int node = row0 + (threadIdx.x >> 4);
    const int strm = s0 + (threadIdx.x & 15);
    const bool mine = node < n && strm < streams;
    const int nd = min(node, n - 1), sd = min(strm, streams - 1);
    const float* m_in = d.m + (int64_t)sd * 3 * ld;
    float mx = m_in[nd], my = m_in[ld + nd], mz = m_in[2 * ld + nd];
    float sx = mx, sy = my, sz = mz, ax = 0.f, ay = 0.f, az = 0.f;
    float* xbuf = d.xchg;                                        // [3][streams][ld]
    const int64_t bstride = (int64_t)streams * ld;

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
                if (!gather_multi(xin, ld, n, s0, ns, xs, abort_flag)) ok_lds = 0;
                __syncthreads();
                if (ok_lds == 0) return;
                // re-arm this pair's entry of the buffer two stages ahead now:
                // every workgroup finished reading it (the gather just saw all
                // outputs of the previous stage, each published after its
                // workgroup's own gather), and its store then completes while
                // the stage is computed
                if (mine)
                    __hip_atomic_store(reinterpret_cast<unsigned*>(xold + (int64_t)strm * ld + node), ~0u,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // partial tile of this wave: D[i][j] = sum over its nodes of W[row0+i][k] X[k][s0+j]
                f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int t = 0; t < KREG; ++t) {
                    if (t < steps) {
                        const int kk = wave * kq + 4 * t + (lane >> 4);
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(areg[t], xs[kk * kTile + (lane & 15)], acc, 0, 0,
                                                                   0);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) cs[(wave * kTile + 4 * (lane >> 4) + r) * kTile + (lane & 15)] = acc[r];
                __syncthreads();
                const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
                const float dot = ((cs[(0 * kTile + ti) * kTile + tj] + cs[(1 * kTile + ti) * kTile + tj]) +
                                   cs[(2 * kTile + ti) * kTile + tj]) +
                                  cs[(3 * kTile + ti) * kTile + tj];
                float fx, fy, fz;
                llg_rhs<float, false>(k, sx, sy, sz, k.a_cp * dot, 0.f, 0.f, hin, fx, fy, fz);
                float nx = rk4_update(k, stage, mx, ax, fx);
                float ny = rk4_update(k, stage, my, ay, fy);
                float nz = rk4_update(k, stage, mz, az, fz);
                if (stage == 3) {
                    if (renorm) renormalize(nx, ny, nz);
                    mx = nx;
                    my = ny;
                    mz = nz;
                }
                sx = nx;
                sy = ny;
                sz = nz;
                if (mine) {
                    const int64_t o = (int64_t)strm * ld + node;
                    // the re-arm store must complete before the publish
                    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                    __hip_atomic_store(xout + o, nx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        if (mine) {
            if (states) {
                float* rec = states + (((int64_t)s * streams + strm) * n + node) * 3;
                rec[0] = mx;
                rec[1] = my;
                rec[2] = mz;
            }
            if (!finite3(mx, my, mz)) atomicMin(d.bad, s);
        }
    }
    if (mine) {
        float* mo = d.m + (int64_t)strm * 3 * ld;
        mo[node] = mx;
        mo[ld + node] = my;
        mo[2 * ld + node] = mz;
    }
}

__global__ void k_multi_prologue(const float* m, float* xchg, int streams, int64_t ld) {
    // buffer 0 <- m^x of every stream; buffers 1 and 2 <- sentinel
    const int64_t per = (int64_t)streams * ld;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * per;
         i += (int64_t)gridDim.x * blockDim.x) {
        unsigned v = ~0u;
        if (i < per) {
            const int64_t st = i / ld, node = i - st * ld;
            v = __builtin_bit_cast(unsigned, m[st * 3 * ld + node]);
        }
        reinterpret_cast<unsigned*>(xchg)[i] = v;
    }
}

constexpr int kMaxKreg = 64;   // N <= 1024

int kreg_for(int n) {
    const int need = ((n + kTile - 1) / kTile * kTile) / 16;
    for (int kr : {4, 8, 16, 32, 64})
        if (kr >= need) return kr;
    return 0;
}

}  // namespace

size_t multi_lds_bytes(int n) {
    const int kp = (n + kTile - 1) / kTile * kTile;
    return ((size_t)kp * kTile + 4 * kTile * kTile) * sizeof(float);
}

bool multi_fits(int n, int streams, int* grid_x, int* grid_y) {
    if (n < 1 || streams < 1 || kreg_for(n) == 0 || n > 16 * kMaxKreg) return false;
    const int gx = (n + kTile - 1) / kTile, gy = (streams + kTile - 1) / kTile;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    const size_t lds = multi_lds_bytes(n);
    if (lds + 64 > 160 * 1024) return false;
    per_cu = (int)std::min<size_t>(8, (160 * 1024) / (lds + 64));
    if ((int64_t)gx * gy > (int64_t)cus * per_cu) return false;
    if (grid_x) *grid_x = gx;
    if (grid_y) *grid_y = gy;
    return true;
}

hipError_t run_multi(const DevState<float>& d, const Coef<float>& k, const RunSpec& r, int streams) {
    int gx = 0, gy = 0;
    if (!multi_fits(d.n, streams, &gx, &gy)) return hipErrorInvalidValue;
    const size_t lds = multi_lds_bytes(d.n);
    hipError_t e = hipMemsetAsync(d.sync, 0, 256, r.stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_multi_prologue, dim3(64), dim3(256), 0, r.stream, (const float*)d.m, d.xchg, streams, d.ld);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    DevState<float> dd = d;
    Coef<float> kk = k;
    const double* u = r.u;
    float* states = static_cast<float*>(r.states);
    int st = streams, samples = r.samples, substeps = r.substeps, renorm = r.renorm;
    void* args[] = {&dd, &kk, &u, &states, &st, &samples, &substeps, &renorm};
    const void* fn = nullptr;
    switch (kreg_for(d.n)) {
        case 4: fn = reinterpret_cast<const void*>(&k_multi<4>); break;
        case 8: fn = reinterpret_cast<const void*>(&k_multi<8>); break;
        case 16: fn = reinterpret_cast<const void*>(&k_multi<16>); break;
        case 32: fn = reinterpret_cast<const void*>(&k_multi<32>); break;
        default: fn = reinterpret_cast<const void*>(&k_multi<64>); break;
    }
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipLaunchCooperativeKernel(fn, dim3(gx, gy), dim3(kBlock), args, (unsigned)lds, r.stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace sto
