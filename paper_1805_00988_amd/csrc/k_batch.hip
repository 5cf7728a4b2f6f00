// Batched circuits: one persistent launch runs thousands of independent
// circuits of different widths.
//
// Workgroups pop circuit indices from a device queue (an atomic counter) in
// the host's longest-first order until the queue is empty, so every
// workgroup exits once all circuits are taken.  A circuit whose state fits
// in one LDS tile (up to 2^13 complex64 / 2^12 complex128 amplitudes) starts
// from |0...0> directly in LDS, runs all its gates there and reduces its
// Z-string expectation without touching HBM.  A wider circuit keeps its
// state in HBM and runs the host's tile passes over it; the first pass
// synthesises |0...0> instead of loading it, and the last pass accumulates
// the expectation while it stores the final tiles.
#include "sv_internal.hpp"
#include "tile_sweep.hpp"

#include <algorithm>
#include <type_traits>

namespace sv {

constexpr int kBatchThreads = 512;

template <typename T>
struct BV;
template <>
struct BV<float> {
    using type = float4;
    static constexpr int amps = 2, bits = 1;
};
template <>
struct BV<double> {
    using type = double2;
    static constexpr int amps = 1, bits = 0;
};

__device__ __forceinline__ uint64_t btile_addr(const TileSpec &sp, uint64_t base, uint32_t l) {
    uint64_t g = base | (l & ((1u << sp.L) - 1u));
    const uint32_t hi = l >> sp.L;
    for (int i = 0; i < sp.K; ++i)
        if ((hi >> i) & 1u) g |= 1ull << sp.high[i];
    return g;
}

__device__ __forceinline__ double bwave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

template <typename T>
__device__ __forceinline__ double zterm(cpx<T> a, uint64_t x, uint64_t zmask) {
    const double p = (double)a.re * a.re + (double)a.im * a.im;
    return (__popcll(x & zmask) & 1) ? -p : p;
}

template <typename T, int W, bool TWOQ>
__global__ __launch_bounds__(kBatchThreads) void k_batch(BatchArgs a) {
    using V = BV<T>;
    extern __shared__ char lds_raw[];
    cpx<T> *lds = reinterpret_cast<cpx<T> *>(lds_raw);
    __shared__ int s_idx;
    __shared__ double s_red[kBatchThreads / 64];
    for (;;) {
        if (threadIdx.x == 0) s_idx = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int qi = s_idx;
        __syncthreads();
        if (qi >= a.n_circuits) break; // uniform: every wave leaves together
        const int ci = a.order[qi];
        const BatchCircuit &c = a.circuits[ci]; // read through memory (uniform)
        typename V::type *state = reinterpret_cast<typename V::type *>(
            reinterpret_cast<char *>(a.states) + c.state_off);
        double zacc = 0.0;
        for (int pi = 0; pi < c.n_passes; ++pi) {
            const BatchPass &p = a.passes[c.pass_off + pi];
            const int m = p.sp.L + p.sp.K;
            const uint32_t tsize = 1u << m, tvec = tsize >> V::bits;
            const uint64_t n_tiles = 1ull << (c.w - m);
            const bool last = pi == c.n_passes - 1;
            for (uint64_t tile = 0; tile < n_tiles; ++tile) {
                uint64_t base = tile << p.sp.L;
                for (int i = 0; i < p.sp.K; ++i) base = insert_zero(base, p.sp.high[i]);
                if (pi == 0) {
                    for (uint32_t l = threadIdx.x; l < tsize; l += kBatchThreads)
                        lds[lds_phys<T>(l)] = cpx<T>{(base == 0 && l == 0) ? T(1) : T(0), T(0)};
                } else {
                    for (uint32_t l = threadIdx.x; l < tvec; l += kBatchThreads) {
                        const uint32_t la = l << V::bits;
                        const typename V::type w = state[btile_addr(p.sp, base, la) >> V::bits];
                        if constexpr (V::bits == 1) {
                            lds[lds_phys<T>(la)] = cpx<T>{w.x, w.y};
                            lds[lds_phys<T>(la + 1)] = cpx<T>{w.z, w.w};
                        } else {
                            lds[lds_phys<T>(la)] = cpx<T>{w.x, w.y};
                        }
                    }
                }
                __syncthreads();
                tile_run_sweeps<T, W, TWOQ>(lds, m, base, a.sweeps + p.sweep_off, p.n_sweeps,
                                      a.recs + p.gate_off);
                if (last) {
                    for (uint32_t l = threadIdx.x; l < tsize; l += kBatchThreads)
                        zacc += zterm(lds[lds_phys<T>(l)], btile_addr(p.sp, base, l), a.zmask);
                }
                if (!last || c.keep) {
                    for (uint32_t l = threadIdx.x; l < tvec; l += kBatchThreads) {
                        const uint32_t la = l << V::bits;
                        typename V::type w;
                        if constexpr (V::bits == 1) {
                            const cpx<T> u0 = lds[lds_phys<T>(la)], u1 = lds[lds_phys<T>(la + 1)];
                            w = float4{u0.re, u0.im, u1.re, u1.im};
                        } else {
                            const cpx<T> u0 = lds[lds_phys<T>(la)];
                            w = double2{u0.re, u0.im};
                        }
                        state[btile_addr(p.sp, base, la) >> V::bits] = w;
                    }
                }
                __syncthreads();
            }
            // the next pass reads what this pass wrote: make the stores visible
            __threadfence();
            __syncthreads();
        }
        zacc = bwave_sum(zacc);
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = zacc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kBatchThreads / 64; ++w) t += s_red[w];
            a.out[ci] = t;
        }
        __syncthreads();
    }
}

__global__ void k_batch_reset(unsigned int *counter) { *counter = 0u; }

template <typename T, int W, bool TWOQ>
static void launch_batch_t(const BatchArgs &args, int grid, size_t lds, hipStream_t s) {
    (void)hipFuncSetAttribute((const void *)k_batch<T, W, TWOQ>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    k_batch<T, W, TWOQ><<<grid, kBatchThreads, lds, s>>>(args);
}

hipError_t launch_batch(const BatchArgs &args, int dtype, int sweep_w, int tile_m, int grid, bool two_qubit,
                        hipStream_t s) {
    const int m = tile_m;
    const size_t lds = (size_t)(1u << m) * (dtype == SV_C64 ? 8 : 16);
    k_batch_reset<<<1, 1, 0, s>>>(args.counter);
#define SV_BATCH_CASE(TT, WW, Q)                                                                   \
    if ((dtype == SV_C64) == std::is_same<TT, float>::value && sweep_w == WW && two_qubit == Q) {  \
        launch_batch_t<TT, WW, Q>(args, grid, lds, s);                                             \
        return hipGetLastError();                                                                  \
    }
    SV_BATCH_CASE(float, 4, false)
    SV_BATCH_CASE(float, 3, false)
    SV_BATCH_CASE(double, 3, false)
    SV_BATCH_CASE(double, 4, false)
    SV_BATCH_CASE(float, 4, true)
    SV_BATCH_CASE(float, 3, true)
    SV_BATCH_CASE(double, 3, true)
    SV_BATCH_CASE(double, 4, true)
#undef SV_BATCH_CASE
    return hipErrorInvalidValue;
}

} // namespace sv
