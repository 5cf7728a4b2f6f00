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

// One pass of a circuit over one tile.  As in the gate tile pass, the first
// sweep takes its register groups straight from the source and the last
// hands them straight to the sink, so the tile crosses LDS only between
// sweeps: the source is |0...0> synthesised in registers on the circuit's
// first pass, else the state; the sink accumulates the Z-string terms on
// the last pass and stores the state unless that pass is the last and the
// states are not kept.  A thread owns at most one group per sweep
// (2^(m-W) <= kBatchThreads).
template <typename T, int W, bool TWOQ>
__device__ void batch_tile(cpx<T> *state, cpx<T> *lds, const TileSpec &sp, int m, uint64_t base,
                           const TileSweep *__restrict__ sweeps, int n_sweeps, const char *__restrict__ recs,
                           bool synth, bool last_pass, bool store, uint64_t zmask, double &zacc) {
    constexpr int D = 1 << W;
    const uint32_t n_groups = (1u << m) >> W;
    for (int si = 0; si < n_sweeps; ++si) {
        const TileSweep &S = sweeps[si];
        const bool first = si == 0, last = si == n_sweeps - 1;
        uint32_t pb[W];
        uint64_t gbit[W];
#pragma unroll
        for (int b = 0; b < W; ++b) {
            pb[b] = lds_phys<T>(1u << S.qpos[b]);
            gbit[b] = tile_offset(sp, 1u << S.qpos[b]);
        }
        auto goff_of = [&](int j) {
            uint64_t o = 0;
#pragma unroll
            for (int b = 0; b < W; ++b)
                if ((j >> b) & 1) o |= gbit[b];
            return o;
        };
        auto poff_of = [&](int j) {
            uint32_t o = 0;
#pragma unroll
            for (int b = 0; b < W; ++b)
                if ((j >> b) & 1) o ^= pb[b];
            return o;
        };
        for (uint32_t g = threadIdx.x; g < n_groups; g += blockDim.x) {
            const uint32_t gb = group_bits<W>(S, g);
            const uint32_t pg = lds_phys<T>(gb);
            const uint64_t row = base | tile_offset(sp, gb);
            cpx<T> v[D];
            if (first && synth) {
#pragma unroll
                for (int j = 0; j < D; ++j) v[j] = cpx<T>{(row | goff_of(j)) == 0 ? T(1) : T(0), T(0)};
            } else if (first) {
#pragma unroll
                for (int j = 0; j < D; ++j) v[j] = state[row | goff_of(j)];
            } else {
#pragma unroll
                for (int j = 0; j < D; ++j) v[j] = lds[pg ^ poff_of(j)];
            }
            PhaseAcc<T, W> acc;
            acc.init();
            const char *rp = recs + S.rec_off;
            for (int gi = 0; gi < S.n_gates; ++gi) {
                const TileGate &G = *reinterpret_cast<const TileGate *>(rp);
                // advance before the gate: its inline assembly would make the
                // compiler read the size again after it
                rp += G.size;
                sweep_gate_t<T, W, TWOQ>(v, acc, gb, G, base);
            }
            if (last) {
                if (last_pass) {
#pragma unroll
                    for (int j = 0; j < D; ++j) zacc += zterm(v[j], row | goff_of(j), zmask);
                }
                if (store) {
#pragma unroll
                    for (int j = 0; j < D; ++j) state[row | goff_of(j)] = v[j];
                }
            } else {
#pragma unroll
                for (int j = 0; j < D; ++j) lds[pg ^ poff_of(j)] = v[j];
            }
        }
        __syncthreads();
    }
}

template <typename T, int W, bool TWOQ>
__global__ __launch_bounds__(kBatchThreads) void k_batch(BatchArgs a) {
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
        cpx<T> *state = reinterpret_cast<cpx<T> *>(reinterpret_cast<char *>(a.states) + c.state_off);
        double zacc = 0.0;
        for (int pi = 0; pi < c.n_passes; ++pi) {
            const BatchPass &p = a.passes[c.pass_off + pi];
            const int m = p.sp.L + p.sp.K;
            const uint64_t n_tiles = 1ull << (c.w - m);
            const bool last = pi == c.n_passes - 1;
            for (uint64_t tile = 0; tile < n_tiles; ++tile) {
                uint64_t base = tile << p.sp.L;
                for (int i = 0; i < p.sp.K; ++i) base = insert_zero(base, p.sp.high[i]);
                batch_tile<T, W, TWOQ>(state, lds, p.sp, m, base, a.sweeps + p.sweep_off, p.n_sweeps,
                                       a.recs + p.gate_off, pi == 0, last, !last || c.keep, a.zmask, zacc);
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
