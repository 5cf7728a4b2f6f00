// Measurement in the computational basis (Sec. 1.3.3, Sec. 2.4): outcome
// probabilities of a few qubits, projection onto an outcome with
// renormalisation, and full-register sampling by the inverse cumulative
// distribution.  All sums are FP64 and run in a fixed order, so results are
// deterministic.
#include "sv_internal.hpp"
#include "tile_sweep.hpp"

#include <algorithm>

namespace sv {

constexpr int kMeasThreads = 256;

__device__ __forceinline__ double meas_wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

template <typename T>
__device__ __forceinline__ double pr(const cpx<T> &a) {
    return (double)a.re * a.re + (double)a.im * a.im;
}

template <typename T>
__device__ __forceinline__ cpx<T> amp_of(const typename Amp16<T>::type &w, int i) {
    if constexpr (sizeof(T) == 4) return i == 0 ? cpx<T>{w.x, w.y} : cpx<T>{w.z, w.w};
    else return cpx<T>{w.x, w.y};
}

// Outcome index of x: bit i = bit pos[i] of x.
__device__ __forceinline__ uint32_t outcome_bits(uint64_t x, const MeasurePos &mp) {
    uint32_t o = 0;
#pragma unroll
    for (int i = 0; i < kMaxMeasureQubits; ++i)
        if (i < mp.k) o |= (uint32_t)((x >> mp.pos[i]) & 1ull) << i;
    return o;
}

// ------------------------------------------------------------- marginals
// Every thread keeps its own 2^k FP64 bins in LDS (bin b of thread t at
// b * kMeasThreads + t: consecutive lanes, consecutive banks), the
// workgroup then sums each bin over its threads in order.
template <typename T>
__global__ __launch_bounds__(kMeasThreads) void k_marginals(const typename Amp16<T>::type *__restrict__ v,
                                                            uint64_t n_vec, MeasurePos mp, double *partials) {
    extern __shared__ double bins[];
    const int nb = 1 << mp.k;
    for (int b = 0; b < nb; ++b) bins[b * kMeasThreads + threadIdx.x] = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kMeasThreads;
    for (uint64_t e = (uint64_t)blockIdx.x * kMeasThreads + threadIdx.x; e < n_vec; e += stride) {
        const typename Amp16<T>::type w = v[e];
#pragma unroll
        for (int i = 0; i < (sizeof(T) == 4 ? 2 : 1); ++i) {
            const uint64_t x = (e << Amp16<T>::bits) + i;
            bins[outcome_bits(x, mp) * kMeasThreads + threadIdx.x] += pr(amp_of<T>(w, i));
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kMeasThreads) {
        double s = 0.0;
        for (int t = 0; t < kMeasThreads; ++t) s += bins[b * kMeasThreads + t];
        partials[(size_t)b * gridDim.x + blockIdx.x] = s;
    }
}

// ------------------------------------------------- masked probability
template <typename T>
__global__ __launch_bounds__(kMeasThreads) void k_masked_prob(const typename Amp16<T>::type *__restrict__ v,
                                                              uint64_t n_vec, uint64_t mask, uint64_t want,
                                                              double *partials) {
    __shared__ double sh[kMeasThreads / 64];
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kMeasThreads;
    for (uint64_t e = (uint64_t)blockIdx.x * kMeasThreads + threadIdx.x; e < n_vec; e += stride) {
        const typename Amp16<T>::type w = v[e];
#pragma unroll
        for (int i = 0; i < (sizeof(T) == 4 ? 2 : 1); ++i) {
            const uint64_t x = (e << Amp16<T>::bits) + i;
            if ((x & mask) == want) acc += pr(amp_of<T>(w, i));
        }
    }
    acc = meas_wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < kMeasThreads / 64; ++i) s += sh[i];
        partials[blockIdx.x] = s;
    }
}

// --------------------------------------------------------------- collapse
template <typename T>
__global__ __launch_bounds__(kMeasThreads) void k_collapse(typename Amp16<T>::type *__restrict__ v, uint64_t n_vec,
                                                           uint64_t mask, uint64_t want, T scale) {
    const uint64_t stride = (uint64_t)gridDim.x * kMeasThreads;
    for (uint64_t e = (uint64_t)blockIdx.x * kMeasThreads + threadIdx.x; e < n_vec; e += stride) {
        typename Amp16<T>::type w = v[e];
        const uint64_t x = e << Amp16<T>::bits;
        const T s0 = ((x & mask) == want) ? scale : T(0);
        if constexpr (sizeof(T) == 4) {
            const T s1 = (((x + 1) & mask) == want) ? scale : T(0);
            w = float4{w.x * s0, w.y * s0, w.z * s1, w.w * s1};
        } else {
            w = double2{w.x * s0, w.y * s0};
        }
        v[e] = w;
    }
}

// --------------------------------------------------------------- sampling
// Sum of each contiguous block of 2^block_log amplitudes (one workgroup per
// block, grid-stride over blocks).
template <typename T>
__global__ __launch_bounds__(kMeasThreads) void k_block_sums(const cpx<T> *__restrict__ v, int block_log,
                                                             uint64_t n_blocks, double *sums) {
    __shared__ double sh[kMeasThreads / 64];
    const uint64_t bsize = 1ull << block_log;
    for (uint64_t b = blockIdx.x; b < n_blocks; b += gridDim.x) {
        const cpx<T> *p = v + b * bsize;
        double acc = 0.0;
        for (uint64_t i = threadIdx.x; i < bsize; i += kMeasThreads) acc += pr(p[i]);
        acc = meas_wave_sum(acc);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int i = 0; i < kMeasThreads / 64; ++i) s += sh[i];
            sums[b] = s;
        }
        __syncthreads();
    }
}

// One wave per sample: scan the sample's block 64 amplitudes at a time
// (FP64 inclusive prefix across the wave plus the running sum) and take the
// first amplitude whose cumulative sum exceeds the sample's target; if
// rounding leaves none, the block's last amplitude with p > 0.
template <typename T>
__global__ __launch_bounds__(kMeasThreads) void k_sample_scan(const cpx<T> *__restrict__ v, int block_log,
                                                              int n_samples, const int64_t *__restrict__ blk,
                                                              const double *__restrict__ target,
                                                              uint64_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int s = (int)((blockIdx.x * kMeasThreads + threadIdx.x) >> 6);
    if (s >= n_samples) return; // whole waves leave together
    const uint64_t bsize = 1ull << block_log;
    const uint64_t base = (uint64_t)blk[s] << block_log;
    const double t = target[s];
    double run = 0.0;
    int64_t last = -1;
    int64_t found = -1;
    for (uint64_t c = 0; c < bsize; c += 64) {
        const uint64_t i = c + lane;
        const double p = i < bsize ? pr(v[base + i]) : 0.0;
        double inc = p;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        const uint64_t hit = __ballot(run + inc > t);
        if (hit) {
            found = (int64_t)(c + __builtin_ctzll(hit));
            break;
        }
        const uint64_t nz = __ballot(p > 0.0);
        if (nz) last = (int64_t)(c + 63 - __builtin_clzll(nz));
        run += __shfl(inc, 63, 64);
    }
    if (lane == 0) out[s] = base + (uint64_t)(found >= 0 ? found : (last >= 0 ? last : 0));
}

// ---------------------------------------------------------------- launchers
static unsigned stream_grid(uint64_t n_vec) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n_vec + kMeasThreads - 1) / kMeasThreads, 1024));
}

int marginal_blocks(int n, int dtype) {
    const uint64_t n_vec = (1ull << n) >> (dtype == SV_C64 ? 1 : 0);
    return (int)stream_grid(std::max<uint64_t>(n_vec, 1));
}

hipError_t launch_marginals(const void *amps, int n, int dtype, const MeasurePos &mp, double *partials,
                            hipStream_t s) {
    if (mp.k < 1 || mp.k > kMaxMeasureQubits) return hipErrorInvalidValue;
    const int vb = dtype == SV_C64 ? 1 : 0;
    if (n < vb) return hipErrorInvalidValue;
    const uint64_t n_vec = (1ull << n) >> vb;
    const unsigned grid = stream_grid(n_vec);
    const size_t lds = (size_t)(1u << mp.k) * kMeasThreads * sizeof(double);
    if (dtype == SV_C64) {
        (void)hipFuncSetAttribute((const void *)k_marginals<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_marginals<float><<<grid, kMeasThreads, lds, s>>>((const float4 *)amps, n_vec, mp, partials);
    } else {
        (void)hipFuncSetAttribute((const void *)k_marginals<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_marginals<double><<<grid, kMeasThreads, lds, s>>>((const double2 *)amps, n_vec, mp, partials);
    }
    return hipGetLastError();
}

hipError_t launch_masked_prob(const void *amps, int n, int dtype, uint64_t mask, uint64_t want,
                              double *partials, hipStream_t s) {
    const int vb = dtype == SV_C64 ? 1 : 0;
    if (n < vb) return hipErrorInvalidValue;
    const uint64_t n_vec = (1ull << n) >> vb;
    const unsigned grid = stream_grid(n_vec);
    if (dtype == SV_C64)
        k_masked_prob<float><<<grid, kMeasThreads, 0, s>>>((const float4 *)amps, n_vec, mask, want, partials);
    else
        k_masked_prob<double><<<grid, kMeasThreads, 0, s>>>((const double2 *)amps, n_vec, mask, want, partials);
    return hipGetLastError();
}

hipError_t launch_collapse(void *amps, int n, int dtype, uint64_t mask, uint64_t want, double scale,
                           hipStream_t s) {
    const int vb = dtype == SV_C64 ? 1 : 0;
    if (n < vb) return hipErrorInvalidValue;
    const uint64_t n_vec = (1ull << n) >> vb;
    const unsigned grid = stream_grid(n_vec);
    if (dtype == SV_C64)
        k_collapse<float><<<grid, kMeasThreads, 0, s>>>((float4 *)amps, n_vec, mask, want, (float)scale);
    else
        k_collapse<double><<<grid, kMeasThreads, 0, s>>>((double2 *)amps, n_vec, mask, want, scale);
    return hipGetLastError();
}

int sample_block_log(int n) { return std::max(std::min(n, 8), n - 16); }

hipError_t launch_block_sums(const void *amps, int n, int dtype, int block_log, double *sums, hipStream_t s) {
    if (block_log > n) return hipErrorInvalidValue;
    const uint64_t nbk = 1ull << (n - block_log);
    const unsigned grid = (unsigned)std::min<uint64_t>(nbk, 4096);
    if (dtype == SV_C64)
        k_block_sums<float><<<grid, kMeasThreads, 0, s>>>((const cpx<float> *)amps, block_log, nbk, sums);
    else
        k_block_sums<double><<<grid, kMeasThreads, 0, s>>>((const cpx<double> *)amps, block_log, nbk, sums);
    return hipGetLastError();
}

hipError_t launch_sample_scan(const void *amps, int dtype, int block_log, int n_samples, const int64_t *blk,
                              const double *target, uint64_t *out, hipStream_t s) {
    if (n_samples <= 0) return hipSuccess;
    const unsigned grid = (unsigned)(((uint64_t)n_samples * 64 + kMeasThreads - 1) / kMeasThreads);
    if (dtype == SV_C64)
        k_sample_scan<float><<<grid, kMeasThreads, 0, s>>>((const cpx<float> *)amps, block_log, n_samples, blk,
                                                           target, out);
    else
        k_sample_scan<double><<<grid, kMeasThreads, 0, s>>>((const cpx<double> *)amps, block_log, n_samples, blk,
                                                            target, out);
    return hipGetLastError();
}

} // namespace sv
