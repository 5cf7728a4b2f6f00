// Dense k-qubit blocks (products of several gates, built by the host fuser).
//
// Each workgroup stages a tile of 2^m amplitudes in LDS (the same tile
// layout as the gate tile pass: low qubits plus extra qubits, here at least
// the block's qubits).  Inside a tile the 2^m amplitudes form 2^(m-k) groups
// of 2^k that differ only in the block's qubits; every group is multiplied
// by the 2^k x 2^k matrix U.
//
// complex64 blocks of k = 4, 5 run on the matrix cores.  With X the groups
// as rows of [Re x | Im x] (M x 2K real) the product is two real GEMMs:
//   Re Y = [Re X | Im X] . [[Re U^T], [-Im U^T]],
//   Im Y = [Re X | Im X] . [[Im U^T], [ Re U^T]].
// The right-hand operands are the same for every group: the host lays them
// out once per block in the exact per-lane order of the MFMA B operand, and
// each wave keeps them in registers.  FP32 uses v_mfma_f32_{32x32x2,16x16x4}
// _f32; split-BF16 represents every FP32 operand as hi + lo (two bf16) and
// accumulates hi*hi + hi*lo + lo*hi in FP32 with v_mfma_f32_{32x32x16,
// 16x16x32}_bf16.
#include "sv_internal.hpp"

#include <algorithm>

namespace sv {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kFuseThreads = 512;

__device__ __forceinline__ uint32_t deposit(uint32_t x, const int *pos, int nbits) {
    uint32_t r = 0;
    for (int b = 0; b < nbits; ++b)
        if ((x >> b) & 1u) r |= 1u << pos[b];
    return r;
}

// Tile staging shared with the gate tile pass (same index mapping).
__device__ __forceinline__ uint64_t tile_base(const TileSpec &sp, uint64_t tile) {
    uint64_t base = tile << sp.L;
    for (int i = 0; i < sp.K; ++i) base = insert_zero(base, sp.high[i]);
    return base;
}

__device__ __forceinline__ uint64_t tile_addr(const TileSpec &sp, uint64_t base, uint32_t l) {
    uint64_t g = base | (l & ((1u << sp.L) - 1u));
    const uint32_t hi = l >> sp.L;
    for (int i = 0; i < sp.K; ++i)
        if ((hi >> i) & 1u) g |= 1ull << sp.high[i];
    return g;
}

template <typename T>
struct V16;
template <>
struct V16<float> {
    using type = float4;
    static constexpr int bits = 1;
};
template <>
struct V16<double> {
    using type = double2;
    static constexpr int bits = 0;
};

template <typename T>
__device__ __forceinline__ void stage_in(const typename V16<T>::type *v, cpx<T> *lds,
                                         const TileSpec &sp, uint64_t base, uint32_t tsize) {
    constexpr int vb = V16<T>::bits;
    for (uint32_t l = threadIdx.x; l < (tsize >> vb); l += blockDim.x) {
        const uint32_t la = l << vb;
        const typename V16<T>::type w = v[tile_addr(sp, base, la) >> vb];
        if constexpr (vb == 1) {
            lds[la] = cpx<T>{w.x, w.y};
            lds[la + 1] = cpx<T>{w.z, w.w};
        } else {
            lds[la] = cpx<T>{w.x, w.y};
        }
    }
}

template <typename T>
__device__ __forceinline__ void stage_out(typename V16<T>::type *v, const cpx<T> *lds,
                                          const TileSpec &sp, uint64_t base, uint32_t tsize) {
    constexpr int vb = V16<T>::bits;
    for (uint32_t l = threadIdx.x; l < (tsize >> vb); l += blockDim.x) {
        const uint32_t la = l << vb;
        typename V16<T>::type w;
        if constexpr (vb == 1) {
            w = float4{lds[la].re, lds[la].im, lds[la + 1].re, lds[la + 1].im};
        } else {
            w = double2{lds[la].re, lds[la].im};
        }
        v[tile_addr(sp, base, la) >> vb] = w;
    }
}

// ------------------------------------------------- native (vector ALU)
// One thread per group: the 2^K amplitudes go to registers, every output is
// a dot product with a row of U (uniform across the wave, read through the
// scalar cache), written back to the group's own LDS slots.  The blocks of a
// pass are applied one after another to the staged tile.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_dense_native(typename V16<T>::type *v, TileSpec sp, int m,
                                                      const DenseBlock *__restrict__ blocks, int n_blocks,
                                                      const char *__restrict__ base_ptr,
                                                      uint64_t n_tiles) {
    extern __shared__ char lds_raw[];
    cpx<T> *lds = reinterpret_cast<cpx<T> *>(lds_raw);
    constexpr int D = 1 << K;
    const uint32_t tsize = 1u << m;
    const uint32_t n_groups = tsize >> K;
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint64_t base = tile_base(sp, tile);
        stage_in<T>(v, lds, sp, base, tsize);
        __syncthreads();
        for (int b = 0; b < n_blocks; ++b) {
            const DenseBlock &B = blocks[b];
            const cpx<T> *U = reinterpret_cast<const cpx<T> *>(base_ptr + B.op_off);
            uint32_t F[D];
#pragma unroll
            for (int j = 0; j < D; ++j) F[j] = deposit((uint32_t)j, B.bp.qpos, K);
            for (uint32_t g = threadIdx.x; g < n_groups; g += blockDim.x) {
                const uint32_t gb = deposit(g, B.bp.gpos, B.bp.ng);
                cpx<T> x[D];
#pragma unroll
                for (int j = 0; j < D; ++j) x[j] = lds[gb | F[j]];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    cpx<T> acc = cmul(U[i * D], x[0]);
#pragma unroll
                    for (int j = 1; j < D; ++j) acc = cfma(U[i * D + j], x[j], acc);
                    lds[gb | F[i]] = acc;
                }
            }
            __syncthreads();
        }
        stage_out<T>(v, lds, sp, base, tsize);
        __syncthreads();
    }
}

// ---------------------------------------------------- MFMA, complex64
// Per-lane B-operand fragments, laid out by the host:
//   FP32:       frag[(part * KSTEPS + s) * 64 + lane]            (float)
//   split-BF16: frag[((part * KSTEPS + s) * 2 + hl) * 64 + lane]  (bf16x8)
// part 0 -> Re Y, part 1 -> Im Y; hl 0 = hi, 1 = lo.
template <int K, int PREC>
struct MfmaShape;
// K = 5, FP32: 32x32x2, 32 K-steps over [Re x | Im x] (64)
template <>
struct MfmaShape<5, 1> {
    static constexpr int rows = 32, ksteps = 32;
};
// K = 4, FP32: 16x16x4, 8 K-steps over 32
template <>
struct MfmaShape<4, 1> {
    static constexpr int rows = 16, ksteps = 8;
};
// K = 5, BF16: 32x32x16, 4 K-steps over 64
template <>
struct MfmaShape<5, 2> {
    static constexpr int rows = 32, ksteps = 4;
};
// K = 4, BF16: 16x16x32, 1 K-step over 32
template <>
struct MfmaShape<4, 2> {
    static constexpr int rows = 16, ksteps = 1;
};

// x ~ hi + lo with hi = bf16(x) and lo = bf16(x - hi)
__device__ __forceinline__ __bf16 bf16_hi(float x) { return (__bf16)x; }
__device__ __forceinline__ __bf16 bf16_lo(float x, __bf16 hi) { return (__bf16)(x - (float)hi); }

template <int K, int PREC>
__global__ __launch_bounds__(kFuseThreads) void k_dense_mfma(float4 *v, TileSpec sp, int m,
                                                             const DenseBlock *__restrict__ blocks,
                                                             int n_blocks, const char *__restrict__ base_ptr,
                                                             uint64_t n_tiles) {
    using S = MfmaShape<K, PREC>;
    constexpr int D = 1 << K;         // amplitudes per group = output columns
    constexpr int ROWS = S::rows;     // groups per wave-tile
    constexpr int KS = S::ksteps;
    constexpr int ACC = ROWS == 32 ? 16 : 4;
    using accT = typename std::conditional<ROWS == 32, floatx16, floatx4>::type;
    extern __shared__ char lds_raw[];
    cpx<float> *lds = reinterpret_cast<cpx<float> *>(lds_raw);
    const uint32_t tsize = 1u << m;
    const uint32_t n_groups = tsize >> K;
    const uint32_t n_wt = n_groups / ROWS;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int r = lane % ROWS;          // A row (group within wave-tile) / D column (output amp)
    const int kk = lane / ROWS;         // K sub-index of the lane

    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint64_t base = tile_base(sp, tile);
        stage_in<float>(v, lds, sp, base, tsize);
        __syncthreads();
        for (int b = 0; b < n_blocks; ++b) {
        const DenseBlock &B = blocks[b];
        const BlockPos &bp = B.bp;
        const void *frag = base_ptr + B.op_off;
        // this block's B fragments in registers (the same for every group)
        float bf32[2][PREC == 1 ? KS : 1];
        bf16x8 bbf[2][PREC == 2 ? KS : 1][2];
        if constexpr (PREC == 1) {
            const float *f = reinterpret_cast<const float *>(frag);
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int s = 0; s < KS; ++s) bf32[p][s] = f[(p * KS + s) * 64 + lane];
        } else {
            const bf16x8 *f = reinterpret_cast<const bf16x8 *>(frag);
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int s = 0; s < KS; ++s)
#pragma unroll
                    for (int hl = 0; hl < 2; ++hl) bbf[p][s][hl] = f[((p * KS + s) * 2 + hl) * 64 + lane];
        }
        const uint32_t Fcol = deposit((uint32_t)r, bp.qpos, K); // this lane's output amplitude
        const uint32_t Grow = deposit((uint32_t)r, bp.gpos, bp.ng);
        for (uint32_t wt = wave; wt < n_wt; wt += nwaves) {
            const uint32_t gw = deposit(wt * ROWS, bp.gpos, bp.ng);
            const uint32_t arow = gw | Grow;
            accT yr = {}, yi = {};
            if constexpr (PREC == 1) {
                // K index q = KS/2 ... : first half Re, second half Im of amp j
                constexpr int half = KS / 2;
                constexpr int per = ROWS == 32 ? 2 : 4; // K per MFMA
#pragma unroll
                for (int s = 0; s < half; ++s) {
                    const int j = per * s + kk;
                    const cpx<float> x = lds[arow | deposit((uint32_t)j, bp.qpos, K)];
                    if constexpr (ROWS == 32) {
                        yr = __builtin_amdgcn_mfma_f32_32x32x2f32(x.re, bf32[0][s], yr, 0, 0, 0);
                        yi = __builtin_amdgcn_mfma_f32_32x32x2f32(x.re, bf32[1][s], yi, 0, 0, 0);
                        yr = __builtin_amdgcn_mfma_f32_32x32x2f32(x.im, bf32[0][s + half], yr, 0, 0, 0);
                        yi = __builtin_amdgcn_mfma_f32_32x32x2f32(x.im, bf32[1][s + half], yi, 0, 0, 0);
                    } else {
                        yr = __builtin_amdgcn_mfma_f32_16x16x4f32(x.re, bf32[0][s], yr, 0, 0, 0);
                        yi = __builtin_amdgcn_mfma_f32_16x16x4f32(x.re, bf32[1][s], yi, 0, 0, 0);
                        yr = __builtin_amdgcn_mfma_f32_16x16x4f32(x.im, bf32[0][s + half], yr, 0, 0, 0);
                        yi = __builtin_amdgcn_mfma_f32_16x16x4f32(x.im, bf32[1][s + half], yi, 0, 0, 0);
                    }
                }
            } else {
                if constexpr (ROWS == 32) {
                    // K-step s < 2: Re of amps 16s + 8kk + e; s >= 2: Im of the same amps
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2) {
                        bf16x8 rh, rl, ih, il;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const int j = 16 * s2 + 8 * kk + e;
                            const cpx<float> x = lds[arow | deposit((uint32_t)j, bp.qpos, K)];
                            const __bf16 a = bf16_hi(x.re), b = bf16_hi(x.im);
                            rh[e] = a;
                            rl[e] = bf16_lo(x.re, a);
                            ih[e] = b;
                            il[e] = bf16_lo(x.im, b);
                        }
#pragma unroll
                        for (int p = 0; p < 2; ++p) {
                            accT &acc = p == 0 ? yr : yi;
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bbf[p][s2][0], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bbf[p][s2][1], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rl, bbf[p][s2][0], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bbf[p][s2 + 2][0], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bbf[p][s2 + 2][1], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(il, bbf[p][s2 + 2][0], acc, 0, 0, 0);
                        }
                    }
                } else {
                    // one K-step of 32: kk = 0,1 -> Re of amps 8kk + e; kk = 2,3 -> Im of amps 8(kk-2) + e
                    bf16x8 ah, al;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int j = 8 * (kk & 1) + e;
                        const cpx<float> x = lds[arow | deposit((uint32_t)j, bp.qpos, K)];
                        const float c = kk < 2 ? x.re : x.im;
                        const __bf16 a = bf16_hi(c);
                        ah[e] = a;
                        al[e] = bf16_lo(c, a);
                    }
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        accT &acc = p == 0 ? yr : yi;
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bbf[p][0][0], acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bbf[p][0][1], acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bbf[p][0][0], acc, 0, 0, 0);
                    }
                }
            }
            // D[row][col]: col = r (output amplitude), rows from the accumulator layout
#pragma unroll
            for (int q = 0; q < ACC; ++q) {
                const int row = ROWS == 32 ? 8 * (q / 4) + 4 * kk + (q % 4) : 4 * kk + q;
                const uint32_t g = gw | deposit((uint32_t)row, bp.gpos, bp.ng);
                lds[g | Fcol] = cpx<float>{yr[q], yi[q]};
            }
        }
        __syncthreads();
        } // blocks
        stage_out<float>(v, lds, sp, base, tsize);
        __syncthreads();
    }
    (void)D;
}

// ---------------------------------------------------------------- launch
int fused_tile_qubits(int dtype) { return dtype == SV_C64 ? 13 : 12; }

hipError_t launch_dense_pass(void *amps, int n, int dtype, const TileSpec &sp, int k,
                             const DenseBlock *dev_blocks, int n_blocks, const char *dev_base, int prec,
                             hipStream_t s) {
    const int m = sp.L + sp.K;
    if (m > n || k > m || k < 1 || k > 5 || n_blocks < 1) return hipErrorInvalidValue;
    const uint64_t n_tiles = 1ull << (n - m);
    const size_t lds = (size_t)(1u << m) * (dtype == SV_C64 ? 8 : 16);
    const unsigned grid = (unsigned)std::min<uint64_t>(n_tiles, 1024);
    if (prec != SV_PREC_NATIVE) {
        if (dtype != SV_C64 || k < 4) return hipErrorInvalidValue;
        const int rows = k == 5 ? 32 : 16;
        if (((1u << m) >> k) % rows) return hipErrorInvalidValue; // whole wave-tiles only
#define SV_MFMA_CASE(KK, PP)                                                                       \
    if (k == KK && prec == PP) {                                                                   \
        (void)hipFuncSetAttribute((const void *)k_dense_mfma<KK, PP>,                              \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);           \
        k_dense_mfma<KK, PP><<<grid, kFuseThreads, lds, s>>>((float4 *)amps, sp, m, dev_blocks,    \
                                                             n_blocks, dev_base, n_tiles);         \
        return hipGetLastError();                                                                  \
    }
        SV_MFMA_CASE(5, 1)
        SV_MFMA_CASE(4, 1)
        SV_MFMA_CASE(5, 2)
        SV_MFMA_CASE(4, 2)
#undef SV_MFMA_CASE
        return hipErrorInvalidValue;
    }
#define SV_NATIVE_CASE(TT, VT, KK)                                                                 \
    if (k == KK) {                                                                                 \
        (void)hipFuncSetAttribute((const void *)k_dense_native<TT, KK>,                            \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);           \
        k_dense_native<TT, KK><<<grid, 256, lds, s>>>((VT *)amps, sp, m, dev_blocks, n_blocks,      \
                                                      dev_base, n_tiles);                          \
        return hipGetLastError();                                                                  \
    }
    if (dtype == SV_C64) {
        SV_NATIVE_CASE(float, float4, 1)
        SV_NATIVE_CASE(float, float4, 2)
        SV_NATIVE_CASE(float, float4, 3)
        SV_NATIVE_CASE(float, float4, 4)
        SV_NATIVE_CASE(float, float4, 5)
    } else {
        SV_NATIVE_CASE(double, double2, 1)
        SV_NATIVE_CASE(double, double2, 2)
        SV_NATIVE_CASE(double, double2, 3)
        SV_NATIVE_CASE(double, double2, 4)
        SV_NATIVE_CASE(double, double2, 5)
    }
#undef SV_NATIVE_CASE
    return hipErrorInvalidValue;
}

} // namespace sv
