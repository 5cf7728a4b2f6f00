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
#include "tile_sweep.hpp"

#include <algorithm>

namespace sv {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kFuseThreads = 512;

__device__ __forceinline__ uint32_t deposit(uint32_t x, const int *pos, int nbits) {
    uint32_t r = 0;
    for (int b = 0; b < nbits; ++b)
        if ((x >> b) & 1u) r |= 1u << pos[b];
    return r;
}

// Tile index mapping and swizzled LDS layout are those of the gate tile
// pass (lds_phys is linear over XOR, so the address of a deposit of
// disjoint index parts is the XOR of the parts' addresses).
__device__ __forceinline__ uint64_t tile_base(const TileSpec &sp, uint64_t tile) {
    uint64_t base = tile << sp.L;
    for (int i = 0; i < sp.K; ++i) base = insert_zero(base, sp.high[i]);
    return base;
}

// Byte offset of the operand variant a block uses in the tile at 'base':
// bit i of the variant index is the tile's value of the i-th lowest qubit of
// the block's vmask (qubits outside the tile, fixed within it).  Uniform per
// tile, so it stays on the scalar unit.
__device__ __forceinline__ int64_t variant_offset(const DenseBlock &B, uint64_t base) {
    uint32_t v = 0;
    int i = 0;
    for (uint64_t vm = B.vmask; vm; vm &= vm - 1, ++i) v |= (uint32_t)((base >> __builtin_ctzll(vm)) & 1ull) << i;
    return (int64_t)v * B.vstride;
}

// ------------------------------------------------- native (vector ALU)
// One thread per group: the 2^K amplitudes go to registers, every output is
// a dot product with a row of U (uniform across the wave, read through the
// scalar cache), written back to the group's own LDS slots.  The blocks of a
// pass are applied one after another to the staged tile.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_dense_native(typename Amp16<T>::type *v, TileSpec sp, int m,
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
        tile_load<T, 256, 8>(v, lds, sp, base, tsize);
        __syncthreads();
        for (int b = 0; b < n_blocks; ++b) {
            const DenseBlock &B = blocks[b];
            const cpx<T> *U = reinterpret_cast<const cpx<T> *>(base_ptr + B.op_off + variant_offset(B, base));
            uint32_t PF[D];
#pragma unroll
            for (int j = 0; j < D; ++j) PF[j] = lds_phys<T>(deposit((uint32_t)j, B.bp.qpos, K));
            for (uint32_t g = threadIdx.x; g < n_groups; g += blockDim.x) {
                const uint32_t pg = lds_phys<T>(deposit(g, B.bp.gpos, B.bp.ng));
                cpx<T> x[D];
#pragma unroll
                for (int j = 0; j < D; ++j) x[j] = lds[pg ^ PF[j]];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    cpx<T> acc = cmul(U[i * D], x[0]);
#pragma unroll
                    for (int j = 1; j < D; ++j) acc = cfma(U[i * D + j], x[j], acc);
                    lds[pg ^ PF[i]] = acc;
                }
            }
            __syncthreads();
        }
        tile_store<T, 256, 8>(v, lds, sp, base, tsize);
        __syncthreads();
    }
}

// ------------------------------------------------------------ matrix cores
// All matrix-core kernels share one addressing scheme.  A wave-tile is ROWS
// groups (MFMA rows) of one block; the group index of row i of wave-tile wt
// is wt*ROWS + i, and its LDS offset is goff_hi[wt] ^ goff_lo[i] since the
// two parts have disjoint bits (the host stores qoff[2^K], goff_lo[ROWS],
// goff_hi[groups / ROWS] consecutively).  So every A-operand and result
// address is a per-lane constant (set once per block) XOR a wave-uniform
// table entry.
//
// Operand fragments (host-built, per lane, in the MFMA B-operand order):
//   split-BF16: frag[((part * KS + s) * 2 + hl) * 64 + lane]   (bf16x8)
//   FP32:       frag[(part * KS + s) * 64 + lane]               (float)
//   FP64:       frag[((part * NT + nt) * KS + s) * 64 + lane]   (double)
// part 0 -> Re Y, part 1 -> Im Y; hl 0 = hi, 1 = lo.  Split-BF16 orders the
// real K index as (amplitude, re/im) interleaved, so a lane's 8 operand
// elements are the real and imaginary parts of 4 amplitudes; FP32 and FP64
// order it [Re x | Im x].

// x ~ hi + lo with hi = bf16(x) and lo = bf16(x - hi)
__device__ __forceinline__ __bf16 bf16_hi(float x) { return (__bf16)x; }
__device__ __forceinline__ __bf16 bf16_lo(float x, __bf16 hi) { return (__bf16)(x - (float)hi); }

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Split-BF16 operands of 4 amplitudes (elements 2i, 2i+1 = re, im of x_i).
__device__ __forceinline__ void split4(const cpx<float> (&x)[4], bf16x8 &h, bf16x8 &l) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const __bf16 a = bf16_hi(x[i].re), c = bf16_hi(x[i].im);
        h[2 * i] = a;
        h[2 * i + 1] = c;
        l[2 * i] = bf16_lo(x[i].re, a);
        l[2 * i + 1] = bf16_lo(x[i].im, c);
    }
}

// Where a block reads its operands and writes its results: the tile in LDS
// (swizzled offsets qoff[2^K], goff = goff_lo[ROWS] then goff_hi) or the
// state itself (global offsets gq, gg in the same layout, OR-combined with
// the tile's base index).  The first block of a pass can read the state and
// the last one write it, so that the tile crosses LDS only between blocks.
struct BlockTabs {
    const uint32_t *qoff, *goff;
    const uint64_t *gq, *gg;
};

template <typename T, bool G>
__device__ __forceinline__ cpx<T> blk_load(const cpx<T> *lds, const cpx<T> *state, uint32_t l, uint64_t g) {
    if constexpr (G) return state[g];
    else return lds[l];
}
template <typename T, bool G>
__device__ __forceinline__ void blk_store(cpx<T> *lds, cpx<T> *state, uint32_t l, uint64_t g, cpx<T> x) {
    if constexpr (G) state[g] = x;
    else lds[l] = x;
}

// The MFMA operand lane layouts are mirror images (A lane l holds
// A[l % R][k(l)], B lane l holds B[k(l)][l % R]), so the fragments, laid
// out as the B operand of Y = X B, serve unchanged as the A operand of
// Y^T = B^T X^T.  The kernels compute that transposed product: the result
// a lane holds is then its own operand row (group), at block indices that
// differ from its operand indices only in fixed bits, and a quarter-wave
// writes consecutive groups.

// complex64, split-BF16 (3 products, FP32 accumulate).  K = 4: 16x16x32,
// one K-step; K = 5: 32x32x16, four K-steps.
template <int K>
struct Bf16Cfg;
template <>
struct Bf16Cfg<4> {
    static constexpr int rows = 16, ksteps = 1, threads = 512;
};
template <>
struct Bf16Cfg<5> {
    static constexpr int rows = 32, ksteps = 4, threads = 256;
};

// One block applied to the tile by this wave's wave-tiles.  f points to the
// block's operand fragments.
template <int K, bool SG, bool DG>
__device__ __forceinline__ void block_bf16(cpx<float> *lds, cpx<float> *state, uint64_t base, const bf16x8 *f,
                                           const BlockTabs &t, uint32_t n_wt, int wave, int nwaves) {
    using C = Bf16Cfg<K>;
    constexpr int ROWS = C::rows, KS = C::ksteps;
    constexpr int ACC = ROWS == 32 ? 16 : 4;
    using accT = typename std::conditional<ROWS == 32, floatx16, floatx4>::type;
    const int lane = threadIdx.x & 63;
    const int r = lane % ROWS, kk = lane / ROWS;
    bf16x8 bw[2][KS][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int hl = 0; hl < 2; ++hl) bw[p][s][hl] = f[((p * KS + s) * 2 + hl) * 64 + lane];
    // lane (r, kk) reads block indices 4kk + 8s + i of row r and holds the
    // results of row r at 4kk + q (16x16) or 4kk + 8(q/4) + q%4 (32x32)
    const uint32_t l_lane = t.goff[r] ^ t.qoff[4 * kk];
    const uint64_t g_lane = base | t.gg[r] | t.gq[4 * kk];
    for (uint32_t wt = wave; wt < n_wt; wt += nwaves) {
        const uint32_t lw = t.goff[ROWS + wt] ^ l_lane; // goff_hi[wt]
        const uint64_t gw = t.gg[ROWS + wt] | g_lane;
        accT yr = {}, yi = {};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            cpx<float> x[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                x[i] = blk_load<float, SG>(lds, state, lw ^ t.qoff[8 * s + i], gw | t.gq[8 * s + i]);
            bf16x8 h, l;
            split4(x, h, l);
            if constexpr (ROWS == 32) {
                yr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bw[0][s][0], h, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bw[1][s][0], h, yi, 0, 0, 0);
                yr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bw[0][s][1], h, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bw[1][s][1], h, yi, 0, 0, 0);
                yr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bw[0][s][0], l, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bw[1][s][0], l, yi, 0, 0, 0);
            } else {
                yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[0][s][0], h, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[1][s][0], h, yi, 0, 0, 0);
                yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[0][s][1], h, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[1][s][1], h, yi, 0, 0, 0);
                yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[0][s][0], l, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[1][s][0], l, yi, 0, 0, 0);
            }
        }
#pragma unroll
        for (int q = 0; q < ACC; ++q) {
            const int c = ROWS == 32 ? 8 * (q / 4) + (q % 4) : q;
            blk_store<float, DG>(lds, state, lw ^ t.qoff[c], gw | t.gq[c], cpx<float>{yr[q], yi[q]});
        }
    }
}

// complex64, FP32 (v_mfma_f32_16x16x4_f32 for K = 4, 32x32x2 for K = 5).
// K-step s uses element s*KPS + kk of [Re x | Im x]: the lane loads
// amplitude KPS*s + kk once and uses its real part at step s and its
// imaginary part at step s + KS/2.
template <int K>
struct F32Cfg;
template <>
struct F32Cfg<4> {
    static constexpr int rows = 16, kps = 4, threads = 512;
};
template <>
struct F32Cfg<5> {
    static constexpr int rows = 32, kps = 2, threads = 256;
};

template <int K, bool SG, bool DG>
__device__ __forceinline__ void block_f32(cpx<float> *lds, cpx<float> *state, uint64_t base, const float *f,
                                          const BlockTabs &t, uint32_t n_wt, int wave, int nwaves) {
    using C = F32Cfg<K>;
    constexpr int D = 1 << K, ROWS = C::rows, KPS = C::kps;
    constexpr int KS = 2 * D / KPS, HALF = KS / 2;
    constexpr int ACC = ROWS == 32 ? 16 : 4;
    using accT = typename std::conditional<ROWS == 32, floatx16, floatx4>::type;
    const int lane = threadIdx.x & 63;
    const int r = lane % ROWS, kk = lane / ROWS;
    float bw[2][KS];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int s = 0; s < KS; ++s) bw[p][s] = f[(p * KS + s) * 64 + lane];
    // reads: index kk + KPS*s of row r; results: 4kk + q (16x16) or
    // 4kk + 8(q/4) + q%4 (32x32) of row r
    const uint32_t la = t.goff[r] ^ t.qoff[kk], lo = t.goff[r] ^ t.qoff[4 * kk];
    const uint64_t ga = base | t.gg[r] | t.gq[kk], go = base | t.gg[r] | t.gq[4 * kk];
    for (uint32_t wt = wave; wt < n_wt; wt += nwaves) {
        const uint32_t lh = t.goff[ROWS + wt];
        const uint64_t gh = t.gg[ROWS + wt];
        accT yr = {}, yi = {};
#pragma unroll
        for (int s = 0; s < HALF; ++s) {
            const cpx<float> x = blk_load<float, SG>(lds, state, lh ^ la ^ t.qoff[KPS * s], gh | ga | t.gq[KPS * s]);
            if constexpr (ROWS == 32) {
                yr = __builtin_amdgcn_mfma_f32_32x32x2f32(bw[0][s], x.re, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_32x32x2f32(bw[1][s], x.re, yi, 0, 0, 0);
                yr = __builtin_amdgcn_mfma_f32_32x32x2f32(bw[0][s + HALF], x.im, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_32x32x2f32(bw[1][s + HALF], x.im, yi, 0, 0, 0);
            } else {
                yr = __builtin_amdgcn_mfma_f32_16x16x4f32(bw[0][s], x.re, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_16x16x4f32(bw[1][s], x.re, yi, 0, 0, 0);
                yr = __builtin_amdgcn_mfma_f32_16x16x4f32(bw[0][s + HALF], x.im, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_16x16x4f32(bw[1][s + HALF], x.im, yi, 0, 0, 0);
            }
        }
#pragma unroll
        for (int q = 0; q < ACC; ++q) {
            const int c = ROWS == 32 ? 8 * (q / 4) + (q % 4) : q;
            blk_store<float, DG>(lds, state, lh ^ lo ^ t.qoff[c], gh | go | t.gq[c], cpx<float>{yr[q], yi[q]});
        }
    }
}

// complex128 on the FP64 matrix cores (v_mfma_f64_16x16x4f64; result
// element q of lane l is row 4q + l/16, column l%16, as measured on the
// device): wave-tiles of 16 groups, D/16 output tiles of 16 amplitudes per
// part, K-steps as in the FP32 kernel.  Fragments stay in registers for
// K = 4 and are read per K-step for K = 5.
template <int K, bool SG, bool DG>
__device__ __forceinline__ void block_f64(cpx<double> *lds, cpx<double> *state, uint64_t base,
                                          const double *frag, const BlockTabs &t, uint32_t n_wt, int wave,
                                          int nwaves) {
    constexpr int D = 1 << K;
    constexpr int NT = D / 16;
    constexpr int KS = 2 * D / 4;
    constexpr int HALF = KS / 2;
    constexpr bool PRELOAD = K == 4;
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, kk = lane >> 4;
    double bpre[PRELOAD ? 2 * NT * KS : 1];
    if constexpr (PRELOAD) {
#pragma unroll
        for (int i = 0; i < 2 * NT * KS; ++i) bpre[i] = frag[i * 64 + lane];
    }
    // reads: index kk + 4s of row r; results: kk + 4q + 16nt of row r
    const uint32_t l_lane = t.goff[r] ^ t.qoff[kk];
    const uint64_t g_lane = base | t.gg[r] | t.gq[kk];
    for (uint32_t wt = wave; wt < n_wt; wt += nwaves) {
        const uint32_t lw = t.goff[16 + wt] ^ l_lane; // goff_hi[wt]
        const uint64_t gw = t.gg[16 + wt] | g_lane;
        doublex4 acc[2][NT];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[p][nt] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < HALF; ++s) {
            const cpx<double> x = blk_load<double, SG>(lds, state, lw ^ t.qoff[4 * s], gw | t.gq[4 * s]);
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int i0 = (p * NT + nt) * KS + s, i1 = i0 + HALF;
                    const double b0 = PRELOAD ? bpre[PRELOAD ? i0 : 0] : frag[i0 * 64 + lane];
                    const double b1 = PRELOAD ? bpre[PRELOAD ? i1 : 0] : frag[i1 * 64 + lane];
                    acc[p][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, x.re, acc[p][nt], 0, 0, 0);
                    acc[p][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, x.im, acc[p][nt], 0, 0, 0);
                }
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = 4 * q + 16 * nt;
                blk_store<double, DG>(lds, state, lw ^ t.qoff[c], gw | t.gq[c],
                                      cpx<double>{acc[0][nt][q], acc[1][nt][q]});
            }
    }
}

// Register-staged passes (any tile size; the only path for K = 5): each
// workgroup loads a tile, applies the blocks, stores it.  ENG: SV_PREC_FP32,
// SV_PREC_SPLIT_BF16 (complex64) or kPrecMfma64 (complex128).
template <int ENG, int K>
struct EngCfg {
    using T = typename std::conditional<ENG == kPrecMfma64, double, float>::type;
    static constexpr int rows = ENG == kPrecMfma64 ? 16 : (K == 5 ? 32 : 16);
    static constexpr int threads = ENG == kPrecMfma64 ? 256 : (K == 5 ? 256 : 512);
};

template <int ENG, int K, bool SG, bool DG>
__device__ __forceinline__ void apply_block_t(cpx<typename EngCfg<ENG, K>::T> *lds,
                                              cpx<typename EngCfg<ENG, K>::T> *state, uint64_t base,
                                              const char *op, const BlockTabs &t, uint32_t n_wt, int wave,
                                              int nwaves) {
    if constexpr (ENG == SV_PREC_SPLIT_BF16)
        block_bf16<K, SG, DG>(lds, state, base, reinterpret_cast<const bf16x8 *>(op), t, n_wt, wave, nwaves);
    else if constexpr (ENG == SV_PREC_FP32)
        block_f32<K, SG, DG>(lds, state, base, reinterpret_cast<const float *>(op), t, n_wt, wave, nwaves);
    else
        block_f64<K, SG, DG>(lds, state, base, reinterpret_cast<const double *>(op), t, n_wt, wave, nwaves);
}

template <int ENG, int K>
__global__ __launch_bounds__((EngCfg<ENG, K>::threads)) void k_dense_mfma(
    typename Amp16<typename EngCfg<ENG, K>::T>::type *v, TileSpec sp, int m, const DenseBlock *__restrict__ blocks,
    int n_blocks, const char *__restrict__ base_ptr, uint64_t n_tiles, uint32_t direct) {
    using Cf = EngCfg<ENG, K>;
    using T = typename Cf::T;
    extern __shared__ char lds_raw[];
    cpx<T> *lds = reinterpret_cast<cpx<T> *>(lds_raw);
    cpx<T> *state = reinterpret_cast<cpx<T> *>(v);
    const uint32_t tsize = 1u << m;
    const uint32_t n_wt = (tsize >> K) / Cf::rows;
    const int wave = wave_id(), nwaves = Cf::threads / 64;
    const bool dfirst = direct & kDirectFirst, dlast = direct & kDirectLast;
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint64_t base = tile_base(sp, tile);
        if (!dfirst) {
            tile_load<T, Cf::threads, 8>(v, lds, sp, base, tsize);
            __syncthreads();
        }
        for (int b = 0; b < n_blocks; ++b) {
            const DenseBlock &B = blocks[b];
            const uint32_t *tab = reinterpret_cast<const uint32_t *>(base_ptr + B.tab_off);
            const uint64_t *gtab = reinterpret_cast<const uint64_t *>(base_ptr + B.gtab_off);
            const BlockTabs t{tab, tab + (1 << K), gtab, gtab + (1 << K)};
            const char *op = base_ptr + B.op_off + variant_offset(B, base);
            const bool sg = b == 0 && dfirst, dg = b == n_blocks - 1 && dlast;
            if (sg && dg) apply_block_t<ENG, K, true, true>(lds, state, base, op, t, n_wt, wave, nwaves);
            else if (sg) apply_block_t<ENG, K, true, false>(lds, state, base, op, t, n_wt, wave, nwaves);
            else if (dg) apply_block_t<ENG, K, false, true>(lds, state, base, op, t, n_wt, wave, nwaves);
            else apply_block_t<ENG, K, false, false>(lds, state, base, op, t, n_wt, wave, nwaves);
            // the next block (or the next tile's first LDS writes) follows
            // every wave's reads of this one
            __syncthreads();
        }
        if (!dlast) {
            tile_store<T, Cf::threads, 8>(v, lds, sp, base, tsize);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- launch
int fused_tile_qubits(int dtype) { return dtype == SV_C64 ? 13 : 12; }

hipError_t launch_dense_pass(void *amps, int n, int dtype, const TileSpec &sp, int k,
                             const DenseBlock *dev_blocks, int n_blocks, const char *dev_base, int prec,
                             uint32_t direct, hipStream_t s) {
    const int m = sp.L + sp.K;
    if (m > n || k > m || k < 1 || k > 5 || n_blocks < 1) return hipErrorInvalidValue;
    const uint64_t n_tiles = 1ull << (n - m);
    const size_t lds = (size_t)(1u << m) * (dtype == SV_C64 ? 8 : 16);
    const unsigned grid = (unsigned)std::min<uint64_t>(n_tiles, 1u << 30);
    if (prec != SV_PREC_NATIVE) {
        const bool f64 = prec == kPrecMfma64;
        if (f64 != (dtype == SV_C128) || k < 4) return hipErrorInvalidValue;
        const int rows = (!f64 && k == 5) ? 32 : 16;
        if (((1u << m) >> k) % rows) return hipErrorInvalidValue; // whole wave-tiles only
#define SV_MFMA_CASE(ENG, KK)                                                                      \
    if (prec == ENG && k == KK) {                                                                  \
        using VT = typename Amp16<typename EngCfg<ENG, KK>::T>::type;                              \
        (void)hipFuncSetAttribute((const void *)k_dense_mfma<ENG, KK>,                             \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);           \
        k_dense_mfma<ENG, KK><<<grid, EngCfg<ENG, KK>::threads, lds, s>>>((VT *)amps, sp, m, dev_blocks, \
                                                                         n_blocks, dev_base, n_tiles, \
                                                                         direct);                      \
        return hipGetLastError();                                                                  \
    }
        SV_MFMA_CASE(SV_PREC_SPLIT_BF16, 4)
        SV_MFMA_CASE(SV_PREC_SPLIT_BF16, 5)
        SV_MFMA_CASE(SV_PREC_FP32, 4)
        SV_MFMA_CASE(SV_PREC_FP32, 5)
        SV_MFMA_CASE(kPrecMfma64, 4)
        SV_MFMA_CASE(kPrecMfma64, 5)
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
