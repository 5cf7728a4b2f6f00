// Adjoint-method gradient kernels.
//
// With psi the circuit output and lam = H psi for a diagonal observable H,
// the reverse sweep undoes the gates, last first, on both vectors.  For a
// parametrised gate U(theta) whose derivative is U' = c M U (c a constant,
// M a 2x2 "probe": the Pauli of a rotation, or the projector |1><1| of the
// phase gate) the gradient term 2 Re <lam| U' |psi_before> equals a real
// multiple of Im <lam| M |psi_after>, evaluated on the vectors before the
// gate is undone.  The sweep runs as tile passes over both vectors staged in
// LDS; each probe's FP64 partial sums go to one slot per gate.
#include "sv_internal.hpp"
#include "tile_sweep.hpp"

#include <algorithm>

namespace sv {

constexpr int kAdjThreads = 256;

template <typename T>
struct AV;
template <>
struct AV<float> {
    using type = float4;
    static constexpr int amps = 2, bits = 1;
    __device__ static cpx<float> get(const float4 &v, int k) {
        return k == 0 ? cpx<float>{v.x, v.y} : cpx<float>{v.z, v.w};
    }
    __device__ static void put(float4 &v, int k, cpx<float> c) {
        if (k == 0) { v.x = c.re; v.y = c.im; } else { v.z = c.re; v.w = c.im; }
    }
};
template <>
struct AV<double> {
    using type = double2;
    static constexpr int amps = 1, bits = 0;
    __device__ static cpx<double> get(const double2 &v, int) { return {v.x, v.y}; }
    __device__ static void put(double2 &v, int, cpx<double> c) { v.x = c.re; v.y = c.im; }
};

// x of another lane of the same 16-lane row, moved by DPP (both halves of
// the double; no LDS round trip)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_f64(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, in a fixed order: within each row of 16 lanes by
// rotations of 8 and 4 and quad swaps of 2 and 1 (every lane then holds its
// row's sum), then the four rows' sums; every lane returns the total.
__device__ __forceinline__ double wave_sum_d(double x) {
    x += dpp_f64<0x128>(x); // row_ror:8
    x += dpp_f64<0x124>(x); // row_ror:4
    x += dpp_f64<0x4E>(x);  // quad_perm [2,3,0,1]
    x += dpp_f64<0xB1>(x);  // quad_perm [1,0,3,2]
    return (lane_f64(x, 0) + lane_f64(x, 16)) + (lane_f64(x, 32) + lane_f64(x, 48));
}

__device__ __forceinline__ double block_sum_d(double x) {
    __shared__ double sh[kAdjThreads / 64];
    x = wave_sum_d(x);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = x;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kAdjThreads / 64; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// Im(conj(y) z) in FP64
template <typename T>
__device__ __forceinline__ double im_conj_mul(cpx<T> y, cpx<T> z) {
    return (double)y.re * (double)z.im - (double)y.im * (double)z.re;
}

// lam = h(x) psi, loss partial = sum h(x) |psi_x|^2, h(x) = sum_j c_j (-1)^popcount(x & m_j)
struct AdjTerms {
    int n;
    uint64_t mask[kMaxTerms];
    double coeff[kMaxTerms];
};

template <typename T>
__global__ __launch_bounds__(kAdjThreads) void k_adjoint_init(const typename AV<T>::type *__restrict__ psi,
                                                              typename AV<T>::type *__restrict__ lam,
                                                              uint64_t n_vec, AdjTerms t,
                                                              double *partials) {
    using V = AV<T>;
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kAdjThreads;
    for (uint64_t e = (uint64_t)blockIdx.x * kAdjThreads + threadIdx.x; e < n_vec; e += stride) {
        const typename V::type w = psi[e];
        typename V::type o;
#pragma unroll
        for (int k = 0; k < V::amps; ++k) {
            const uint64_t x = (e << V::bits) | (uint64_t)k;
            double h = 0.0;
            for (int j = 0; j < t.n; ++j) h += (__popcll(x & t.mask[j]) & 1) ? -t.coeff[j] : t.coeff[j];
            const cpx<T> a = V::get(w, k);
            V::put(o, k, cpx<T>{(T)(h * (double)a.re), (T)(h * (double)a.im)});
            acc += h * ((double)a.re * a.re + (double)a.im * a.im);
        }
        lam[e] = o;
    }
    acc = block_sum_d(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// Sum each slot's partials: out[s] = sum_b partials[s * n_blocks + b].
__global__ __launch_bounds__(kAdjThreads) void k_sum_slots(const double *partials, int n_blocks,
                                                           double *out) {
    double acc = 0.0;
    const double *p = partials + (size_t)blockIdx.x * n_blocks;
    for (int i = threadIdx.x; i < n_blocks; i += kAdjThreads) acc += p[i];
    acc = block_sum_d(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// Workgroups of the adjoint launches (each owns at least one tile and writes
// one partial per slot): more of them than fit at once, so that tiles are
// handed out as workgroups finish; at 24 qubits one tile each (measured:
// 24.9 ms per loss and gradient against 25.3 with 4096 workgroups and 26.5
// with 768 looping ones).
int adjoint_blocks() { return 8192; }

hipError_t launch_adjoint_init(const void *psi, void *lam, int n, int dtype, int n_terms,
                               const uint64_t *masks, const double *coeffs, double *partials,
                               hipStream_t s) {
    if (n_terms < 1 || n_terms > kMaxTerms) return hipErrorInvalidValue;
    AdjTerms t{};
    t.n = n_terms;
    for (int j = 0; j < n_terms; ++j) {
        t.mask[j] = masks[j];
        t.coeff[j] = coeffs[j];
    }
    const uint64_t N = 1ull << n;
    const unsigned grid = (unsigned)adjoint_blocks();
    if (dtype == SV_C64)
        k_adjoint_init<float><<<grid, kAdjThreads, 0, s>>>((const float4 *)psi, (float4 *)lam, N / 2, t,
                                                            partials);
    else
        k_adjoint_init<double><<<grid, kAdjThreads, 0, s>>>((const double2 *)psi, (double2 *)lam, N, t,
                                                             partials);
    return hipGetLastError();
}

// ------------------------------------------------------ tiled reverse sweep
// Both vectors of a tile sit in LDS; each register sweep loads the same group
// of psi and lam and undoes the sweep's gates on both.  A parametrised gate
// is preceded by a probe record that adds the group's share of
// Im <lam| M |psi> to the gate's slot (wave reduction, then lane 0 adds it
// to its wave's row of slots).  The slot sums of a workgroup cover all its
// tiles and are written once at the end.
int adjoint_tile_qubits(int dtype) { return dtype == SV_C64 ? 12 : 11; } // 2 x 32 KiB of LDS

// Re(conj(y) z) in FP64
template <typename T>
__device__ __forceinline__ double re_conj_mul(cpx<T> y, cpx<T> z) {
    return (double)y.re * (double)z.re + (double)y.im * (double)z.im;
}

// The pair (j, c = j | 2^P) of psi (v) and lam (w): Im(conj(w_j) z_0) +
// Im(conj(w_c) z_1) with z = M (v_j, v_c).  For M = X: z = (v_c, v_j); Y:
// (-i v_c, i v_j), so Im(conj(w) (+-i) v) = +-Re(conj(w) v); Z: (v_j, -v_c);
// |1><1|: (0, v_c).
template <typename T, int KIND>
__device__ __forceinline__ double probe_pair(const cpx<T> &vj, const cpx<T> &vc, const cpx<T> &wj,
                                             const cpx<T> &wc, const TileGate &G) {
    if constexpr (KIND == SK_PROBE_X) {
        return im_conj_mul(wj, vc) + im_conj_mul(wc, vj);
    } else if constexpr (KIND == SK_PROBE_Y) {
        return re_conj_mul(wc, vj) - re_conj_mul(wj, vc);
    } else if constexpr (KIND == SK_PROBE_Z) {
        return im_conj_mul(wj, vj) - im_conj_mul(wc, vc);
    } else if constexpr (KIND == SK_PROBE_P1) {
        return im_conj_mul(wc, vc);
    } else {
        const cpx<T> m0 = gmat<T>(G, 0), m1 = gmat<T>(G, 1), m2 = gmat<T>(G, 2), m3 = gmat<T>(G, 3);
        const cpx<T> z0 = cfma(m0, vj, cmul(m1, vc));
        const cpx<T> z1 = cfma(m2, vj, cmul(m3, vc));
        return im_conj_mul(wj, z0) + im_conj_mul(wc, z1);
    }
}

template <typename T, int W, int P, int KIND>
__device__ __forceinline__ double probe_pos(const cpx<T> (&v)[1 << W], const cpx<T> (&w)[1 << W],
                                            uint32_t gb, const TileGate &G) {
    constexpr int D = 1 << W;
    double acc = 0.0;
    if ((gb & G.lane) != G.lane) return acc;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (j & (1 << P)) continue;
        if (!((G.amask >> j) & 1u)) continue;
        const int c = j | (1 << P);
        acc += probe_pair<T, KIND>(v[j], v[c], w[j], w[c], G);
    }
    return acc;
}

template <typename T, int W, int KIND>
__device__ __forceinline__ double probe_kind(const cpx<T> (&v)[1 << W], const cpx<T> (&w)[1 << W],
                                             uint32_t gb, const TileGate &G) {
    const int p = G.b0;
    if (p == 0) return probe_pos<T, W, 0, KIND>(v, w, gb, G);
    if constexpr (W >= 2) if (p == 1) return probe_pos<T, W, 1, KIND>(v, w, gb, G);
    if constexpr (W >= 3) if (p == 2) return probe_pos<T, W, 2, KIND>(v, w, gb, G);
    if constexpr (W >= 4) if (p == 3) return probe_pos<T, W, 3, KIND>(v, w, gb, G);
    return 0.0;
}

__device__ __forceinline__ bool is_probe(int kind) {
    return kind == SK_PARAM || (kind >= SK_PROBE_X && kind <= SK_PROBE_P1);
}

template <typename T, int W>
__device__ __forceinline__ double probe_gate(const cpx<T> (&v)[1 << W], const cpx<T> (&w)[1 << W],
                                             uint32_t gb, const TileGate &G) {
    switch (G.kind) {
    case SK_PROBE_X: return probe_kind<T, W, SK_PROBE_X>(v, w, gb, G);
    case SK_PROBE_Y: return probe_kind<T, W, SK_PROBE_Y>(v, w, gb, G);
    case SK_PROBE_Z: return probe_kind<T, W, SK_PROBE_Z>(v, w, gb, G);
    case SK_PROBE_P1: return probe_kind<T, W, SK_PROBE_P1>(v, w, gb, G);
    default: return probe_kind<T, W, SK_PARAM>(v, w, gb, G);
    }
}

template <typename T, int W, bool TWOQ>
__global__ __launch_bounds__(kAdjThreads) void k_adjoint_tile(typename AV<T>::type *psi, typename AV<T>::type *lam,
                                                      TileSpec sp, int m, const TileSweep *__restrict__ sweeps,
                                                      int n_sweeps, const char *__restrict__ recs,
                                                      int slot0, int n_slots, double *partials,
                                                      uint64_t n_tiles) {
    constexpr int D = 1 << W;
    extern __shared__ char lds_raw[];
    const uint32_t tsize = 1u << m;
    // one LDS tile, used by psi and then by lam at each exchange (half the
    // LDS of a tile per vector: more workgroups per CU)
    cpx<T> *lt = reinterpret_cast<cpx<T> *>(lds_raw);
    // one row of slot sums per wave, written only by that wave's lane 0 (no
    // atomics): the workgroup's sums are then formed in a fixed order and the
    // gradient is the same bit for bit on every run
    constexpr int kWaves = kAdjThreads / 64;
    __shared__ double slot_acc[kWaves][kMaxAdjSlots];
    for (int i = threadIdx.x; i < kWaves * kMaxAdjSlots; i += blockDim.x) (&slot_acc[0][0])[i] = 0.0;
    __syncthreads();
    // one register group per thread (at most blockDim groups, checked at
    // launch); a thread past the last group holds zeros, adds 0 to the
    // probes' wave sums and takes part in every barrier
    const uint32_t n_groups = tsize >> W;
    const uint32_t g = threadIdx.x;
    const bool act = g < n_groups;
    cpx<T> *ps = reinterpret_cast<cpx<T> *>(psi);
    cpx<T> *ls = reinterpret_cast<cpx<T> *>(lam);
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        uint64_t base = tile << sp.L;
        for (int i = 0; i < sp.K; ++i) base = insert_zero(base, sp.high[i]);
        // psi's group in vw[0, D), lam's in vw[D, 2D): one record walk
        // applies each gate to both, as a gate on W + 1 register positions
        // whose top position (the vector) no gate targets.  The first sweep
        // reads both groups straight from HBM and the last writes them
        // straight back; between sweeps the groups move to the next sweep's
        // register layout through the LDS tile, psi first, then lam.
        cpx<T> vw[2 * D];
        cpx<T>(&v)[D] = *reinterpret_cast<cpx<T>(*)[D]>(&vw[0]);
        cpx<T>(&w)[D] = *reinterpret_cast<cpx<T>(*)[D]>(&vw[D]);
        PhaseAcc<T, W + 1> acc_unused;
        acc_unused.init();
        for (int si = 0; si < n_sweeps; ++si) {
            const TileSweep &S = sweeps[si];
            const int ng = S.n_gates;
            const bool first = si == 0, last = si == n_sweeps - 1;
            const uint32_t gb = group_bits<W>(S, act ? g : 0u);
            const uint64_t row = base | tile_offset(sp, gb);
            uint64_t gbit[W];
#pragma unroll
            for (int b = 0; b < W; ++b) gbit[b] = tile_offset(sp, 1u << S.qpos[b]);
            auto goff_of = [&](int j) {
                uint64_t o = 0;
#pragma unroll
                for (int b = 0; b < W; ++b)
                    if ((j >> b) & 1) o |= gbit[b];
                return o;
            };
            if (first) {
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    v[j] = act ? ps[row | goff_of(j)] : cpx<T>{T(0), T(0)};
                    w[j] = act ? ls[row | goff_of(j)] : cpx<T>{T(0), T(0)};
                }
            }
            const char *rp = recs + S.rec_off;
            for (int gi = 0; gi < ng; ++gi) {
                const TileGate &G = *reinterpret_cast<const TileGate *>(rp);
                rp += G.size;
                if (is_probe(G.kind)) {
                    if ((base & G.cout) != G.cout) continue; // uniform
                    const double mine = act ? probe_gate<T, W>(v, w, gb, G) : 0.0;
                    const double c = wave_sum_d(mine);
                    if ((threadIdx.x & 63) == 0) slot_acc[threadIdx.x >> 6][G.b1] += c;
                } else {
                    // adjoint passes carry no gathered phases (their probes
                    // read the amplitudes between gates); the register-index
                    // mask repeats for lam's half
                    GateHot h = *reinterpret_cast<const GateHot *>(&G);
                    h.amask |= h.amask << D;
                    sweep_gate_h<T, W + 1, TWOQ, false>(vw, acc_unused, gb, h, G, base);
                }
            }
            if (last) {
                if (act) {
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        ps[row | goff_of(j)] = v[j];
                        ls[row | goff_of(j)] = w[j];
                    }
                }
            } else {
                const TileSweep &N = sweeps[si + 1];
                uint32_t PF[D], PN[D];
                register_offsets<T, W>(S, PF);
                register_offsets<T, W>(N, PN);
                const uint32_t pg = lds_phys<T>(gb);
                const uint32_t pn = lds_phys<T>(group_bits<W>(N, act ? g : 0u));
                // each barrier orders one vector's writes before its reads,
                // and its reads before the next writes to the tile
                if (act) {
#pragma unroll
                    for (int j = 0; j < D; ++j) lt[pg ^ PF[j]] = v[j];
                }
                __syncthreads();
                if (act) {
#pragma unroll
                    for (int j = 0; j < D; ++j) v[j] = lt[pn ^ PN[j]];
                }
                __syncthreads();
                if (act) {
#pragma unroll
                    for (int j = 0; j < D; ++j) lt[pg ^ PF[j]] = w[j];
                }
                __syncthreads();
                if (act) {
#pragma unroll
                    for (int j = 0; j < D; ++j) w[j] = lt[pn ^ PN[j]];
                }
                __syncthreads();
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_slots; i += blockDim.x) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += slot_acc[w][i];
        partials[(size_t)(slot0 + i) * gridDim.x + blockIdx.x] = t;
    }
}

hipError_t launch_adjoint_tile(void *psi, void *lam, int n, int dtype, const TileSpec &spec,
                               const TileSweep *dev_sweeps, int n_sweeps, const char *dev_gates,
                               int slot0, int n_slots, double *partials, int n_blocks, bool two_qubit,
                               hipStream_t s) {
    const int m = spec.L + spec.K;
    const int vbits = dtype == SV_C64 ? 1 : 0;
    if (m > n || m > adjoint_tile_qubits(dtype) || spec.L < vbits || n_slots > kMaxAdjSlots || m < 1)
        return hipErrorInvalidValue;
    const uint64_t n_tiles = 1ull << (n - m);
    if ((uint64_t)n_blocks > n_tiles) return hipErrorInvalidValue; // every workgroup owns a tile
    const size_t lds = (size_t)(1u << m) * (dtype == SV_C64 ? 8 : 16);
    const int W = std::min(m, sweep_width(dtype));
    if (((1u << m) >> W) > (unsigned)kAdjThreads) return hipErrorInvalidValue; // one group per thread
#define SV_ADJ_CASE(TT, VT, WW)                                                                    \
    if (W == WW) {                                                                                 \
        if (two_qubit) {                                                                           \
            (void)hipFuncSetAttribute((const void *)k_adjoint_tile<TT, WW, true>,                  \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);       \
            k_adjoint_tile<TT, WW, true><<<n_blocks, 256, lds, s>>>(                               \
                (VT *)psi, (VT *)lam, spec, m, dev_sweeps, n_sweeps, dev_gates, slot0, n_slots,    \
                partials, n_tiles);                                                                \
        } else {                                                                                   \
            (void)hipFuncSetAttribute((const void *)k_adjoint_tile<TT, WW, false>,                 \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);       \
            k_adjoint_tile<TT, WW, false><<<n_blocks, 256, lds, s>>>(                              \
                (VT *)psi, (VT *)lam, spec, m, dev_sweeps, n_sweeps, dev_gates, slot0, n_slots,    \
                partials, n_tiles);                                                                \
        }                                                                                          \
        return hipGetLastError();                                                                  \
    }
    if (dtype == SV_C64) {
        SV_ADJ_CASE(float, float4, 4)
        SV_ADJ_CASE(float, float4, 3)
        SV_ADJ_CASE(float, float4, 2)
        SV_ADJ_CASE(float, float4, 1)
    } else {
        SV_ADJ_CASE(double, double2, 3)
        SV_ADJ_CASE(double, double2, 2)
        SV_ADJ_CASE(double, double2, 1)
    }
#undef SV_ADJ_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_sum_slots(const double *partials, int n_slots, int n_blocks, double *out,
                            hipStream_t s) {
    if (n_slots <= 0) return hipSuccess;
    k_sum_slots<<<n_slots, kAdjThreads, 0, s>>>(partials, n_blocks, out);
    return hipGetLastError();
}

} // namespace sv
