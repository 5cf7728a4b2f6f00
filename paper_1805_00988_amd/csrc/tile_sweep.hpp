// Applying a run of gates to a tile of amplitudes staged in LDS.
//
// A tile holds 2^m amplitudes (local index l, m <= 13).  The gates of a pass
// are grouped by the host into sweeps: a sweep names W = 4 local qubit
// positions and a list of gates whose targets lie among them (diagonal
// gates may target any tile position).  For each sweep every thread takes
// groups of 2^W amplitudes that differ only in those positions, holds them
// in registers, applies the sweep's gates in order and writes them back, so
// the tile crosses LDS once per sweep instead of once per gate.
//
// LDS addresses are swizzled (lds_swizzle): positions within one 128-byte
// LDS row (16 complex64 or 8 complex128 amplitudes) are XOR-ed with a fold of
// the row index, so the lanes of a wave, whose groups differ in arbitrary
// tile bits, spread over the banks.
#pragma once

#include "sv_internal.hpp"

#include <cstddef>
#include <type_traits>

namespace sv {


template <typename T>
__device__ __forceinline__ uint32_t lds_phys(uint32_t l) {
    return lds_swizzle(l, 2 * (int)sizeof(T));
}

// ------------------------------------------------------------ tile staging
// 16-byte vectors of amplitudes: two complex64 or one complex128.
template <typename T>
struct Amp16;
template <>
struct Amp16<float> {
    using type = float4;
    static constexpr int bits = 1;
};
template <>
struct Amp16<double> {
    using type = double2;
    static constexpr int bits = 0;
};

// Offset of local amplitude l from the tile's base index: the low L bits in
// place, bit L + i at global position high[i].  The map is linear over the
// OR of parts with disjoint bits.
__device__ __forceinline__ uint64_t tile_offset(const TileSpec &sp, uint32_t l) {
    uint64_t g = l & ((1u << sp.L) - 1u);
    const uint32_t hi = l >> sp.L;
#pragma unroll
    for (int i = 0; i < kMaxTileHigh; ++i) {
        if (i >= sp.K) break;
        if ((hi >> i) & 1u) g |= 1ull << sp.high[i];
    }
    return g;
}

// Copy a tile of tsize amplitudes between the state and the swizzled LDS
// tile with NTH threads.  Thread t moves the 16-byte vectors at local index
// t*VA + r*STRIDE (VA amplitudes per vector, STRIDE = NTH*VA) for rounds r;
// U rounds are issued before any of their results is used, so a lane keeps
// U memory accesses in flight.  Both addresses split into a per-thread part
// and a wave-uniform per-round part (disjoint bits, combined by OR / XOR).
template <typename T, int NTH, int U>
__device__ __forceinline__ void tile_load(const typename Amp16<T>::type *__restrict__ v, cpx<T> *lds,
                                          const TileSpec &sp, uint64_t base, uint32_t tsize) {
    constexpr int vb = Amp16<T>::bits;
    constexpr uint32_t STRIDE = (uint32_t)NTH << vb;
    const uint32_t lt = threadIdx.x << vb;
    const uint64_t gt = base | tile_offset(sp, lt);
    const uint32_t pt = lds_phys<T>(lt);
    for (uint32_t r0 = 0; r0 < tsize; r0 += U * STRIDE) {
        typename Amp16<T>::type w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t ru = r0 + u * STRIDE;
            if (ru + lt < tsize) w[u] = v[(gt | tile_offset(sp, ru)) >> vb];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t ru = r0 + u * STRIDE;
            if (ru + lt < tsize) {
                const uint32_t p = lds_phys<T>(ru) ^ pt;
                lds[p] = cpx<T>{w[u].x, w[u].y};
                if constexpr (vb == 1) lds[p ^ 1u] = cpx<T>{w[u].z, w[u].w};
            }
        }
    }
}

template <typename T, int NTH, int U>
__device__ __forceinline__ void tile_store(typename Amp16<T>::type *__restrict__ v, const cpx<T> *lds,
                                           const TileSpec &sp, uint64_t base, uint32_t tsize) {
    constexpr int vb = Amp16<T>::bits;
    constexpr uint32_t STRIDE = (uint32_t)NTH << vb;
    const uint32_t lt = threadIdx.x << vb;
    const uint64_t gt = base | tile_offset(sp, lt);
    const uint32_t pt = lds_phys<T>(lt);
    for (uint32_t r0 = 0; r0 < tsize; r0 += U * STRIDE) {
        typename Amp16<T>::type w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t ru = r0 + u * STRIDE;
            if (ru + lt < tsize) {
                const uint32_t p = lds_phys<T>(ru) ^ pt;
                const cpx<T> a = lds[p];
                if constexpr (vb == 1) {
                    const cpx<T> b = lds[p ^ 1u];
                    w[u] = typename Amp16<T>::type{a.re, a.im, b.re, b.im};
                } else {
                    w[u] = typename Amp16<T>::type{a.re, a.im};
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t ru = r0 + u * STRIDE;
            if (ru + lt < tsize) v[(gt | tile_offset(sp, ru)) >> vb] = w[u];
        }
    }
}

// Matrix entry i of a record, stored in the state's own precision.
template <typename T>
__device__ __forceinline__ cpx<T> gmat(const TileGate &G, int i) {
    const T *m = reinterpret_cast<const T *>(G.m);
    return cpx<T>{m[2 * i], m[2 * i + 1]};
}
template <typename T>
__device__ __forceinline__ T gre(const TileGate &G, int i) {
    return reinterpret_cast<const T *>(G.m)[2 * i];
}

// ------------------------------------------------ in-place register updates
// The amplitudes of a group stay in the registers they were loaded into for
// the whole sweep.  Every update is inline assembly whose outputs are tied
// to their inputs.  With TEST it checks its own enable bit, bit J of the
// uniform mask 'am' (a scalar test and branch inside the block); without,
// it runs unconditionally.  A gate path is then one straight run of such
// blocks, so the per-gate dispatch merges its paths with the group in place
// and without copies.  Each output first collects the terms that do not
// read its own input component and takes that component in one final FMA.
#define SV_SKIP_BEGIN "s_bitcmp1_b32 %[am], %[bit]\n\ts_cbranch_scc0 .Lsv_skip%=\n\t"
#define SV_SKIP_END "\n.Lsv_skip%=:"
#define SV_ASM(TEXT, OUTS, INS)                                                                    \
    if constexpr (TEST)                                                                            \
        asm volatile(SV_SKIP_BEGIN TEXT SV_SKIP_END : OUTS : INS, [am] "s"(am), [bit] "n"(J) : "scc"); \
    else                                                                                           \
        asm volatile(TEXT : OUTS : INS)
#define SV_ASM_NOIN(TEXT, OUTS)                                                                    \
    if constexpr (TEST)                                                                            \
        asm volatile(SV_SKIP_BEGIN TEXT SV_SKIP_END : OUTS : [am] "s"(am), [bit] "n"(J) : "scc");  \
    else                                                                                           \
        asm volatile(TEXT : OUTS)
#define SV_REG_ARITH(T, S)                                                                         \
    /* x <- d x */                                                                                 \
    template <int J, bool TEST>                                                                    \
    __device__ __forceinline__ void rmul(cpx<T> &x, cpx<T> d, uint32_t am) {                       \
        T t0, t1;                                                                                  \
        SV_ASM("v_mul_" S " %2, %5, %1\n\t"                                                        \
               "v_mul_" S " %3, %5, %0\n\t"                                                        \
               "v_fma_" S " %0, %4, %0, -%2\n\t"                                                   \
               "v_fma_" S " %1, %4, %1, %3",                                                       \
               SV_OUTS("+v"(x.re), "+v"(x.im), "=&v"(t0), "=&v"(t1)),                               \
               SV_INS("v"(d.re), "v"(d.im)));                                                      \
    }                                                                                              \
    /* (x0, x1) <- (g0 x0 + g1 x1, g2 x0 + g3 x1) */                                               \
    template <int J, bool TEST>                                                                    \
    __device__ __forceinline__ void rgen(cpx<T> &x0, cpx<T> &x1, const cpx<T> (&g)[4], uint32_t am) { \
        T ar, ai, br, bi;                                                                          \
        SV_ASM("v_mul_" S " %4, -%9, %1\n\t"                                                       \
               "v_fma_" S " %4, -%11, %3, %4\n\t"                                                  \
               "v_fma_" S " %4, %10, %2, %4\n\t"                                                   \
               "v_mul_" S " %5, %9, %0\n\t"                                                        \
               "v_fma_" S " %5, %11, %2, %5\n\t"                                                   \
               "v_fma_" S " %5, %10, %3, %5\n\t"                                                   \
               "v_mul_" S " %6, -%15, %3\n\t"                                                      \
               "v_fma_" S " %6, -%13, %1, %6\n\t"                                                  \
               "v_fma_" S " %6, %12, %0, %6\n\t"                                                   \
               "v_mul_" S " %7, %15, %2\n\t"                                                       \
               "v_fma_" S " %7, %13, %0, %7\n\t"                                                   \
               "v_fma_" S " %7, %12, %1, %7\n\t"                                                   \
               "v_fma_" S " %0, %8, %0, %4\n\t"                                                    \
               "v_fma_" S " %1, %8, %1, %5\n\t"                                                    \
               "v_fma_" S " %2, %14, %2, %6\n\t"                                                   \
               "v_fma_" S " %3, %14, %3, %7",                                                      \
               SV_OUTS("+v"(x0.re), "+v"(x0.im), "+v"(x1.re), "+v"(x1.im), "=&v"(ar), "=&v"(ai),    \
                       "=&v"(br), "=&v"(bi)),                                                      \
               SV_INS("v"(g[0].re), "v"(g[0].im), "v"(g[1].re), "v"(g[1].im), "v"(g[2].re),        \
                      "v"(g[2].im), "v"(g[3].re), "v"(g[3].im)));                                  \
    }                                                                                              \
    /* (x0, x1) <- (r0 x0 + r1 x1, r2 x0 + r3 x1), r real */                                       \
    template <int J, bool TEST>                                                                    \
    __device__ __forceinline__ void rreal(cpx<T> &x0, cpx<T> &x1, const T (&r)[4], uint32_t am) {  \
        T ar, ai, br, bi;                                                                          \
        SV_ASM("v_mul_" S " %4, %9, %2\n\t"                                                        \
               "v_mul_" S " %5, %9, %3\n\t"                                                        \
               "v_mul_" S " %6, %10, %0\n\t"                                                       \
               "v_mul_" S " %7, %10, %1\n\t"                                                       \
               "v_fma_" S " %0, %8, %0, %4\n\t"                                                    \
               "v_fma_" S " %1, %8, %1, %5\n\t"                                                    \
               "v_fma_" S " %2, %11, %2, %6\n\t"                                                   \
               "v_fma_" S " %3, %11, %3, %7",                                                      \
               SV_OUTS("+v"(x0.re), "+v"(x0.im), "+v"(x1.re), "+v"(x1.im), "=&v"(ar), "=&v"(ai),    \
                       "=&v"(br), "=&v"(bi)),                                                      \
               SV_INS("v"(r[0]), "v"(r[1]), "v"(r[2]), "v"(r[3])));                                \
    }                                                                                              \
    /* (x0, x1) <- (r0 x0 + i q1 x1, i q2 x0 + r3 x1), r, q real: w = {r0, q1, q2, r3} */          \
    template <int J, bool TEST>                                                                    \
    __device__ __forceinline__ void rrimag(cpx<T> &x0, cpx<T> &x1, const T (&w)[4], uint32_t am) { \
        T ar, ai, br, bi;                                                                          \
        SV_ASM("v_mul_" S " %4, -%9, %3\n\t"                                                       \
               "v_mul_" S " %5, %9, %2\n\t"                                                        \
               "v_mul_" S " %6, -%10, %1\n\t"                                                      \
               "v_mul_" S " %7, %10, %0\n\t"                                                       \
               "v_fma_" S " %0, %8, %0, %4\n\t"                                                    \
               "v_fma_" S " %1, %8, %1, %5\n\t"                                                    \
               "v_fma_" S " %2, %11, %2, %6\n\t"                                                   \
               "v_fma_" S " %3, %11, %3, %7",                                                      \
               SV_OUTS("+v"(x0.re), "+v"(x0.im), "+v"(x1.re), "+v"(x1.im), "=&v"(ar), "=&v"(ai),    \
                       "=&v"(br), "=&v"(bi)),                                                      \
               SV_INS("v"(w[0]), "v"(w[1]), "v"(w[2]), "v"(w[3])));                                \
    }                                                                                              \
    /* x <- dr x + a (dr real) */                                                                  \
    template <int J, bool TEST>                                                                    \
    __device__ __forceinline__ void rfin(cpx<T> &x, T dr, cpx<T> a, uint32_t am) {                 \
        SV_ASM("v_fma_" S " %0, %2, %0, %3\n\t"                                                    \
               "v_fma_" S " %1, %2, %1, %4",                                                       \
               SV_OUTS("+v"(x.re), "+v"(x.im)), SV_INS("v"(dr), "v"(a.re), "v"(a.im)));            \
    }
#define SV_OUTS(...) __VA_ARGS__
#define SV_INS(...) __VA_ARGS__
SV_REG_ARITH(float, "f32")
SV_REG_ARITH(double, "f64")
#undef SV_REG_ARITH

// Exchange two amplitudes held in registers, in place.
template <int J, bool TEST>
__device__ __forceinline__ void rswap(cpx<float> &a, cpx<float> &b, uint32_t am) {
    SV_ASM_NOIN("v_swap_b32 %0, %2\n\t"
                "v_swap_b32 %1, %3",
                SV_OUTS("+v"(a.re), "+v"(a.im), "+v"(b.re), "+v"(b.im)));
}
template <int J, bool TEST>
__device__ __forceinline__ void rswap(cpx<double> &a, cpx<double> &b, uint32_t am) {
    double t0, t1;
    SV_ASM_NOIN("v_mov_b64 %4, %0\n\t"
                "v_mov_b64 %5, %1\n\t"
                "v_mov_b64 %0, %2\n\t"
                "v_mov_b64 %1, %3\n\t"
                "v_mov_b64 %2, %4\n\t"
                "v_mov_b64 %3, %5",
                SV_OUTS("+v"(a.re), "+v"(a.im), "+v"(b.re), "+v"(b.im), "=&v"(t0), "=&v"(t1)));
}
// The same exchange in the lanes of 'lm' only (per-lane controls), complex64:
// two selects and a copy per component.
template <int J, bool TEST>
__device__ __forceinline__ void rswap_lanes(cpx<float> &a, cpx<float> &b, uint64_t lm, uint32_t am) {
    float t0, t1;
    SV_ASM("v_cndmask_b32 %4, %0, %2, %6\n\t"
           "v_cndmask_b32 %5, %1, %3, %6\n\t"
           "v_cndmask_b32 %2, %2, %0, %6\n\t"
           "v_cndmask_b32 %3, %3, %1, %6\n\t"
           "v_mov_b32 %0, %4\n\t"
           "v_mov_b32 %1, %5",
           SV_OUTS("+v"(a.re), "+v"(a.im), "+v"(b.re), "+v"(b.im), "=&v"(t0), "=&v"(t1)), SV_INS("s"(lm)));
}
// x <- 1, in place
__device__ __forceinline__ void rone(cpx<float> &x) {
    asm volatile("v_mov_b32 %0, 1.0\n\tv_mov_b32 %1, 0" : "+v"(x.re), "+v"(x.im));
}
__device__ __forceinline__ void rone(cpx<double> &x) {
    asm volatile("v_mov_b64 %0, 1.0\n\tv_mov_b64 %1, 0" : "+v"(x.re), "+v"(x.im));
}
#undef SV_OUTS
#undef SV_INS
#undef SV_ASM
#undef SV_ASM_NOIN
#undef SV_SKIP_BEGIN
#undef SV_SKIP_END

// Calls f(integral_constant<j>) for j = 0 .. N-1 with j in MASK.
template <uint32_t MASK, int N, int J = 0, typename F>
__device__ __forceinline__ void for_each_index(F &&f) {
    if constexpr (J < N) {
        if constexpr ((MASK >> J) & 1u) f(std::integral_constant<int, J>{});
        for_each_index<MASK, N, J + 1>(f);
    }
}

// f over the register indices of FULL (compile-time) that am enables: as
// unconditional updates when am is all of FULL (the common case: no control
// on a register position), else each behind its own enable test.  f takes
// the index and the TEST flag as integral constants.
template <uint32_t FULL, int N, typename F>
__device__ __forceinline__ void over_mask(uint32_t am, F &&f) {
    if (am == FULL) {
        for_each_index<FULL, N>([&](auto jc) { f(jc, std::false_type{}); });
    } else {
        for_each_index<FULL, N>([&](auto jc) { f(jc, std::true_type{}); });
    }
}

// Register indices of a group of 2^W whose bits in 'clear' are 0.
template <int W>
constexpr uint32_t index_set(uint32_t clear) {
    uint32_t m = 0;
    for (int j = 0; j < (1 << W); ++j)
        if (!(j & clear)) m |= 1u << j;
    return m;
}

// The leading 96 bytes of a record: the header and the matrix entries a
// one-qubit record uses, read with one batch of scalar loads per gate.
struct GateHot {
    int32_t kind, b0, b1;
    uint32_t lane, amask, pad; // pad: the record's packed size (TileGate::size)
    uint64_t cout;
    uint32_t m[16];
};
static_assert(offsetof(TileGate, m) == offsetof(GateHot, m), "record layout");
static_assert(offsetof(TileGate, size) == offsetof(GateHot, pad), "record layout");
template <typename T>
__device__ __forceinline__ cpx<T> hmat(const GateHot &h, int i) {
    const T *m = reinterpret_cast<const T *>(h.m);
    return cpx<T>{m[2 * i], m[2 * i + 1]};
}
template <typename T>
__device__ __forceinline__ T hre(const GateHot &h, int i) {
    return reinterpret_cast<const T *>(h.m)[2 * i];
}

#define SV_J constexpr int j = decltype(jc)::value; constexpr bool t = decltype(tc)::value
// One-qubit gate on register position P (pairs j, j | 2^P).  A lane whose
// group fails the per-lane controls applies the identity instead.
template <typename T, int W, int P>
__device__ __forceinline__ void sweep_1q(cpx<T> (&v)[1 << W], bool ok, const GateHot &h, uint32_t am) {
    constexpr int D = 1 << W;
    constexpr uint32_t PAIRS = index_set<W>(1u << P);
    const int kind = h.kind;
    if (kind == SK_GEN) {
        const cpx<T> one{T(1), T(0)}, zero{T(0), T(0)};
        const cpx<T> g[4] = {ok ? hmat<T>(h, 0) : one, ok ? hmat<T>(h, 1) : zero, ok ? hmat<T>(h, 2) : zero,
                             ok ? hmat<T>(h, 3) : one};
        over_mask<PAIRS, D>(am, [&](auto jc, auto tc) { SV_J; rgen<j, t>(v[j], v[j | (1 << P)], g, am); });
    } else if (kind == SK_REAL) {
        const T r[4] = {ok ? hre<T>(h, 0) : T(1), ok ? hre<T>(h, 1) : T(0), ok ? hre<T>(h, 2) : T(0),
                        ok ? hre<T>(h, 3) : T(1)};
        over_mask<PAIRS, D>(am, [&](auto jc, auto tc) { SV_J; rreal<j, t>(v[j], v[j | (1 << P)], r, am); });
    } else if (kind == SK_RIMAG) {
        const cpx<T> m1 = hmat<T>(h, 1), m2 = hmat<T>(h, 2);
        const T w[4] = {ok ? hre<T>(h, 0) : T(1), ok ? m1.im : T(0), ok ? m2.im : T(0), ok ? hre<T>(h, 3) : T(1)};
        over_mask<PAIRS, D>(am, [&](auto jc, auto tc) { SV_J; rrimag<j, t>(v[j], v[j | (1 << P)], w, am); });
    } else if (kind == SK_SWAP) {
        if (h.lane == 0) {
            over_mask<PAIRS, D>(am, [&](auto jc, auto tc) { SV_J; rswap<j, t>(v[j], v[j | (1 << P)], am); });
        } else if constexpr (std::is_same<T, float>::value) { // per-lane controls
            const uint64_t lm = __builtin_amdgcn_ballot_w64(ok);
            over_mask<PAIRS, D>(am, [&](auto jc, auto tc) {
                SV_J;
                rswap_lanes<j, t>(v[j], v[j | (1 << P)], lm, am);
            });
        }
    } else { // SK_DIAGR: amplitude j takes d1 if its bit P is set, else d0
        const cpx<T> one{T(1), T(0)};
        const cpx<T> d0 = ok ? hmat<T>(h, 0) : one, d1 = ok ? hmat<T>(h, 1) : one;
        constexpr uint32_t UP = index_set<W>(0) & ~PAIRS;
        auto f = [&](auto jc, auto tc) { SV_J; rmul<j, t>(v[j], ((j >> P) & 1) ? d1 : d0, am); };
        if (am == UP) for_each_index<UP, D>([&](auto jc) { f(jc, std::false_type{}); }); // phase gate
        else over_mask<index_set<W>(0), D>(am, f);
    }
}

// Two-qubit gate on register positions P < Q.  Lanes failing the per-lane
// controls add nothing and keep their own terms (identity).
template <typename T, int W, int P, int Q>
__device__ __forceinline__ void sweep_2q(cpx<T> (&v)[1 << W], bool ok, const TileGate &G, uint32_t am) {
    constexpr uint32_t QUADS = index_set<W>((1u << P) | (1u << Q));
    T dr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) dr[r] = ok ? gre<T>(G, 5 * r) : T(1);
    for_each_index<QUADS, (1 << W)>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int i1 = j | (1 << P), i2 = j | (1 << Q), i3 = j | (1 << P) | (1 << Q);
        const cpx<T> x[4] = {v[j], v[i1], v[i2], v[i3]};
        cpx<T> a[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const cpx<T> d = gmat<T>(G, 5 * r);
            cpx<T> acc{-d.im * x[r].im, d.im * x[r].re};
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c != r) acc = cfma(gmat<T>(G, 4 * r + c), x[c], acc);
            a[r] = ok ? acc : cpx<T>{T(0), T(0)};
        }
        // every read of the old amplitudes happens before the first of them
        // is overwritten in place
        asm volatile("" : "+v"(a[0].re), "+v"(a[0].im), "+v"(a[1].re), "+v"(a[1].im), "+v"(a[2].re),
                     "+v"(a[2].im), "+v"(a[3].re), "+v"(a[3].im));
        rfin<j, true>(v[j], dr[0], a[0], am);
        rfin<j, true>(v[i1], dr[1], a[1], am);
        rfin<j, true>(v[i2], dr[2], a[2], am);
        rfin<j, true>(v[i3], dr[3], a[3], am);
    });
}

// diag(d0, d1) on tile bit b0 outside the registers: one factor per lane.
template <typename T, int W>
__device__ __forceinline__ void sweep_diag_lane(cpx<T> (&v)[1 << W], uint32_t gb, bool ok, const GateHot &h,
                                                uint32_t am) {
    const bool up = (gb >> h.b0) & 1u;
    const cpx<T> d0 = hmat<T>(h, 0), d1 = hmat<T>(h, 1);
    const cpx<T> d = ok ? (up ? d1 : d0) : cpx<T>{T(1), T(0)};
    over_mask<index_set<W>(0), (1 << W)>(am, [&](auto jc, auto tc) { SV_J; rmul<j, t>(v[j], d, am); });
}
#undef SV_J

// Phase factors gathered per lane (SK_PHASE) until a flush applies them:
// f[W] multiplies every amplitude of the group, f[p] those with register
// bit p set.
template <typename T, int W>
struct PhaseAcc {
    cpx<T> f[W + 1];
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int s = 0; s <= W; ++s) f[s] = cpx<T>{T(1), T(0)};
    }
};

template <typename T, int W, int S = 0>
__device__ __forceinline__ void phase_gather(PhaseAcc<T, W> &acc, int slot, cpx<T> d) {
    if constexpr (S == W) {
        rmul<0, false>(acc.f[W], d, 0u);
    } else {
        if (slot == S) rmul<0, false>(acc.f[S], d, 0u);
        else phase_gather<T, W, S + 1>(acc, slot, d);
    }
}

// v[j] *= f[p] for the register indices j with bit p set, p = B .. W-1,
// where slot p is in 'used' (one uniform branch per slot around untested
// updates)
template <typename T, int W, int B = 0>
__device__ __forceinline__ void phase_flush_bits(cpx<T> (&v)[1 << W], PhaseAcc<T, W> &acc, uint32_t used) {
    if constexpr (B < W) {
        constexpr uint32_t UP = index_set<W>(0) & ~index_set<W>(1u << B);
        if ((used >> B) & 1u) {
            for_each_index<UP, (1 << W)>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                rmul<j, false>(v[j], acc.f[B], 0u);
            });
            rone(acc.f[B]);
        }
        phase_flush_bits<T, W, B + 1>(v, acc, used);
    }
}

// v[j] *= f[W] * prod_{p in j} f[p] over the slots in 'used'; the used
// slots are reset to 1.
template <typename T, int W>
__device__ __forceinline__ void phase_flush(cpx<T> (&v)[1 << W], PhaseAcc<T, W> &acc, uint32_t used) {
    if ((used >> W) & 1u) {
        for_each_index<index_set<W>(0), (1 << W)>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            rmul<j, false>(v[j], acc.f[W], 0u);
        });
        rone(acc.f[W]);
    }
    phase_flush_bits<T, W>(v, acc, used);
}

// Apply one record to a group held in registers; gb holds the group's own
// tile bits, base is the global index of the tile's amplitude 0 (the
// record's controls outside the tile hold for the whole tile or not at all:
// then its enable mask is 0).  Every branch of the dispatch ends in the
// updates of one path (no empty path), so that the paths merge with the
// group in its registers.  Two-qubit records are handled only by the TWOQ
// instances: their partial sums, which read the old amplitudes while others
// are rewritten, keep the compiler from holding the group in place across
// the dispatch, so passes without them use kernels without that path.
// PHASES = false compiles the gathered-phase kinds out, for streams that
// carry none (the adjoint's reverse passes); LPH compiles in the lane-bit
// phase lists (always for complex128; complex64 streams carry them only for
// the kernel instances launched with them).
template <typename T, int W, bool TWOQ, bool PHASES = true, bool LPH = std::is_same<T, double>::value>
__device__ __forceinline__ void sweep_gate_h(cpx<T> (&v)[1 << W], PhaseAcc<T, W> &acc, uint32_t gb,
                                             const GateHot &h, const TileGate &G, uint64_t base) {
    const int kind = h.kind;
    const bool ok = (gb & h.lane) == h.lane;
    const uint32_t am = __builtin_amdgcn_readfirstlane((base & h.cout) == h.cout ? h.amask : 0u);
    if (PHASES && kind == SK_PHASE) {
        // tile factor: product of the entries' phases whose condition holds
        const char *e = reinterpret_cast<const char *>(&G) + kRecordHead;
        cpx<T> u{T(1), T(0)};
        // the entry's phase or 1, chosen on the scalar unit: no branch, so
        // the loads of consecutive entries issue together
#pragma unroll 4
        for (int i = 0; i < h.b1; ++i) {
            const char *ei = e + (size_t)i * (8 + sizeof(cpx<T>));
            const uint64_t c = *reinterpret_cast<const uint64_t *>(ei);
            const cpx<T> ph = *reinterpret_cast<const cpx<T> *>(ei + 8);
            const bool on = (base & c) == c;
            u = cmul(u, cpx<T>{on ? ph.re : T(1), on ? ph.im : T(0)});
        }
        phase_gather<T, W>(acc, h.b0, ok ? u : cpx<T>{T(1), T(0)});
    } else if (PHASES && kind == SK_PTAB) {
        // tile factor: one table entry per window of the tile's index bits
        // (uniform addresses, no branch: scalar loads issued together)
        const char *tab = reinterpret_cast<const char *>(&G) + kRecordHead + kPtabDesc;
        cpx<T> f[kPtabWindows];
#pragma unroll
        for (int w = 0; w < kPtabWindows; ++w) {
            const uint32_t x = (uint32_t)(base >> h.m[4 * w]) & h.m[4 * w + 1];
            f[w] = *reinterpret_cast<const cpx<T> *>(tab + h.m[4 * w + 2] + (size_t)x * sizeof(cpx<T>));
        }
        cpx<T> u = f[0];
#pragma unroll
        for (int w = 1; w < kPtabWindows; ++w) u = cmul(u, f[w]);
        phase_gather<T, W>(acc, h.b0, ok ? u : cpx<T>{T(1), T(0)});
    } else if (PHASES && LPH && kind == SK_LPH) {
        // per-lane factor: the phases of the lane bits its group holds
        const char *e = reinterpret_cast<const char *>(&G) + kRecordHead;
        cpx<T> u{T(1), T(0)};
#pragma unroll 2
        for (int i = 0; i < h.b1; ++i) {
            const char *ei = e + (size_t)i * (8 + sizeof(cpx<T>));
            const uint32_t bm = *reinterpret_cast<const uint32_t *>(ei);
            const cpx<T> ph = *reinterpret_cast<const cpx<T> *>(ei + 8);
            const bool on = (gb & bm) != 0u;
            u = cmul(u, cpx<T>{on ? ph.re : T(1), on ? ph.im : T(0)});
        }
        phase_gather<T, W>(acc, h.b0, u);
    } else if (PHASES && kind == SK_FLUSH) {
        phase_flush<T, W>(v, acc, am);
    } else if (kind == SK_DIAG) {
        sweep_diag_lane<T, W>(v, gb, ok, h, am);
    } else if (TWOQ && W >= 2 && kind == SK_2Q) {
        if constexpr (TWOQ && W >= 2) {
            const int pq = h.b0 * 4 + h.b1;
            if constexpr (W == 2) {
                sweep_2q<T, W, 0, 1>(v, ok, G, am);
            } else if constexpr (W == 3) {
                if (pq == 1) sweep_2q<T, W, 0, 1>(v, ok, G, am);
                else if (pq == 2) sweep_2q<T, W, 0, 2>(v, ok, G, am);
                else sweep_2q<T, W, 1, 2>(v, ok, G, am);
            } else {
                if (pq == 1) sweep_2q<T, W, 0, 1>(v, ok, G, am);
                else if (pq == 2) sweep_2q<T, W, 0, 2>(v, ok, G, am);
                else if (pq == 6) sweep_2q<T, W, 1, 2>(v, ok, G, am);
                else if (pq == 3) sweep_2q<T, W, 0, 3>(v, ok, G, am);
                else if (pq == 7) sweep_2q<T, W, 1, 3>(v, ok, G, am);
                else sweep_2q<T, W, 2, 3>(v, ok, G, am);
            }
        }
    } else {
        const int p = h.b0;
        if constexpr (W == 1) {
            sweep_1q<T, W, 0>(v, ok, h, am);
        } else if constexpr (W == 2) {
            if (p == 0) sweep_1q<T, W, 0>(v, ok, h, am);
            else sweep_1q<T, W, 1>(v, ok, h, am);
        } else if constexpr (W == 3) {
            if (p == 0) sweep_1q<T, W, 0>(v, ok, h, am);
            else if (p == 1) sweep_1q<T, W, 1>(v, ok, h, am);
            else sweep_1q<T, W, 2>(v, ok, h, am);
        } else {
            if (p == 0) sweep_1q<T, W, 0>(v, ok, h, am);
            else if (p == 1) sweep_1q<T, W, 1>(v, ok, h, am);
            else if (p == 2) sweep_1q<T, W, 2>(v, ok, h, am);
            else sweep_1q<T, W, 3>(v, ok, h, am);
        }
    }
}

template <typename T, int W, bool TWOQ, bool LPH = std::is_same<T, double>::value>
__device__ __forceinline__ void sweep_gate_t(cpx<T> (&v)[1 << W], PhaseAcc<T, W> &acc, uint32_t gb,
                                             const TileGate &G, uint64_t base) {
    const GateHot h = *reinterpret_cast<const GateHot *>(&G);
    sweep_gate_h<T, W, TWOQ, true, LPH>(v, acc, gb, h, G, base);
}

// Apply the ng packed records starting at rp to one register group.  (A
// variant that loads record i+1's head while record i is applied needs a
// second set of scalar registers for it and spills.)
template <typename T, int W, bool TWOQ, bool LPH = std::is_same<T, double>::value>
__device__ __forceinline__ void run_records(cpx<T> (&v)[1 << W], PhaseAcc<T, W> &acc, uint32_t gb,
                                            const char *__restrict__ rp, int ng, uint64_t base) {
    for (int gi = 0; gi < ng; ++gi) {
        const TileGate &G = *reinterpret_cast<const TileGate *>(rp);
        // advance before the gate: its inline assembly would make the
        // compiler read the size again after it
        rp += G.size;
        sweep_gate_t<T, W, TWOQ, LPH>(v, acc, gb, G, base);
    }
}

// Tile bits of the sweep's register positions: gb (the group's own bits,
// per lane) spreads group index g around them.
template <int W>
__device__ __forceinline__ uint32_t group_bits(const TileSweep &S, uint32_t g) {
#pragma unroll
    for (int b = 0; b < W; ++b) {
        const uint32_t low = (1u << S.qpos[b]) - 1u;
        g = (g & low) | ((g & ~low) << 1);
    }
    return g;
}

// LDS offsets (swizzled) of the register indices' bits, uniform per sweep.
template <typename T, int W>
__device__ __forceinline__ void register_offsets(const TileSweep &S, uint32_t (&PF)[1 << W]) {
#pragma unroll
    for (int j = 0; j < (1 << W); ++j) {
        uint32_t f = 0;
#pragma unroll
        for (int b = 0; b < W; ++b)
            if ((j >> b) & 1) f |= 1u << S.qpos[b];
        PF[j] = lds_phys<T>(f);
    }
}

// Apply the sweeps of one pass to the tile in LDS.  'base' is the global
// index of the tile's local amplitude 0 (for controls outside the tile).
// Caller synchronises before (tile loaded); every sweep ends with a barrier.
// The LDS swizzle is linear over XOR and a group's bits are disjoint from
// the register bits, so amplitude j of the group sits at
// lds_phys(gb) ^ lds_phys(register bits of j).
template <typename T, int W, bool TWOQ>
__device__ void tile_run_sweeps(cpx<T> *lds, int m, uint64_t base, const TileSweep *__restrict__ sweeps,
                                int n_sweeps, const char *__restrict__ recs) {
    constexpr int D = 1 << W;
    const uint32_t n_groups = (1u << m) >> W;
    for (int si = 0; si < n_sweeps; ++si) {
        const TileSweep &S = sweeps[si];
        const int ng = S.n_gates;
        const char *r0 = recs + S.rec_off;
        uint32_t PF[D];
        register_offsets<T, W>(S, PF);
        for (uint32_t g = threadIdx.x; g < n_groups; g += blockDim.x) {
            const uint32_t gb = group_bits<W>(S, g);
            const uint32_t pg = lds_phys<T>(gb);
            cpx<T> v[D];
            uint32_t addr[D];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                addr[j] = pg ^ PF[j];
                v[j] = lds[addr[j]];
            }
            PhaseAcc<T, W> acc;
            acc.init();
            const char *rp = r0;
            for (int gi = 0; gi < ng; ++gi) {
                const TileGate &G = *reinterpret_cast<const TileGate *>(rp);
                // advance before the gate: its inline assembly would make the
                // compiler read the size again after it
                rp += G.size;
                sweep_gate_t<T, W, TWOQ>(v, acc, gb, G, base);
            }
#pragma unroll
            for (int j = 0; j < D; ++j) lds[addr[j]] = v[j];
        }
        __syncthreads();
    }
}

} // namespace sv
